"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/treecode.h declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2412_01733_amd import _lib
    return _lib


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "treecode.h")).read()
    return sorted(set(re.findall(r"\b(tc_[a-z_]+)\s*\(", text)) - {"tc_alloc_fn", "tc_free_fn"})


def test_header_and_binding_agree():
    assert sorted(_lib().EXPORTS) == declared_symbols()


def test_stats_struct_layout_matches_header(tmp_path):
    """The binding's tc_stats mirrors the C struct byte for byte (compiled with gcc)."""
    import subprocess
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "treecode.h"\n'
                   'int main(void){printf("%zu %zu %zu", sizeof(tc_stats), offsetof(tc_stats, stage_ms),'
                   ' offsetof(tc_stats, lists_stored)); printf(" %zu", offsetof(tc_stats, list_bytes)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    size, off_stage, off_lists, off_bytes = map(int, subprocess.check_output([str(exe)]).split())
    S = _lib().TcStats
    assert ctypes.sizeof(S) == size
    assert S.stage_ms.offset == off_stage and S.lists_stored.offset == off_lists
    assert S.list_bytes.offset == off_bytes


def test_library_exports_every_symbol():
    L = _lib().load()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert L.tc_version().decode().startswith("treecode-gfx950")


def test_argument_validation_without_device():
    m = _lib()
    L = m.load()
    h = ctypes.c_void_p()
    assert L.tc_build(None, None, 5, m.TC_F32, None, ctypes.byref(h)) == m.TC_ERR_INVALID
    assert b"non-NULL" in L.tc_last_error()
    assert L.tc_build(None, None, -1, m.TC_F32, None, ctypes.byref(h)) == m.TC_ERR_INVALID
    assert L.tc_build(None, None, 1 << 31, m.TC_F32, None, ctypes.byref(h)) == m.TC_ERR_INVALID
    assert L.tc_build(None, None, 0, 7, None, ctypes.byref(h)) == m.TC_ERR_INVALID
    assert L.tc_build(None, None, 0, m.TC_F32, None, None) == m.TC_ERR_INVALID
    assert L.tc_moments(None, None) == m.TC_ERR_INVALID
    assert L.tc_forces(None, 0.5, 0.01, 1.0, 0, 0, None, None, None) == m.TC_ERR_INVALID
    assert L.tc_forces_backward(None, None, None, None, None, None) == m.TC_ERR_INVALID
    assert L.tc_tree_stats(None, None, None) == m.TC_ERR_INVALID
    assert L.tc_tree_set_timing(None, 1) == m.TC_ERR_INVALID
    assert L.tc_tree_set_walk_status(None, 1, None) == m.TC_ERR_INVALID
    assert L.tc_tree_export(None, None, None, None, None, None, None, None, None) == m.TC_ERR_INVALID
    assert L.tc_interaction_counts(None, None, None) == m.TC_ERR_INVALID
    assert L.tc_tree_target_order(None, None, None) == m.TC_ERR_INVALID
    L.tc_tree_free(None)  # no-op


def test_allocator_must_be_paired():
    m = _lib()
    L = m.load()
    alloc = m.ALLOC_FN(lambda b, s, c: None)
    assert L.tc_set_allocator(alloc, m.FREE_FN(), None) == m.TC_ERR_INVALID
    assert L.tc_set_allocator(m.ALLOC_FN(), m.FREE_FN(), None) == m.TC_OK


def test_no_device_is_reported(monkeypatch):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    m = _lib()
    L = m.load()
    h = ctypes.c_void_p()
    assert L.tc_build(None, None, 0, m.TC_F32, None, ctypes.byref(h)) == m.TC_ERR_DEVICE
    assert b"device" in L.tc_last_error()


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2412_01733_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "treecode_oracle" not in text, f
