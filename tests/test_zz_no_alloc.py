"""tc_forces_noalloc, the allocation-free variant of tc_build + tc_moments +
tc_forces, called through the C ABI: its outputs must equal those of the
three calls bit for bit (the same kernels run in the same order), on two calls
in a row, the second with a smaller input, and sizes beyond its static
scratch must be refused before anything is written."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _reference(L, m, p, mm, n, dt, theta, eps, walk, out_dt, stream):
    h = ctypes.c_void_p()
    acc = torch.empty((n, 3), dtype=out_dt, device="cuda:0")
    pot = torch.empty((n,), dtype=out_dt, device="cuda:0")
    assert L.tc_build(_ptr(p), _ptr(mm), n, dt, stream, ctypes.byref(h)) == m.TC_OK, L.tc_last_error()
    assert L.tc_moments(h, stream) == m.TC_OK, L.tc_last_error()
    assert L.tc_forces(h, theta, eps, 1.0, walk, 0, _ptr(acc), _ptr(pot), stream) == m.TC_OK, L.tc_last_error()
    torch.cuda.synchronize()
    L.tc_tree_free(h)
    return acc.cpu(), pot.cpu()


@pytest.mark.parametrize("walk", ["f32c", "f64"])
def test_noalloc_matches_handle_path(walk):
    from paper_2412_01733_amd import _lib as m
    L = m.load()
    dev = torch.device("cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    mode = m.TC_WALK_F32C if walk == "f32c" else m.TC_WALK_F64
    out_dt = torch.float32 if walk == "f32c" else torch.float64
    # two calls in a row on the same static scratch, the second smaller
    for n, seed, dtype, theta, eps in ((1 << 18, 31, np.float32, 0.5, 0.01), (5000, 32, np.float64, 0.7, 0.02)):
        print("noalloc case", walk, n, seed, flush=True)
        pos, mass = workloads.plummer(n, seed, dtype=dtype)
        p = torch.from_numpy(pos).to(dev)
        mm = torch.from_numpy(mass).to(dev)
        dt = m.TC_F32 if dtype == np.float32 else m.TC_F64
        acc = torch.full((n, 3), float("nan"), dtype=out_dt, device=dev)
        pot = torch.full((n,), float("nan"), dtype=out_dt, device=dev)
        st = L.tc_forces_noalloc(_ptr(p), _ptr(mm), n, dt, theta, eps, 1.0, mode, _ptr(acc), _ptr(pot), stream)
        assert st == m.TC_OK, L.tc_last_error()
        torch.cuda.synchronize()
        ra, rp = _reference(L, m, p, mm, n, dt, theta, eps, mode, out_dt, stream)
        a, ph = acc.cpu(), pot.cpu()
        assert torch.equal(a, ra), float((a - ra).abs().max())
        assert torch.equal(ph, rp), float((ph - rp).abs().max())


def test_noalloc_refuses_sizes_beyond_its_scratch():
    from paper_2412_01733_amd import _lib as m
    L = m.load()
    dev = torch.device("cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n = (1 << 18) + 1
    p = torch.zeros((n, 3), dtype=torch.float32, device=dev)
    mm = torch.ones(n, dtype=torch.float32, device=dev)
    acc = torch.full((n, 3), 7.0, dtype=torch.float32, device=dev)
    st = L.tc_forces_noalloc(_ptr(p), _ptr(mm), n, m.TC_F32, 0.5, 0.01, 1.0, m.TC_WALK_F32C, _ptr(acc), None, stream)
    assert st == m.TC_ERR_INVALID and b"outside" in L.tc_last_error()
    torch.cuda.synchronize()
    assert bool((acc == 7.0).all())
    # empty input is valid and writes nothing
    st = L.tc_forces_noalloc(None, None, 0, m.TC_F32, 0.5, 0.01, 1.0, m.TC_WALK_F32C, None, None, stream)
    assert st == m.TC_OK


def test_noalloc_refuses_a_tree_beyond_its_scratch():
    """2^17 close pairs: each pair shares its cell down to level ~19, so the
    octree has ~20 nodes per pair, more than the static array holds; the call
    is refused after the node count, before any node kernel or output write."""
    from paper_2412_01733_amd import _lib as m
    L = m.load()
    dev = torch.device("cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n = 1 << 18
    g = np.random.default_rng(5)
    base = g.random((n // 2, 3))
    pos = np.empty((n, 3))
    pos[0::2] = base
    pos[1::2] = base + 3e-6
    p = torch.from_numpy(pos).to(dev)
    mm = torch.full((n,), 1.0 / n, dtype=torch.float64, device=dev)
    acc = torch.full((n, 3), 7.0, dtype=torch.float64, device=dev)
    st = L.tc_forces_noalloc(_ptr(p), _ptr(mm), n, m.TC_F64, 0.5, 0.01, 1.0, m.TC_WALK_F64, _ptr(acc), None, stream)
    assert st == m.TC_ERR_OVERFLOW, (st, L.tc_last_error())
    assert b"static scratch" in L.tc_last_error()
    torch.cuda.synchronize()
    assert bool((acc == 7.0).all())
