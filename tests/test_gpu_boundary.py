"""The Python binding and the C ABI at their edges, on the GPU: caller
buffers are checked before any launch (a wrong shape, dtype, layout or a
strided view that would be updated through a copy raises and leaves the
buffers untouched), the library's buffers come from torch's caching
allocator, and the walk status is clean after every walk kind and reported
when set."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _set(n=3000, seed=41, dtype=np.float32):
    pos, m = workloads.plummer(n, seed, dtype=dtype)
    return torch.from_numpy(pos).to(dev()), torch.from_numpy(m).to(dev())


def test_leapfrog_refuses_a_strided_position_view():
    """A position view that is not contiguous would be drifted through a
    temporary copy, leaving the caller's positions unchanged: refused."""
    import paper_2412_01733_amd as tc
    p, m = _set()
    n = p.shape[0]
    state = torch.cat([p, torch.zeros_like(p)], dim=1)  # [n, 6]: positions are a strided view
    pos_view = state[:, :3]
    assert not pos_view.is_contiguous()
    vel = torch.zeros_like(p)
    acc = torch.zeros((n, 3), dtype=torch.float32, device=dev())
    before = state.clone()
    with pytest.raises(ValueError, match="pos must be contiguous"):
        tc.leapfrog_step(pos_view, vel, m, acc, 1e-3, 0.5, 0.01)
    torch.cuda.synchronize()
    assert torch.equal(state, before) and bool((vel == 0).all()) and bool((acc == 0).all())


@pytest.mark.parametrize("bad", ["dtype", "shape", "strided"])
def test_forces_out_buffers_checked(bad):
    import paper_2412_01733_amd as tc
    p, m = _set()
    n = p.shape[0]
    t = tc.Tree().build(p, m).moments()
    acc = torch.full((n, 3), 5.0, dtype=torch.float32, device=dev())
    pot = torch.full((n,), 5.0, dtype=torch.float32, device=dev())
    if bad == "dtype":  # an FP32 buffer handed to the FP64 walk
        exc, kw = TypeError, dict(walk="f64", out=(acc, pot))
    elif bad == "shape":
        exc, kw = ValueError, dict(walk="f32c", out=(acc[: n - 1], pot))
    else:
        exc, kw = ValueError, dict(walk="f32c", out=(acc, torch.full((2 * n,), 5.0, device=dev())[::2]))
    with pytest.raises(exc):
        t.forces(0.5, 0.01, **kw)
    torch.cuda.synchronize()
    assert bool((acc == 5.0).all()) and bool((pot == 5.0).all())


def test_leapfrog_buffers_checked():
    import paper_2412_01733_amd as tc
    p, m = _set()
    n = p.shape[0]
    vel = torch.zeros_like(p)
    with pytest.raises(TypeError):  # FP64 acc for the FP32 walk
        tc.leapfrog_step(p, vel, m, torch.zeros((n, 3), dtype=torch.float64, device=dev()), 1e-3, 0.5, 0.01)
    with pytest.raises(ValueError):  # short potential
        tc.leapfrog_step(p, vel, m, torch.zeros((n, 3), device=dev()), 1e-3, 0.5, 0.01,
                         pot=torch.zeros(n - 1, device=dev()))


def test_backward_gradient_shapes_checked():
    import paper_2412_01733_amd as tc
    p, m = _set()
    n = p.shape[0]
    t = tc.Tree().build(p, m).moments()
    t.forces(0.5, 0.01)
    with pytest.raises(ValueError):
        t.backward(torch.ones((n - 1, 3), device=dev()))
    with pytest.raises(ValueError):
        t.backward(torch.ones((n, 3), device=dev()), torch.ones(n + 1, device=dev()))


def test_buffers_come_from_torch_allocator():
    import paper_2412_01733_amd as tc
    tc.treecode.bind_torch_allocator()
    p, m = _set(200_000, 42)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    t = tc.Tree().build(p, m).moments()
    t.forces(0.5, 0.01)
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - before
    # keys, sort buffers, particle records and the node arrays: well over 50 B per particle
    assert held > 50 * 200_000, held
    t.free()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before < held


@pytest.mark.parametrize("walk", ["f32c", "f64"])
def test_walk_status_clean(walk):
    """Forward, counted, storing and adjoint walks leave the status word clear
    (tc_tree_stats would report an overflow or a corrupt tree otherwise), and
    a rebuild on the handle reads it at its synchronisation."""
    import paper_2412_01733_amd as tc
    p, m = _set(20000, 43)
    t = tc.Tree().build(p, m).moments()
    for kw in (dict(), dict(count=True), dict(store_lists=True)):
        acc, _ = t.forces(0.5, 0.01, walk=walk, **kw)
        t.stats()  # raises TreecodeError on a non-zero status
    t.backward(torch.ones_like(acc))
    t.stats()
    t.forces(0.5, 0.01, walk=walk)
    t.build(p, m)  # checks the previous walk's status at its sync


@pytest.mark.parametrize("bits,status,word", [(1, 5, "overflowed"), (2, 3, "corrupt"), (3, 5, "overflowed")])
def test_walk_status_reported(bits, status, word):
    """The walk status word reaches the caller: set from the host (as a walk
    whose stack push was refused, bit 0, or that met a node with more than 8
    children, bit 1, would leave it; no kernel is made to misbehave), it is
    reported once by tc_tree_stats, and by the next tc_build when a walk's
    status is pending; the failed build leaves the handle unbuilt, and a
    rebuild clears the word."""
    import paper_2412_01733_amd as tc
    from paper_2412_01733_amd import _lib as L
    p, m = _set(20000, 44)
    t = tc.Tree().build(p, m).moments()
    t.forces(0.5, 0.01)
    lib = L.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev()).cuda_stream)
    L.check(lib.tc_tree_set_walk_status(t._h, bits, stream))
    with pytest.raises(L.TreecodeError) as e:
        t.stats()
    assert e.value.status == status and word in str(e.value), str(e.value)
    t.stats()  # reported once
    L.check(lib.tc_tree_set_walk_status(t._h, bits, stream))
    with pytest.raises(L.TreecodeError) as e:
        t.build(p, m)
    assert e.value.status == status and word in str(e.value), str(e.value)
    with pytest.raises(L.TreecodeError) as e:
        t.forces(0.5, 0.01)
    assert e.value.status == L.TC_ERR_STATE
    t.build(p, m).moments()
    acc, _ = t.forces(0.5, 0.01)
    t.stats()
    assert torch.isfinite(acc).all()
    assert lib.tc_tree_set_walk_status(t._h, 4, stream) == L.TC_ERR_INVALID


def test_default_allocator_is_stream_ordered():
    """With no allocator installed the library takes its buffers from the
    device's default memory pool in stream order (hipMallocAsync /
    hipFreeAsync on the call's stream): a handle built, grown (a larger
    rebuild frees and re-allocates on the stream) and freed through the C ABI
    gives results bitwise equal to the same calls on torch's pool."""
    import paper_2412_01733_amd as tc
    from paper_2412_01733_amd import _lib as L
    lib = L.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev()).cuda_stream)
    sets = [_set(n, 45 + i) for i, n in enumerate((5000, 60000))]

    def run(h):
        outs = []
        for p, m in sets:
            acc = torch.empty((p.shape[0], 3), dtype=torch.float32, device=dev())
            pot = torch.empty(p.shape[0], dtype=torch.float32, device=dev())
            L.check(lib.tc_build(ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(m.data_ptr()), p.shape[0],
                                 L.TC_F32, stream, ctypes.byref(h)))
            L.check(lib.tc_moments(h, stream))
            L.check(lib.tc_forces(h, 0.5, 0.01, 1.0, L.TC_WALK_F32C, 0, ctypes.c_void_p(acc.data_ptr()),
                                  ctypes.c_void_p(pot.data_ptr()), stream))
            outs.append((acc, pot))
        torch.cuda.synchronize()
        return outs

    try:
        assert lib.tc_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None) == L.TC_OK  # the default
        h = ctypes.c_void_p()
        got = run(h)
        lib.tc_tree_free(h)
    finally:
        tc.treecode.bind_torch_allocator()
    h = ctypes.c_void_p()
    ref = run(h)
    lib.tc_tree_free(h)
    for (a, p), (ra, rp) in zip(got, ref):
        assert torch.equal(a, ra) and torch.equal(p, rp)
