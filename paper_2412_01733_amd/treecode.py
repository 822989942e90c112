"""Python binding of libtreecode: argument marshalling only.

torch supplies device memory and the stream; every step of the computation
runs in the library's HIP kernels.  Functions here mirror the C ABI names:

  Tree.build / Tree.moments / Tree.forces   -> tc_build / tc_moments / tc_forces
  Tree.backward, TreeForces (autograd)      -> tc_forces_backward
  leapfrog_step                             -> tc_leapfrog_step
  forces(pos, mass, theta, eps, ...)        -> build + moments + forces
"""
from __future__ import annotations

import atexit
import ctypes
import threading
import weakref

import torch

from . import _lib
from ._lib import check

_WALKS = {"f32c": _lib.TC_WALK_F32C, "f64": _lib.TC_WALK_F64}
_DT = {torch.float32: _lib.TC_F32, torch.float64: _lib.TC_F64}


# torch's caching allocator serves every buffer the library owns (tc_set_allocator).
# A block is handed back to the pool of the stream it was allocated on, so a free
# is ordered after the work already enqueued on that stream: no device sync.
_alloc_lock = threading.Lock()
_alloc_cbs = None
_live_trees = weakref.WeakSet()


def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=None, stream=int(stream or 0))
    except Exception:  # out of memory or no device: the library reports TC_ERR_NOMEM
        return None


def _torch_free(ptr, stream, ctx):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


def _ensure_allocator(lib, force=False):
    global _alloc_cbs
    with _alloc_lock:
        if _alloc_cbs is None or force:
            cbs = _alloc_cbs or (_lib.ALLOC_FN(_torch_alloc), _lib.FREE_FN(_torch_free))
            check(lib.tc_set_allocator(cbs[0], cbs[1], None))
            _alloc_cbs = cbs  # the C side keeps the pointers: keep the thunks alive


def bind_torch_allocator():
    """(Re)install torch's caching allocator for handles created from now on
    (done automatically by the first Tree; needed again only after another
    allocator was installed through tc_set_allocator)."""
    _ensure_allocator(_lib.load(), force=True)


@atexit.register
def _free_live_trees():
    # release handles while torch's allocator is still up
    for t in list(_live_trees):
        t.free()


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _check_particles(pos, mass):
    """Type, device and shape checks of (pos [n,3], mass [n]); returns the
    tensors unchanged (callers decide whether a contiguous copy is allowed)."""
    if not (isinstance(pos, torch.Tensor) and isinstance(mass, torch.Tensor)):
        raise TypeError("pos and mass must be torch tensors")
    if pos.device.type != "cuda" or mass.device != pos.device:
        raise ValueError("pos and mass must live on the same GPU")
    if pos.dtype not in _DT or mass.dtype != pos.dtype:
        raise TypeError("pos and mass must both be float32 or both float64")
    if pos.dim() != 2 or pos.shape[1] != 3 or mass.dim() != 1 or mass.shape[0] != pos.shape[0]:
        raise ValueError("pos must be [n,3] and mass [n]")
    return pos, mass


def _check_buffer(name, t, shape, dtype, device, required=True):
    """A caller-supplied buffer the library reads or writes in place: it must
    have exactly this shape, dtype and device and be contiguous, otherwise the
    kernels would touch memory outside it.  Raises before any launch."""
    if t is None:
        if required:
            raise ValueError("%s is required" % name)
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.device != device:
        raise ValueError("%s must live on %s, got %s" % (name, device, t.device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _walk_dtype(walk):
    if walk not in _WALKS:
        raise ValueError("walk must be one of %s" % sorted(_WALKS))
    return torch.float32 if walk == "f32c" else torch.float64


class Tree:
    """A tc_tree handle bound to one GPU."""

    def __init__(self):
        self._lib = _lib.load()
        _ensure_allocator(self._lib)
        self._h = ctypes.c_void_p(None)
        _live_trees.add(self)
        self.n = 0
        self.device = None
        self._walk = None
        self._timing = None
        self._timing_applied = False

    def free(self):
        """Release the handle (waits for its enqueued work)."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.tc_tree_free(h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        self.free()

    # -- C ABI calls ---------------------------------------------------------
    def build(self, pos, mass):
        pos, mass = _check_particles(pos, mass)
        pos, mass = pos.contiguous(), mass.contiguous()  # read only: a copy is harmless
        self.device = pos.device
        self.n = pos.shape[0]
        with torch.cuda.device(pos.device):
            check(self._lib.tc_build(_ptr(pos), _ptr(mass), self.n, _DT[pos.dtype],
                                     _stream_ptr(pos.device), ctypes.byref(self._h)))
            if self._timing is not None and not self._timing_applied:
                check(self._lib.tc_tree_set_timing(self._h, 1 if self._timing else 0))
                self._timing_applied = True
        self._keep = (pos, mass)
        return self

    def moments(self):
        with torch.cuda.device(self.device):
            check(self._lib.tc_moments(self._h, _stream_ptr(self.device)))
        return self

    def forces(self, theta, eps, G=1.0, walk="f32c", count=False, store_lists=False, potential=True,
               out=None):
        """(acc [n,3], pot [n] or None) in caller order; float32 for f32c, float64 for f64."""
        dt = _walk_dtype(walk)
        mode = _WALKS[walk]
        if out is None:
            acc = torch.empty((self.n, 3), dtype=dt, device=self.device)
            pot = torch.empty((self.n,), dtype=dt, device=self.device) if potential else None
        else:
            acc, pot = out
            _check_buffer("acc", acc, (self.n, 3), dt, self.device)
            _check_buffer("pot", pot, (self.n,), dt, self.device, required=False)
        flags = (_lib.TC_COUNT if count else 0) | (_lib.TC_STORE_LISTS if store_lists else 0)
        with torch.cuda.device(self.device):
            check(self._lib.tc_forces(self._h, float(theta), float(eps), float(G), mode, flags,
                                      _ptr(acc), _ptr(pot), _stream_ptr(self.device)))
        self._walk = walk
        return acc, pot

    def backward(self, g_acc, g_pot=None, need_pos=True, need_mass=True):
        if self._walk is None:
            raise RuntimeError("backward needs a forces() call on this tree first")
        dt = _walk_dtype(self._walk)
        # read only: converted copies are allowed, but shape and device must match
        for name, g, shape in (("g_acc", g_acc, (self.n, 3)), ("g_pot", g_pot, (self.n,))):
            if g is None:
                continue
            if not isinstance(g, torch.Tensor) or tuple(g.shape) != shape or g.device != self.device:
                raise ValueError("%s must be a tensor of shape %s on %s" % (name, shape, self.device))
        g_acc = g_acc.to(dt).contiguous()
        g_pot = g_pot.to(dt).contiguous() if g_pot is not None else None
        g_pos = torch.empty((self.n, 3), dtype=dt, device=self.device) if need_pos else None
        g_mass = torch.empty((self.n,), dtype=dt, device=self.device) if need_mass else None
        with torch.cuda.device(self.device):
            check(self._lib.tc_forces_backward(self._h, _ptr(g_acc), _ptr(g_pot), _ptr(g_pos), _ptr(g_mass),
                                               _stream_ptr(self.device)))
        return g_pos, g_mass

    def set_timing(self, on=True):
        """Record per-stage HIP-event durations (applied at the next build if no handle yet)."""
        self._timing = bool(on)
        self._timing_applied = False
        if self._h.value:
            check(self._lib.tc_tree_set_timing(self._h, 1 if on else 0))
            self._timing_applied = True

    def stats(self):
        s = _lib.TcStats()
        with torch.cuda.device(self.device):
            check(self._lib.tc_tree_stats(self._h, ctypes.byref(s), _stream_ptr(self.device)))
        return dict(n=s.n, n_nodes=s.n_nodes, n_leaves=s.n_leaves, n_multi_leaves=s.n_multi_leaves,
                    lo=list(s.lo), L=s.L, log2L=s.log2L, max_level=s.max_level, state=s.state,
                    last_mode=s.last_mode, interactions=int(s.interactions), node_visits=int(s.node_visits),
                    lane_visits=int(s.lane_visits), momentum=list(s.momentum),
                    sum_m_abs_a=s.sum_m_abs_a, kinetic=s.kinetic, potential=s.potential,
                    lin_momentum=list(s.lin_momentum), ang_momentum=list(s.ang_momentum),
                    stage_ms=list(s.stage_ms), lists_stored=bool(s.lists_stored),
                    max_stack=int(s.max_stack), group_pops=int(s.group_pops),
                    visits_no_accept=int(s.visits_no_accept), visits_all_accept=int(s.visits_all_accept),
                    visits_box_open=int(s.visits_box_open), visits_box_accept=int(s.visits_box_accept),
                    walk_steps=int(s.walk_steps), walk_single_steps=int(s.walk_single_steps),
                    visits_overlap=int(s.visits_overlap),
                    visits_overlap_all_accept=int(s.visits_overlap_all_accept), list_bytes=int(s.list_bytes))

    def export(self, moments=True):
        st = self.stats()
        n, nn = st["n"], st["n_nodes"]
        dev = self.device
        out = dict(
            keys=torch.empty(n, dtype=torch.int64, device=dev),
            perm=torch.empty(n, dtype=torch.int32, device=dev),
            level=torch.empty(nn, dtype=torch.uint8, device=dev),
            first=torch.empty(nn, dtype=torch.int32, device=dev),
            count=torch.empty(nn, dtype=torch.int32, device=dev),
        )
        if moments:
            out["com"] = torch.empty((nn, 3), dtype=torch.float64, device=dev)
            out["mass"] = torch.empty(nn, dtype=torch.float64, device=dev)
        with torch.cuda.device(dev):
            check(self._lib.tc_tree_export(self._h, _ptr(out["keys"]), _ptr(out["perm"]), _ptr(out["level"]),
                                           _ptr(out["first"]), _ptr(out["count"]), _ptr(out.get("com")),
                                           _ptr(out.get("mass")), _stream_ptr(dev)))
        return out

    def target_order(self):
        """Sorted positions of the particles in the walk's target order (Hilbert order)."""
        o = torch.empty(self.n, dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            check(self._lib.tc_tree_target_order(self._h, _ptr(o), _stream_ptr(self.device)))
        return o

    def interaction_counts(self):
        c = torch.empty(self.n, dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            check(self._lib.tc_interaction_counts(self._h, _ptr(c), _stream_ptr(self.device)))
        return c


class TreeForces(torch.autograd.Function):
    """(acc, pot) = TreeForces.apply(pos, mass, theta, eps, G, walk, store_lists).

    Forward: tc_build + tc_moments + tc_forces (storing the interaction lists
    if store_lists and they fit the library's budget; re-walking in the
    backward is as fast on MI355X).  Backward: tc_forces_backward,
    the adjoint of the same walk with the tree membership and every
    interaction set held fixed (the opening decisions are piecewise constant
    in x, so this is the derivative wherever no decision sits on its
    threshold).  Gradients come back in the dtype of pos.
    """

    @staticmethod
    def forward(ctx, pos, mass, theta, eps, G=1.0, walk="f32c", store_lists=False):
        tree = Tree()
        tree.build(pos.detach(), mass.detach()).moments()
        acc, pot = tree.forces(theta, eps, G, walk=walk, store_lists=store_lists)
        ctx.tree = tree
        ctx.in_dtype = pos.dtype
        return acc, pot

    @staticmethod
    def backward(ctx, g_acc, g_pot):
        tree = ctx.tree
        if g_acc is None:
            dt = torch.float32 if tree._walk == "f32c" else torch.float64
            g_acc = torch.zeros((tree.n, 3), dtype=dt, device=tree.device)
        gpos, gmass = tree.backward(g_acc, g_pot, need_pos=ctx.needs_input_grad[0],
                                    need_mass=ctx.needs_input_grad[1])
        gpos = gpos.to(ctx.in_dtype) if gpos is not None else None
        gmass = gmass.to(ctx.in_dtype) if gmass is not None else None
        return gpos, gmass, None, None, None, None, None


def leapfrog_step(pos, vel, mass, acc, tau, theta, eps, G=1.0, walk="f32c", pot=None, tree=None):
    """One kick-drift-kick step (Eqs.(2)-(5)) in place through tc_leapfrog_step.

    pos, vel, mass: [n,3], [n,3], [n] of one float dtype; acc (and pot) are of
    the walk's precision and hold a^n on entry, a^{n+1} on exit.  Returns the
    tree handle (reuse it for the next step)."""
    # pos, vel, acc and pot are updated in place: they are checked as given, never copied
    pos, mass = _check_particles(pos, mass)
    n = pos.shape[0]
    _check_buffer("pos", pos, (n, 3), pos.dtype, pos.device)
    mass = mass.contiguous()  # read only
    _check_buffer("vel", vel, (n, 3), pos.dtype, pos.device)
    adt = _walk_dtype(walk)
    _check_buffer("acc", acc, (n, 3), adt, pos.device)
    _check_buffer("pot", pot, (n,), adt, pos.device, required=False)
    t = tree if tree is not None else Tree()
    t.device = pos.device
    t.n = pos.shape[0]
    with torch.cuda.device(pos.device):
        check(t._lib.tc_leapfrog_step(ctypes.byref(t._h), _ptr(pos), _ptr(vel), _ptr(mass), _ptr(acc), _ptr(pot),
                                      t.n, _DT[pos.dtype], float(tau), float(theta), float(eps), float(G),
                                      _WALKS[walk], _stream_ptr(pos.device)))
    t._walk = walk
    t._keep = (pos, mass)
    return t


def forces(pos, mass, theta, eps, G=1.0, walk="f32c", count=False, tree=None, store_lists=False):
    """Barnes-Hut accelerations and potentials of Eq.(1): (acc, pot, tree).
    store_lists keeps the walk's interaction lists for a later tree.backward."""
    t = tree if tree is not None else Tree()
    t.build(pos, mass).moments()
    acc, pot = t.forces(theta, eps, G, walk=walk, count=count, store_lists=store_lists)
    return acc, pot, t


def version():
    return _lib.load().tc_version().decode()
