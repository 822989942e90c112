"""Python binding of libtreecode: argument marshalling only.

torch supplies device memory and the stream; every step of the computation
runs in the library's HIP kernels.  Functions here mirror the C ABI names:

  Tree.build / Tree.moments / Tree.forces   -> tc_build / tc_moments / tc_forces
  Tree.backward, TreeForces (autograd)      -> tc_forces_backward
  leapfrog_step                             -> tc_leapfrog_step
  forces(pos, mass, theta, eps, ...)        -> build + moments + forces
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check

_WALKS = {"f32c": _lib.TC_WALK_F32C, "f64": _lib.TC_WALK_F64}
_DT = {torch.float32: _lib.TC_F32, torch.float64: _lib.TC_F64}


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _check_particles(pos, mass):
    if not (isinstance(pos, torch.Tensor) and isinstance(mass, torch.Tensor)):
        raise TypeError("pos and mass must be torch tensors")
    if pos.device.type != "cuda" or mass.device != pos.device:
        raise ValueError("pos and mass must live on the same GPU")
    if pos.dtype not in _DT or mass.dtype != pos.dtype:
        raise TypeError("pos and mass must both be float32 or both float64")
    if pos.dim() != 2 or pos.shape[1] != 3 or mass.dim() != 1 or mass.shape[0] != pos.shape[0]:
        raise ValueError("pos must be [n,3] and mass [n]")
    return pos.contiguous(), mass.contiguous()


class Tree:
    """A tc_tree handle bound to one GPU."""

    def __init__(self):
        self._lib = _lib.load()
        self._h = ctypes.c_void_p(None)
        self.n = 0
        self.device = None
        self._walk = None
        self._timing = None
        self._timing_applied = False

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.tc_tree_free(h)
            self._h = ctypes.c_void_p(None)

    # -- C ABI calls ---------------------------------------------------------
    def build(self, pos, mass):
        pos, mass = _check_particles(pos, mass)
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
        mode = _WALKS[walk]
        dt = torch.float32 if walk == "f32c" else torch.float64
        if out is None:
            acc = torch.empty((self.n, 3), dtype=dt, device=self.device)
            pot = torch.empty((self.n,), dtype=dt, device=self.device) if potential else None
        else:
            acc, pot = out
        flags = (_lib.TC_COUNT if count else 0) | (_lib.TC_STORE_LISTS if store_lists else 0)
        with torch.cuda.device(self.device):
            check(self._lib.tc_forces(self._h, float(theta), float(eps), float(G), mode, flags,
                                      _ptr(acc), _ptr(pot), _stream_ptr(self.device)))
        self._walk = walk
        return acc, pot

    def backward(self, g_acc, g_pot=None, need_pos=True, need_mass=True):
        dt = torch.float32 if self._walk == "f32c" else torch.float64
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
                    stage_ms=list(s.stage_ms), lists_stored=bool(s.lists_stored))

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
    pos, mass = _check_particles(pos, mass)
    if not (vel.is_contiguous() and pos.is_contiguous() and acc.is_contiguous()):
        raise ValueError("pos, vel and acc must be contiguous (they are updated in place)")
    if vel.shape != pos.shape or vel.dtype != pos.dtype or vel.device != pos.device:
        raise ValueError("vel must match pos")
    adt = torch.float32 if walk == "f32c" else torch.float64
    if acc.dtype != adt or acc.shape != pos.shape:
        raise ValueError("acc must be [n,3] of the walk precision")
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
