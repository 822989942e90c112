"""FP64 CPU oracle for TreeCode (Barnes-Hut) gravity — test infrastructure.

This package is the slow, plainly written reference that the GPU library is
checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import it; the product path never does.  It shares no
code with the HIP library: the arithmetic lives in ``treecode_oracle.c``
(built with gcc, ``-O3 -fno-fast-math -ffp-contract=off``) and in the few
plain numpy companions below.

Every function follows a passage of Kuzmin, Sirotin & Khoperskov (2024):
Eq.(1) for the softened interaction, the TreeCode description of section 2
for the octree, the monopole moments and the opening angle, Eqs.(2)-(5) for
the kick-drift-kick leapfrog.  The readings taken where the paper is silent
are stated in the header of ``treecode_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "treecode_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The mutation tests point this at a copy of the oracle built with one
# planted mistake, to show that the pins catch it; it is never rebuilt.
_LIB_OVERRIDE = os.environ.get("TREECODE_ORACLE_LIB")

CFLAGS = ["-O3", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-pthread"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if _LIB_OVERRIDE:
        return _LIB_OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        L.or_root_cube.argtypes = [P, I64, P, P, P]
        L.or_root_cube.restype = ctypes.c_int
        L.or_keys.argtypes = [P, I64, P, ctypes.c_int, P, P]
        L.or_sort.argtypes = [P, I64, P]
        L.or_tree_new.argtypes = [P, P, I64]
        L.or_tree_new.restype = P
        L.or_tree_free.argtypes = [P]
        L.or_tree_nnodes.argtypes = [P]
        L.or_tree_nnodes.restype = I64
        L.or_tree_geometry.argtypes = [P, P, P, P]
        L.or_tree_sorted.argtypes = [P, P, P]
        L.or_tree_nodes.argtypes = [P] + [P] * 8
        L.or_tree_forces.argtypes = [P, D, D, D, P, I64, P, P, P, ctypes.c_int]
        L.or_direct.argtypes = [P, P, I64, D, D, P, I64, P, P, ctypes.c_int]
        PP = ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))
        L.or_tree_lists.argtypes = [P, D, PP, PP, ctypes.c_int]
        L.or_free.argtypes = [P]
        L.or_frozen_forces.argtypes = [P, P, P, P, P, D, D, P, P, ctypes.c_int]
        L.or_frozen_adjoint.argtypes = [P, P, P, D, D, P, P, P, P]
        L.or_leapfrog_step.argtypes = [P, P, P, P, P, I64, D, D, D, D, ctypes.c_int]
        L.or_leapfrog_step.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _threads(nthreads):
    if nthreads is None:
        nthreads = int(os.environ.get("ORACLE_THREADS", "0")) or (os.cpu_count() or 1)
    return int(nthreads)


def _f64pos(pos):
    # FP32 inputs are widened exactly; the oracle computes in FP64.
    return np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))


def root_cube(pos):
    """(lo[3], L, log2L): the root cube of the particle set."""
    x = _f64pos(pos)
    lo = np.zeros(3)
    L = ctypes.c_double()
    e = ctypes.c_int()
    if lib().or_root_cube(_ptr(x), x.shape[0], _ptr(lo), ctypes.byref(L), ctypes.byref(e)) != 0:
        raise ValueError("non-finite position")
    return lo, L.value, e.value


def keys(pos):
    """(keys u64[n], q int64[n,3]) in caller order."""
    x = _f64pos(pos)
    lo, _, e = root_cube(x)
    k = np.zeros(x.shape[0], np.uint64)
    q = np.zeros((x.shape[0], 3), np.int64)
    lib().or_keys(_ptr(x), x.shape[0], _ptr(lo), e, _ptr(q), _ptr(k))
    return k, q


def stable_sort(k):
    k = np.ascontiguousarray(k, dtype=np.uint64)
    perm = np.zeros(k.shape[0], np.int64)
    lib().or_sort(_ptr(k), k.shape[0], _ptr(perm))
    return perm


class Tree:
    """Keys, sort, top-down octree and monopole moments of one particle set."""

    def __init__(self, pos, mass):
        x = _f64pos(pos)
        m = np.ascontiguousarray(np.asarray(mass, dtype=np.float64).reshape(-1))
        if m.shape[0] != x.shape[0]:
            raise ValueError("pos and mass disagree on n")
        self.n = x.shape[0]
        self._x, self._m = x, m
        h = lib().or_tree_new(_ptr(x), _ptr(m), self.n)
        if not h:
            raise ValueError("non-finite position or negative mass")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_tree_free(h)
            self._h = None

    @property
    def nnodes(self) -> int:
        return int(lib().or_tree_nnodes(self._h))

    def geometry(self):
        lo = np.zeros(3)
        L = ctypes.c_double()
        e = ctypes.c_int()
        lib().or_tree_geometry(self._h, _ptr(lo), ctypes.byref(L), ctypes.byref(e))
        return lo, L.value, e.value

    def sorted(self):
        """(sorted keys u64[n], perm int64[n]: sorted position -> caller index)."""
        k = np.zeros(self.n, np.uint64)
        p = np.zeros(self.n, np.int64)
        lib().or_tree_sorted(self._h, _ptr(k), _ptr(p))
        return k, p

    def nodes(self):
        """Pre-order node table as a dict of arrays."""
        nn = self.nnodes
        out = dict(
            level=np.zeros(nn, np.int32),
            first=np.zeros(nn, np.int64),
            count=np.zeros(nn, np.int64),
            nchild=np.zeros(nn, np.int32),
            child=np.zeros((nn, 8), np.int64),
            parent=np.zeros(nn, np.int64),
            com=np.zeros((nn, 3)),
            mass=np.zeros(nn),
        )
        lib().or_tree_nodes(self._h, *[_ptr(out[k]) for k in
                                      ("level", "first", "count", "nchild", "child", "parent", "com", "mass")])
        return out

    def forces(self, theta, eps, G=1.0, targets=None, nthreads=None):
        """Barnes-Hut (acc[nt,3], pot[nt], ninteractions[nt]) for caller-index targets."""
        if targets is None:
            tg, nt = None, self.n
        else:
            tg = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
            nt = tg.shape[0]
            if nt and (tg.min() < 0 or tg.max() >= self.n):
                raise IndexError("target out of range")
        acc = np.zeros((nt, 3))
        pot = np.zeros(nt)
        nint = np.zeros(nt, np.int64)
        lib().or_tree_forces(self._h, float(theta), float(eps), float(G), _ptr(tg), nt,
                             _ptr(acc), _ptr(pot), _ptr(nint), _threads(nthreads))
        return acc, pot, nint


    # -- frozen interaction lists (for the adjoint) --------------------------
    def lists(self, theta, nthreads=None):
        """Every particle's interaction list (caller order) as CSR arrays
        (offsets[n+1], codes): code >= 0 is a pre-order node, code < 0 the
        particle at sorted position -(code + 1)."""
        off = ctypes.POINTER(ctypes.c_int64)()
        cod = ctypes.POINTER(ctypes.c_int64)()
        lib().or_tree_lists(self._h, float(theta), ctypes.byref(off), ctypes.byref(cod), _threads(nthreads))
        o = np.ctypeslib.as_array(off, shape=(self.n + 1,)).copy()
        c = np.ctypeslib.as_array(cod, shape=(max(int(o[-1]), 1),))[:int(o[-1])].copy()
        lib().or_free(ctypes.cast(off, ctypes.c_void_p))
        lib().or_free(ctypes.cast(cod, ctypes.c_void_p))
        return o, c

    def frozen_forces(self, pos, mass, lists, eps, G=1.0, nthreads=1):
        """F(x, m; lists): forces with this tree's membership and the given lists frozen
        (targets shared by nthreads; the result does not depend on it)."""
        x = _f64pos(pos)
        m = np.ascontiguousarray(np.asarray(mass, dtype=np.float64).reshape(-1))
        o, c = lists
        acc = np.zeros((self.n, 3))
        pot = np.zeros(self.n)
        lib().or_frozen_forces(self._h, _ptr(x), _ptr(m), _ptr(o), _ptr(c), float(eps), float(G),
                               _ptr(acc), _ptr(pot), _threads(nthreads))
        return acc, pot

    def frozen_adjoint(self, lists, eps, g_acc, g_pot=None, G=1.0):
        """(dL/dx [n,3], dL/dm [n]) of L(F(x, m; lists)) at this tree's (x, m)."""
        o, c = lists
        ga = np.ascontiguousarray(np.asarray(g_acc, dtype=np.float64).reshape(-1, 3))
        gp = None if g_pot is None else np.ascontiguousarray(np.asarray(g_pot, dtype=np.float64))
        gx = np.zeros((self.n, 3))
        gm = np.zeros(self.n)
        lib().or_frozen_adjoint(self._h, _ptr(o), _ptr(c), float(eps), float(G), _ptr(ga), _ptr(gp),
                                _ptr(gx), _ptr(gm))
        return gx, gm


def leapfrog_step(pos, vel, mass, acc, tau, theta, eps, G=1.0, nthreads=None):
    """One kick-drift-kick step, Eqs.(2)-(5) with a rebuild for Eq.(4).
    Returns new (pos, vel, acc, pot) as FP64 arrays."""
    x = _f64pos(pos).copy()
    v = _f64pos(vel).copy()
    a = _f64pos(acc).copy()
    m = np.ascontiguousarray(np.asarray(mass, dtype=np.float64).reshape(-1))
    pot = np.zeros(x.shape[0])
    if lib().or_leapfrog_step(_ptr(x), _ptr(v), _ptr(m), _ptr(a), _ptr(pot), x.shape[0], float(tau),
                              float(theta), float(eps), float(G), _threads(nthreads)) != 0:
        raise ValueError("non-finite position after the drift")
    return x, v, a, pot


def direct(pos, mass, eps, G=1.0, targets=None, nthreads=None):
    """Direct-summation (acc[nt,3], pot[nt]) of Eq.(1), j != i, FP64."""
    x = _f64pos(pos)
    m = np.ascontiguousarray(np.asarray(mass, dtype=np.float64).reshape(-1))
    if targets is None:
        tg, nt = None, x.shape[0]
    else:
        tg = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt = tg.shape[0]
    acc = np.zeros((nt, 3))
    pot = np.zeros(nt)
    lib().or_direct(_ptr(x), _ptr(m), x.shape[0], float(eps), float(G), _ptr(tg), nt,
                    _ptr(acc), _ptr(pot), _threads(nthreads))
    return acc, pot


def forces(pos, mass, theta, eps, G=1.0, targets=None, nthreads=None):
    """Convenience: build a Tree and evaluate Barnes-Hut forces."""
    return Tree(pos, mass).forces(theta, eps, G, targets, nthreads)
