"""Pins of the oracle's moments and Barnes-Hut walk.

Each test fixes the oracle against something other than itself: exact
rational arithmetic, the textbook direct sum written independently in numpy,
closed forms (N = 1, 2; the Plummer profile), conservation of momentum,
exact power-of-two scaling, and a brute-force set definition of the
Barnes-Hut interaction set.
Passages: Eq.(1) (softened pairwise gravity, j != i); the TreeCode
description of section 2 (monopole at the centre of mass, opening angle
theta, theta -> 0 gives the direct sum).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads


def numpy_direct(pos, m, eps, G=1.0):
    """Direct sum of Eq.(1) by dense numpy broadcasting (independent code)."""
    x = np.asarray(pos, np.float64)
    d = x[None, :, :] - x[:, None, :]          # d[i, j] = x_j - x_i
    q = (d * d).sum(-1) + eps * eps
    np.fill_diagonal(q, np.inf)                 # j != i
    inv = q ** -0.5
    a = G * ((m[None, :] * inv ** 3)[:, :, None] * d).sum(1)
    phi = -G * (m[None, :] * inv).sum(1)
    return a, phi


def rel_err(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


# ---------------------------------------------------------------- moments

def test_root_moments_closed_form():
    pos, m = workloads.plummer(5000, 11)
    m = m * (1.0 + np.arange(5000) % 7)
    T = oracle.Tree(pos, m)
    nd = T.nodes()
    assert abs(nd["mass"][0] - m.sum()) <= 1e-15 * m.sum()
    com = (m[:, None] * pos).sum(0) / m.sum()
    assert np.abs(nd["com"][0] - com).max() < 1e-14


def test_moments_exact_definition_dyadic():
    """Dyadic inputs: every node's M equals the exact particle sum, and X
    is within a few ulps of the exact centre of mass of its particles."""
    g = np.random.default_rng(5)
    n = 700
    pos = g.integers(0, 1024, size=(n, 3)) * 2.0 ** -10
    pos[:10] = pos[10]  # coincident particles -> a level-21 leaf
    m = 2.0 ** -g.integers(3, 9, size=n).astype(np.float64)
    T = oracle.Tree(pos, m)
    nd = T.nodes()
    _, perm = T.sorted()
    sx, sm = pos[perm], m[perm]
    for i in range(T.nnodes):
        b, c = nd["first"][i], nd["count"][i]
        Mx = sum(Fraction(v) for v in sm[b:b + c])
        assert Fraction(nd["mass"][i]) == Mx
        for a in range(3):
            X = sum(Fraction(mm) * Fraction(xx) for mm, xx in zip(sm[b:b + c], sx[b:b + c, a])) / Mx
            assert abs(float(Fraction(nd["com"][i, a]) - X)) <= 8 * np.spacing(1.0)


def test_single_particle_leaf_is_verbatim_and_zero_mass_centre():
    pos = np.array([[0.1, 0.2, 0.3], [0.9, 0.8, 0.7], [0.11, 0.2, 0.31]])
    m = np.array([0.0, 1.0, 0.0])
    T = oracle.Tree(pos, m)
    nd = T.nodes()
    _, perm = T.sorted()
    leaves = np.where(nd["nchild"] == 0)[0]
    for i in leaves:
        s = nd["first"][i]
        assert (nd["com"][i] == pos[perm[s]]).all()  # bit-for-bit
    # an internal node whose particles all have zero mass sits at its cell centre
    lo, L, _ = T.geometry()
    for i in np.where((nd["nchild"] > 0) & (nd["mass"] == 0.0))[0]:
        side = L * 2.0 ** -nd["level"][i]
        corner = lo + np.floor((nd["com"][i] - lo) / side) * side
        assert np.allclose(nd["com"][i], corner + side / 2, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- walk

def test_direct_matches_numpy():
    pos, m = workloads.plummer(1500, 21)
    a, p = oracle.direct(pos, m, 0.01)
    a2, p2 = numpy_direct(pos, m, 0.01)
    assert rel_err(a, a2).max() < 1e-13
    assert np.abs(p - p2).max() / np.abs(p2).max() < 1e-13


@pytest.mark.parametrize("eps", [0.0, 0.01])
def test_theta_zero_is_direct_sum(eps):
    pos, m = workloads.plummer(2048, 22)
    m = m * np.linspace(0.5, 1.5, 2048)
    a, p, ni = oracle.forces(pos, m, 0.0, eps)
    a2, p2 = numpy_direct(pos, m, eps)
    assert rel_err(a, a2).max() < 1e-13
    assert np.abs(p - p2).max() / np.abs(p2).max() < 1e-13
    assert (ni == 2047).all()


def test_n1_and_n2_closed_forms():
    a, p, ni = oracle.forces(np.array([[0.3, -1.0, 2.0]]), np.array([2.0]), 0.7, 0.1)
    assert (a == 0).all() and (p == 0).all() and ni[0] == 0
    x = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    m = np.array([2.0, 5.0])
    eps, G = 0.5, 1.5
    for theta in (0.0, 0.5, 1.0, 10.0):   # the containing root is never accepted
        a, p, ni = oracle.forces(x, m, theta, eps, G)
        q = 25.0 + eps * eps
        assert np.allclose(a[0], G * 5.0 * np.array([3.0, 4.0, 0.0]) / q ** 1.5, rtol=1e-15, atol=0)
        assert np.allclose(a[1], -G * 2.0 * np.array([3.0, 4.0, 0.0]) / q ** 1.5, rtol=1e-15, atol=0)
        assert np.allclose(p, [-G * 5.0 / q ** 0.5, -G * 2.0 / q ** 0.5], rtol=1e-15, atol=0)
    # two particles sharing a key form one level-21 leaf; still a direct pair
    x = np.array([[0.0, 0.0, 0.0], [1e-12, 0.0, 0.0], [1.0, 1.0, 1.0]])
    T = oracle.Tree(x, np.ones(3))
    nd = T.nodes()
    assert ((nd["level"] == 21) & (nd["count"] == 2)).any()
    a, p, ni = T.forces(0.9, 0.01)
    a2, p2 = numpy_direct(x, np.ones(3), 0.01)
    assert rel_err(a[:2], a2[:2]).max() < 1e-12


def bruteforce_bh(T, pos, m, theta, eps, G=1.0):
    """Barnes-Hut by set definition: node n is accepted for target i iff the
    opening test passes, n does not contain i, and every strict ancestor of n
    is rejected (fails the test or contains i).  Leaves whose ancestors are
    all rejected and which are rejected themselves give direct terms."""
    nd = T.nodes()
    _, perm = T.sorted()
    lo, L, _ = T.geometry()
    sx, sm = pos[perm], m[perm]
    lev, first, count, par = nd["level"], nd["first"], nd["count"], nd["parent"]
    leaf = nd["nchild"] == 0
    side = L * 2.0 ** -lev.astype(np.float64)
    n, nn = len(m), len(lev)
    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    nint = np.zeros(n, np.int64)
    for s in range(n):
        x = sx[s]
        d = nd["com"] - x
        dist = np.sqrt((d * d).sum(1))
        contains = (first <= s) & (s < first + count)
        ok = (theta > 0) & (side < theta * dist) & ~contains
        blocked = np.zeros(nn, bool)          # some strict ancestor accepted
        for l in range(1, 22):
            sel = lev == l
            p = par[sel]
            blocked[sel] = blocked[p] | ok[p]
        accepted = ok & ~blocked
        srcs_x = [nd["com"][accepted]]
        srcs_m = [nd["mass"][accepted]]
        dl = np.where(leaf & ~blocked & ~accepted)[0]
        js = np.concatenate([np.arange(first[i], first[i] + count[i]) for i in dl]) if len(dl) else np.zeros(0, int)
        js = js[js != s]
        srcs_x.append(sx[js])
        srcs_m.append(sm[js])
        y = np.concatenate(srcs_x)
        mu = np.concatenate(srcs_m)
        dd = y - x
        q = (dd * dd).sum(1) + eps * eps
        inv = q ** -0.5
        acc[perm[s]] = G * ((mu * inv ** 3)[:, None] * dd).sum(0)
        pot[perm[s]] = -G * (mu * inv).sum()
        nint[perm[s]] = len(mu)
    return acc, pot, nint


@pytest.mark.parametrize("theta", [0.3, 0.7, 1.2])
def test_walk_equals_set_definition(theta):
    pos, m = workloads.plummer(1200, 31)
    pos = np.concatenate([pos, _dup_cluster()])
    m = np.concatenate([m, np.full(8, 1e-3)])
    m = m * (1 + 0.3 * np.sin(np.arange(len(m))))
    T = oracle.Tree(pos, m)
    a, p, ni = T.forces(theta, 0.02)
    a2, p2, n2 = bruteforce_bh(T, pos, m, theta, 0.02)
    assert (ni == n2).all()
    assert rel_err(a, a2).max() < 1e-12
    assert np.abs(p - p2).max() / np.abs(p2).max() < 1e-13


def _dup_cluster():
    c = np.array([[0.2, 0.1, -0.3]])
    return np.concatenate([np.repeat(c, 5, 0), c + [[1e-9, 0, 0]], c + [[0, 3e-9, 0]], c + [[0, 0, 2e-7]]])


def test_error_shrinks_with_theta():
    pos, m = workloads.plummer(4096, 41)
    ad, _ = oracle.direct(pos, m, 0.01)
    T = oracle.Tree(pos, m)
    errs = []
    for th in (0.8, 0.5, 0.3, 0.1):
        a, _, _ = T.forces(th, 0.01)
        errs.append(np.median(rel_err(a, ad)))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[0] < 0.05 and errs[3] < 1e-4


def test_target_subset_equals_full():
    pos, m = workloads.plummer(3000, 42)
    T = oracle.Tree(pos, m)
    a, p, ni = T.forces(0.5, 0.01)
    tg = workloads.target_sample(3000, 200, 9)
    a2, p2, n2 = T.forces(0.5, 0.01, targets=tg)
    assert (a2 == a[tg]).all() and (p2 == p[tg]).all() and (n2 == ni[tg]).all()


def test_thread_count_does_not_change_results():
    pos, m = workloads.plummer(3000, 43)
    T = oracle.Tree(pos, m)
    a1, p1, _ = T.forces(0.6, 0.01, nthreads=1)
    a4, p4, _ = T.forces(0.6, 0.01, nthreads=4)
    assert (a1 == a4).all() and (p1 == p4).all()


def test_momentum_direct_sum():
    pos, m = workloads.plummer(3000, 44)
    a, _ = oracle.direct(pos, m, 0.01)
    P = (m[:, None] * a).sum(0)
    assert np.linalg.norm(P) / (m * np.linalg.norm(a, axis=1)).sum() < 1e-14


def test_plummer_radial_profile():
    """Shell-averaged radial acceleration against -G M(<r) / r^2 (Newton's
    shell theorem for the truncated Plummer sphere)."""
    pos, m = workloads.plummer(16384, 1000)
    a, _, _ = oracle.forces(pos, m, 0.7, 0.01)
    r = np.linalg.norm(pos, axis=1)
    ar = (a * pos).sum(1) / r
    # enclosed mass of the drawn sample (removes its Poisson noise) and of the
    # analytic profile (noise of ~1/sqrt(count) left in)
    o = np.argsort(r)
    m_emp = np.empty_like(r)
    m_emp[o] = np.concatenate([[0.0], np.cumsum(m[o])[:-1]])
    edges = np.quantile(r[(r > 0.1) & (r < 5.0)], np.linspace(0, 1, 11))
    for lo_, hi_ in zip(edges[:-1], edges[1:]):
        sel = (r >= lo_) & (r < hi_)
        want = -(workloads.plummer_enclosed(r[sel]) / r[sel] ** 2).mean()
        want_emp = -(m_emp[sel] / r[sel] ** 2).mean()
        assert abs(ar[sel].mean() / want_emp - 1.0) < 0.01
        assert abs(ar[sel].mean() / want - 1.0) < 0.04


@pytest.mark.parametrize("k", [-3, 2])
def test_power_of_two_scaling_is_exact(k):
    pos, m = workloads.plummer(2000, 45)
    s = 2.0 ** k
    a, p, ni = oracle.forces(pos, m, 0.6, 0.01)
    k0, _ = oracle.keys(pos)
    ks, _ = oracle.keys(pos * s)
    assert (k0 == ks).all()
    a2, p2, n2 = oracle.forces(pos * s, m, 0.6, 0.01 * s)
    assert (n2 == ni).all()
    assert (a2 == a / (s * s)).all() and (p2 == p / s).all()
    a3, p3, _ = oracle.forces(pos, m * s, 0.6, 0.01)
    assert (a3 == a * s).all() and (p3 == p * s).all()
