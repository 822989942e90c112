"""Pins of the oracle's frozen-list adjoint and its leapfrog step.

The adjoint of F(x, m; lists) — forces with the tree membership and every
target's interaction set held fixed — is checked against torch's CPU
autograd of independent torch implementations (the direct sum of Eq.(1) at
theta = 0, and the frozen Barnes-Hut sum built from flat centre-of-mass
sums at theta > 0) and against central finite differences.  The
kick-drift-kick step of Eqs.(2)-(5) is checked for time reversibility and
against a circular two-body orbit.
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")


def _problem(n, seed, theta):
    x, m = workloads.plummer(n, seed)
    m = m * (1.0 + 0.3 * np.sin(np.arange(n)))
    T = oracle.Tree(x, m)
    L = T.lists(theta)
    g = np.random.default_rng(seed + 1).standard_normal((n, 3))
    h = np.random.default_rng(seed + 2).standard_normal(n)
    return x, m, T, L, g, h


def test_frozen_forces_reproduce_the_walk():
    x, m, T, L, _, _ = _problem(700, 11, 0.6)
    a, p, ni = T.forces(0.6, 0.02)
    a2, p2 = T.frozen_forces(x, m, L, 0.02)
    assert (a == a2).all() and (p == p2).all()
    assert (np.diff(L[0]) == ni).all()


def torch_direct(x, m, eps):
    d = x[None, :, :] - x[:, None, :]
    q = (d * d).sum(-1) + eps * eps
    n = x.shape[0]
    off = ~torch.eye(n, dtype=torch.bool)
    inv = torch.where(off, q, torch.ones_like(q)).rsqrt() * off
    a = ((m[None, :] * inv ** 3)[:, :, None] * d).sum(1)
    phi = -(m[None, :] * inv).sum(1)
    return a, phi


def test_adjoint_theta0_equals_autograd_of_direct_sum():
    n, eps = 300, 0.02
    x, m, T, L, g, h = _problem(n, 21, 0.0)
    gx, gm = T.frozen_adjoint(L, eps, g, h)
    xt = torch.tensor(x, requires_grad=True)
    mt = torch.tensor(m, requires_grad=True)
    a, phi = torch_direct(xt, mt, eps)
    (a * torch.tensor(g)).sum().add((phi * torch.tensor(h)).sum()).backward()
    assert np.abs(gx - xt.grad.numpy()).max() <= 1e-11 * np.abs(gx).max()
    assert np.abs(gm - mt.grad.numpy()).max() <= 1e-11 * np.abs(gm).max()


def torch_frozen_bh(T, L, x, m, eps):
    """Frozen Barnes-Hut forces in torch: node moments as flat sums over each
    node's (fixed) particle range, sources taken from the recorded lists."""
    nd = T.nodes()
    _, perm = T.sorted()
    permt = torch.tensor(perm)
    sx, sm = x[permt], m[permt]
    n, nn = x.shape[0], len(nd["level"])
    # membership matrix: node -> particles (sorted positions)
    rows, cols = [], []
    for i in range(nn):
        for j in range(nd["first"][i], nd["first"][i] + nd["count"][i]):
            rows.append(i)
            cols.append(j)
    W = torch.zeros((nn, n), dtype=torch.float64)
    W[rows, cols] = 1.0
    M = W @ sm
    X = (W @ (sm[:, None] * sx)) / M[:, None]
    single = torch.tensor((nd["nchild"] == 0) & (nd["count"] == 1))
    first = torch.tensor(nd["first"])
    X = torch.where(single[:, None], sx[first], X)
    off, codes = L
    spos = np.empty(n, np.int64)
    spos[perm] = np.arange(n)
    tgt = np.repeat(np.arange(n), np.diff(off))
    node = codes >= 0
    y = torch.empty((len(codes), 3), dtype=torch.float64)
    mu = torch.empty(len(codes), dtype=torch.float64)
    y = torch.where(torch.tensor(node)[:, None], X[torch.tensor(np.where(node, codes, 0))],
                    sx[torch.tensor(np.where(node, 0, -codes - 1))])
    mu = torch.where(torch.tensor(node), M[torch.tensor(np.where(node, codes, 0))],
                     sm[torch.tensor(np.where(node, 0, -codes - 1))])
    xi = sx[torch.tensor(spos[tgt])]
    d = y - xi
    q = (d * d).sum(1) + eps * eps
    inv = q.rsqrt()
    a = torch.zeros((n, 3), dtype=torch.float64).index_add(0, torch.tensor(tgt), (mu * inv ** 3)[:, None] * d)
    phi = torch.zeros(n, dtype=torch.float64).index_add(0, torch.tensor(tgt), -mu * inv)
    return a, phi


@pytest.mark.parametrize("theta", [0.5, 0.9])
def test_adjoint_equals_autograd_of_frozen_bh(theta):
    n, eps = 400, 0.02
    x, m, T, L, g, h = _problem(n, 31, theta)
    a0, p0, _ = T.forces(theta, eps)
    xt = torch.tensor(x, requires_grad=True)
    mt = torch.tensor(m, requires_grad=True)
    a, phi = torch_frozen_bh(T, L, xt, mt, eps)
    assert np.abs(a.detach().numpy() - a0).max() <= 1e-12 * np.abs(a0).max()
    (a * torch.tensor(g)).sum().add((phi * torch.tensor(h)).sum()).backward()
    gx, gm = T.frozen_adjoint(L, eps, g, h)
    assert np.abs(gx - xt.grad.numpy()).max() <= 1e-10 * np.abs(gx).max()
    assert np.abs(gm - mt.grad.numpy()).max() <= 1e-10 * np.abs(gm).max()


def test_adjoint_against_central_differences():
    n, eps, theta = 600, 0.01, 0.5
    x, m, T, L, g, h = _problem(n, 41, theta)
    gx, gm = T.frozen_adjoint(L, eps, g, h)

    def loss(xx, mm):
        a, p = T.frozen_forces(xx, mm, L, eps)
        return (a * g).sum() + (p * h).sum()

    rng = np.random.default_rng(5)
    for i, k in zip(rng.integers(0, n, 12), rng.integers(0, 3, 12)):
        hh = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[i, k] += hh
        xm[i, k] -= hh
        fd = (loss(xp, m) - loss(xm, m)) / (2 * hh)
        assert abs(fd - gx[i, k]) <= 1e-6 * max(abs(gx[i, k]), 1e-3 * np.abs(gx).max())
    for i in rng.integers(0, n, 12):
        hh = 1e-5 * m[i]
        mp, mm = m.copy(), m.copy()
        mp[i] += hh
        mm[i] -= hh
        fd = (loss(x, mp) - loss(x, mm)) / (2 * hh)
        assert abs(fd - gm[i]) <= 1e-6 * max(abs(gm[i]), 1e-3 * np.abs(gm).max())


def test_leapfrog_time_reversible():
    x, m = workloads.plummer(500, 51)
    v = np.random.default_rng(2).standard_normal((500, 3)) * 0.3
    a0, _, _ = oracle.forces(x, m, 0.6, 0.02)
    x1, v1, a1, _ = oracle.leapfrog_step(x, v, m, a0, 1e-3, 0.6, 0.02)
    x2, v2, a2, _ = oracle.leapfrog_step(x1, v1, m, a1, -1e-3, 0.6, 0.02)
    assert np.abs(x2 - x).max() < 1e-13
    assert np.abs(v2 - v).max() < 1e-12
    assert np.abs(x1 - x).max() > 1e-5  # it did move


def test_leapfrog_circular_two_body_orbit():
    # two equal masses 1/2 on a circle of radius 1/2 about the origin: omega = 1
    x = np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
    v = np.array([[0.0, 0.5, 0.0], [0.0, -0.5, 0.0]])
    m = np.array([0.5, 0.5])
    a, _, _ = oracle.forces(x, m, 0.5, 0.0)
    tau, steps = 1e-2, 100
    for _ in range(steps):
        x, v, a, pot = oracle.leapfrog_step(x, v, m, a, tau, 0.5, 0.0)
    t = tau * steps
    want = 0.5 * np.array([np.cos(t), np.sin(t), 0.0])
    assert np.abs(x[0] - want).max() < 2e-5  # leapfrog phase error ~ (omega tau)^2 omega t / 24
    # the separation oscillates with relative amplitude ~ (omega tau)^2 / 8
    assert abs(np.linalg.norm(x[0] - x[1]) - 1.0) < 2e-5


def test_frozen_forces_do_not_depend_on_the_thread_count():
    """Targets are independent: sharing them among threads leaves every sum,
    and so every bit of the result, unchanged."""
    x, m = workloads.plummer(3000, 17)
    T = oracle.Tree(x, m)
    L = T.lists(0.6)
    a1, p1 = T.frozen_forces(x, m, L, 0.01, nthreads=1)
    a8, p8 = T.frozen_forces(x, m, L, 0.01, nthreads=8)
    assert (a1 == a8).all() and (p1 == p8).all()
