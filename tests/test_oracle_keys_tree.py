"""Pins of the oracle's root cube, Morton keys, sort and octree topology.

Everything here is checked against hand-worked values, brute force written
differently from the oracle, or a library routine — never against the
oracle itself.  Passage: the TreeCode description of section 2 (recursive
split into eight octants until a cell holds at most one particle).
"""
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_keys_fixture():
    rows = []
    with open(os.path.join(GOLDEN, "keys_handworked.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            x, y, z, k = line.split()
            rows.append(((float(x), float(y), float(z)), int(k)))
    return rows


def test_keys_handworked():
    rows = _load_keys_fixture()
    pos = np.array([r[0] for r in rows])
    want = np.array([r[1] for r in rows], dtype=np.uint64)
    lo, L, e = oracle.root_cube(pos)
    assert list(lo) == [0.0, 0.0, 0.0] and L == 1.0 and e == 0
    got, _ = oracle.keys(pos)
    assert (got == want).all(), (got, want)


@pytest.mark.parametrize("extent,expect", [(1.0, 1.0), (3.0, 4.0), (4.0, 4.0), (0.3, 0.5),
                                           (2.0 ** -30, 2.0 ** -30), (5e5, 2.0 ** 19), (0.0, 1.0)])
def test_root_cube_power_of_two(extent, expect):
    pos = np.array([[1.0, -2.0, 7.0], [1.0 + extent, -2.0 + extent / 2, 7.0]])
    lo, L, e = oracle.root_cube(pos)
    assert L == expect and L == 2.0 ** e
    assert list(lo) == [1.0, -2.0, 7.0]


def test_root_cube_rejects_nonfinite():
    with pytest.raises(ValueError):
        oracle.root_cube(np.array([[0.0, np.nan, 0.0]]))
    with pytest.raises(ValueError):
        oracle.Tree(np.array([[0.0, 0.0, np.inf], [1.0, 1.0, 1.0]]), np.ones(2))
    with pytest.raises(ValueError):
        oracle.Tree(np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]]), np.array([1.0, -1.0]))


def _interleave_by_strings(q):
    """Brute-force key: interleave binary digit strings, x first."""
    out = []
    for qx, qy, qz in q:
        bx, by, bz = (format(int(v), "021b") for v in (qx, qy, qz))
        s = "".join(a + b + c for a, b, c in zip(bx, by, bz))
        out.append(int(s, 2))
    return np.array(out, dtype=np.uint64)


def test_keys_bruteforce_and_roundtrip():
    pos, _ = workloads.plummer(3000, 7)
    k, q = oracle.keys(pos)
    assert (k == _interleave_by_strings(q)).all()
    assert (k >> np.uint64(63) == 0).all()
    # quantisation by exact rational arithmetic (power-of-two scale)
    lo, L, e = oracle.root_cube(pos)
    from fractions import Fraction
    for i in range(0, 3000, 97):
        for a in range(3):
            d = Fraction(pos[i, a] - lo[a])  # the FP64 subtraction, then exact scaling
            qq = min((d * Fraction(2) ** 21 / Fraction(L)).__floor__(), 2 ** 21 - 1)
            assert qq == q[i, a]
    # decode: the child digit at level l is 4x+2y+z of bit 21-l
    for i in range(0, 3000, 131):
        for l in range(1, 22):
            d = (int(k[i]) >> (3 * (21 - l))) & 7
            b = 21 - l
            assert d == 4 * ((q[i, 0] >> b) & 1) + 2 * ((q[i, 1] >> b) & 1) + ((q[i, 2] >> b) & 1)


def test_stable_sort_matches_library():
    g = np.random.default_rng(3)
    k = g.integers(0, 50, size=5000).astype(np.uint64)  # many ties
    perm = oracle.stable_sort(k)
    assert (perm == np.argsort(k, kind="stable")).all()
    big = g.integers(0, 2 ** 63 - 1, size=4096, dtype=np.int64).astype(np.uint64)
    assert (oracle.stable_sort(big) == np.argsort(big, kind="stable")).all()


def _bruteforce_nodes(skeys):
    """Enumerate the canonical octree by prefixes: a level-l cell (distinct
    top-3l-bit prefix) is a node iff l == 0 or its parent cell holds >= 2
    particles.  Returns (level, first, count) sorted by (first, level)."""
    n = len(skeys)
    keys = [int(v) for v in skeys]
    nodes = []
    for l in range(22):
        sh = 3 * (21 - l)
        groups = {}
        for s, kk in enumerate(keys):
            p = kk >> sh
            if p not in groups:
                groups[p] = [s, 0]
            groups[p][1] += 1
        psh = 3 * (21 - (l - 1)) if l > 0 else None
        pcount = {}
        if l > 0:
            for kk in keys:
                pp = kk >> psh
                pcount[pp] = pcount.get(pp, 0) + 1
        for p, (first, cnt) in groups.items():
            if l == 0 or pcount[p >> 3] >= 2:
                nodes.append((first, l, cnt))
    nodes.sort()
    return [(l, f, c) for f, l, c in nodes]


def _clustered(n, seed):
    g = np.random.default_rng(seed)
    pos = g.random((n, 3))
    # duplicates and near-duplicates so that level-21 multi-particle leaves occur
    pos[n // 2:n // 2 + 6] = pos[1]
    pos[n // 2 + 6:n // 2 + 9] = pos[2] + 1e-9
    return pos


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 0), (5, 1), (64, 2), (300, 3)])
def test_topology_bruteforce(n, seed):
    pos = _clustered(n, seed) if n >= 20 else np.random.default_rng(seed).random((n, 3))
    T = oracle.Tree(pos, np.ones(n))
    skeys, perm = T.sorted()
    nd = T.nodes()
    got = list(zip(nd["level"].tolist(), nd["first"].tolist(), nd["count"].tolist()))
    assert got == _bruteforce_nodes(skeys)


def test_topology_invariants():
    pos = np.concatenate([workloads.plummer(2000, 5)[0], _clustered(200, 9)])
    n = pos.shape[0]
    T = oracle.Tree(pos, np.ones(n))
    nd = T.nodes()
    lev, first, count, nch, child, parent = (nd[k] for k in ("level", "first", "count", "nchild", "child", "parent"))
    nn = lev.shape[0]
    assert first[0] == 0 and count[0] == n and lev[0] == 0 and parent[0] == -1
    order = np.lexsort((lev, first))
    assert (order == np.arange(nn)).all(), "pre-order must equal (first, level) order"
    leaf_cover = np.zeros(n, np.int64)
    for i in range(nn):
        if nch[i] == 0:
            assert count[i] == 1 or lev[i] == 21
            leaf_cover[first[i]:first[i] + count[i]] += 1
        else:
            ch = child[i, :nch[i]]
            assert (lev[ch] == lev[i] + 1).all()
            assert (parent[ch] == i).all()
            assert first[ch[0]] == first[i]
            assert (first[ch[1:]] == first[ch[:-1]] + count[ch[:-1]]).all()
            assert count[ch].sum() == count[i]
            assert count[i] >= 2 and lev[i] < 21
    assert (leaf_cover == 1).all(), "every particle in exactly one leaf"
    # duplicated keys gave multi-particle leaves at level 21
    assert ((nch == 0) & (count > 1)).any()
