"""GPU parity at the full benchmark size: Plummer sphere, N = 1e7, FP32
storage (seed 1002), eps = 0.005, the launch configuration the benchmark
times (one tc_build + tc_moments + tc_forces through the C ABI).

  * keys, permutation, node table and FP64 moments: bit-exact against the
    oracle over all 1e7 particles and ~1.5e7 nodes; the walk's target order a
    permutation of all 1e7 targets;
  * accelerations and potentials at theta in {0.3, 0.5, 0.8}: on 4096 seeded
    targets the oracle evaluates one by one, the bars of tests/bars.py
    (F32C median <= 1e-5, p99 <= 1e-4, every count-matching target <= 1e-4;
    F64 median <= 1e-13, p99 <= 1e-11, count-matching targets <= 1e-12);
  * interaction counts on the sample: F64 differs from the oracle on at most
    0.1% of targets, F32C on under 1% (distances within FP32 rounding of the
    opening threshold);
  * momentum ratio |sum m a| / sum m |a| over all N: the F32C walk within
    1e-6 (absolute) of the F64 walk, which matches the oracle per target;
  * Newton's shell theorem over the whole F32C field (theta = 0.5): shell means
    of the radial acceleration for 0.1 < r < 5 against -G M(<r) / r^2 to 0.2%,
    a pin independent of the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads
from bars import check_errors, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, SEED, EPS, SAMPLE = 10_000_000, 1002, 0.005, 4096


@pytest.fixture(scope="module")
def big():
    import paper_2412_01733_amd as tc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    print("fullsize: generating Plummer N=%d" % N, flush=True)
    pos, m = workloads.plummer(N, SEED, dtype=np.float32)
    dev = torch.device("cuda:0")
    tree = tc.Tree()
    tree.build(torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev)).moments()
    torch.cuda.synchronize()
    print("fullsize: oracle build", flush=True)
    T = oracle.Tree(pos, m)
    tg = workloads.target_sample(N, SAMPLE, 2002)
    return dict(pos=pos, m=m, tree=tree, T=T, tg=tg, dev=dev)


def test_fullsize_tree_bit_exact(big):
    ex = {k: v.cpu().numpy() for k, v in big["tree"].export(moments=True).items()}
    T = big["T"]
    ok, op = T.sorted()
    assert (ex["keys"].view(np.uint64) == ok).all(), "keys differ"
    assert (ex["perm"].astype(np.int64) == op).all(), "permutation differs"
    nd = T.nodes()
    assert len(ex["level"]) == len(nd["level"]), (len(ex["level"]), len(nd["level"]))
    assert (ex["level"].astype(np.int32) == nd["level"]).all()
    assert (ex["first"].astype(np.int64) == nd["first"]).all()
    assert (ex["count"].astype(np.int64) == nd["count"]).all()
    assert (ex["mass"] == nd["mass"]).all(), "moments (mass) not bit-exact"
    assert (ex["com"] == nd["com"]).all(), "moments (com) not bit-exact"


def test_fullsize_target_order_is_a_permutation(big):
    """Every one of the 1e7 targets is served by exactly one wavefront."""
    order = big["tree"].target_order().cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(N))


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8])
def test_fullsize_sampled_forces(big, theta):
    tree, tg = big["tree"], big["tg"]
    ra, rp, rn = big["T"].forces(theta, EPS, targets=tg)
    sel = torch.from_numpy(tg).to(big["dev"])
    rp_ratio = {}
    for walk, flip_bar in (("f32c", 0.01), ("f64", 1e-3)):
        print("fullsize: theta=%g walk=%s" % (theta, walk), flush=True)
        acc, pot = tree.forces(theta, EPS, walk=walk, count=True)
        cnt = tree.interaction_counts()[sel].cpu().numpy().astype(np.int64)
        st = tree.stats()
        a = acc[sel].double().cpu().numpy()
        p = pot[sel].double().cpu().numpy()
        e = rel_err(a, ra)
        ep = rel_err(p, rp)
        same = cnt == rn
        print("fullsize: max over count-matching targets %.3g (pot %.3g)" % (e[same].max(), ep[same].max()), flush=True)
        check_errors(e, walk, same, "acc")
        check_errors(ep, walk, same, "pot")
        assert np.mean(cnt != rn) <= flip_bar, (walk, np.mean(cnt != rn))
        rp_ratio[walk] = np.linalg.norm(st["momentum"]) / st["sum_m_abs_a"]
    assert abs(rp_ratio["f32c"] - rp_ratio["f64"]) <= 1e-6, rp_ratio


def test_fullsize_plummer_radial_profile(big):
    """Newton's shell theorem for the whole 1e7 field of the F32C walk: the
    mean radial acceleration over shells 0.1 < r < 5 (20 equal-count bins)
    equals -G M(<r) / r^2, with M(<r) the enclosed mass of the drawn sample
    (its Poisson noise removed) to 0.2%, and the truncated-Plummer closed
    form to that plus 4 sigma of the sample's Poisson noise in M(<r)."""
    tree, pos, m = big["tree"], big["pos"].astype(np.float64), big["m"].astype(np.float64)
    acc, _ = tree.forces(0.5, EPS, walk="f32c")
    a = acc.double().cpu().numpy()
    r = np.linalg.norm(pos, axis=1)
    ar = (a * pos).sum(1) / r
    o = np.argsort(r)
    m_emp = np.empty_like(r)
    m_emp[o] = np.concatenate([[0.0], np.cumsum(m[o])[:-1]])
    inner = (r > 0.1) & (r < 5.0)
    edges = np.quantile(r[inner], np.linspace(0, 1, 21))
    worst_emp = worst_cf = 0.0
    for lo_, hi_ in zip(edges[:-1], edges[1:]):
        sel = (r >= lo_) & (r < hi_)
        got = ar[sel].mean()
        want_emp = -(m_emp[sel] / r[sel] ** 2).mean()
        f = workloads.plummer_enclosed(r[sel])
        want_cf = -(f / r[sel] ** 2).mean()
        fm = float(np.median(f))
        sigma = np.sqrt(fm * (1.0 - fm) / N) / fm  # relative Poisson noise of M(<r)
        e_emp, e_cf = abs(got / want_emp - 1.0), abs(got / want_cf - 1.0)
        print("shell %.3f-%.3f: vs drawn %.2e, vs closed form %.2e (sigma %.1e)" % (lo_, hi_, e_emp, e_cf, sigma), flush=True)
        assert e_emp < 2e-3, (lo_, hi_, e_emp)
        assert e_cf < 2e-3 + 4 * sigma, (lo_, hi_, e_cf, sigma)
        worst_emp, worst_cf = max(worst_emp, e_emp), max(worst_cf, e_cf)
    print("worst: vs drawn %.2e, vs closed form %.2e" % (worst_emp, worst_cf), flush=True)
