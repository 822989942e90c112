"""GPU parity at the paper's top size (section 3: N up to 1e8): an exponential
disc of 2e7 particles inside a Hernquist halo of 8e7, FP32 positions,
velocities and masses, theta = 0.5, eps = 0.01, seed 1004 - one tree build,
one force evaluation with the interaction lists recomputed by the walk (never
stored), and one kick-drift-kick step, all through the C ABI in the launch
configuration the benchmark's 1e8 mode times.

  * keys and permutation over all 1e8 particles: bit-exact against the oracle;
  * node table (level, first, count) over all ~1.5e8 nodes: bit-exact (u32
    node indices near their range, and the multi-particle leaves that FP32
    duplicates form at level 21);
  * accelerations and potentials on 2^16 seeded targets the oracle evaluates
    one by one: the bars of tests/bars.py, per-target maximum included, and
    interaction counts differing from the oracle's on < 1% of them;
  * the leapfrog step: kick and drift bit-exact against FP64 arithmetic
    rounded to FP32, and the keys of the drifted positions bit-exact against
    the oracle's keys of the same positions.
The module builds once and checks in separate tests, so progress shows
between the long steps (drawing 1e8 particles, the oracle's build).
"""
import numpy as np
import pytest

import oracle
import workloads
from bars import check_errors, rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

N_DISC, N_HALO, SEED, THETA, EPS, TAU, SAMPLE = 20_000_000, 80_000_000, 1004, 0.5, 0.01, 1e-3, 1 << 16


@pytest.fixture(scope="module")
def big():
    import paper_2412_01733_amd as tc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    print("disc100m: drawing %d + %d particles" % (N_DISC, N_HALO), flush=True)
    pos, vel, m = workloads.disc_galaxy(N_DISC, N_HALO, SEED, dtype=np.float32)
    dev = torch.device("cuda:0")
    p, v, mm = (torch.from_numpy(a).to(dev) for a in (pos, vel, m))
    tree = tc.Tree()
    tree.build(p, mm).moments()
    acc, pot = tree.forces(THETA, EPS, walk="f32c", count=True)
    torch.cuda.synchronize()
    st = tree.stats()
    ex = {k: t.cpu().numpy() for k, t in tree.export(moments=False).items()}
    tg = workloads.target_sample(pos.shape[0], SAMPLE, 2004)
    sel = torch.from_numpy(tg).to(dev)
    out = dict(pos=pos, vel=vel, m=m, p=p, v=v, mm=mm, tree=tree, st=st, ex=ex, tg=tg,
               acc=acc[sel].double().cpu().numpy(), pot=pot[sel].double().cpu().numpy(),
               counts=tree.interaction_counts()[sel].cpu().numpy().astype(np.int64), acc_full=acc, pot_full=pot)
    print("disc100m: GPU tree %d nodes (%d multi-particle leaves)" % (st["n_nodes"], st["n_multi_leaves"]), flush=True)
    return out


@pytest.fixture(scope="module")
def otree(big):
    print("disc100m: oracle build at N = 1e8", flush=True)
    return oracle.Tree(big["pos"], big["m"])


def test_disc100m_keys_and_permutation(big, otree):
    ok, op = otree.sorted()
    assert (big["ex"]["keys"].view(np.uint64) == ok).all(), "keys differ"
    assert (big["ex"]["perm"].astype(np.int64) == op).all(), "permutation differs"


def test_disc100m_node_table(big, otree):
    nd = otree.nodes()
    ex = big["ex"]
    assert big["st"]["n_nodes"] == otree.nnodes == len(ex["level"]), (big["st"]["n_nodes"], otree.nnodes)
    assert (ex["level"].astype(np.int32) == nd["level"]).all()
    assert (ex["first"].astype(np.uint32).astype(np.int64) == nd["first"]).all()
    assert (ex["count"].astype(np.uint32).astype(np.int64) == nd["count"]).all()
    assert big["st"]["n_multi_leaves"] == int(((nd["nchild"] == 0) & (nd["count"] > 1)).sum())


def test_disc100m_sampled_forces(big, otree):
    ra, rp, rn = otree.forces(THETA, EPS, targets=big["tg"], nthreads=16)
    same = big["counts"] == rn
    e = rel_err(big["acc"], ra)
    ep = rel_err(big["pot"], rp)
    print("disc100m: median %.3g p99 %.3g max(count-matching) %.3g, count mismatches %.4f" %
          (np.median(e), np.quantile(e, 0.99), e[same].max(), 1 - same.mean()), flush=True)
    check_errors(e, "f32c", same, "acc")
    check_errors(ep, "f32c", same, "pot")
    assert 1 - same.mean() < 0.01


def test_disc100m_leapfrog_step(big):
    import paper_2412_01733_amd as tc
    p, v, mm, tree = big["p"], big["v"], big["mm"], big["tree"]
    acc, pot = big["acc_full"], big["pot_full"]
    x0 = big["pos"].astype(np.float64)
    v0 = big["vel"].astype(np.float64)
    a0 = acc.cpu().numpy().astype(np.float64)
    tc.leapfrog_step(p, v, mm, acc, TAU, THETA, EPS, walk="f32c", pot=pot, tree=tree)
    torch.cuda.synchronize()
    vh = (v0 + 0.5 * TAU * a0).astype(np.float32)
    xn = (x0 + TAU * vh.astype(np.float64)).astype(np.float32)
    assert (p.cpu().numpy() == xn).all(), "drift differs from FP64-then-round"
    vn = (vh.astype(np.float64) + 0.5 * TAU * acc.cpu().numpy().astype(np.float64)).astype(np.float32)
    assert (v.cpu().numpy() == vn).all(), "second kick differs from FP64-then-round"
    k_gpu = tree.export(moments=False)["keys"].cpu().numpy().view(np.uint64)
    k_ref, _ = oracle.keys(xn)
    assert (k_gpu == np.sort(k_ref)).all(), "keys of the drifted positions differ"
