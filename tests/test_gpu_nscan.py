"""Sampled parity along the benchmark's N-scan (the N range of the paper's
efficiency-versus-N figure): Plummer spheres N = 2^17 ... 2^24, FP32, theta
= 0.5, eps = 0.005, seed 1002, the configuration `bench.py --mode nscan`
times.  At every N: 512 seeded targets against the oracle (its full tree,
each target evaluated one by one) within the bars of tests/bars.py, and
interaction counts differing on < 1% of them, for both walks."""
import numpy as np
import pytest

import oracle
import workloads
from bars import check_errors, rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("e", list(range(17, 25)))
def test_nscan_sampled_parity(e):
    import paper_2412_01733_amd as tc
    n = 1 << e
    pos, m = workloads.plummer(n, 1002, dtype=np.float32)
    dev = torch.device("cuda:0")
    tg = workloads.target_sample(n, 512, 3000 + e)
    sel = torch.from_numpy(tg).to(dev)
    T = oracle.Tree(pos, m)
    ra, rp, rn = T.forces(0.5, 0.005, targets=tg, nthreads=16)
    tree = tc.Tree().build(torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev)).moments()
    for walk in ("f32c", "f64"):
        acc, pot = tree.forces(0.5, 0.005, walk=walk, count=True)
        cnt = tree.interaction_counts()[sel].cpu().numpy().astype(np.int64)
        same = cnt == rn
        check_errors(rel_err(acc[sel].double().cpu().numpy(), ra), walk, same, "acc N=2^%d" % e)
        check_errors(rel_err(pot[sel].double().cpu().numpy(), rp), walk, same, "pot N=2^%d" % e)
        assert 1 - same.mean() < 0.01, (walk, e, 1 - same.mean())
