"""The walk's target order (tc_tree_target_order) through the C ABI.

The order groups targets into wavefronts and decides no result, so its bars
are: it is a permutation of the sorted positions (every target is served
exactly once), and it is the Hilbert order of the particles' level-21 cells,
ties (particles sharing a cell) in key order.  The Hilbert index here comes
from tests/hilbert_ref.py (numpy, pinned on the CPU by the unit steps of the
curve), for comparison with the library's top-down construction from the
tree.
"""
import numpy as np
import pytest

import workloads
from hilbert_ref import hilbert_from_morton

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _dups(n, seed):
    g = np.random.default_rng(seed)
    pos = g.random((n, 3))
    pos[n // 3:n // 3 + 7] = pos[0]
    pos[n // 2:n // 2 + 300] = pos[5]
    return pos


CASES = [
    ("plummer16k", lambda: workloads.plummer(16384, 1000)),
    ("disc20k_f32", lambda: workloads.disc_galaxy(16000, 4000, 5, dtype=np.float32)[0::2]),
    ("dups4097", lambda: (_dups(4097, 4), np.full(4097, 1.0 / 4097))),
    ("n1", lambda: workloads.plummer(1, 7)),
    ("n2", lambda: workloads.plummer(2, 7)),
    ("n65", lambda: workloads.plummer(65, 7)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_target_order_is_the_hilbert_permutation(name, make):
    import paper_2412_01733_amd as tc
    pos, m = make()
    print("case", name, flush=True)
    t = tc.Tree()
    t.build(torch.from_numpy(np.ascontiguousarray(pos)).to(dev()),
            torch.from_numpy(np.ascontiguousarray(m)).to(dev())).moments()
    order = t.target_order().cpu().numpy().astype(np.int64)
    n = pos.shape[0]
    assert np.array_equal(np.sort(order), np.arange(n)), "not a permutation"
    keys = t.export(moments=False)["keys"].cpu().numpy().view(np.uint64)
    h = hilbert_from_morton(keys)
    assert np.array_equal(order, np.argsort(h, kind="stable")), "not the Hilbert order"


def test_target_order_needs_moments():
    import paper_2412_01733_amd as tc
    pos, m = workloads.plummer(100, 3)
    t = tc.Tree()
    t.build(torch.from_numpy(pos).to(dev()), torch.from_numpy(m).to(dev()))
    with pytest.raises(RuntimeError):
        t.target_order()
