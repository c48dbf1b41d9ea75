"""Host-side checks of the SVD plan (no GPU): sector structure, new-bond
order and factor descriptors against the oracle's, and error statuses."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2401_01921_amd import bst
from tests.helpers import _random_sym_pair


def _same_sectors(O, rowrank):
    sym = None if O.sym == orc.U1 else list(O.sym)
    T = bst.Tensor(O.labels, O.legs, sym=sym)
    plan = bst.Svd(T, rowrank)
    ref = orc.svd_sectors(O, rowrank)
    assert plan.nsectors == len(ref)
    assert plan.nvalues == sum(min(s["M"].shape) for s in ref)
    for k, s in enumerate(ref):
        q, m, n = plan.sector(k)
        assert (q, m, n) == (s["q"], s["M"].shape[0], s["M"].shape[1])
    return T, plan, ref


def test_paper_example_sectors():
    legs = [(1, [(1, 2), (-1, 2)]), (1, [(1, 2), (-1, 2)]), (-1, [(2, 2), (0, 4), (-2, 2)])]
    O = orc.BlockTensor(["a", "b", "c"], legs)
    T, plan, ref = _same_sectors(O, 2)
    assert [plan.sector(k)[0] for k in range(3)] == [2, 0, -2]


@pytest.mark.parametrize("sym", [(0,), (3,), (0, 2)])
def test_random_structures_match_oracle(sym):
    rng = np.random.default_rng(31 + len(sym) + sum(sym))
    for case in range(25):
        A, _ = _random_sym_pair(rng, int(rng.integers(2, 6)), 2, 0, sym, dmax=4)
        if A.numel == 0:
            continue
        rr = int(rng.integers(1, A.rank))
        T, plan, ref = _same_sectors(A, rr)
        # factor descriptors for random kept counts equal the oracle's
        kept = [int(rng.integers(0, min(s["M"].shape) + 1)) for s in ref]
        if sum(kept) == 0:
            kept[0] = 1
        U, Vd = plan.factors(kept, "m")
        ou, _, ov, _ = orc.svd_truncate(A, rr, 1 << 30, 0.0, bond="m")
        bond = [(s["q"], k) for s, k in zip(ref, kept) if k > 0]
        exp_u = orc.BlockTensor(A.labels[:rr] + ["m"], A.legs[:rr] + [(-1, bond)], sym=A.sym)
        exp_v = orc.BlockTensor(["m"] + A.labels[rr:], [(1, bond)] + A.legs[rr:], sym=A.sym)
        assert U.labels == exp_u.labels and Vd.labels == exp_v.labels
        assert U.table() == [(tuple(t), tuple(s), o) for t, s, o in exp_u.table()]
        assert Vd.table() == [(tuple(t), tuple(s), o) for t, s, o in exp_v.table()]


def test_errors():
    legs = [(1, [(1, 2), (-1, 2)]), (1, [(1, 2), (-1, 2)]), (-1, [(2, 2), (0, 4), (-2, 2)])]
    T = bst.Tensor(["a", "b", "c"], legs)
    for rr in (0, 3):
        with pytest.raises(bst.BstError) as e:
            bst.Svd(T, rr)
        assert e.value.status == "E_INVALID"
    plan = bst.Svd(T, 2)
    with pytest.raises(bst.BstError) as e:
        plan.factors([0, 0, 0], "m")
    assert e.value.status == "E_INVALID"
    with pytest.raises(bst.BstError) as e:
        plan.factors([3, 1, 1], "m")          # more than min(rows, cols) = 2
    assert e.value.status == "E_INVALID"
    with pytest.raises(bst.BstError) as e:
        plan.factors([1, 1, 1], "a")          # bond label taken by a row leg
    assert e.value.status == "E_LABEL"
