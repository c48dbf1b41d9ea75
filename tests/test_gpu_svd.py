"""GPU parity of the symmetric SVD with truncation (Sec. "Singular value
decomposition") through the C ABI, against the float64 oracle on the same
seeded inputs.  Singular values are compared directly; the singular vectors
are unique only up to sign, so what is compared is the truncated product
U S V^dagger (unique when the cut falls between distinct values) and the
orthonormality of the factors.  Kept counts are bit-exact: the oracle's
rule is applied to the GPU's own values (the decision taken in the same
precision) and, where no value lies within 1e-9 of the cut, also equals the
oracle's counts on its own values."""
import numpy as np
import pytest

from tests.gpu_common import DEV, dev, host, require_gpu, torch
from tests.helpers import _random_sym_pair
from oracle import oracle as orc
from paper_2401_01921_amd import bst
from paper_2401_01921_amd.dmrg import legs_full

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _gpu_svd(O, rowrank, keepdim, err=0.0, mb=None, absorb=None):
    sym = None if O.sym == orc.U1 else list(O.sym)
    T = bst.Tensor(O.labels, O.legs, sym=sym)
    plan = bst.Svd(T, rowrank)
    ws = bst.workspace(plan.workspace_bytes)
    ws.fill_(255)
    plan.execute(dev(O.data), ws)
    kept, s_err = plan.truncate(keepdim, err, mb, ws)
    full, _ = plan.truncate(1 << 40, 0.0, None, ws)
    Ut, Vt = plan.factors(full, "m")
    U = torch.full((Ut.numel,), np.nan, dtype=torch.float64, device=DEV)
    V = torch.full((Vt.numel,), np.nan, dtype=torch.float64, device=DEV)
    S = torch.full((sum(full),), np.nan, dtype=torch.float64, device=DEV)
    plan.write(full, 0, U, S, V, ws)
    sv_all = host(S)
    # per-sector values of the full decomposition
    svals, o = [], 0
    for k in full:
        svals.append(sv_all[o:o + k])
        o += k
    res = dict(kept=kept, s_err=s_err, svals=svals)
    if sum(kept) > 0:
        Ut, Vt = plan.factors(kept, "m")
        U = torch.full((Ut.numel,), np.nan, dtype=torch.float64, device=DEV)
        V = torch.full((Vt.numel,), np.nan, dtype=torch.float64, device=DEV)
        S = torch.full((max(sum(kept), 1),), np.nan, dtype=torch.float64, device=DEV)
        plan.write(kept, bst.ABSORB[absorb], U, S, V, ws)
        torch.cuda.synchronize()
        lu, legu, _ = legs_full(Ut)
        lv, legv, _ = legs_full(Vt)
        res["U"] = orc.BlockTensor(lu, legu, host(U), sym=O.sym)
        res["Vd"] = orc.BlockTensor(lv, legv, host(V), sym=O.sym)
        res["S"] = host(S)[:sum(kept)]
    return res


def _compare(O, rr, keepdim, err=0.0, mb=None, what=""):
    ref_full = orc.svd(O, rr)
    ref_s = [s for _, _, s, _ in ref_full]
    g = _gpu_svd(O, rr, keepdim, err, mb, absorb="u")
    smax = max([float(s[0]) for s in ref_s if s.size] + [1e-300])
    assert len(g["svals"]) == len(ref_s)
    for a, b in zip(g["svals"], ref_s):
        assert a.shape == b.shape
        assert np.max(np.abs(a - b), initial=0.0) <= 1e-12 * smax, (what, a, b)
        assert np.all(np.diff(a) <= 0)
    # kept counts: the oracle's rule on the GPU's values, bit for bit
    kept_g, serr_g = orc.truncation_counts(g["svals"], keepdim, err, mb)
    assert g["kept"] == kept_g, what
    assert g["s_err"] == serr_g, what
    kept_o, serr_o = orc.truncation_counts(ref_s, keepdim, err, mb)
    allv = np.sort(np.concatenate(ref_s + [np.zeros(0)]))
    cut = serr_o
    near = np.any((np.abs(allv - cut) < 1e-9 * smax) & (allv != cut)) if cut > 0 else False
    if not near:
        assert g["kept"] == kept_o, what
        assert abs(g["s_err"] - serr_o) <= 1e-12 * smax
    if sum(g["kept"]) == 0:
        return g
    # U S V^dagger against the oracle's truncated product (absorbed into U)
    R = orc.permute(orc.contract(g["U"], g["Vd"]), O.labels)
    ou, _, ov, _ = orc.svd_truncate(O, rr, keepdim, err, mb, bond="m", absorb="u")
    Ro = orc.permute(orc.contract(ou, ov), O.labels)
    if not near:
        assert np.max(np.abs(R.data - Ro.data), initial=0.0) <= 1e-11 * smax, what
    # V^dagger rows orthonormal per sector; U columns orthogonal with norms S
    for s in orc.svd_sectors(g["Vd"], 1):
        M = s["M"]
        assert np.allclose(M @ M.T, np.eye(M.shape[0]), atol=1e-12), what
    return g


def _paper_tensor(seed=4):
    legs = [(1, [(1, 2), (-1, 2)]), (1, [(1, 2), (-1, 2)]), (-1, [(2, 2), (0, 4), (-2, 2)])]
    T = orc.BlockTensor(["a", "b", "c"], legs)
    T.data[:] = np.random.default_rng(seed).uniform(-1, 1, T.numel)
    return T


@pytest.mark.parametrize("keep,mb", [(100, None), (4, None), (4, [1, 1, 1]), (0, [1, 0, 2])])
def test_paper_example(keep, mb):
    _compare(_paper_tensor(), 2, keep, 1e-10, mb, f"paper keep {keep} mb {mb}")


@pytest.mark.parametrize("sym", [(0,), (3,), (0, 2)])
def test_random_structures(sym):
    rng = np.random.default_rng(101 + sum(sym) + 7 * len(sym))
    done = 0
    for case in range(40):
        A, _ = _random_sym_pair(rng, int(rng.integers(2, 6)), 2, 0, sym, dmax=6)
        if A.numel == 0:
            continue
        rr = int(rng.integers(1, A.rank))
        total = sum(min(s["M"].shape) for s in orc.svd_sectors(A, rr))
        keep = int(rng.integers(0, total + 2))
        err = float(rng.choice([0.0, 0.5]))
        mb = None if case % 3 else [int(rng.integers(0, 3)) for _ in orc.svd_sectors(A, rr)]
        _compare(A, rr, keep, err, mb, f"{sym} case {case} rr {rr} keep {keep} err {err} mb {mb}")
        done += 1
    assert done >= 20


def test_large_sector_matrices():
    """Sector matrices of a few hundred rows and columns (many Jacobi rounds
    over all 16 waves), tall and wide, from a DMRG-like two-site tensor."""
    va = [(-2, 30), (0, 80), (2, 30)]
    vb = [(-2, 40), (0, 90), (2, 40)]
    ph = [(1, 1), (-1, 1)]
    O = orc.BlockTensor(["a", "s1", "s2", "b"], [(1, va), (1, ph), (1, ph), (-1, vb)])
    assert O.numel > 0
    secs = orc.svd_sectors(O, 2)
    assert max(max(s["M"].shape) for s in secs) >= 130
    O.data[:] = np.random.default_rng(9).standard_normal(O.numel)
    g = _compare(O, 2, 120, 1e-12, None, "large")
    assert sum(g["kept"]) == 120


def test_sector_residency_paths():
    """The three places a sector's Jacobi sweeps run: X and Vh in LDS (the
    30 x 40 sectors), X in LDS with Vh in global memory (110 x 130: X 114 KB,
    Vh 97 KB), and above the LDS budget a round per launch over the device
    (110 x 240: X 211 KB)."""
    va = [(-2, 30), (0, 80), (2, 30)]
    for vb, big in (([(-2, 40), (0, 90), (2, 40)], 130), ([(-2, 40), (0, 200), (2, 40)], 240)):
        ph = [(1, 1), (-1, 1)]
        O = orc.BlockTensor(["a", "s1", "s2", "b"], [(1, va), (1, ph), (1, ph), (-1, vb)])
        secs = orc.svd_sectors(O, 2)
        assert max(max(s["M"].shape) for s in secs) == big
        O.data[:] = np.random.default_rng(11).standard_normal(O.numel)
        g = _compare(O, 2, 150, 1e-12, None, f"residency {big}")
        assert sum(g["kept"]) == 150


def test_sweep_report():
    """bst_svd_sweeps: a diagonal sector (columns already orthogonal) rotates
    in no sweep, a one-column sector has none, and a random 300 x 260 one
    (rotated a round per launch) converges within the cap."""
    legs = [(1, [(0, 6), (1, 30), (2, 300)]), (-1, [(0, 6), (1, 1), (2, 260)])]
    O = orc.BlockTensor(["a", "b"], legs)
    O.block(0)[...] = np.diag(np.arange(1.0, 7.0))
    rng = np.random.default_rng(5)
    O.block(1)[...] = rng.standard_normal((30, 1))
    O.block(2)[...] = rng.standard_normal((300, 260))
    plan = bst.Svd(bst.Tensor(O.labels, O.legs), 1)
    assert [plan.sector(k)[1:] for k in range(plan.nsectors)] == [(6, 6), (30, 1), (300, 260)]
    ws = bst.workspace(plan.workspace_bytes)
    plan.execute(dev(O.data), ws)
    sw = plan.sweeps(ws)
    assert sw[0] == 0 and sw[1] == 0
    assert 1 <= sw[2] < 60


def test_big_sectors_run_a_round_per_launch():
    """Sectors above the LDS budget rotate a round per launch, a workgroup
    per pair: a tall 300 x 260 sector of rank 200 (60 zero values), a wide
    150 x 400 one and a 2100 x 20 one (fewer rounds, so their workgroups of
    the later rounds exit at once), beside a 5 x 7 sector on the
    one-workgroup path, in one execute."""
    legs = [(1, [(0, 300), (1, 150), (2, 5), (3, 2100)]), (-1, [(0, 260), (1, 400), (2, 7), (3, 20)])]
    O = orc.BlockTensor(["a", "b"], legs)
    rng = np.random.default_rng(23)
    O.block(0)[...] = rng.standard_normal((300, 200)) @ rng.standard_normal((200, 260))
    O.block(1)[...] = rng.standard_normal((150, 400))
    O.block(2)[...] = rng.standard_normal((5, 7))
    O.block(3)[...] = rng.standard_normal((2100, 20))
    assert [s["M"].shape for s in orc.svd_sectors(O, 1)] == [(300, 260), (150, 400), (5, 7), (2100, 20)]
    g = _compare(O, 1, 300, 0.0, None, "big sectors")
    assert sum(g["kept"]) == 300
    assert np.sum(g["svals"][0] > 1e-9 * g["svals"][0][0]) == 200
    # the rounds' fixed order makes a second run bit-identical
    h = _gpu_svd(O, 1, 300)
    for x, y in zip(g["svals"], h["svals"]):
        assert np.array_equal(x, y)
    assert np.array_equal(h["U"].data, _gpu_svd(O, 1, 300)["U"].data)


def test_rank_deficient_and_thin():
    """Zero singular values (a rank-deficient sector), a sector with a
    single column, and exact repeats."""
    legs = [(1, [(0, 6), (1, 1)]), (-1, [(0, 3), (1, 5)])]
    O = orc.BlockTensor(["a", "b"], legs)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 1))
    O.block(0)[...] = x @ rng.standard_normal((1, 3))   # rank 1 of 3
    O.block(1)[...] = rng.standard_normal((1, 5))
    g = _compare(O, 1, 10, 0.0, None, "deficient")
    assert np.sum(g["svals"][0] > 1e-12) == 1


def test_svd_is_deterministic():
    O = _paper_tensor(7)
    a = _gpu_svd(O, 2, 5)
    b = _gpu_svd(O, 2, 5)
    for x, y in zip(a["svals"], b["svals"]):
        assert np.array_equal(x, y)
    assert np.array_equal(a["U"].data, b["U"].data) and np.array_equal(a["Vd"].data, b["Vd"].data)
