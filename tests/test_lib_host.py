"""Host-side checks of the C-ABI library (no GPU): exported symbols, block
tables bit-exact against the oracle, plan bookkeeping (output structure,
algorithmic flops) and error statuses."""
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import oracle as orc
from paper_2401_01921_amd import bst, workloads as wl
from tests.helpers import _random_pair, _random_sym_pair

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "bst.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"^(?:bst_status|const char\*|int32_t)\s+(bst_\w+)\s*\(", hdr, re.M))
    assert declared == set(bst.EXPORTS)
    lib = bst.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert "gfx950" in bst.version()


def same_table(legs, labels=None):
    labels = labels or [f"l{i}" for i in range(len(legs))]
    O = orc.BlockTensor(labels, legs)
    T = bst.Tensor(labels, legs)
    assert (T.nblocks, T.numel) == (len(O.blocks), O.numel)
    assert T.table() == [(tuple(t), tuple(s), o) for t, s, o in O.table()]
    return O, T


def test_paper_block_table():
    legs = [(1, [(1, 1), (-1, 1)]), (1, [(1, 1), (-1, 1)]), (-1, [(2, 1), (0, 2), (-2, 1)])]
    O, T = same_table(legs, ["a", "b", "c"])
    assert T.find_block([1, 1, 2]) == 3
    with pytest.raises(bst.BstError) as e:
        T.find_block([0, 0, 1])
    assert e.value.status == "E_NOBLOCK"


@pytest.mark.parametrize("k", [2, 3, 5])
def test_workload_tables_bit_exact(k):
    for name, (labels, legs) in wl.heff_workload_specs(k).items():
        same_table(legs, labels)


def test_pairwise_tables_bit_exact():
    for name, (labels, legs) in wl.pairwise_specs().items():
        same_table(legs, labels)


@settings(max_examples=80, deadline=None)
@given(st.integers(0, 100000))
def test_random_structures_bit_exact(seed):
    rng = np.random.default_rng(seed)
    rank = int(rng.integers(0, 7))
    legs = []
    for _ in range(rank):
        ns = int(rng.integers(1, 10))
        qs = rng.integers(-6, 7, ns).tolist()   # repeated charges allowed
        legs.append((int(rng.choice([1, -1])), [(int(q), int(rng.integers(1, 10))) for q in qs]))
    same_table(legs)


def test_invalid_descriptors():
    with pytest.raises(bst.BstError) as e:
        bst.Tensor(["a"], [(1, [(0, 0)])])
    assert e.value.status == "E_INVALID"
    with pytest.raises(bst.BstError) as e:
        bst.Tensor(["a", "a"], [(1, [(0, 1)]), (-1, [(0, 1)])])
    assert e.value.status == "E_LABEL"
    with pytest.raises(bst.BstError):
        bst.Tensor(["a"], [(2, [(0, 1)])])
    T = bst.Tensor(["a", "b"], [(1, [(0, 2)]), (-1, [(1, 2)])])
    assert (T.nblocks, T.numel) == (0, 0)


SYMS = [(2,), (3,), (5,), (0, 2), (0, 3), (2, 3)]


@pytest.mark.parametrize("sym", SYMS)
def test_symmetric_structures_bit_exact(sym):
    """Z_n and product symmetries: the library's block table equals the
    oracle's, bit for bit, on random structures (repeated charges allowed)."""
    rng = np.random.default_rng(sum(sym) * 31 + len(sym))
    for _ in range(25):
        rank = int(rng.integers(0, 6))
        legs = []
        for _ in range(rank):
            ns = int(rng.integers(1, 7))
            secs = []
            for _ in range(ns):
                c = tuple(int(rng.integers(-3, 4)) if n == 0 else int(rng.integers(0, n)) for n in sym)
                secs.append((c if len(sym) > 1 else c[0], int(rng.integers(1, 6))))
            legs.append((int(rng.choice([1, -1])), secs))
        labels = [f"l{i}" for i in range(rank)]
        O = orc.BlockTensor(labels, legs, sym=sym)
        T = bst.Tensor(labels, legs, sym=list(sym))
        assert (T.nblocks, T.numel) == (len(O.blocks), O.numel)
        assert T.table() == [(tuple(t), tuple(sh), o) for t, sh, o in O.table()]
        if rank:
            assert T.symmetry() == list(sym)
            want = [q if len(sym) > 1 else (q,) for q, _ in O.legs[0][1]]
            assert T.leg_charges(0) == want


@pytest.mark.parametrize("sym", SYMS)
def test_symmetric_contract_plan_structure_and_flops(sym):
    rng = np.random.default_rng(1000 + sum(sym) * 7 + len(sym))
    for _ in range(20):
        ra, rb = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        A, B = _random_sym_pair(rng, ra, rb, min(int(rng.integers(0, 3)), ra, rb), sym)
        C = orc.contract(A, B)
        tA = bst.Tensor(A.labels, A.legs, sym=list(sym))
        tB = bst.Tensor(B.labels, B.legs, sym=list(sym))
        tC, plan = bst.contract_plan(tA, tB)
        assert tC.labels == C.labels
        if C.rank:   # a scalar result has no leg to carry the symmetries
            assert tC.symmetry() == list(sym)
        assert tC.table() == [(tuple(t), tuple(sh), o) for t, sh, o in C.table()]
        assert plan.stats().gemm_flops == orc._contract_flops(A, B)


def test_symmetric_errors_match_oracle():
    with pytest.raises(bst.BstError) as e:
        bst.Tensor(["a"], [(1, [(3, 1)])], sym=[3])
    assert e.value.status == "E_QNUM"
    with pytest.raises(bst.BstError) as e:
        bst.Tensor(["a"], [(1, [(0, 1)])], sym=[1])
    assert e.value.status == "E_INVALID"
    legs = [(1, [(0, 1), (1, 1)]), (-1, [(0, 1), (1, 1)])]
    A = bst.Tensor(["a", "x"], legs, sym=[2])
    B = bst.Tensor(["x", "b"], [(1, [(0, 1), (1, 1)]), (-1, [(0, 1), (1, 1)])], sym=[3])
    with pytest.raises(bst.BstError) as e:
        bst.contract_plan(A, B)
    assert e.value.status == "E_QNUM"
    # a U(1) leg against a Z_2 leg with the same charge values
    U = bst.Tensor(["x", "b"], [(1, [(0, 1), (1, 1)]), (-1, [(0, 1), (1, 1)])])
    with pytest.raises(bst.BstError) as e:
        bst.contract_plan(A, U)
    assert e.value.status == "E_QNUM"


def _legs_of(T):
    return T.legs()


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 100000))
def test_contract_plan_structure_and_flops(seed):
    rng = np.random.default_rng(seed)
    ra, rb = int(rng.integers(1, 5)), int(rng.integers(1, 5))
    A, B = _random_pair(rng, ra, rb, min(int(rng.integers(0, 3)), ra, rb))
    C = orc.contract(A, B)
    tA = bst.Tensor(A.labels, A.legs)
    tB = bst.Tensor(B.labels, B.legs)
    tC, plan = bst.contract_plan(tA, tB)
    labels, legs = tC.legs()
    assert labels == C.labels and legs == C.legs
    assert tC.table() == [(tuple(t), tuple(s), o) for t, s, o in C.table()]
    assert plan.stats().gemm_flops == orc._contract_flops(A, B)


def test_contract_plan_errors_match_oracle():
    a = (1, [(0, 2), (1, 3)])
    A = bst.Tensor(["x", "y"], [a, (-1, [(0, 2), (1, 3)])])
    cases = [
        ([(-1, [(0, 2), (1, 3)]), (-1, [(0, 2)])], "E_DIRECTION"),
        ([(1, [(0, 2), (2, 3)]), (-1, [(0, 2)])], "E_QNUM"),
        ([(1, [(0, 2), (1, 4)]), (-1, [(0, 2)])], "E_DIM"),
        ([(1, [(1, 3), (0, 2)]), (-1, [(0, 2)])], "E_QNUM"),
    ]
    for legs, status in cases:
        B = bst.Tensor(["y", "z"], legs)
        with pytest.raises(bst.BstError) as e:
            bst.contract_plan(A, B)
        assert e.value.status == status
        OA = orc.BlockTensor(["x", "y"], [a, (-1, [(0, 2), (1, 3)])])
        OB = orc.BlockTensor(["y", "z"], legs)
        with pytest.raises(orc.OracleError) as eo:
            orc.contract(OA, OB)
        assert eo.value.status == status


@pytest.mark.parametrize("k", [2, 3, 5])
def test_heff_plan_flops_match_oracle(k):
    specs = wl.heff_workload_specs(k)
    O = {n: orc.BlockTensor(*v) for n, v in specs.items()}
    T = {n: bst.Tensor(*v) for n, v in specs.items()}
    plan = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"])
    f = orc.heff_flops(O["L"], O["W1"], O["W2"], O["R"], O["psi"])
    steps = {s["name"]: s for s in plan.steps()}
    assert steps["gemm_L_psi"]["flops"] == f[0]
    assert steps["mpo_apply"]["flops"] == f[1] + f[2]
    assert steps["gemm_T3_R"]["flops"] == f[3]
    assert plan.stats().flops == sum(f)


def test_heff_plan_rejects_mismatched_operands():
    v = wl.gaussian_sector_dims(32, 2)
    specs = wl.heff_specs("1/2", v, v)
    T = {n: bst.Tensor(*s) for n, s in specs.items()}
    bad_R = bst.Tensor(specs["R"][0], [(1, v)] + specs["R"][1][1:])   # b leg direction flipped
    with pytest.raises(bst.BstError) as e:
        bst.heff_plan(T["L"], T["W1"], T["W2"], bad_R, T["psi"])
    assert e.value.status in ("E_STRUCTURE", "E_DIRECTION")
    other = wl.gaussian_sector_dims(34, 2)
    Lx = bst.Tensor(specs["L"][0], [specs["L"][1][0], specs["L"][1][1], (-1, other)])
    with pytest.raises(bst.BstError) as e:
        bst.heff_plan(Lx, T["W1"], T["W2"], T["R"], T["psi"])
    assert e.value.status == "E_DIM"


def test_permute_plan_structure():
    rng = np.random.default_rng(7)
    legs = [(1, [(0, 2), (1, 3)]), (-1, [(0, 1), (1, 2)]), (1, [(-1, 2), (0, 3)]), (-1, [(0, 2), (-1, 1)])]
    O = orc.BlockTensor(["a", "b", "c", "d"], legs)
    T = bst.Tensor(["a", "b", "c", "d"], legs)
    for order in (["c", "a", "d", "b"], ["a", "b", "c", "d"], ["d", "c", "b", "a"]):
        P = orc.permute(O, order)
        out, plan = bst.permute_plan(T, order)
        labels, lg = out.legs()
        assert labels == P.labels and lg == P.legs
        assert out.table() == [(tuple(t), tuple(s), o) for t, s, o in P.table()]
    with pytest.raises(bst.BstError) as e:
        bst.permute_plan(T, ["a", "b", "c", "x"])
    assert e.value.status == "E_LABEL"


def test_batch_plan_sums_members():
    plans = []
    total = 0.0
    for chi, q in wl.batch_draws()[:4]:
        v = wl.gaussian_sector_dims(chi, q)
        T = {n: bst.Tensor(*s) for n, s in wl.heff_specs("1/2", v, v).items()}
        p = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], "bf16x3")
        total += p.stats().flops
        plans.append(p)
    b = bst.heff_batch_plan(plans)
    assert b.stats().flops == total
    assert b.n_in == 20 and b.n_out == 4


def test_binding_fails_loudly_without_library(tmp_path):
    """The binding has no fallback: a package copy without libbst.so must not import."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2401_01921_amd"
    pkg.mkdir()
    src = os.path.join(ROOT, "paper_2401_01921_amd")
    for f in ("__init__.py", "bst.py"):
        shutil.copy(os.path.join(src, f), pkg / f)
    code = ("import sys\n"
            "try:\n"
            "    from paper_2401_01921_amd import bst\n"
            "except ImportError as e:\n"
            "    print('IMPORT_ERROR', e); sys.exit(0)\n"
            "sys.exit(3)\n")
    env = {k: v for k, v in os.environ.items() if k != "BST_LIB"}
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True,
                       text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "not built" in r.stdout


def test_complex_plans_structure_and_errors():
    """Complex plans: output descriptors equal the float64 ones, buffers are
    two float64 per element, reserved labels and rank limits are refused."""
    rng = np.random.default_rng(12)
    A, B = _random_pair(rng, 3, 3, 2)
    tA, tB = bst.Tensor(A.labels, A.legs), bst.Tensor(B.labels, B.legs)
    tC, plan = bst.contract_plan(tA, tB, "fp64", dtype="c128")
    rC, rplan = bst.contract_plan(tA, tB, "fp64")
    assert tC.table() == rC.table() and tC.labels == rC.labels
    assert plan.in_numel == [2 * tA.numel, 2 * tB.numel] and plan.out_numel == [2 * tC.numel]
    assert plan.stats().flops == pytest.approx(4 * rplan.stats().flops)
    tP, pplan = bst.permute_plan(tA, list(reversed(tA.labels)), dtype="c128")
    assert pplan.in_numel == [2 * tA.numel]
    with pytest.raises(bst.BstError) as e:
        bst.permute_plan(bst.Tensor(["#re", "x"], [(1, [(0, 2)]), (-1, [(0, 2)])]), ["x", "#re"], dtype="c128")
    assert e.value.status == "E_LABEL"
    big = bst.Tensor([f"l{i}" for i in range(8)], [(1, [(0, 1)])] * 8)
    with pytest.raises(bst.BstError) as e:
        bst.permute_plan(big, [f"l{i}" for i in range(8)], dtype="c128")
    assert e.value.status == "E_INVALID"


def test_complex_output_rank_limit():
    A = bst.Tensor([f"a{i}" for i in range(4)], [(1, [(0, 1)])] * 4)
    B = bst.Tensor([f"b{i}" for i in range(4)], [(1, [(0, 1)])] * 4)
    with pytest.raises(bst.BstError) as e:
        bst.contract_plan(A, B, "fp64", dtype="c128")
    assert e.value.status == "E_INVALID" and "rank 7" in str(e.value)


@pytest.mark.parametrize("k", [2, 5])
def test_fused_mpo_schedule_built(k, monkeypatch):
    """The plan builds the fused L.psi + MPO schedule for the H_eff operators
    (spin-1/2 chi = 512, spin-1 chi = 4096): with BST_FUSED_MPO=1 the BF16x3
    form reports the fused step and no L.psi GEMM; FP64 never fuses."""
    from paper_2401_01921_amd import workloads as wl
    T = {n: bst.Tensor(*s) for n, s in wl.heff_workload_specs(k).items()}
    plan = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], "bf16x3")
    monkeypatch.setenv("BST_FUSED_MPO", "1")
    tiles = plan.tiles()
    assert "mpo_apply:fused" in tiles and "gemm_L_psi" not in tiles, tiles
    plan.set_precision("fp64")
    assert "gemm_L_psi" in plan.tiles()
    monkeypatch.setenv("BST_FUSED_MPO", "0")
    plan.set_precision("bf16x3")
    assert "gemm_L_psi" in plan.tiles()
