"""GPU parity through the C ABI: permute (bit-exact), pairwise contraction and
H_eff.psi in every arithmetic form against the float64 oracle, on seeded
inputs shared by both sides."""
import numpy as np
import pytest

from tests.gpu_common import (DEV, TOL, check, dev, heff_operands, host, lib_heff, rel_err,
                              require_gpu, run_heff, torch)
from tests.helpers import _random_pair, _random_sym_pair
from oracle import oracle as orc
from paper_2401_01921_amd import bst, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _print(*a):
    print(*a, flush=True)


def test_permute_bit_exact_random_structures():
    rng = np.random.default_rng(11)
    for case in range(25):
        rank = int(rng.integers(1, 6))
        legs = []
        for _ in range(rank):
            ns = int(rng.integers(1, 4))
            qs = sorted(rng.choice(np.arange(-2, 3), ns, replace=False).tolist())
            legs.append((int(rng.choice([1, -1])), [(q, int(rng.integers(1, 40))) for q in qs]))
        labels = [f"l{i}" for i in range(rank)]
        O = orc.BlockTensor(labels, legs)
        if O.numel == 0 or O.numel > 3_000_000:
            continue
        O.data[:] = wl.normal(100 + case, O.numel)
        order = [labels[i] for i in rng.permutation(rank)]
        _print("permute case", case, rank, O.numel, order)
        P = orc.permute(O, order)
        T = bst.Tensor(labels, legs)
        out_t, plan = bst.permute_plan(T, order)
        x = dev(O.data)
        y = torch.full((out_t.numel,), np.nan, dtype=torch.float64, device=DEV)
        ws = bst.workspace(plan.workspace_bytes)
        plan.execute([x], [y], ws)
        torch.cuda.synchronize()
        assert np.array_equal(host(y), P.data)


@pytest.mark.parametrize("order", [["b", "a", "c"], ["c", "a", "b"], ["a", "c", "b"], ["c", "b", "a"]])
def test_permute_bit_exact_large_blocks(order):
    """Blocks wider than one tile and rows longer than a wave in both
    directions, odd extents (odd block offsets), fastest leg kept or moved."""
    legs = [(1, [(-1, 70), (0, 131), (1, 3)]), (1, [(0, 150), (1, 9)]), (-1, [(-1, 67), (0, 130), (1, 41), (2, 5)])]
    O = orc.BlockTensor(["a", "b", "c"], legs)
    O.data[:] = wl.normal(77, O.numel)
    P = orc.permute(O, order)
    T = bst.Tensor(["a", "b", "c"], legs)
    out_t, plan = bst.permute_plan(T, order)
    y = torch.full((out_t.numel,), np.nan, dtype=torch.float64, device=DEV)
    plan.execute([dev(O.data)], [y], bst.workspace(plan.workspace_bytes))
    torch.cuda.synchronize()
    assert np.array_equal(host(y), P.data)


@pytest.mark.parametrize("cdim", [90, 150, 16, 48])
def test_permute_narrow_last_strips(cdim):
    """Transposing tiles of every shape: the last strip of the last dim is
    26, 22, 16 or 48 elements wide (128 x 32, 256 x 16 or 64 x 64 tiles)."""
    legs = [(1, [(-1, 37), (0, 150), (1, 21)]), (1, [(0, 70), (1, 33)]), (-1, [(-1, cdim), (0, cdim + 3), (1, 7)])]
    O = orc.BlockTensor(["a", "b", "c"], legs)
    O.data[:] = wl.normal(78, O.numel)
    for order in (["c", "a", "b"], ["c", "b", "a"], ["a", "c", "b"]):
        P = orc.permute(O, order)
        T = bst.Tensor(["a", "b", "c"], legs)
        out_t, plan = bst.permute_plan(T, order)
        y = torch.full((out_t.numel,), np.nan, dtype=torch.float64, device=DEV)
        plan.execute([dev(O.data)], [y], bst.workspace(plan.workspace_bytes))
        torch.cuda.synchronize()
        assert np.array_equal(host(y), P.data), (cdim, order)


def test_permute_paper_example():
    T = bst.Tensor(["a", "b", "c"], [(1, [(0, 2)]), (1, [(0, 2)]), (-1, [(0, 2)])])
    out_t, plan = bst.permute_plan(T, ["a", "c", "b"])
    y = torch.empty(8, dtype=torch.float64, device=DEV)
    plan.execute([dev(np.arange(8.0))], [y], bst.workspace(plan.workspace_bytes))
    torch.cuda.synchronize()
    assert host(y).tolist() == [0, 2, 1, 3, 4, 6, 5, 7]


def _contract_case(A, B, prec):
    C = orc.contract(A, B)
    sym = None if A.sym == orc.U1 else list(A.sym)
    tA, tB = bst.Tensor(A.labels, A.legs, sym=sym), bst.Tensor(B.labels, B.legs, sym=sym)
    tC, plan = bst.contract_plan(tA, tB, prec)
    out = torch.full((tC.numel,), np.nan, dtype=torch.float64, device=DEV)
    plan.execute([dev(A.data), dev(B.data)], [out], bst.workspace(plan.workspace_bytes))
    torch.cuda.synchronize()
    return host(out), C.data


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_pairwise_workload(prec):
    specs = wl.pairwise_specs()
    A = orc.BlockTensor(*specs["A"])
    B = orc.BlockTensor(*specs["B"])
    A.data[:] = wl.normal(wl.seed_for(1, "A"), A.numel)
    B.data[:] = wl.normal(wl.seed_for(1, "B"), B.numel)
    got, ref = _contract_case(A, B, prec)
    check(got, ref, prec, "pairwise")
    # the two output blocks nothing reaches are exact zeros
    zero = np.zeros_like(ref, dtype=bool)
    C = orc.contract(A, B)
    for b in range(len(C.blocks)):
        if not np.any(C.block(b)):
            zero[C.offsets[b]:C.offsets[b] + C.block(b).size] = True
    assert zero.sum() > 0 and np.all(got[zero] == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_random_contractions(prec):
    """Random structures and label orders: covers A packing, B packing,
    transposed B, outer products, full contractions and ragged tiles."""
    rng = np.random.default_rng(21)
    for case in range(30):
        ra, rb = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        nc = min(int(rng.integers(0, 4)), ra, rb)
        A, B = _random_pair(rng, ra, rb, nc)
        # stretch the dims so that tiles are ragged and span several tiles
        free = [i for i, l in enumerate(A.labels) if l not in B.labels]
        if free:
            scale = int(rng.integers(1, 30))
            A = orc.BlockTensor(A.labels, [(d, [(q, g * scale if i == free[0] else g) for q, g in s])
                                           for i, (d, s) in enumerate(A.legs)])
            A.data[:] = rng.standard_normal(A.numel)
        if A.numel == 0 or B.numel == 0:
            continue
        got, ref = _contract_case(A, B, prec)
        check(got, ref, prec, f"contract case {case} {A.labels} {B.labels}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_heff_spin_half_chi512(prec):
    specs, O = heff_operands(2)
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T, plan = lib_heff(specs, prec)
    got = run_heff(plan, O)
    check(got, ref, prec, "heff chi512")


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_heff_mpo_64bit_indexing(prec, monkeypatch):
    """The MPO apply with 64-bit plane indexing (chosen by the plan only for
    operators whose plane offsets pass 2^32 bytes; forced here) gives the
    same result as the 32-bit indexing and the oracle's."""
    specs, O = heff_operands(2)
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T, plan32 = lib_heff(specs, prec)
    assert "mpo_apply:i32" in plan32.tiles()
    monkeypatch.setenv("BST_MPO_INDEX64", "1")
    T, plan64 = lib_heff(specs, prec)
    monkeypatch.delenv("BST_MPO_INDEX64")
    assert "mpo_apply:i64" in plan64.tiles(), plan64.tiles()
    got64 = run_heff(plan64, O)
    got32 = run_heff(plan32, O)
    assert np.array_equal(got64, got32)
    check(got64, ref, prec, "heff chi512 64-bit MPO indexing")


@pytest.mark.parametrize("spin", ["1/2", "1"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_heff_xx_mpo(prec, spin):
    """The XX MPO (the paper's benchmark model; bond of 4 channels, so other
    MPO coefficient classes and T1/T3 row groups than the Heisenberg MPO)."""
    specs, O = heff_operands(2, spin=spin, model="xx")
    assert O["W1"].legs[0][1][1] == (0, 2)
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T, plan = lib_heff(specs, prec)
    got = run_heff(plan, O)
    check(got, ref, prec, f"heff xx chi512 spin {spin}")


@pytest.mark.parametrize("sym", [(2,), (3,), (0, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_symmetric_contractions(prec, sym):
    """Z_n and U(1) x Z_2 structures (Sec. "Symmetry and quantum numbers"):
    random pairs, dims stretched so that tiles are ragged."""
    rng = np.random.default_rng(5 + sum(sym) + 10 * len(sym))
    for case in range(12):
        ra, rb = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        nc = min(int(rng.integers(0, 4)), ra, rb)
        A, B = _random_sym_pair(rng, ra, rb, nc, sym, dmax=5)
        free = [i for i, l in enumerate(A.labels) if l not in B.labels]
        if free:
            scale = int(rng.integers(1, 25))
            A = orc.BlockTensor(A.labels, [(d, [(q, g * scale if i == free[0] else g) for q, g in s])
                                           for i, (d, s) in enumerate(A.legs)], sym=sym)
            A.data[:] = rng.standard_normal(A.numel)
        if A.numel == 0 or B.numel == 0:
            continue
        got, ref = _contract_case(A, B, prec)
        check(got, ref, prec, f"sym contract {sym} {case} {A.labels} {B.labels}")


def _heff_sym_operands(sym, virt, phys, bond, seed):
    """Random L, W, R, psi of a two-site H_eff under `sym` (legs as in the
    U(1) workloads: psi in, in, in, out; L in, out, out; R out, in, in;
    W in, in, out, out)."""
    rng = np.random.default_rng(seed)
    specs = {"L": (["a", "w", "ap"], [(1, virt), (-1, bond), (-1, virt)]),
             "R": (["b", "w", "bp"], [(-1, virt), (1, bond), (1, virt)]),
             "W1": (["wl", "s", "sp", "wr"], [(1, bond), (1, phys), (-1, phys), (-1, bond)]),
             "psi": (["a", "s1", "s2", "b"], [(1, virt), (1, phys), (1, phys), (-1, virt)])}
    specs["W2"] = specs["W1"]
    O = {n: orc.BlockTensor(*sp, sym=sym) for n, sp in specs.items()}
    for n in ("L", "R", "W1", "psi"):
        O[n].data[:] = rng.standard_normal(O[n].numel)
    O["W2"] = O["W1"]
    return specs, O


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("which", ["z2", "u1xz2"])
def test_heff_symmetric_operands(prec, which):
    """H_eff with Z_2 legs (virtual {0: 96, 1: 80}, MPO bond {0: 3, 1: 2}) or
    U(1) x Z_2 legs, random operands, against the oracle's apply."""
    if which == "z2":
        sym = (2,)
        virt, phys, bond = [(0, 96), (1, 80)], [(0, 1), (1, 1)], [(0, 3), (1, 2)]
    else:
        sym = (0, 2)
        virt = [((q, p), 20 + 7 * abs(q) + 5 * p) for q in range(-3, 4) for p in (0, 1)]
        phys = [((1, 0), 1), ((-1, 1), 1)]
        bond = [((-2, 1), 1), ((0, 0), 2), ((0, 1), 1), ((2, 1), 1)]
    specs, O = _heff_sym_operands(sym, virt, phys, bond, 77)
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T = {n: bst.Tensor(*sp, sym=list(sym)) for n, sp in specs.items()}
    plan = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], prec)
    got = run_heff(plan, O)
    check(got, ref, prec, f"heff {which} {O['psi'].numel}")


def test_heff_fp64_is_deterministic():
    specs, O = heff_operands(2)
    T, plan = lib_heff(specs, "fp64")
    a = run_heff(plan, O)
    b = run_heff(plan, O)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_heff_spin_half_chi2048_error_table(prec):
    specs, O = heff_operands(3)
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T, plan = lib_heff(specs, prec)
    got = run_heff(plan, O)
    check(got, ref, prec, "heff chi2048")


_CHI4096 = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_heff_spin_one_chi4096(prec):
    """The Lanczos workload's operator at full size, every form, against the
    oracle at the form's tolerance (the oracle's apply is computed once)."""
    if not _CHI4096:
        specs, O = heff_operands(5, recipe="dmrg_like")
        _CHI4096.update(specs=specs, O=O,
                        ref=orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data)
    specs, O, ref = _CHI4096["specs"], _CHI4096["O"], _CHI4096["ref"]
    T, plan = lib_heff(specs, prec)
    got = run_heff(plan, O)
    check(got, ref, prec, "heff chi4096")


def test_heff_graph_replay_matches_eager():
    specs, O = heff_operands(2)
    T, plan = lib_heff(specs, "bf16x3")
    eager = run_heff(plan, O)
    plan.use_graph(True)
    ins = [dev(O[n].data) for n in ("L", "W1", "W2", "R", "psi")]
    ws = bst.workspace(plan.workspace_bytes)
    for rep in range(4):
        out = torch.full((O["psi"].numel,), np.nan, dtype=torch.float64, device=DEV)
        plan.execute(ins, [out], ws)
        torch.cuda.synchronize()
        junk = torch.randn(1000, device=DEV).sum().item()   # eager work between replays
        assert np.array_equal(host(out), eager), rep
    plan.use_graph(False)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_every_gemm_variant(prec):
    """Every compiled GEMM variant (tile shape, LDS-staged or direct) that the
    autotuner may pick gives the oracle's result on the chi = 512 H_eff."""
    specs, O = heff_operands(2)
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T, plan = lib_heff(specs, prec)
    for tile in range(plan.tile_count(prec)):
        plan.set_tile(prec, tile)
        got = run_heff(plan, O)
        check(got, ref, prec, f"variant {tile} {plan.tiles()}")
    # the generic contraction path (no pre-split planes) with every variant
    rng = np.random.default_rng(5)
    A, B = _random_pair(rng, 3, 3, 2)
    free = [i for i, l in enumerate(A.labels) if l not in B.labels]
    A = orc.BlockTensor(A.labels, [(d, [(q, g * 23 if i == free[0] else g) for q, g in s])
                                   for i, (d, s) in enumerate(A.legs)])
    A.data[:] = rng.standard_normal(A.numel)
    C = orc.contract(A, B)
    tA, tB = bst.Tensor(A.labels, A.legs), bst.Tensor(B.labels, B.legs)
    tC, cplan = bst.contract_plan(tA, tB, prec)
    for tile in range(cplan.tile_count(prec)):
        cplan.set_tile(prec, tile)
        out = torch.full((tC.numel,), np.nan, dtype=torch.float64, device=DEV)
        cplan.execute([dev(A.data), dev(B.data)], [out], bst.workspace(cplan.workspace_bytes))
        torch.cuda.synchronize()
        check(host(out), C.data, prec, f"contract variant {tile}")


def _pipelined_tiles(plan, prec):
    """Indices of the pipelined (k-step schedule) plane-GEMM shapes."""
    out = []
    for tile in range(plan.tile_count(prec)):
        plan.set_tile(prec, tile)
        if "s" in plan.tiles().split(";")[0].split(":")[1]:
            out.append(tile)
    return out


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
def test_pipelined_gemm_full_size(prec):
    """The pipelined plane GEMMs on the spin-1 chi = 4096 operator: every
    shape equals the LDS-staged kernel bit for bit (same products, same
    k order) and the oracle within the form's tolerance."""
    specs, O = heff_operands(5, recipe="dmrg_like")
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T, plan = lib_heff(specs, prec)
    plan.set_tile(prec, 0)   # LDS-staged 64x64
    base = run_heff(plan, O)
    check(base, ref, prec, "pipelined base (LDS kernel)")
    tiles = _pipelined_tiles(plan, prec)
    assert tiles
    for tile in tiles:
        plan.set_tile(prec, tile)
        got = run_heff(plan, O)
        _print("pipelined", prec, tile, plan.tiles(), "max|diff| vs LDS kernel",
               float(np.max(np.abs(got - base))))
        assert np.array_equal(got, base), plan.tiles()
        check(got, ref, prec, f"pipelined {tile}")


def test_workspace_overwritten_between_calls():
    """The plan's tables live in the workspace; after the caller overwrites
    the workspace (here with NaN bytes) the binding makes the plan upload
    them again, and the result is unchanged."""
    specs, O = heff_operands(2)
    T, plan = lib_heff(specs, "bf16x3")
    ins = [dev(O[n].data) for n in ("L", "W1", "W2", "R", "psi")]
    out = torch.empty(O["psi"].numel, dtype=torch.float64, device=DEV)
    ws = bst.workspace(plan.workspace_bytes)
    plan.execute(ins, [out], ws)
    torch.cuda.synchronize()
    first = host(out)
    ws.fill_(255)
    out.fill_(float("nan"))
    plan.execute(ins, [out], ws)
    torch.cuda.synchronize()
    assert np.array_equal(host(out), first)


def test_fp64_panels_full_size(monkeypatch):
    """Float64 sector GEMMs on the padded layouts (pipelined kernel) on the
    spin-1 chi = 4096 operator: every tile shape gives the same bits (same
    products, same k order), the oracle's result to float64 rounding, and
    the per-block-pair kernels' result to the same tolerance."""
    specs, O = heff_operands(5, recipe="dmrg_like")
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T, bplan = lib_heff(specs, "fp64")
    assert "p;" not in bplan.tiles(), bplan.tiles()   # the default: per-block-pair kernels
    blocks = run_heff(bplan, O)
    check(blocks, ref, "fp64", "fp64 per-block kernels")
    monkeypatch.setenv("BST_FP64_PANELS", "1")
    T, plan = lib_heff(specs, "fp64")
    tiles = _pipelined_tiles(plan, "fp64")
    assert len(tiles) == plan.tile_count("fp64")   # float64 panels: pipelined shapes only
    base = None
    for tile in tiles:
        plan.set_tile("fp64", tile)
        assert "p;" in plan.tiles(), plan.tiles()
        got = run_heff(plan, O)
        check(got, ref, "fp64", f"fp64 panels {plan.tiles()}")
        if base is None:
            base = got
        assert np.array_equal(got, base), plan.tiles()


@pytest.mark.parametrize("k", [2, 3])
def test_fp64_autotuned_variant(k):
    """The autotuner times the FP64 apply on the per-block-pair kernels and on
    the float64 panels and keeps the faster; either way the result is the
    oracle's to float64 rounding and repeats bit for bit."""
    specs, O = heff_operands(k)
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    T, plan = lib_heff(specs, "fp64")
    ins = [dev(O[n].data) for n in ("L", "W1", "W2", "R", "psi")]
    out = torch.empty(O["psi"].numel, dtype=torch.float64, device=DEV)
    plan.autotune(ins, [out], bst.workspace(plan.workspace_bytes), reps=2)
    _print("fp64 autotuned", k, plan.tiles())
    a = run_heff(plan, O)
    b = run_heff(plan, O)
    check(a, ref, "fp64", f"fp64 autotuned {plan.tiles()}")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("case", ["chi512", "chi4096"])
def test_fused_lpsi_mpo(case, monkeypatch):
    """L.psi fused into the MPO apply (BF16x3): T1 is formed in registers
    with the same products in the same order as the L.psi GEMM and folded
    into the outputs in the MPO apply's order, so the result equals the
    two-kernel path bit for bit, and the oracle within the form's bar.
    chi512: spin-1/2 operator; chi4096: the spin-1 Lanczos operator."""
    if case == "chi512":
        specs, O = heff_operands(2)
    else:
        specs, O = heff_operands(5, recipe="dmrg_like")
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    monkeypatch.setenv("BST_FUSED_MPO", "0")
    T, plan = lib_heff(specs, "bf16x3")
    two = run_heff(plan, O)
    assert "mpo_apply:i" in plan.tiles()
    monkeypatch.setenv("BST_FUSED_MPO", "1")
    assert "mpo_apply:fused" in plan.tiles() and "gemm_L_psi" not in plan.tiles(), plan.tiles()
    fused = run_heff(plan, O)
    _print("fused", case, plan.tiles(), "max|diff| vs two kernels", float(np.max(np.abs(fused - two))))
    assert np.array_equal(fused, two)
    check(fused, ref, "bf16x3", f"fused L.psi + MPO {case}")
