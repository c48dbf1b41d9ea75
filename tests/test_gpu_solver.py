"""GPU parity of the batched H_eff launch, the autotuner and the Lanczos
ground-state solver (singlets, exact diagonalisation of whole chains through
exact environments, and the float64 oracle's Lanczos on the same inputs)."""
import json
import os

import numpy as np
import pytest

from tests import chain_env
from tests.gpu_common import (DEV, TOL, check, dev, heff_operands, host, lib_heff, rel_err,
                              require_gpu, run_heff, torch)
from oracle import oracle as orc
from paper_2401_01921_amd import bst, workloads as wl

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _print(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ batch
def _batch_members(n):
    members = []
    for i, (chi, q) in enumerate(wl.batch_draws()[:n]):
        v = wl.gaussian_sector_dims(chi, q)
        specs = wl.heff_specs("1/2", v, v)
        T = {k: bst.Tensor(*s) for k, s in specs.items()}
        data = {
            "L": wl.normal(wl.seed_for(4, "L", i), T["L"].numel),
            "R": wl.normal(wl.seed_for(4, "R", i), T["R"].numel),
            "psi": wl.normal(wl.seed_for(4, "psi", i), T["psi"].numel),
            "W1": T["W1"].from_dense(wl.heisenberg_mpo_dense("1/2")),
        }
        data["W2"] = data["W1"]
        members.append((specs, T, data))
    return members


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_batched_heff_matches_single_applies(prec):
    """The 64 uneven applies in one grouped launch per step (float32 bulk is
    the batched workload's stated form), captured in a hipGraph: the first
    execute captures and runs it, the second replays it into outputs that
    were refilled with NaN, so a replay that writes nothing fails."""
    members = _batch_members(64)
    plans = [bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], prec) for _, T, _ in members]
    batch = bst.heff_batch_plan(plans)
    ins, outs = [], []
    for _, T, d in members:
        ins += [dev(d[k]) for k in ("L", "W1", "W2", "R", "psi")]
        outs.append(torch.full((T["psi"].numel,), np.nan, dtype=torch.float64, device=DEV))
    batch.use_graph(True)
    ws = bst.workspace(batch.workspace_bytes)
    batch.execute(ins, outs, ws)    # capture and run
    torch.cuda.synchronize()
    first = [host(o) for o in outs]
    for o in outs:
        o.fill_(float("nan"))
    batch.execute(ins, outs, ws)    # graph replay
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(host(o), first[i]), i
    # every member equals its own single-apply plan (same tiles, same order)
    for i, (p, (_, T, d)) in enumerate(zip(plans, members)):
        single = torch.empty_like(outs[i])
        p.execute(ins[5 * i:5 * i + 5], [single], bst.workspace(p.workspace_bytes))
        torch.cuda.synchronize()
        assert np.array_equal(host(single), host(outs[i])), i
    # and a few members against the oracle
    for i in (0, 17, 63):
        specs, T, d = members[i]
        O = {k: orc.BlockTensor(*specs[k], d[k]) for k in ("L", "W1", "W2", "R", "psi")}
        ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
        check(host(outs[i]), ref, prec, f"batch member {i}")


def test_batched_heff_pipelined_gemm():
    """The batch's merged problem lists (operands in many buffers) through
    the pipelined plane GEMM: bit-identical to the LDS-staged kernel."""
    members = _batch_members(64)
    plans = [bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], "bf16x3") for _, T, _ in members]
    batch = bst.heff_batch_plan(plans)
    ins, outs = [], []
    for _, T, d in members:
        ins += [dev(d[k]) for k in ("L", "W1", "W2", "R", "psi")]
        outs.append(torch.full((T["psi"].numel,), np.nan, dtype=torch.float64, device=DEV))
    ws = bst.workspace(batch.workspace_bytes)
    batch.set_tile("bf16x3", 0)   # LDS-staged 64x64
    batch.execute(ins, outs, ws)
    torch.cuda.synchronize()
    base = [host(o) for o in outs]
    for tile in range(batch.tile_count("bf16x3")):
        batch.set_tile("bf16x3", tile)
        if "s" not in batch.tiles().split(";")[0].split(":")[1]:
            continue
        for o in outs:
            o.fill_(float("nan"))
        batch.execute(ins, outs, ws)
        torch.cuda.synchronize()
        _print("batch pipelined", tile, batch.tiles())
        for i, o in enumerate(outs):
            assert np.array_equal(host(o), base[i]), (tile, i)


def test_autotune_keeps_results():
    specs, O = heff_operands(3)
    ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
    for prec in ("fp64", "bf16x3"):
        T, plan = lib_heff(specs, prec)
        ins = [dev(O[n].data) for n in ("L", "W1", "W2", "R", "psi")]
        out = torch.empty(O["psi"].numel, dtype=torch.float64, device=DEV)
        ws = bst.workspace(plan.workspace_bytes)
        plan.autotune(ins, [out], ws, reps=2)
        _print("tuned", prec, plan.tiles())
        out.fill_(float("nan"))
        plan.execute(ins, [out], ws)
        torch.cuda.synchronize()
        check(host(out), ref, prec, "autotuned")


def test_empty_and_degenerate_buffers():
    # a tensor with no valid block contracts to an empty result
    A = bst.Tensor(["x", "y"], [(1, [(0, 2)]), (-1, [(1, 2)])])
    B = bst.Tensor(["y", "z"], [(1, [(1, 2)]), (-1, [(1, 3)])])
    C, plan = bst.contract_plan(A, B)
    assert C.numel == 0
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    b = dev(np.ones(B.numel))
    plan.execute([e, b], [e], bst.workspace(plan.workspace_bytes))
    torch.cuda.synchronize()


# ---------------------------------------------------------------- Lanczos
def _lanczos_lib(specs, O, nsteps, prec, refine=True, psi0=None, three_pass=False, f32_basis=False):
    T, plan = lib_heff(specs, "fp64")
    ops = [dev(O[n].data) for n in ("L", "W1", "W2", "R")]
    p0 = dev(psi0 if psi0 is not None else wl.normal(999, O["psi"].numel))
    r = bst.lanczos_ground(plan, ops, p0, nsteps, prec, refine, three_pass=three_pass,
                           f32_basis=f32_basis)
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("three_pass", [False, True])
@pytest.mark.parametrize("spin,singlet", [("1/2", -0.75), ("1", -2.0)])
def test_lanczos_two_site_singlet(spin, singlet, three_pass):
    """Two sites: the Krylov space is exhausted (breakdown) before nsteps."""
    Ld, Rd, Wd, specs = chain_env.chain_heff_dense(2, spin)
    O = {"L": orc.from_dense(*specs["L"], Ld), "R": orc.from_dense(*specs["R"], Rd),
         "W1": orc.from_dense(*specs["W1"], Wd), "W2": orc.from_dense(*specs["W2"], Wd),
         "psi": orc.BlockTensor(*specs["psi"])}
    r = _lanczos_lib(specs, O, O["psi"].numel, "fp64", three_pass=three_pass)
    _print("singlet", spin, three_pass, r["energy"], r["steps"])
    assert abs(r["energy"] - singlet) < 1e-13


@pytest.mark.parametrize("spin,nsites", [("1/2", 6), ("1/2", 10), ("1", 6)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_lanczos_matches_exact_diagonalisation(spin, nsites, prec):
    Ld, Rd, Wd, specs = chain_env.chain_heff_dense(nsites, spin)
    O = {"L": orc.from_dense(*specs["L"], Ld), "R": orc.from_dense(*specs["R"], Rd),
         "W1": orc.from_dense(*specs["W1"], Wd), "W2": orc.from_dense(*specs["W2"], Wd),
         "psi": orc.BlockTensor(*specs["psi"])}
    E_ed = orc.heisenberg_chain_ground(nsites, spin)
    n = min(O["psi"].numel, 128)
    r = _lanczos_lib(specs, O, n, prec)
    _print("ED", spin, nsites, prec, r["energy"], E_ed, r["energy"] - E_ed, r["steps"], r["residual"])
    assert abs(r["energy"] - E_ed) < 1e-10 * max(1.0, abs(E_ed))


@pytest.mark.parametrize("prec", ["fp64", "bf16x6", "bf16x3"])
def test_lanczos_xx_chain_free_fermions(prec):
    """A 10-site XX chain through exact environments (MPO bond 4): the refined
    energy equals the free-fermion closed form (fp64 and bf16x6 to 1e-10
    relative; bf16x3 to the 1e-6 that the Heisenberg chain test allows it)."""
    from tests.test_oracle_xx import free_fermion_ground
    Ld, Rd, Wd, specs = chain_env.chain_heff_dense(10, "1/2", "xx")
    O = {"L": orc.from_dense(*specs["L"], Ld), "R": orc.from_dense(*specs["R"], Rd),
         "W1": orc.from_dense(*specs["W1"], Wd), "W2": orc.from_dense(*specs["W2"], Wd),
         "psi": orc.BlockTensor(*specs["psi"])}
    E0 = free_fermion_ground(10)
    r = _lanczos_lib(specs, O, min(O["psi"].numel, 128), prec)
    _print("XX chain", prec, r["energy"], E0, r["energy"] - E0, r["steps"], r["residual"])
    if prec == "bf16x3":
        assert abs(r["energy"] - E0) < 1e-6
    else:
        assert abs(r["energy"] - E0) < 1e-10 * abs(E0)


@pytest.mark.parametrize("prec", ["fp64", "bf16x6"])
@pytest.mark.parametrize("h", [0.7, 1.0])
def test_lanczos_tfim_z2_chain(prec, h):
    """Lanczos on Z_2-symmetric tensors: a 10-site transverse-field Ising
    chain through exact parity environments; the refined energy equals the
    free-fermion closed form."""
    from tests.test_oracle_zn import tfim_closed_form
    Ld, Rd, Wd, specs = chain_env.tfim_chain_heff_dense(10, h)
    sym = wl.TFIM_SYM
    O = {"L": orc.from_dense(*specs["L"], Ld, sym=sym), "R": orc.from_dense(*specs["R"], Rd, sym=sym),
         "W1": orc.from_dense(*specs["W1"], Wd, sym=sym), "psi": orc.BlockTensor(*specs["psi"], sym=sym)}
    T = {n: bst.Tensor(*sp, sym=list(sym)) for n, sp in specs.items()}
    plan = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], "fp64")
    ops = [dev(O[n].data) for n in ("L", "W1", "W1", "R")]
    n = O["psi"].numel
    r = bst.lanczos_ground(plan, ops, dev(wl.normal(7, n)), min(n, 128), prec, True)
    torch.cuda.synchronize()
    E0 = tfim_closed_form(10, h)
    _print("TFIM Z2", h, prec, r["energy"], E0, r["energy"] - E0, r["steps"])
    assert abs(r["energy"] - E0) < 1e-10 * abs(E0)


def test_lanczos_bf16x3_reports_its_error():
    """bf16x3 matvecs: the refined energy of a 10-site chain, stated (not
    bounded at 1e-10: the split's 2^-17 product error limits the Ritz vector)."""
    Ld, Rd, Wd, specs = chain_env.chain_heff_dense(10, "1/2")
    O = {"L": orc.from_dense(*specs["L"], Ld), "R": orc.from_dense(*specs["R"], Rd),
         "W1": orc.from_dense(*specs["W1"], Wd), "W2": orc.from_dense(*specs["W2"], Wd),
         "psi": orc.BlockTensor(*specs["psi"])}
    E_ed = orc.heisenberg_chain_ground(10, "1/2")
    r = _lanczos_lib(specs, O, 128, "bf16x3")
    _print("ED bf16x3", r["energy"] - E_ed, r["theta"] - E_ed)
    assert abs(r["energy"] - E_ed) < 1e-6


@pytest.mark.parametrize("three_pass", [False, True])
def test_lanczos_matches_oracle_medium(three_pass):
    """Spin-1, chi = 256: the float64 GPU Lanczos reproduces the oracle's
    alpha/beta (all 40 steps) and energies under either reorthogonalisation
    schedule; the split forms reach the same refined energy."""
    specs, O = heff_operands(5, recipe="dmrg_like", chi=256, qmax=8)
    psi0 = wl.normal(wl.seed_for(5, "psi0"), O["psi"].numel)
    mv = lambda v: orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"],
                                  orc.BlockTensor(O["psi"].labels, O["psi"].legs, v)).data
    ref = orc.lanczos_ground(mv, psi0, 40)
    r = _lanczos_lib(specs, O, 40, "fp64", psi0=psi0, three_pass=three_pass)
    da = np.max(np.abs(r["alpha"] - ref["alpha"]))
    db = np.max(np.abs(r["beta"][:39] - ref["beta"][:39]))
    _print("medium fp64", three_pass, r["energy"], ref["energy"], r["theta"] - ref["theta"], da, db)
    assert r["steps"] == ref["steps"]
    assert da < 1e-11 and db < 1e-11
    assert abs(r["energy"] - ref["energy"]) <= 1e-12 * abs(ref["energy"])
    y = host(r["psi"])
    assert abs(abs(float(y @ ref["y"]) / np.linalg.norm(ref["y"])) - 1.0) < 1e-10
    # every split form meets the 1e-10 refined-energy bar, with float64
    # Krylov rows (the default) and with float32 rows
    for prec, f32b in (("fp32", False), ("bf16x6", False), ("bf16x3", False), ("bf16x6", True),
                       ("bf16x3", True)):
        if three_pass and f32b:
            continue   # the three-pass schedule always keeps float64 rows
        rs = _lanczos_lib(specs, O, 40, prec, psi0=psi0, three_pass=three_pass, f32_basis=f32b)
        err = abs(rs["energy"] - ref["energy"]) / abs(ref["energy"])
        _print("medium", prec, "f32 rows" if f32b else "f64 rows", "refined rel err", err,
               "theta rel err", abs(rs["theta"] - ref["theta"]) / abs(ref["theta"]))
        assert err <= 1e-10, (prec, f32b, err)


@pytest.mark.parametrize("nsteps", [1, 2, 3])
def test_lanczos_few_steps(nsteps):
    """One to three steps (the first and last steps of the one-pass schedule
    at once, C of size 1 to 3): alpha, beta and the refined energy against
    the oracle's textbook Lanczos with the same steps; the split forms,
    whose few-step Ritz vector is far from an eigenvector, to their matvec
    error."""
    specs, O = heff_operands(5, recipe="dmrg_like", chi=256, qmax=8)
    psi0 = wl.normal(wl.seed_for(5, "psi0"), O["psi"].numel)
    mv = lambda v: orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"],
                                  orc.BlockTensor(O["psi"].labels, O["psi"].legs, v)).data
    ref = orc.lanczos_ground(mv, psi0, nsteps)
    scale = np.max(np.abs(ref["alpha"]))
    for prec, f32b, tol in (("fp64", False, 1e-12), ("bf16x3", False, 1e-5), ("bf16x3", True, 1e-5)):
        r = _lanczos_lib(specs, O, nsteps, prec, psi0=psi0, f32_basis=f32b)
        _print("few steps", nsteps, prec, f32b, r["alpha"], ref["alpha"], r["energy"], ref["energy"])
        assert r["steps"] == ref["steps"] == nsteps
        assert np.max(np.abs(r["alpha"] - ref["alpha"])) <= tol * scale
        assert np.max(np.abs(r["beta"][:nsteps] - ref["beta"][:nsteps])) <= tol * scale
        assert abs(r["energy"] - ref["energy"]) <= tol * abs(ref["energy"])


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
def test_lanczos_float32_z_is_exact(prec, monkeypatch):
    """With float64 rows and a split form, H u_j is kept as float32 during the
    steps: the split GEMMs accumulate in float32, so the values stored are
    the ones a float64 H u_j holds, and the whole solve (every alpha and
    beta, the Ritz value, the refined energy) is bit-identical to the one
    that keeps H u_j float64 (BST_LANCZOS_Z64)."""
    specs, O = heff_operands(5, recipe="dmrg_like", chi=256, qmax=8)
    psi0 = wl.normal(wl.seed_for(5, "psi0"), O["psi"].numel)
    r32 = _lanczos_lib(specs, O, 40, prec, psi0=psi0)
    monkeypatch.setenv("BST_LANCZOS_Z64", "1")
    r64 = _lanczos_lib(specs, O, 40, prec, psi0=psi0)
    _print("z float32", prec, r32["z32"], r64["z32"], r32["energy"], r64["energy"])
    assert r32["z32"] and not r64["z32"]
    assert r32["steps"] == r64["steps"]
    assert np.array_equal(r32["alpha"], r64["alpha"])
    assert np.array_equal(r32["beta"], r64["beta"])
    assert r32["theta"] == r64["theta"] and r32["energy"] == r64["energy"]
    assert np.array_equal(host(r32["psi"]), host(r64["psi"]))


def test_lanczos_full_size_matches_oracle_golden():
    """Spin-1 chi = 4096, 40 steps: refined energies against the oracle's
    value stored by tests/golden/make_lanczos_golden.py."""
    path = os.path.join(GOLD, "lanczos_spin1_chi4096.json")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    with open(path) as f:
        gold = json.load(f)
    specs, O = heff_operands(5, recipe="dmrg_like")
    psi0 = wl.normal(wl.seed_for(5, "psi0"), O["psi"].numel)
    for prec, f32b in (("fp64", False), ("fp32", False), ("bf16x6", False), ("bf16x3", False),
                       ("bf16x6", True), ("bf16x3", True)):
        r = _lanczos_lib(specs, O, 40, prec, psi0=psi0, f32_basis=f32b)
        err = abs(r["energy"] - gold["energy"]) / abs(gold["energy"])
        _print("chi4096", prec, "f32 rows" if f32b else "f64 rows", r["energy"], gold["energy"],
               "rel err", err, "residual", r["residual"])
        if prec == "fp64":
            assert err <= 1e-12
            assert abs(r["theta"] - gold["theta"]) <= 1e-12 * abs(gold["theta"])
        else:
            assert err <= 1e-10, (prec, f32b, err)
