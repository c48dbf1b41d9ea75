"""Benchmark: Lanczos ground state of the two-site H_eff on one MI355X.

One step = one 40-step Lanczos solve of the spin-1 Heisenberg two-site
H_eff at chi = 4096 (41 charge sectors, 4,589,718 psi elements): 40 H_eff.psi
applies in a reduced-precision MFMA form, full reorthogonalisation against
float64 Krylov rows, the float64 tridiagonal eigensolve, and one float64
apply for the refined energy.  Inputs are resident on the GPU before timing
starts.  The same solve in plain float64 is timed beside it, and the refined
energies of both are compared.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec bf16x6]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H_eff·psi GFLOP/s & % MFMA peak, split-prec vs FP64 at 1e-10 energy err"
PEAK = {  # MI355X published dense peaks
    "hbm_gbs": 8000.0,
    "fp64_tflops": 78.6,
    "fp32_tflops": 157.3,
    "bf16_tflops": 2516.6,
}
MFMA_MULT = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6}
MFMA_PEAK = {"fp64": PEAK["fp64_tflops"], "fp32": PEAK["fp32_tflops"], "bf16x3": PEAK["bf16_tflops"],
             "bf16x6": PEAK["bf16_tflops"]}
WORKLOAD = 5
# the algorithmic steps of one apply (the W1, W2 pair runs fused as mpo_apply)
APPLY_STEPS = ("gemm_L_psi", "mpo_apply", "gemm_T3_R")

# HBM bytes per launch of a kernel, from FETCH_SIZE / WRITE_SIZE counter runs
# scaled by a copy of known size (profiles/hbm_traffic_lanczos40-spin1-chi4096.md).
# Valid only for the kernel source they were taken on: `src_sha` is the first
# 16 hex digits of that file's sha256; any change reports traffic as null.
TRAFFIC = {
    "gs_update": {"bytes_per_launch": 807744972.1, "src": "paper_2401_01921_amd/csrc/kernels_aux.hip",
                  "src_sha": "79718e1e8af89904",
                  "profile": "profiles/hbm_traffic_lanczos40-spin1-chi4096.md"},
}


def measured_traffic(kernel):
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None or t["bytes_per_launch"] is None:
        return None
    with open(os.path.join(ROOT, t["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["src_sha"]:
            return None
    return t["bytes_per_launch"]


WIDENED_ROWS = ("svd256", "svd1024", "dmrg16", "dmrg64", "complex")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="bf16x3", choices=["fp32", "bf16x3", "bf16x6", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads, forms and calibration measurements")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tile variants (short runs under a profiler)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run the library's streaming copy over this many MiB (a kernel "
                         "of known traffic that calibrates hardware byte counters)")
    ap.add_argument("--widened-only", metavar="ROWS", default=None,
                    help="run only the named rows beyond the H_eff solve, comma separated, "
                         f"from {','.join(WIDENED_ROWS)} (one JSON line of their results; "
                         "for per-workload profiles)")
    return ap.parse_args()


def onepass_vector_flops(n: int, m: int) -> float:
    """Flops of the vector work a solve executes with the one-pass schedule
    (float64 arithmetic throughout): the start vector's norm and scaling;
    per step j the u_j.z and z.z dot (4n) and the basis pass (per element
    2(j+1) for the residual's combination of the stored rows 0..j, 2 for the
    scaled z term, 2(j+1) for the measures u_m.w and 2 for w.w); the Ritz
    vector (2nm); the refinement's two dots, residual and scaling.  The
    scalar work on the triangular row map is O(j^2) per step, not counted."""
    f = 5.0 * n
    for j in range(m):
        f += 4.0 * n + (4.0 * j + 8.0) * n
    return f + 2.0 * n * m + 9.0 * n


def cgs2_vector_flops(n: int, m: int) -> float:
    """Flops of the oracle's textbook solve besides its applies: per step
    with nv rows two classical Gram-Schmidt passes (8 n nv), the norm and
    the scaling; then the Ritz vector and the refinement."""
    f = 3.0 * n
    for j in range(m):
        f += 8.0 * n * (j + 1) + 3.0 * n
    return f + 2.0 * n * m + 6.0 * n


def apply_roofline_ms(steps, prec):
    """Roofline time (ms) of one apply: per algorithmic step the larger of
    its MFMA time (algorithmic flops times the form's MFMA multiplicity over
    the form's peak) and its HBM time (algorithmic bytes at the storage
    precision over 8 TB/s)."""
    by = "bytes_fp64" if prec == "fp64" else "bytes_fp32"
    t = 0.0
    for s in steps:
        if s["name"] not in APPLY_STEPS:
            continue
        mm = 1.0 if s["name"] == "mpo_apply" else MFMA_MULT[prec]
        peak = PEAK["fp64_tflops"] if prec == "fp64" else (
            PEAK["fp32_tflops"] if (prec == "fp32" or s["name"] == "mpo_apply") else PEAK["bf16_tflops"])
        t += max(s["flops"] * mm / (peak * 1e9), s[by] / (PEAK["hbm_gbs"] * 1e6))
    return t


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not part "
                                   "of this build (the path would shard by left charge sector)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2401_01921_amd import bst, workloads as wl

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = "cuda"
    if a.widened_only is not None:
        rows = [r for r in a.widened_only.split(",") if r]
        bad = [r for r in rows if r not in WIDENED_ROWS]
        if bad or not rows:
            raise SystemExit(f"--widened-only takes rows from {','.join(WIDENED_ROWS)}")
        print(json.dumps({"widened": bench_widened(bst, wl, torch, dev, set(rows))}), flush=True)
        return
    copy_cal = copy_calibration(bst, torch, dev, a.copy_mib) if a.copy_mib > 0 else None
    w = wl.WORKLOADS[WORKLOAD]
    v = wl.gaussian_sector_dims(w["chi"], w["qmax"])
    specs = wl.heff_specs(w["spin"], v, v)
    T = {k: bst.Tensor(*s) for k, s in specs.items()}
    plan = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], "fp64")
    n = T["psi"].numel
    m = w["steps"]
    host = {
        "L": wl.dmrg_like_env(T["L"].table(), T["L"].numel, wl.seed_for(WORKLOAD, "L"), "L", v),
        "R": wl.dmrg_like_env(T["R"].table(), T["R"].numel, wl.seed_for(WORKLOAD, "R"), "R", v),
        "W1": T["W1"].from_dense(wl.heisenberg_mpo_dense(w["spin"])),
        "psi0": wl.normal(wl.seed_for(WORKLOAD, "psi0"), n),
    }
    host["W2"] = host["W1"]
    g = {k: torch.from_numpy(x).to(dev) for k, x in host.items()}
    ops = [g["L"], g["W1"], g["W2"], g["R"]]
    ws = bst.workspace(bst.lanczos_workspace(plan, m))
    psi_out = torch.empty(n, dtype=torch.float64, device=dev)
    apply_flops = plan.stats().flops
    step_flops = (m + 1) * apply_flops + onepass_vector_flops(n, m)

    # autotune the tile variant of every GEMM step for both forms (untimed)
    tune_out = torch.empty(n, dtype=torch.float64, device=dev)
    tune_ws = bst.workspace(plan.workspace_bytes)
    tuned = {}
    for prec in (a.prec, "fp64"):
        plan.set_precision(prec)
        if not a.no_tune:
            plan.autotune([g["L"], g["W1"], g["W2"], g["R"], g["psi0"]], [tune_out], tune_ws,
                          reps=5)
        tuned[prec] = plan.tiles()
    del tune_ws, tune_out

    def solve(prec, timing=False, three_pass=False, f32_basis=False):
        return bst.lanczos_ground(plan, ops, g["psi0"], m, prec, True, ws=ws, psi_out=psi_out,
                                  timing=timing, three_pass=three_pass, f32_basis=f32_basis)

    def timed(prec, steps, warmup, three_pass=False, f32_basis=False):
        for _ in range(warmup):
            solve(prec, three_pass=three_pass, f32_basis=f32_basis)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        for _ in range(steps):
            res = solve(prec, three_pass=three_pass, f32_basis=f32_basis)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res

    # ---- timed region: the split-precision solve (float64 Krylov rows) ----
    ms_split, res_split = timed(a.prec, a.steps, a.warmup)
    # plain float64 solve on the same inputs
    ms64, res64 = timed("fp64", max(2, a.steps // 2), 1)
    # per-kernel HIP-event times of one solve of each form
    prof_split = solve(a.prec, timing=True)
    prof64 = solve("fp64", timing=True)

    e64, es = res64["energy"], res_split["energy"]
    err = abs(es - e64) / abs(e64)

    # ---- roofline of the kernels (algorithmic work / HIP-event time) ------
    steps = {s["name"]: s for s in plan.steps()}
    km, kc = prof_split["kernel_ms"], prof_split["kernel_calls"]
    inter32 = a.prec != "fp64"

    def gemm_roof(name, prof, prec):
        calls = prof["kernel_calls"][name]
        avg_ms = prof["kernel_ms"][name] / max(calls, 1)
        fl = steps[name]["flops"]
        mult = MFMA_MULT[prec]
        return dict(kernel=name, avg_ms=avg_ms, alg_tflops=fl / avg_ms / 1e9,
                    mfma_tflops=fl * mult / avg_ms / 1e9, peak_tflops=MFMA_PEAK[prec],
                    mfma_frac=fl * mult / avg_ms / 1e9 / MFMA_PEAK[prec])

    def gs_bytes(kind, res, rowb=8.0):
        # algorithmic bytes of one solve's Gram-Schmidt kernels (one-pass
        # schedule): the dot reads u_j and z; the pass of step j (0-based)
        # reads basis rows 0..j and z and (except on the last step) writes
        # row j+1.  Rows are float64 (4 bytes with float32 rows); z is float64,
        # or float32 when the solve reports it kept H u_j in float32.
        zb = 4.0 if res.get("z32") else rowb
        tot = 0.0
        for j in range(m):
            if kind == "dots":
                tot += rowb * n + zb * n
            else:
                tot += rowb * n * (j + 1) + zb * n + (rowb * n if j + 1 < m else 0.0)
        return tot

    def hbm_roof(key, total_bytes, prof):
        ms = prof["kernel_ms"][key]
        calls = prof["kernel_calls"][key]
        return dict(kernel=key, avg_ms=ms / max(calls, 1), calls=calls,
                    achieved_gbs=total_bytes / ms / 1e6, frac=total_bytes / ms / 1e6 / PEAK["hbm_gbs"])

    mpo_bytes = steps["mpo_apply"]["bytes_fp32" if inter32 else "bytes_fp64"]
    kern = {
        # with the fused L.psi + MPO kernel the split solve has no L.psi launches
        # of its own (the refinement's FP64 one remains): no roofline of its own
        "gemm_L_psi": (None if "mpo_apply:fused" in tuned[a.prec]
                       else gemm_roof("gemm_L_psi", prof_split, a.prec)),
        "gemm_T3_R": gemm_roof("gemm_T3_R", prof_split, a.prec),
        "mpo_apply": hbm_roof("mpo_apply", mpo_bytes * kc["mpo_apply"], prof_split),
        "gs_dots": hbm_roof("gs_dots", gs_bytes("dots", prof_split), prof_split),
        "gs_update": hbm_roof("gs_update", gs_bytes("update", prof_split), prof_split),
        "fp64_gemm_L_psi": gemm_roof("gemm_L_psi", prof64, "fp64"),
        "fp64_gemm_T3_R": gemm_roof("gemm_T3_R", prof64, "fp64"),
        "fp64_gs_update": hbm_roof("gs_update", gs_bytes("update", prof64), prof64),
    }
    # dominant kernel of the step = largest summed time
    dom = max((k for k in km if kern.get(k) is not None), key=km.get)
    r = kern[dom]
    if dom.startswith("gemm"):
        roof = {"bound": "mfma", "kernel": dom, "achieved": round(r["mfma_tflops"], 2),
                "peak": MFMA_PEAK[a.prec], "unit": "TFLOP/s", "frac": round(r["mfma_frac"], 4),
                "traffic": None}
    else:
        per_launch = r["achieved_gbs"] * r["avg_ms"] * 1e6
        tr = measured_traffic(dom)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(r["achieved_gbs"], 1),
                "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(r["frac"], 4),
                "traffic": tr, "alg_bytes_per_launch": per_launch,
                "traffic_over_alg": None if tr is None else round(tr / per_launch, 4)}

    extras = {}
    if not a.no_extras:
        # the same split solve with float32 Krylov rows (and float32 H u_j)
        msf, resf = timed(a.prec, max(2, a.steps // 2), 1, f32_basis=True)
        extras["float32_rows"] = {
            "ms_per_solve": round(msf * 1e3, 3),
            "energy_rel_err_vs_fp64": abs(resf["energy"] - e64) / abs(e64),
            "speedup_vs_fp64": round(ms64 / msf, 3)}
        # the same split solve under the textbook three-pass schedule
        ms3, res3 = timed(a.prec, max(2, a.steps // 2), 1, three_pass=True)
        extras["three_pass_schedule"] = {
            "ms_per_solve": round(ms3 * 1e3, 3),
            "kernels": {k: round(v, 4) for k, v in
                        solve(a.prec, timing=True, three_pass=True)["kernel_ms"].items()},
            "energy_rel_diff_vs_one_pass": abs(res3["energy"] - es) / abs(es)}
        extras.update(bench_extras(bst, wl, torch, dev, plan, ins_apply=[
            g["L"], g["W1"], g["W2"], g["R"], g["psi0"]], apply_flops=apply_flops))
        extras.update(bench_widened(bst, wl, torch, dev))

    # ---- CPU baseline: the oracle's Lanczos solve on the host cores -------
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(specs, host, apply_flops, n, m, a.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(step_flops / ms_split / 1e9, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_split * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16x3(f32 acc)+f64", "bf16x6": "bf16x6(f32 acc)+f64",
                  "fp32": "f32+f64", "fp64": "f64"}[a.prec],
        "data": "synthetic",
        "config": {"workload": w["name"], "chi": w["chi"], "sectors": len(v), "spin": w["spin"],
                   "psi_elements": n, "lanczos_steps": m, "matvec": a.prec, "krylov_rows": "fp64",
                   "h_u": ("fp32 (the matvec's float32 accumulators, exact)" if res_split.get("z32")
                           else "fp64"),
                   "reorthogonalisation": "full, fp64, one basis pass per step",
                   "refine": "fp64", "flops_per_step": step_flops,
                   "heff_flops_per_apply": apply_flops},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64_ms_per_step": round(ms64 * 1e3, 3),
        "speedup_vs_fp64": round(ms64 / ms_split, 3),
        "energy": {"split": es, "fp64": e64, "rel_err_vs_fp64": err,
                   "theta_rel_err": abs(res_split["theta"] - res64["theta"]) / abs(e64),
                   "residual_split": res_split["residual"], "residual_fp64": res64["residual"],
                   "meets_1e-10": bool(err <= 1e-10)},
        "kernels_split": {k: round(v, 4) for k, v in km.items()},
        "kernels_fp64": {k: round(v, 4) for k, v in prof64["kernel_ms"].items()},
        "kernel_roofline": kern,
        "tiles": tuned,
        "extras": extras,
        "copy_calibration": copy_cal,
    }
    print(json.dumps(out), flush=True)


def copy_calibration(bst, torch, dev, mib):
    """Three runs of the library's streaming copy over `mib` MiB: each reads
    and writes exactly mib MiB, which scales the FETCH_SIZE / WRITE_SIZE
    counters."""
    src = torch.ones(mib * 2**20 // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    ms = _time_ms(torch, lambda: bst.calib_copy(src, dst), 3, warm=0)
    del src, dst
    return {"mib": mib, "reps": 3, "ms": round(ms, 4),
            "gbs": round(2 * mib * 2**20 / ms / 1e6, 1)}


def _time_ms(torch, fn, reps, warm=2):
    """Median time (ms) of fn over reps runs, each between HIP events on the
    current stream (the stream the library launches on)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _apply_forms(bst, torch, dev, plan, ins, flops, forms, ref=None, tune=True):
    """Per form: median apply time, GFLOP/s, roofline fraction of the apply,
    per-GEMM MFMA fraction and (with ref) the errors against the oracle."""
    res = torch.empty_like(ins[4])
    ws = bst.workspace(plan.workspace_bytes)
    steps = plan.steps()
    out = {}
    for prec in forms:
        plan.set_precision(prec)
        if tune:
            plan.autotune(ins, [res], ws, reps=3)
        ms = _time_ms(torch, lambda: plan.execute(ins, [res], ws), 20, warm=5)
        prof = dict(plan.profile(ins, [res], ws, reps=10))
        roof = apply_roofline_ms(steps, prec)
        d = {"ms": round(ms, 4), "gflops": round(flops / ms / 1e6, 1),
             "roofline_ms": round(roof, 5), "roofline_frac": round(roof / ms, 4),
             "tiles": plan.tiles()}
        for s in steps:
            if s["name"].startswith("gemm") and prof.get(s["name"], 0) > 0:
                t = prof[s["name"]]
                d["mfma_frac_" + s["name"]] = round(
                    s["flops"] * MFMA_MULT[prec] / t / 1e9 / MFMA_PEAK[prec], 4)
                d["ms_" + s["name"]] = round(t, 4)
        if "mpo_apply" in prof:
            d["ms_mpo_apply"] = round(prof["mpo_apply"], 4)
        if ref is not None:
            res.fill_(float("nan"))
            plan.execute(ins, [res], ws)
            got = res.cpu().numpy()
            d["err_normwise"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            d["err_max"] = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        out[prec] = d
    return out


def bench_extras(bst, wl, torch, dev, plan, ins_apply, apply_flops):
    """The other workloads: single applies per form at chi = 512, 2048 and
    4096, the 64-apply batch per form, the XX-chain apply, the block permute
    on a tensor above 1 GiB, and the calibration kernels."""
    from oracle import oracle as orc
    out = {}
    forms = ("fp64", "fp32", "bf16x3", "bf16x6")
    # chi = 512 and 2048 spin-1/2 applies, every form, errors vs the oracle
    for k, key in ((2, "apply_chi512"), (3, "apply_chi2048")):
        wk = wl.WORKLOADS[k]
        v = wl.gaussian_sector_dims(wk["chi"], wk["qmax"])
        sp = wl.heff_specs(wk["spin"], v, v)
        O = {n_: orc.BlockTensor(*s) for n_, s in sp.items()}
        for n_ in ("L", "R", "psi"):
            O[n_].data[:] = wl.normal(wl.seed_for(k, n_), O[n_].numel)
        Wd = wl.heisenberg_mpo_dense(wk["spin"])
        O["W1"] = orc.from_dense(*sp["W1"], Wd)
        O["W2"] = orc.from_dense(*sp["W2"], Wd)
        ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
        Tk = {n_: bst.Tensor(*s) for n_, s in sp.items()}
        pk = bst.heff_plan(Tk["L"], Tk["W1"], Tk["W2"], Tk["R"], Tk["psi"], "fp64")
        ins = [torch.from_numpy(O[n_].data.copy()).to(dev) for n_ in ("L", "W1", "W2", "R", "psi")]
        fl = pk.stats().flops
        out[key] = {"workload": wk["name"], "flops": fl,
                    "forms": _apply_forms(bst, torch, dev, pk, ins, fl, forms, ref=ref)}
        del pk, ins
    # chi = 4096 spin-1 applies, every form
    out["apply_chi4096"] = _apply_forms(bst, torch, dev, plan, ins_apply, apply_flops, forms)
    # batched: 64 uneven spin-1/2 applies, all sector GEMMs of a step in one
    # launch; per form, with the sum of the members' apply rooflines
    draws = wl.batch_draws()
    members, ins, outs, W = [], [], [], None
    for i, (chi, q) in enumerate(draws):
        v = wl.gaussian_sector_dims(chi, q)
        Tb = {k_: bst.Tensor(*s) for k_, s in wl.heff_specs("1/2", v, v).items()}
        if W is None:
            W = torch.from_numpy(Tb["W1"].from_dense(wl.heisenberg_mpo_dense("1/2"))).to(dev)
        members.append(bst.heff_plan(Tb["L"], Tb["W1"], Tb["W2"], Tb["R"], Tb["psi"], "fp64"))
        ins += [torch.from_numpy(wl.normal(wl.seed_for(4, "L", i), Tb["L"].numel)).to(dev), W, W,
                torch.from_numpy(wl.normal(wl.seed_for(4, "R", i), Tb["R"].numel)).to(dev),
                torch.from_numpy(wl.normal(wl.seed_for(4, "psi", i), Tb["psi"].numel)).to(dev)]
        outs.append(torch.empty(Tb["psi"].numel, dtype=torch.float64, device=dev))
    member_steps = [p.steps() for p in members]
    batch = bst.heff_batch_plan(members)
    bflops = batch.stats().flops
    wsb = bst.workspace(batch.workspace_bytes)
    bres = {"flops": bflops, "kernels_per_execute": batch.stats().nsteps,
            "gemm_problems": batch.stats().gemm_problems}
    for prec in ("fp32", "fp64", "bf16x3"):
        batch.set_precision(prec)
        batch.autotune(ins, outs, wsb, reps=3)
        batch.use_graph(True)
        ms_b = _time_ms(torch, lambda: batch.execute(ins, outs, wsb), 20, warm=3)
        batch.use_graph(False)
        ms_e = _time_ms(torch, lambda: batch.execute(ins, outs, wsb), 20, warm=3)
        roof = sum(apply_roofline_ms(st, prec) for st in member_steps)
        best = min(ms_b, ms_e)
        bres[prec] = {"ms_graph": round(ms_b, 4), "ms_eager": round(ms_e, 4),
                      "gflops": round(bflops / best / 1e6, 1), "roofline_sum_ms": round(roof, 5),
                      "roofline_frac": round(roof / best, 4), "tiles": batch.tiles()}
    bres["split_over_fp64_speedup"] = round(
        min(bres["fp64"]["ms_graph"], bres["fp64"]["ms_eager"]) /
        min(bres["bf16x3"]["ms_graph"], bres["bf16x3"]["ms_eager"]), 3)
    out["batch64"] = bres
    del wsb, ins, outs, batch, members
    # the XX chain's MPO (bond of 4 channels; the model of the paper's DMRG
    # benchmark): one spin-1/2 apply at chi = 4096, q in [-20, 20]
    v = wl.gaussian_sector_dims(4096, 20)
    Tx = {k_: bst.Tensor(*s) for k_, s in wl.heff_specs("1/2", v, v, "xx").items()}
    Wx = torch.from_numpy(Tx["W1"].from_dense(wl.mpo_dense("1/2", "xx"))).to(dev)
    ins_x = [torch.randn(Tx["L"].numel, dtype=torch.float64, device=dev), Wx, Wx,
             torch.randn(Tx["R"].numel, dtype=torch.float64, device=dev),
             torch.randn(Tx["psi"].numel, dtype=torch.float64, device=dev)]
    px = bst.heff_plan(Tx["L"], Tx["W1"], Tx["W2"], Tx["R"], Tx["psi"], "fp64")
    fl_x = px.stats().flops
    out["apply_xx_spin_half_chi4096"] = {
        "psi_elements": Tx["psi"].numel, "flops": fl_x,
        "forms": _apply_forms(bst, torch, dev, px, ins_x, fl_x, ("fp64", "bf16x3"))}
    del ins_x, px
    # block permute of a 1.2 GiB tensor (c, a, b) <- (a, b, c)
    sec = [(q, 150) for q in range(-3, 4)]
    Tp = bst.Tensor(["a", "b", "c"], [(1, sec), (1, sec), (-1, [(q, 150) for q in range(-6, 7)])])
    _, pplan = bst.permute_plan(Tp, ["c", "a", "b"])
    x = torch.randn(Tp.numel, dtype=torch.float64, device=dev)
    y = torch.empty(Tp.numel, dtype=torch.float64, device=dev)
    wsp = bst.workspace(pplan.workspace_bytes)
    ms_p = _time_ms(torch, lambda: pplan.execute([x], [y], wsp), 10)
    kms = pplan.profile([x], [y], wsp, reps=5)[0][1]
    out["permute"] = {"numel": Tp.numel, "gib": round(Tp.numel * 8 / 2**30, 3), "blocks": Tp.nblocks,
                      "order": "(c,a,b) <- (a,b,c)",
                      "ms": round(ms_p, 4), "kernel_ms": round(kms, 4),
                      "gbs": round(2 * 8 * Tp.numel / kms / 1e6, 1),
                      "hbm_frac": round(2 * 8 * Tp.numel / kms / 1e6 / PEAK["hbm_gbs"], 4)}
    # the same tensor with its fastest leg kept: block rows are copied whole
    _, qplan = bst.permute_plan(Tp, ["b", "a", "c"])
    wsq = bst.workspace(qplan.workspace_bytes)
    kq = qplan.profile([x], [y], wsq, reps=5)[0][1]
    out["permute_rows"] = {"order": "(b,a,c) <- (a,b,c)", "kernel_ms": round(kq, 4),
                           "gbs": round(2 * 8 * Tp.numel / kq / 1e6, 1),
                           "hbm_frac": round(2 * 8 * Tp.numel / kq / 1e6 / PEAK["hbm_gbs"], 4)}
    # calibration: the library's streaming copy and read over the same
    # 1.23 GiB, and MFMA loops (the device's practical ceilings)
    cal = {}
    ms_c = _time_ms(torch, lambda: bst.calib_copy(x, y), 10)
    cal["copy_gbs"] = round(2 * 8 * Tp.numel / ms_c / 1e6, 1)
    part = torch.empty(bst.calib_grid(), dtype=torch.float64, device=dev)
    ms_r = _time_ms(torch, lambda: bst.calib_read(x, part), 10)
    cal["read_gbs"] = round(8 * Tp.numel / ms_r / 1e6, 1)
    cal["bytes"] = 8 * Tp.numel
    del x, y, wsp, wsq
    mo = torch.empty(256 * bst.calib_grid(), dtype=torch.float64, device=dev)
    for prec, key, peak in (("fp64", "mfma_f64_tflops", PEAK["fp64_tflops"]),
                            ("bf16x3", "mfma_bf16_tflops", PEAK["bf16_tflops"])):
        iters = 2000 if prec == "fp64" else 4000
        fl = [0.0]

        def run():
            fl[0] = bst.calib_mfma(prec, iters, mo)
        ms_m = _time_ms(torch, run, 5)
        cal[key] = round(fl[0] / ms_m / 1e9, 1)
        cal[key.replace("tflops", "frac_of_peak")] = round(fl[0] / ms_m / 1e9 / peak, 4)
    out["calibration"] = cal
    return out


def bench_widened(bst, wl, torch, dev, rows=None):
    """The rows built beyond the H_eff path, each beside the oracle on the
    host: the symmetric truncated SVD of a two-site state, a two-site DMRG
    sweep of the XX chain, and a complex contraction.  rows: the subset of
    WIDENED_ROWS to run (all when None)."""
    import math
    from oracle import oracle as orc
    from paper_2401_01921_amd import dmrg
    out = {}
    want = (lambda r: True) if rows is None else (lambda r: r in rows)
    ph = wl.physical_sectors("1/2")
    # -- Svd_truncate of a spin-1/2 two-site state, bonds chi = 256 and 1024
    # (q in [-6, 6]); at 1024, seven sectors (170 x 170 to 266 x 266) exceed
    # the LDS budget and run a launch per Jacobi round
    for chi, key, row in ((256, "svd_truncate", "svd256"), (1024, "svd_truncate_chi1024", "svd1024")):
        if not want(row):
            continue
        v = wl.gaussian_sector_dims(chi, 6)
        O = orc.BlockTensor(["a", "s1", "s2", "b"], [(1, v), (1, ph), (1, ph), (-1, v)])
        O.data[:] = wl.normal(wl.seed_for(2, "psi", 7), O.numel)
        T = bst.Tensor(O.labels, O.legs)
        x = torch.from_numpy(O.data.copy()).to(dev)
        plan = bst.Svd(T, 2)
        ws = bst.workspace(plan.workspace_bytes)
        shapes = [plan.sector(k)[1:] for k in range(plan.nsectors)]

        def run_svd():
            plan.execute(x, ws)
            kept, _ = plan.truncate(chi, 1e-12, None, ws)
            Ut, Vt = plan.factors(kept, "m")
            U = torch.empty(Ut.numel, dtype=torch.float64, device=dev)
            Vd = torch.empty(Vt.numel, dtype=torch.float64, device=dev)
            S = torch.empty(sum(kept), dtype=torch.float64, device=dev)
            plan.write(kept, 2, U, S, Vd, ws)
            return S
        ms_svd = _time_ms(torch, run_svd, 5 if chi <= 256 else 2)
        S = run_svd().cpu().numpy()
        t0 = time.perf_counter()
        ou, os_, ov, _ = orc.svd_truncate(O, 2, chi, 1e-12, bond="m", absorb="v")
        cpu_ms = (time.perf_counter() - t0) * 1e3
        ref = np.concatenate(os_)
        out[key] = {
            "workload": f"two-site spin-1/2 state, chi = {chi} bonds ({len(v)} sectors), rows (a, s1), keepdim {chi}",
            "elements": O.numel, "sectors": plan.nsectors,
            "largest_sector": [int(max(m for m, _ in shapes)), int(max(n_ for _, n_ in shapes))],
            "ms": round(ms_svd, 3), "oracle_ms": round(cpu_ms, 2),
            "max_value_err": float(np.max(np.abs(np.sort(S) - np.sort(ref))) / ref.max())}
    # -- the XX MPO and the boundary environments of both chains
    if want("dmrg16") or want("dmrg64"):
        Ws = wl.heff_specs("1/2", [(0, 1)], [(0, 1)], "xx")["W1"]
        Wo = orc.from_dense(*Ws, wl.mpo_dense("1/2", "xx"))
        Wg = dmrg.DevTensor(bst.Tensor(*Ws), torch.from_numpy(Wo.data.copy()).to(dev))
        Ls, lpos, Rs, rpos = wl.boundary_env_specs("1/2", "xx", 0)
        envs = []
        for sp, pos in ((Ls, lpos), (Rs, rpos)):
            D = np.zeros(orc.BlockTensor(*sp).dims())
            D[pos] = 1.0
            envs.append(dmrg.DevTensor(bst.Tensor(*sp), torch.from_numpy(orc.from_dense(*sp, D).data).to(dev)))
    # -- two-site DMRG of the XX chain (N = 16, keepdim 64, 2 sweeps)
    if want("dmrg16"):
        N, keep = 16, 64
        specs = wl.mps_specs(N, "1/2", 0)
        mps = []
        for i, (lab, legs) in enumerate(specs):
            t = bst.Tensor(lab, legs)
            mps.append(dmrg.DevTensor(t, torch.from_numpy(wl.normal(wl.seed_for(2, "A", i), t.numel)).to(dev)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, errs, _ = dmrg.dmrg_two_site(mps, Wg, envs[0], envs[1], 2, keep, 1e-12)
        torch.cuda.synchronize()
        sweep_s = (time.perf_counter() - t0) / 2
        exact = sum(min(0.0, math.cos(math.pi * k / (N + 1))) for k in range(1, N + 1))
        out["dmrg_sweep_xx"] = {
            "workload": f"open XX chain, spin 1/2, N = {N}, total Sz 0, keepdim {keep}, 2 sweeps from a random MPS",
            "s_per_sweep": round(sweep_s, 3), "bond_updates": len(E),
            "energy": E[-1], "exact_free_fermion": exact, "abs_err": abs(E[-1] - exact),
            "max_s_err": max(errs)}
    # -- the same chain at N = 64, keepdim 256 (random start with every sector
    # of every bond capped at 16, so that the first sweep grows the bonds)
    if want("dmrg64"):
        N, keep, cap, nsw = 64, 256, 16, 2
        specs = wl.mps_specs(N, "1/2", 0, cap=cap)
        mps = []
        for i, (lab, legs) in enumerate(specs):
            t = bst.Tensor(lab, legs)
            mps.append(dmrg.DevTensor(t, torch.from_numpy(wl.normal(wl.seed_for(2, "A", i), t.numel)).to(dev)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, errs, fin = dmrg.dmrg_two_site(mps, Wg, envs[0], envs[1], nsw, keep, 1e-12)
        torch.cuda.synchronize()
        sweep_s = (time.perf_counter() - t0) / nsw
        exact = sum(min(0.0, math.cos(math.pi * k / (N + 1))) for k in range(1, N + 1))
        out["dmrg_sweep_xx_n64_chi256"] = {
            "workload": f"open XX chain, spin 1/2, N = {N}, total Sz 0, keepdim {keep}, {nsw} sweeps from a random MPS "
                        f"with sectors capped at {cap}",
            "s_per_sweep": round(sweep_s, 3), "bond_updates": len(E),
            "largest_bond": max(int(sum(g for _, g in T.t.legs()[1][2][1])) for T in fin),
            "energy": E[-1], "exact_free_fermion": exact, "abs_err": abs(E[-1] - exact),
            "max_s_err": max(errs)}
    # -- complex contraction A[l, s, m] . B[m, t, r], chi = 2048 (q in [-16, 16])
    if want("complex"):
        v = wl.gaussian_sector_dims(2048, 16)
        A = (["l", "s", "m"], [(1, v), (1, ph), (-1, v)])
        B = (["m", "t", "r"], [(1, v), (1, ph), (-1, v)])
        tA, tB = bst.Tensor(*A), bst.Tensor(*B)
        res = {}
        for dt in ("f64", "c128"):
            w_ = 2 if dt == "c128" else 1
            tC, cp = bst.contract_plan(tA, tB, "fp64", dtype=dt)
            a_ = torch.randn(w_ * tA.numel, dtype=torch.float64, device=dev)
            b_ = torch.randn(w_ * tB.numel, dtype=torch.float64, device=dev)
            c_ = torch.empty(w_ * tC.numel, dtype=torch.float64, device=dev)
            wsc = bst.workspace(cp.workspace_bytes)
            cp.autotune([a_, b_], [c_], wsc, reps=3)
            ms = _time_ms(torch, lambda: cp.execute([a_, b_], [c_], wsc), 10)
            fl = cp.stats().flops
            res[dt] = {"ms": round(ms, 4), "gflops": round(fl / ms / 1e6, 1), "flops": fl, "tiles": cp.tiles()}
        # the oracle's complex contraction of a smaller state (chi = 512) on the host
        v5 = wl.gaussian_sector_dims(512, 8)
        Ao = orc.BlockTensor(["l", "s", "m"], [(1, v5), (1, ph), (-1, v5)], dtype=np.complex128)
        Bo = orc.BlockTensor(["m", "t", "r"], [(1, v5), (1, ph), (-1, v5)], dtype=np.complex128)
        Ao.data[:] = wl.normal(11, Ao.numel) + 1j * wl.normal(12, Ao.numel)
        Bo.data[:] = wl.normal(13, Bo.numel) + 1j * wl.normal(14, Bo.numel)
        t0 = time.perf_counter()
        Co = orc.contract(Ao, Bo)
        cpu_s = time.perf_counter() - t0
        t5A, t5B = bst.Tensor(*(Ao.labels, Ao.legs)), bst.Tensor(*(Bo.labels, Bo.legs))
        t5C, p5 = bst.contract_plan(t5A, t5B, "fp64", dtype="c128")
        a5 = torch.view_as_real(torch.from_numpy(Ao.data).to(dev)).reshape(-1)
        b5 = torch.view_as_real(torch.from_numpy(Bo.data).to(dev)).reshape(-1)
        c5 = torch.empty(2 * t5C.numel, dtype=torch.float64, device=dev)
        p5.execute([a5, b5], [c5], bst.workspace(p5.workspace_bytes))
        got = c5.cpu().numpy().reshape(-1, 2)
        got = got[:, 0] + 1j * got[:, 1]
        out["complex_contract"] = {
            "workload": "A[l,s,m].B[m,t,r], spin-1/2 physical legs, chi = 2048 virtual legs (33 sectors), FP64 arithmetic",
            "c128": res["c128"], "f64_same_structure": res["f64"],
            "oracle_chi512_gflops": round(p5.stats().flops / cpu_s / 1e9, 2),
            "chi512_max_err_vs_oracle": float(np.max(np.abs(got - Co.data)) / np.max(np.abs(Co.data)))}
    return out


def _cpu_info():
    model, pairs = None, set()
    phys = core = None
    allowed = os.sched_getaffinity(0)
    proc = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, val = line.partition(":")
                k, val = k.strip(), val.strip()
                if k == "processor":
                    proc = int(val)
                elif k == "model name" and model is None:
                    model = val
                elif k == "physical id":
                    phys = val
                elif k == "core id":
                    core = val
                elif not k and proc is not None:
                    if proc in allowed:
                        pairs.add((phys, core))
                    proc = phys = core = None
        if proc is not None and proc in allowed:
            pairs.add((phys, core))
    except OSError:
        pass
    return model, len(pairs) or None, len(allowed)


def cpu_baseline(specs, host, apply_flops, n, m, seconds):
    """The float64 oracle's Lanczos solve of the same operator on this
    host (numpy; BLAS threads as configured): textbook CGS2 steps plus the
    refinement apply, with as many steps as fit about `seconds` (at most the
    solve's m), from a first timed apply."""
    from oracle import oracle as orc
    O = {k: orc.BlockTensor(*specs[k]) for k in ("L", "R", "psi")}
    O["L"].data[:] = host["L"]
    O["R"].data[:] = host["R"]
    W1 = orc.BlockTensor(*specs["W1"], host["W1"])
    W2 = orc.BlockTensor(*specs["W2"], host["W2"])
    mv = lambda x: orc.heff_apply(O["L"], W1, W2, O["R"],
                                  orc.BlockTensor(O["psi"].labels, O["psi"].legs, x)).data
    t0 = time.perf_counter()
    mv(host["psi0"])
    t_apply = time.perf_counter() - t0
    steps = int(max(2, min(m, seconds / max(t_apply, 1e-3) - 1)))
    t0 = time.perf_counter()
    r = orc.lanczos_ground(mv, host["psi0"], steps)
    el = time.perf_counter() - t0
    flops = (r["steps"] + 1) * apply_flops + cgs2_vector_flops(n, r["steps"])
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads") or 0) for i in threadpool_info()) or None
    except Exception:
        pass
    model, phys, logical = _cpu_info()
    if threads is None:
        threads = logical
    return {"value": round(flops / el / 1e9, 2), "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle", "cpu_model": model, "physical_cores": phys, "logical_cpus": logical,
            "sample": f"{r['steps']}-step Lanczos solve (of the {m} timed on the GPU) of the "
                      f"chi=4096 spin-1 H_eff: {r['steps'] + 1} float64 applies and textbook "
                      f"CGS2 reorthogonalisation, numpy oracle, {el:.1f} s; cores = BLAS threads"}


if __name__ == "__main__":
    main()
