"""Benchmark: Lanczos ground state of the two-site H_eff on one MI355X.

One step = one 40-step Lanczos solve of the spin-1 Heisenberg two-site
H_eff at chi = 4096 (41 charge sectors, 4,589,718 psi elements): 40 H_eff.psi
applies in a reduced-precision MFMA form, CGS2 reorthogonalisation,
tridiagonal eigensolve and one float64 apply for the refined energy.  Inputs
are resident on the GPU before timing starts.  The same solve in plain
float64 is timed beside it, and the refined energies of both are compared.

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
WORKLOAD = 5

# HBM bytes per launch of a kernel, from FETCH_SIZE / WRITE_SIZE counter runs
# scaled by a 1 GiB copy (profiles/hbm_traffic_lanczos40-spin1-chi4096.md).
# Valid only for the kernel source they were taken on: `src_sha` is the first
# 16 hex digits of that file's sha256; any change reports traffic as null.
TRAFFIC = {
    "gs_update": {"bytes_per_launch": 4.315e+08, "src": "paper_2401_01921_amd/csrc/kernels_aux.hip",
                  "src_sha": "8ced2cc2cba32584",
                  "profile": "profiles/hbm_traffic_lanczos40-spin1-chi4096.md"},
}


def measured_traffic(kernel):
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    with open(os.path.join(ROOT, t["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["src_sha"]:
            return None
    return t["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="bf16x3", choices=["fp32", "bf16x3", "bf16x6", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the single-apply, batched-apply and permute measurements")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tile variants (short runs under a profiler)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first time a plain device copy of this many MiB (a kernel of known "
                         "traffic that calibrates hardware byte counters)")
    return ap.parse_args()


def lanczos_vector_flops(n: int, m: int) -> float:
    """Algorithmic flops of CGS2 reorthogonalisation, normalisation and Ritz
    vector for m steps on vectors of n elements."""
    f = 0.0
    for j in range(1, m + 1):
        f += 4 * 2.0 * n * j      # two passes of V^T w and w -= V c
        f += 2.0 * n + n          # |w|^2 and scaling
    return f + 2.0 * n * m + 6.0 * n


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
    copy_cal = copy_calibration(torch, dev, a.copy_mib) if a.copy_mib > 0 else None
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
    step_flops = (m + 1) * apply_flops + lanczos_vector_flops(n, m)

    # autotune the tile variant of every GEMM step for both forms (untimed)
    tune_out = torch.empty(n, dtype=torch.float64, device=dev)
    tune_ws = bst.workspace(plan.workspace_bytes)
    tuned = {}
    for prec in (a.prec, "fp64"):
        plan.set_precision(prec)
        if not a.no_tune:
            plan.autotune([g["L"], g["W1"], g["W2"], g["R"], g["psi0"]], [tune_out], tune_ws,
                          reps=3)
        tuned[prec] = plan.tiles()
    del tune_ws, tune_out

    def solve(prec, timing=False, three_pass=False, f64_basis=False):
        return bst.lanczos_ground(plan, ops, g["psi0"], m, prec, True, ws=ws, psi_out=psi_out,
                                  timing=timing, three_pass=three_pass, f64_basis=f64_basis)

    def timed(prec, steps, warmup, three_pass=False, f64_basis=False):
        for _ in range(warmup):
            solve(prec, three_pass=three_pass, f64_basis=f64_basis)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        for _ in range(steps):
            res = solve(prec, three_pass=three_pass, f64_basis=f64_basis)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res

    # ---- timed region: the split-precision solve --------------------------
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
    inter32 = a.prec != "fp64"
    km, kc = prof_split["kernel_ms"], prof_split["kernel_calls"]
    mf = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6}[a.prec]
    peak_mm = {"fp64": PEAK["fp64_tflops"], "fp32": PEAK["fp32_tflops"]}.get(a.prec, PEAK["bf16_tflops"])

    def gemm_roof(name, ms_key, prof, prec, peak):
        calls = prof["kernel_calls"][ms_key]
        avg_ms = prof["kernel_ms"][ms_key] / max(calls, 1)
        fl = steps[name]["flops"]
        mult = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16x6": 6}[prec]
        by = steps[name]["bytes_fp32" if prec != "fp64" else "bytes_fp64"]
        if name == "gemm_T3_R" and prec in ("bf16x3", "bf16x6"):
            by -= 4.0 * n   # inside the solve H u_j is written as float32
        return dict(kernel=name, avg_ms=avg_ms, alg_tflops=fl / avg_ms / 1e9,
                    mfma_tflops=fl * mult / avg_ms / 1e9, peak_tflops=peak,
                    mfma_frac=fl * mult / avg_ms / 1e9 / peak,
                    bytes_gbs=by / avg_ms / 1e6)

    # Krylov rows are float32 with the split matvec forms, float64 otherwise
    vb = 4.0 if a.prec in ("bf16x3", "bf16x6") else 8.0

    def gs_bytes(kind, rowb=None):
        # algorithmic bytes of one solve's Gram-Schmidt kernels (default
        # schedule): the dot reads u_j and z; the pass of step j (0-based)
        # reads basis rows 0..j and z and writes row j and (except on the
        # last step) row j+1.  z = H u_j has the rows' element type (float32
        # rows with the split forms, float64 otherwise).
        rb = vb if rowb is None else rowb
        tot = 0.0
        for j in range(m):
            if kind == "dots":
                tot += 2.0 * rb * n
            else:
                tot += rb * n * (j + 1) + rb * n + rb * n * (2 if j + 1 < m else 1)
        return tot

    def hbm_roof(key, total_bytes, prof):
        ms = prof["kernel_ms"][key]
        calls = prof["kernel_calls"][key]
        return dict(kernel=key, avg_ms=ms / max(calls, 1), calls=calls,
                    achieved_gbs=total_bytes / ms / 1e6, frac=total_bytes / ms / 1e6 / PEAK["hbm_gbs"])

    mpo_bytes = steps["mpo_apply"]["bytes_fp32" if inter32 else "bytes_fp64"]
    kern = {
        "gemm_L_psi": gemm_roof("gemm_L_psi", "gemm_L_psi", prof_split, a.prec, peak_mm),
        "gemm_T3_R": gemm_roof("gemm_T3_R", "gemm_T3_R", prof_split, a.prec, peak_mm),
        "mpo_apply": hbm_roof("mpo_apply", mpo_bytes * kc["mpo_apply"], prof_split),
        "gs_dots": hbm_roof("gs_dots", gs_bytes("dots"), prof_split),
        "gs_update": hbm_roof("gs_update", gs_bytes("update"), prof_split),
        "fp64_gemm_L_psi": gemm_roof("gemm_L_psi", "gemm_L_psi", prof64, "fp64", PEAK["fp64_tflops"]),
        "fp64_gemm_T3_R": gemm_roof("gemm_T3_R", "gemm_T3_R", prof64, "fp64", PEAK["fp64_tflops"]),
    }
    # dominant kernel of the step = largest summed time
    dom = max((k for k in km if k in kern), key=km.get)
    if dom.startswith("gemm"):
        r = kern[dom]
        roof = {"bound": "mfma", "kernel": dom, "achieved": round(r["mfma_tflops"], 2),
                "peak": peak_mm, "unit": "TFLOP/s", "frac": round(r["mfma_frac"], 4), "traffic": None}
    else:
        r = kern[dom]
        per_launch = r["achieved_gbs"] * r["avg_ms"] * 1e6
        tr = measured_traffic(dom)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(r["achieved_gbs"], 1),
                "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": round(r["frac"], 4),
                "traffic": tr, "alg_bytes_per_launch": per_launch,
                "traffic_over_alg": None if tr is None else round(tr / per_launch, 4)}

    extras = {}
    if not a.no_extras:
        # the same split solve under the textbook three-pass schedule
        ms3, res3 = timed(a.prec, max(2, a.steps // 2), 1, three_pass=True)
        extras["three_pass_schedule"] = {
            "ms_per_solve": round(ms3 * 1e3, 3),
            "kernels": {k: round(v, 4) for k, v in
                        solve(a.prec, timing=True, three_pass=True)["kernel_ms"].items()},
            "energy_rel_diff_vs_lagged": abs(res3["energy"] - es) / abs(es)}
        # the same split solve with float64 Krylov rows (and float64 H u_j)
        msb, resb = timed(a.prec, max(2, a.steps // 2), 1, f64_basis=True)
        extras["float64_basis"] = {
            "ms_per_solve": round(msb * 1e3, 3),
            "energy_rel_err_vs_fp64": abs(resb["energy"] - e64) / abs(e64),
            "speedup_vs_fp64": round(ms64 / msb, 3)}
    extras.update({} if a.no_extras else bench_extras(bst, wl, torch, dev, plan, ins_apply=[
        g["L"], g["W1"], g["W2"], g["R"], g["psi0"]], apply_flops=apply_flops))

    # ---- CPU baseline: the oracle's H_eff apply on the host cores ----------
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(specs, host, apply_flops, a.cpu_seconds)

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
                   "psi_elements": n, "lanczos_steps": m, "matvec": a.prec, "refine": "fp64",
                   "flops_per_step": step_flops, "heff_flops_per_apply": apply_flops},
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


def copy_calibration(torch, dev, mib):
    """Three device-to-device copies of `mib` MiB: each reads and writes
    exactly mib MiB, which scales the FETCH_SIZE / WRITE_SIZE counters."""
    src = torch.ones(mib * 2**20 // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    ms = _time_ms(torch, lambda: dst.copy_(src), 3, warm=0)
    del src, dst
    return {"mib": mib, "reps": 3, "ms": round(ms, 4),
            "gbs": round(2 * mib * 2**20 / ms / 1e6, 1)}


def _time_ms(torch, fn, reps, warm=2):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def bench_extras(bst, wl, torch, dev, plan, ins_apply, apply_flops):
    """Single H_eff applies per form, the 64-apply batched launch (one
    hipGraph per step sequence) and the block permute on a tensor above 1 GiB."""
    out = {}
    # single applies of the chi=4096 operator, every form (tuned tiles)
    res = torch.empty_like(ins_apply[4])
    ws = bst.workspace(plan.workspace_bytes)
    forms = {}
    for prec in ("fp64", "fp32", "bf16x3", "bf16x6"):
        plan.set_precision(prec)
        if prec in ("fp32", "bf16x6"):
            plan.autotune(ins_apply, [res], ws, reps=3)
        ms = _time_ms(torch, lambda: plan.execute(ins_apply, [res], ws), 20)
        forms[prec] = {"ms": round(ms, 4), "gflops": round(apply_flops / ms / 1e6, 1)}
    out["apply_chi4096"] = forms
    del ws, res
    # batched: 64 uneven spin-1/2 applies, all sector GEMMs of a step in one launch
    members, ins, outs = [], [], []
    W = None
    for i, (chi, q) in enumerate(wl.batch_draws()):
        v = wl.gaussian_sector_dims(chi, q)
        T = {k: bst.Tensor(*s) for k, s in wl.heff_specs("1/2", v, v).items()}
        if W is None:
            W = torch.from_numpy(T["W1"].from_dense(wl.heisenberg_mpo_dense("1/2"))).to(dev)
        p = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], "bf16x3")
        members.append(p)
        ins += [torch.randn(T["L"].numel, dtype=torch.float64, device=dev), W, W,
                torch.randn(T["R"].numel, dtype=torch.float64, device=dev),
                torch.randn(T["psi"].numel, dtype=torch.float64, device=dev)]
        outs.append(torch.empty(T["psi"].numel, dtype=torch.float64, device=dev))
    batch = bst.heff_batch_plan(members)
    bflops = batch.stats().flops
    wsb = bst.workspace(batch.workspace_bytes)
    batch.autotune(ins, outs, wsb, reps=3)
    batch.use_graph(True)
    ms_b = _time_ms(torch, lambda: batch.execute(ins, outs, wsb), 20)
    batch.use_graph(False)
    ms_e = _time_ms(torch, lambda: batch.execute(ins, outs, wsb), 20)
    out["batch64_bf16x3"] = {"ms_graph": round(ms_b, 4), "ms_eager": round(ms_e, 4),
                             "gflops_graph": round(bflops / ms_b / 1e6, 1), "flops": bflops,
                             "kernels_per_execute": batch.stats().nsteps,
                             "gemm_problems": batch.stats().gemm_problems}
    del wsb, ins, outs, batch, members
    # the XX chain's MPO (bond of 4 channels; the model of the paper's DMRG
    # benchmark): one spin-1/2 apply at chi = 4096, q in [-20, 20]
    v = wl.gaussian_sector_dims(4096, 20)
    T = {k: bst.Tensor(*s) for k, s in wl.heff_specs("1/2", v, v, "xx").items()}
    Wx = torch.from_numpy(T["W1"].from_dense(wl.mpo_dense("1/2", "xx"))).to(dev)
    ins_x = [torch.randn(T["L"].numel, dtype=torch.float64, device=dev), Wx, Wx,
             torch.randn(T["R"].numel, dtype=torch.float64, device=dev),
             torch.randn(T["psi"].numel, dtype=torch.float64, device=dev)]
    px = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], "fp64")
    res_x = torch.empty(T["psi"].numel, dtype=torch.float64, device=dev)
    ws_x = bst.workspace(px.workspace_bytes)
    fl_x = px.stats().flops
    xx = {"psi_elements": T["psi"].numel, "flops": fl_x}
    for prec in ("fp64", "bf16x3"):
        px.set_precision(prec)
        px.autotune(ins_x, [res_x], ws_x, reps=3)
        ms = _time_ms(torch, lambda: px.execute(ins_x, [res_x], ws_x), 20)
        xx[prec] = {"ms": round(ms, 4), "gflops": round(fl_x / ms / 1e6, 1)}
    out["apply_xx_spin_half_chi4096"] = xx
    del ws_x, res_x, ins_x, px
    # block permute of a 1.2 GiB tensor (c, a, b) <- (a, b, c)
    sec = [(q, 150) for q in range(-3, 4)]
    T = bst.Tensor(["a", "b", "c"], [(1, sec), (1, sec), (-1, [(q, 150) for q in range(-6, 7)])])
    Tp, pplan = bst.permute_plan(T, ["c", "a", "b"])
    x = torch.randn(T.numel, dtype=torch.float64, device=dev)
    y = torch.empty(T.numel, dtype=torch.float64, device=dev)
    wsp = bst.workspace(pplan.workspace_bytes)
    ms_p = _time_ms(torch, lambda: pplan.execute([x], [y], wsp), 10)
    prof = pplan.profile([x], [y], wsp, reps=5)
    kms = prof[0][1]
    out["permute"] = {"numel": T.numel, "gib": round(T.numel * 8 / 2**30, 3), "blocks": T.nblocks,
                      "order": "(c,a,b) <- (a,b,c)",
                      "ms": round(ms_p, 4), "kernel_ms": round(kms, 4),
                      "gbs": round(2 * 8 * T.numel / kms / 1e6, 1),
                      "hbm_frac": round(2 * 8 * T.numel / kms / 1e6 / PEAK["hbm_gbs"], 4)}
    # the same tensor with its fastest leg kept: block rows are copied whole
    Tq, qplan = bst.permute_plan(T, ["b", "a", "c"])
    wsq = bst.workspace(qplan.workspace_bytes)
    kq = qplan.profile([x], [y], wsq, reps=5)[0][1]
    out["permute_rows"] = {"order": "(b,a,c) <- (a,b,c)", "kernel_ms": round(kq, 4),
                           "gbs": round(2 * 8 * T.numel / kq / 1e6, 1),
                           "hbm_frac": round(2 * 8 * T.numel / kq / 1e6 / PEAK["hbm_gbs"], 4)}
    del x, y, wsp, wsq
    return out


def cpu_baseline(specs, host, apply_flops, seconds):
    """The float64 oracle's H_eff apply on this host (numpy; BLAS threads as
    configured), repeated for about `seconds`."""
    from oracle import oracle as orc
    O = {k: orc.BlockTensor(*specs[k]) for k in ("L", "R", "psi")}
    O["L"].data[:] = host["L"]
    O["R"].data[:] = host["R"]
    O["psi"].data[:] = host["psi0"]
    W1 = orc.BlockTensor(*specs["W1"], host["W1"])
    W2 = orc.BlockTensor(*specs["W2"], host["W2"])
    reps, t0 = 0, time.perf_counter()
    while True:
        orc.heff_apply(O["L"], W1, W2, O["R"], O["psi"])
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds or reps >= 20:
            break
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads") or 0) for i in threadpool_info()) or None
    except Exception:
        pass
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    return {"value": round(apply_flops * reps / el / 1e9, 2), "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} float64 H_eff.psi applies of the chi=4096 spin-1 workload "
                      f"({el:.1f} s, numpy oracle)"}


if __name__ == "__main__":
    main()
