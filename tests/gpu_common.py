"""Shared pieces of the GPU parity tests: operand generation on the host
(seeded, identical buffers for the oracle and the library), device copies
and error metrics."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as orc  # noqa: E402
from paper_2401_01921_amd import bst, workloads as wl  # noqa: E402

DEV = "cuda"


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel_err(got: np.ndarray, ref: np.ndarray):
    """(normwise relative error, max-abs error over max |ref|)."""
    nr = np.linalg.norm(ref)
    if nr == 0:
        return float(np.linalg.norm(got)), float(np.max(np.abs(got), initial=0.0))
    return (float(np.linalg.norm(got - ref) / nr),
            float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))


# Tolerances of the arithmetic forms against the float64 oracle, for one
# contraction or H_eff apply: float64 rounding; float32 operands and
# accumulation; bf16 split with 2 and 3 planes.  TOL bounds the normwise
# error |y - y_ref| / |y_ref|.  A bf16x3 product drops terms of at most
# 3 * 2^-18 of |a b| (a1 b1, and the rounding of a1 and b1), so one product
# is good to 1.1e-5 and sums of random-sign products come out near 4e-6;
# bf16x6 and float32 sit at the float32 accumulation error.  TOL_MAX bounds
# the max-abs error over max |y_ref|, which on N(0,1) data tracks the
# normwise error within a small factor.
TOL = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 2e-5, "bf16x6": 2e-6}
TOL_MAX = {"fp64": 1e-12, "fp32": 8e-6, "bf16x3": 8e-5, "bf16x6": 8e-6}


def check(got: np.ndarray, ref: np.ndarray, prec: str, what: str = "", steps: int = 1):
    """Assert both error measures of `got` against the oracle's `ref`
    within the tolerances of form `prec` (times `steps` for a chain of that
    many rounded contractions); returns (normwise, max-abs)."""
    nrm, mx = rel_err(got, ref)
    print(what, prec, "normwise", nrm, "max-abs", mx, flush=True)
    assert nrm <= steps * TOL[prec], (what, prec, "normwise", nrm)
    assert mx <= steps * TOL_MAX[prec], (what, prec, "max-abs", mx)
    return nrm, mx


def heff_operands(k: int, recipe: str = "normal", chi=None, qmax=None, spin=None,
                  model: str = "heisenberg"):
    """Oracle tensors and host data of an H_eff workload (Heisenberg MPO, or
    the XX MPO with its bond of 4 channels)."""
    wlk = wl.WORKLOADS[k]
    spin = spin or wlk["spin"]
    v = wl.gaussian_sector_dims(chi or wlk["chi"], qmax if qmax is not None else wlk["qmax"])
    specs = wl.heff_specs(spin, v, v, model)
    O = {n: orc.BlockTensor(*s) for n, s in specs.items()}
    if recipe == "normal":
        O["L"].data[:] = wl.normal(wl.seed_for(k, "L"), O["L"].numel)
        O["R"].data[:] = wl.normal(wl.seed_for(k, "R"), O["R"].numel)
    else:
        O["L"].data[:] = wl.dmrg_like_env(O["L"].table(), O["L"].numel, wl.seed_for(k, "L"), "L", v)
        O["R"].data[:] = wl.dmrg_like_env(O["R"].table(), O["R"].numel, wl.seed_for(k, "R"), "R", v)
    if recipe != "normal" and model != "heisenberg":
        raise ValueError("DMRG-like environments are built for the Heisenberg MPO")
    Wd = wl.mpo_dense(spin, model)
    O["W1"] = orc.from_dense(*specs["W1"], Wd)
    O["W2"] = orc.from_dense(*specs["W2"], Wd)
    O["psi"].data[:] = wl.normal(wl.seed_for(k, "psi"), O["psi"].numel)
    return specs, O


def lib_heff(specs, prec="fp64"):
    T = {n: bst.Tensor(*s) for n, s in specs.items()}
    plan = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], prec)
    return T, plan


def run_heff(plan, O, prec=None):
    if prec is not None:
        plan.set_precision(prec)
    ins = [dev(O[n].data) for n in ("L", "W1", "W2", "R", "psi")]
    # output and workspace start as NaN bytes: a value the kernels forget to
    # write, or an unwritten intermediate they read, shows up as NaN
    out = torch.full((O["psi"].numel,), float("nan"), dtype=torch.float64, device=DEV)
    ws = bst.workspace(plan.workspace_bytes)
    ws.fill_(255)
    plan.execute(ins, [out], ws)
    torch.cuda.synchronize()
    return host(out)
