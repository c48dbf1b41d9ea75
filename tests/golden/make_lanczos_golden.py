"""Writes lanczos_spin1_chi4096.json: the float64 oracle's 40-step Lanczos
on the spin-1, chi = 4096 workload (DMRG-like environments, seeded start
vector).  Calls only the oracle and the seeded input generators.

    python tests/golden/make_lanczos_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2401_01921_amd import workloads as wl  # noqa: E402


def main():
    k = 5
    w = wl.WORKLOADS[k]
    v = wl.gaussian_sector_dims(w["chi"], w["qmax"])
    specs = wl.heff_specs(w["spin"], v, v)
    O = {n: orc.BlockTensor(*s) for n, s in specs.items()}
    O["L"].data[:] = wl.dmrg_like_env(O["L"].table(), O["L"].numel, wl.seed_for(k, "L"), "L", v)
    O["R"].data[:] = wl.dmrg_like_env(O["R"].table(), O["R"].numel, wl.seed_for(k, "R"), "R", v)
    Wd = wl.heisenberg_mpo_dense(w["spin"])
    O["W1"] = orc.from_dense(*specs["W1"], Wd)
    O["W2"] = orc.from_dense(*specs["W2"], Wd)
    psi0 = wl.normal(wl.seed_for(k, "psi0"), O["psi"].numel)
    t0 = time.time()

    def mv(x):
        return orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"],
                              orc.BlockTensor(O["psi"].labels, O["psi"].legs, x)).data

    r = orc.lanczos_ground(mv, psi0, w["steps"])
    out = dict(workload=w["name"], steps=r["steps"], theta=r["theta"], energy=r["energy"],
               residual=r["residual"], alpha=r["alpha"].tolist(), beta=r["beta"].tolist(),
               oracle_seconds=time.time() - t0)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "lanczos_spin1_chi4096.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("theta", "energy", "residual", "oracle_seconds")}))


if __name__ == "__main__":
    main()
