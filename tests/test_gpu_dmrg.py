"""Two-site DMRG sweep on the GPU (Sec. "Benchmarks": DMRG of the XX chain):
every numeric step runs in the library (contraction plans, H_eff Lanczos,
symmetric truncated SVD).  Untruncated sweeps of short open chains end at
the exact-diagonalisation ground-state energy and follow the oracle's sweep
update by update; a truncated sweep stays variational."""
import numpy as np
import pytest

from tests.gpu_common import DEV, dev, host, require_gpu, torch
from oracle import oracle as orc
from paper_2401_01921_amd import bst, dmrg, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _inputs(nsites, spin, model, seed):
    specs = wl.mps_specs(nsites, spin, 0)
    mps_o, mps_g = [], []
    for i, (labels, legs) in enumerate(specs):
        T = orc.BlockTensor(labels, legs)
        T.data[:] = wl.normal(seed * 100 + i, T.numel)
        mps_o.append(T)
        mps_g.append(dmrg.DevTensor(bst.Tensor(labels, legs), dev(T.data)))
    Ws = wl.heff_specs(spin, [(0, 1)], [(0, 1)], model)["W1"]
    Wo = orc.from_dense(*Ws, wl.mpo_dense(spin, model))
    Wg = dmrg.DevTensor(bst.Tensor(*Ws), dev(Wo.data))
    Ls, lpos, Rs, rpos = wl.boundary_env_specs(spin, model, 0)
    D = np.zeros(orc.BlockTensor(*Ls).dims())
    D[lpos] = 1.0
    Lo = orc.from_dense(*Ls, D)
    D = np.zeros(orc.BlockTensor(*Rs).dims())
    D[rpos] = 1.0
    Ro = orc.from_dense(*Rs, D)
    Lg = dmrg.DevTensor(bst.Tensor(*Ls), dev(Lo.data))
    Rg = dmrg.DevTensor(bst.Tensor(*Rs), dev(Ro.data))
    return (mps_o, Wo, Lo, Ro), (mps_g, Wg, Lg, Rg)


@pytest.mark.parametrize("nsites,spin,model", [(6, "1/2", "xx"), (10, "1/2", "xx"), (8, "1/2", "heisenberg"),
                                               (6, "1", "heisenberg")])
def test_untruncated_sweep_matches_exact_and_oracle(nsites, spin, model):
    (mo, Wo, Lo, Ro), (mg, Wg, Lg, Rg) = _inputs(nsites, spin, model, 11)
    E, errs, A = dmrg.dmrg_two_site(mg, Wg, Lg, Rg, 2, 1 << 20, 1e-12)
    exact = orc.chain_ground(nsites, spin, model, charge=0)
    print("dmrg", nsites, spin, model, "E", E[-1], "exact", exact, "updates", len(E), flush=True)
    assert abs(E[-1] - exact) <= 1e-10 * max(1.0, abs(exact))
    Eo, _ = orc.dmrg_two_site(mo, Wo, Lo, Ro, 2, 1 << 20, 1e-12)
    assert len(Eo) == len(E)
    assert np.max(np.abs(np.array(E) - np.array(Eo))) <= 1e-9 * max(1.0, abs(exact))
    # the final MPS: right-orthonormal sites 1.. (V^dagger factors)
    for T in A[1:]:
        labels, legs = T.t.legs()
        O = orc.BlockTensor(labels, legs, host(T.data))
        for s in orc.svd_sectors(O, 1):
            assert np.allclose(s["M"] @ s["M"].T, np.eye(s["M"].shape[0]), atol=1e-10)


def test_truncated_sweep_is_variational():
    nsites, spin, model = 10, "1/2", "xx"
    _, (mg, Wg, Lg, Rg) = _inputs(nsites, spin, model, 5)
    E, errs, _ = dmrg.dmrg_two_site(mg, Wg, Lg, Rg, 2, 6, 1e-12)
    exact = orc.chain_ground(nsites, spin, model, charge=0)
    print("truncated dmrg E", E[-1], "exact", exact, "max s_err", max(errs), flush=True)
    assert min(E) >= exact - 1e-10
    assert E[-1] <= E[0] + 1e-12
    assert max(errs) > 0.0


def test_bf16x3_matvec_sweep():
    """The split-precision matvec inside the sweep's Lanczos, with the float64
    refinement apply, still ends at the exact energy."""
    nsites, spin, model = 8, "1/2", "xx"
    _, (mg, Wg, Lg, Rg) = _inputs(nsites, spin, model, 7)
    E, _, _ = dmrg.dmrg_two_site(mg, Wg, Lg, Rg, 2, 1 << 20, 1e-12, prec="bf16x3")
    exact = orc.chain_ground(nsites, spin, model, charge=0)
    assert abs(E[-1] - exact) <= 1e-9 * max(1.0, abs(exact))
