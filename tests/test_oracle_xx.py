"""The XX chain, the model of the paper's DMRG benchmark (Sec. "Benchmarks"):
its MPO (bond dimension 4) pinned to J (Sx Sx + Sy Sy) built from the complex
spin matrices, the oracle's exact diagonalisation pinned to the free-fermion
closed form (Jordan-Wigner), and the oracle's H_eff and Lanczos on exact
environments of whole XX chains."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2401_01921_amd import workloads as wl
from tests import chain_env
from tests.test_oracle_heff import heff_matrix, heff_tensors


def free_fermion_ground(nsites: int, J: float = 1.0) -> float:
    """Open spin-1/2 XX chain = free fermions hopping with amplitude J/2:
    single-particle energies J cos(pi k / (N + 1)), k = 1..N; the ground
    state fills every negative level (N/2 of them for even N, i.e. total
    Sz = 0)."""
    return sum(min(0.0, J * math.cos(math.pi * k / (nsites + 1))) for k in range(1, nsites + 1))


@pytest.mark.parametrize("spin", ["1/2", "1"])
def test_xx_mpo_bond_term(spin):
    """sum_w W[left-boundary, w] (x) W[w, right-boundary] = Sx Sx + Sy Sy,
    with Sx = (S+ + S-)/2 and Sy = (S+ - S-)/(2i) as complex matrices."""
    W = wl.mpo_dense(spin, "xx")
    assert W.shape[0] == 4 and W.shape[3] == 4
    sp, sm, _, _ = orc._spin_ops(spin)
    sx = (sp + sm).astype(complex) / 2
    sy = (sp - sm).astype(complex) / 2j
    ref = np.kron(sx, sx) + np.kron(sy, sy)
    assert np.max(np.abs(ref.imag)) == 0.0
    first = wl.grouped_index(4, "xx")
    last = wl.grouped_index(0, "xx")
    d = sp.shape[0]
    acc = np.zeros((d * d, d * d))
    for w in range(4):
        acc += np.kron(W[first, :, :, w], W[w, :, :, last])
    assert np.allclose(acc, ref.real, rtol=0, atol=1e-15)
    # no Sz Sz term, unlike the Heisenberg MPO
    H = wl.mpo_dense(spin, "heisenberg")
    acc_h = np.zeros_like(acc)
    for w in range(5):
        acc_h += np.kron(H[wl.grouped_index(4), :, :, w], H[w, :, :, wl.grouped_index(0)])
    sz = orc._spin_ops(spin)[2]
    assert np.allclose(acc_h - acc, np.kron(sz, sz), rtol=0, atol=1e-15)
    # charge conserving on its grouped legs (bond [-d:1, 0:2, +d:1])
    assert wl.mpo_bond(spin, "xx")[1] == (0, 2)
    orc.from_dense(*wl.heff_specs(spin, [(0, 1)], [(0, 1)], "xx")["W1"], W)


@pytest.mark.parametrize("nsites", [2, 4, 6, 8, 10])
def test_xx_chain_free_fermion_closed_form(nsites):
    E = orc.chain_ground(nsites, "1/2", "xx")
    assert abs(E - free_fermion_ground(nsites)) < 1e-12


def test_xx_chain_odd_length_any_sector():
    """Three sites: levels cos(pi/4), 0, -cos(pi/4); the lowest state is
    -1/sqrt(2) (the zero mode leaves two degenerate sectors)."""
    E = orc.chain_ground(3, "1/2", "xx", charge=None)
    assert abs(E + 1.0 / math.sqrt(2.0)) < 1e-14


@pytest.mark.parametrize("spin,nsites", [("1/2", 4), ("1/2", 6), ("1/2", 8), ("1", 4)])
def test_xx_heff_with_exact_environments(spin, nsites):
    """The centre two-site H_eff of an XX chain with exact environments (MPO
    bond 4) has the chain's ground energy as its lowest eigenvalue, found by
    the dense matrix and by the oracle's Lanczos."""
    Ld, Rd, Wd, specs = chain_env.chain_heff_dense(nsites, spin, "xx")
    assert Ld.shape[1] == 4 and Rd.shape[1] == 4
    ops = heff_tensors(Ld, Rd, Wd, specs)
    E_ed = orc.chain_ground(nsites, spin, "xx")
    if spin == "1/2":
        assert abs(E_ed - free_fermion_ground(nsites)) < 1e-12
    H = heff_matrix(*ops)
    assert np.allclose(H, H.T, atol=1e-13)
    assert abs(np.linalg.eigvalsh(H)[0] - E_ed) < 1e-10
    psi0 = wl.normal(4321 + nsites, ops[4].numel)
    mv = lambda v: orc.heff_apply(*ops[:4], orc.BlockTensor(ops[4].labels, ops[4].legs, v)).data
    res = orc.lanczos_ground(mv, psi0, ops[4].numel)
    assert abs(res["energy"] - E_ed) < 1e-10
