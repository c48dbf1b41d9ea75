"""Pins of the oracle's H_eff.psi, MPO input, Lanczos and exact
diagonalisation: closed-form spin energies (angular momentum addition),
brute-force dense H_eff, exact diagonalisation of whole chains through exact
environments, symmetry of H_eff, and a library tridiagonal eigensolver."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as orc
from paper_2401_01921_amd import workloads as wl
from tests import chain_env


def heff_tensors(Ld, Rd, Wd, specs, psi_data=None):
    L = orc.from_dense(*specs["L"], Ld)
    R = orc.from_dense(*specs["R"], Rd)
    W1 = orc.from_dense(*specs["W1"], Wd)
    W2 = orc.from_dense(*specs["W2"], Wd)
    psi = orc.BlockTensor(*specs["psi"])
    if psi_data is not None:
        psi.data[:] = psi_data
    return L, W1, W2, R, psi


def heff_matrix(L, W1, W2, R, psi):
    n = psi.numel
    H = np.zeros((n, n))
    for i in range(n):
        e = orc.BlockTensor(psi.labels, psi.legs)
        e.data[i] = 1.0
        H[:, i] = orc.heff_apply(L, W1, W2, R, e).data
    return H


@pytest.mark.parametrize("spin", ["1/2", "1"])
def test_mpo_bond_term_is_heisenberg(spin):
    """sum_w W[left-boundary, w] (x) W[w, right-boundary] = S1.S2."""
    W = wl.heisenberg_mpo_dense(spin)
    sp, sm, sz, _ = orc._spin_ops(spin)
    first = wl.grouped_index(4)
    last = wl.grouped_index(0)
    d = sp.shape[0]
    acc = np.zeros((d * d, d * d))
    for w in range(5):
        acc += np.kron(W[first, :, :, w], W[w, :, :, last])
    ref = 0.5 * (np.kron(sp, sm) + np.kron(sm, sp)) + np.kron(sz, sz)
    assert np.array_equal(acc, ref)
    # and the MPO is charge conserving on its grouped legs
    orc.from_dense(*wl.heff_specs(spin, [(0, 1)], [(0, 1)])["W1"], W)


@pytest.mark.parametrize("spin,singlet,others", [("1/2", -0.75, [0.25]), ("1", -2.0, [-1.0, 1.0])])
def test_two_site_singlet_energy(spin, singlet, others):
    """Two sites with trivial environments: S1.S2 = [S(S+1) - 2s(s+1)]/2, so the
    singlet is -3/4 (spin 1/2) or -2 (spin 1); psi's right bond {0:1} keeps
    the total-Sz-zero states."""
    Ld, Rd, Wd, specs = chain_env.chain_heff_dense(2, spin)
    ops = heff_tensors(Ld, Rd, Wd, specs)
    H = heff_matrix(*ops)
    ev = np.linalg.eigvalsh(H)
    assert abs(ev[0] - singlet) < 1e-14
    for o in others:
        assert np.min(np.abs(ev - o)) < 1e-14


def test_open_chain_closed_forms():
    """Angular-momentum closed forms for the exact diagonalisation."""
    assert abs(orc.heisenberg_chain_ground(2, "1/2") + 0.75) < 1e-14
    assert abs(orc.heisenberg_chain_ground(3, "1/2", charge=None) + 1.0) < 1e-14
    assert abs(orc.heisenberg_chain_ground(2, "1") + 2.0) < 1e-14


@pytest.mark.parametrize("spin,nsites", [("1/2", 4), ("1/2", 6), ("1/2", 8), ("1/2", 10), ("1", 4), ("1", 6)])
def test_heff_with_exact_environments_matches_ed(spin, nsites):
    """The centre two-site H_eff with exact environments spans the whole
    zero-charge space of the chain, so its lowest eigenvalue (both by the
    dense matrix and by the oracle's Lanczos run to breakdown) equals the
    exact ground-state energy of the chain."""
    Ld, Rd, Wd, specs = chain_env.chain_heff_dense(nsites, spin)
    ops = heff_tensors(Ld, Rd, Wd, specs)
    E_ed = orc.heisenberg_chain_ground(nsites, spin)
    H = heff_matrix(*ops)
    assert np.allclose(H, H.T, atol=1e-13)
    assert abs(np.linalg.eigvalsh(H)[0] - E_ed) < 1e-10
    psi0 = wl.normal(12345 + nsites, ops[4].numel)
    mv = lambda v: orc.heff_apply(*ops[:4], orc.BlockTensor(ops[4].labels, ops[4].legs, v)).data
    res = orc.lanczos_ground(mv, psi0, ops[4].numel)
    assert abs(res["energy"] - E_ed) < 1e-10
    assert abs(res["theta"] - E_ed) < 1e-10


def test_heff_equals_dense_contraction():
    """Tiny random operands: block-sparse H_eff.psi equals the dense einsum of
    the embedded L, W, W, R and psi; outside psi's blocks it is exactly 0."""
    v = wl.gaussian_sector_dims(12, 2)
    specs = wl.heff_specs("1/2", v, v)
    L = orc.BlockTensor(*specs["L"])
    R = orc.BlockTensor(*specs["R"])
    psi = orc.BlockTensor(*specs["psi"])
    L.data[:] = wl.normal(1, L.numel)
    R.data[:] = wl.normal(2, R.numel)
    psi.data[:] = wl.normal(3, psi.numel)
    W = orc.from_dense(*specs["W1"], wl.heisenberg_mpo_dense("1/2"))
    out = orc.heff_apply(L, W, W, R, psi)
    assert out.blocks == psi.blocks and out.legs == psi.legs
    # t, u: bra legs of W1, W2 contracted with psi's physical legs
    ref = np.einsum("awx,xtuy,wstv,vpuz,bzy->aspb", orc.embed(L), orc.embed(psi),
                    orc.embed(W), orc.embed(W), orc.embed(R), optimize=True)
    dense = orc.embed(out)
    assert np.max(np.abs(dense - ref)) <= 1e-13 * np.max(np.abs(ref))
    mask = np.abs(orc.embed(orc.BlockTensor(psi.labels, psi.legs, np.ones(psi.numel)))) > 0
    assert np.all(ref[~mask] == 0.0)


@pytest.mark.parametrize("recipe", ["symmetrized", "dmrg_like"])
def test_environment_recipes_make_heff_symmetric(recipe):
    """<phi, H psi> = <H phi, psi> for the environment recipes used by the
    Lanczos workload (random operands otherwise)."""
    v = wl.gaussian_sector_dims(16, 2)
    specs = wl.heff_specs("1", v, v)
    L = orc.BlockTensor(*specs["L"])
    R = orc.BlockTensor(*specs["R"])
    if recipe == "symmetrized":
        L.data[:] = wl.symmetrized_env(L.table(), L.numel, 7)
        R.data[:] = wl.symmetrized_env(R.table(), R.numel, 8)
    else:
        L.data[:] = wl.dmrg_like_env(L.table(), L.numel, 7, "L", v)
        R.data[:] = wl.dmrg_like_env(R.table(), R.numel, 8, "R", v)
    W = orc.from_dense(*specs["W1"], wl.heisenberg_mpo_dense("1"))
    H = heff_matrix(L, W, W, R, orc.BlockTensor(*specs["psi"]))
    assert np.max(np.abs(H - H.T)) < 1e-13 * np.max(np.abs(H))


def test_tridiagonal_solver_matches_library():
    rng = np.random.default_rng(3)
    for n in [1, 2, 3, 10, 40]:
        a = rng.standard_normal(n)
        b = np.abs(rng.standard_normal(n - 1)) + 0.1
        theta, s = orc.tridiag_lowest(a, b)
        w, v = scipy.linalg.eigh_tridiagonal(a, b)
        assert abs(theta - w[0]) <= 4e-15 * max(1.0, abs(w[0])) * n
        ref = v[:, 0] * np.sign(v[np.argmax(np.abs(v[:, 0])), 0])
        assert np.max(np.abs(s - ref)) < 1e-10


def test_lanczos_on_small_symmetric_matrices():
    rng = np.random.default_rng(4)
    for n in [5, 17, 40]:
        X = rng.standard_normal((n, n))
        A = (X + X.T) / 2
        res = orc.lanczos_ground(lambda v: A @ v, rng.standard_normal(n), n)
        w = np.linalg.eigvalsh(A)
        assert abs(res["theta"] - w[0]) < 1e-12 * max(1.0, abs(w[0]))
        assert abs(res["energy"] - w[0]) < 1e-12 * max(1.0, abs(w[0]))
        V = res["V"]
        assert np.max(np.abs(V @ V.T - np.eye(V.shape[0]))) < 1e-13


def test_lanczos_breakdown_on_invariant_subspace():
    """A start vector inside a 3-dim invariant subspace ends after 3 steps."""
    A = np.diag([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    v0 = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    res = orc.lanczos_ground(lambda v: A @ v, v0, 6)
    assert res["steps"] == 3
    assert abs(res["theta"] - 1.0) < 1e-14


def test_planted_mpo_sign_error_is_caught():
    """Flipping the sign of the Sz.Sz term (a plausible slip in the MPO input)
    moves the two-site spin-1/2 spectrum off the closed form."""
    Ld, Rd, Wd, specs = chain_env.chain_heff_dense(2, "1/2")
    bad = Wd.copy()
    bad[wl.grouped_index(4), :, :, wl.grouped_index(3)] *= -1
    ops = heff_tensors(Ld, Rd, bad, specs)
    ev = np.linalg.eigvalsh(heff_matrix(*ops))
    assert abs(ev[0] + 0.75) > 1e-3


def test_heff_flop_count_closed_form():
    """With one sector per leg (dense tensors) the algorithmic flops of the
    four steps have closed forms: 2 chi^2 D (chi d^2) for L.psi, 2 (chi d^2
    chi D) d D for each MPO step (K = D d, N = d D), 2 (chi d^2) chi (D chi)
    for T3.R."""
    chi, D, d = 6, 5, 2
    legs_v = [(0, chi)]
    ph = [(0, d)]
    mb = [(0, D)]
    L = orc.BlockTensor(["a", "w", "ap"], [(1, legs_v), (-1, mb), (-1, legs_v)])
    R = orc.BlockTensor(["b", "w", "bp"], [(-1, legs_v), (1, mb), (1, legs_v)])
    W = orc.BlockTensor(["wl", "s", "sp", "wr"], [(1, mb), (1, ph), (-1, ph), (-1, mb)])
    psi = orc.BlockTensor(["a", "s1", "s2", "b"], [(1, legs_v), (1, ph), (1, ph), (-1, legs_v)])
    f = orc.heff_flops(L, W, W, R, psi)
    assert f[0] == 2 * (chi * D) * chi * (d * d * chi)
    assert f[1] == 2 * (chi * d * chi) * (D * d) * (d * D)
    assert f[2] == 2 * (chi * d * chi) * (D * d) * (d * D)
    assert f[3] == 2 * (chi * d * d) * (D * chi) * chi
