"""Pins of the oracle's Z_n and product (U(1) x Z_n) symmetries (Sec.
"Symmetry and quantum numbers": a Z_n charge combines by addition modulo n
and is negated on outgoing legs; several symmetries act component by
component): reduction to U(1) when no flux can wrap, the closed-form Z_2
block count, product symmetries as the intersection of their factors,
contraction against the dense einsum of the embeddings, and the grouped
combine rule."""
import numpy as np
import pytest

from oracle import oracle as orc
from tests.helpers import _einsum_reference, _random_sym_pair


@pytest.mark.parametrize("seed", range(6))
def test_zn_equals_u1_when_no_flux_wraps(seed):
    """Non-negative charges whose total flux stays inside (-n, n): the Z_n
    blocks are the U(1) blocks."""
    rng = np.random.default_rng(seed)
    r = int(rng.integers(1, 5))
    legs = []
    for _ in range(r):
        qs = sorted(rng.choice(3, int(rng.integers(1, 4)), replace=False).tolist())
        legs.append((int(rng.choice([1, -1])), [(q, int(rng.integers(1, 4))) for q in qs]))
    n = 2 * r + 1   # |flux| <= 2 r < n
    labels = [f"l{i}" for i in range(r)]
    U = orc.BlockTensor(labels, legs)
    Z = orc.BlockTensor(labels, legs, sym=(n,))
    assert U.blocks == Z.blocks and U.numel == Z.numel


@pytest.mark.parametrize("r,g0,g1", [(1, 2, 3), (2, 2, 3), (3, 1, 4), (4, 3, 2), (5, 1, 1)])
def test_z2_block_count_closed_form(r, g0, g1):
    """Every leg {0: g0, 1: g1}, any directions: half of the 2^r tuples have
    even parity, and the kept elements number ((g0+g1)^r + (g0-g1)^r) / 2."""
    rng = np.random.default_rng(r)
    legs = [(int(rng.choice([1, -1])), [(0, g0), (1, g1)]) for _ in range(r)]
    T = orc.BlockTensor([f"l{i}" for i in range(r)], legs, sym=(2,))
    assert len(T.blocks) == 2 ** (r - 1)
    assert T.numel == ((g0 + g1) ** r + (g0 - g1) ** r) // 2


def test_z3_rank3_by_hand():
    """Z_3, legs in, in, out: for every (q_a, q_b) exactly one q_c = q_a + q_b
    mod 3 closes the flux, so 9 blocks; elements sum g_a g_b g_c."""
    ga, gb, gc = [2, 3, 1], [1, 2, 2], [2, 1, 3]
    legs = [(1, list(enumerate(ga))), (1, list(enumerate(gb))), (-1, list(enumerate(gc)))]
    T = orc.BlockTensor(["a", "b", "c"], legs, sym=(3,))
    assert T.blocks == [(a, b, (a + b) % 3) for a in range(3) for b in range(3)]
    assert T.numel == sum(ga[a] * gb[b] * gc[(a + b) % 3] for a in range(3) for b in range(3)) == 62


@pytest.mark.parametrize("seed", range(5))
def test_product_symmetry_is_the_intersection(seed):
    rng = np.random.default_rng(100 + seed)
    A, _ = _random_sym_pair(rng, int(rng.integers(1, 5)), 1, 0, (0, 2))
    U = orc.BlockTensor(A.labels, [(d, [(q[0], g) for q, g in s]) for d, s in A.legs])
    Z = orc.BlockTensor(A.labels, [(d, [(q[1], g) for q, g in s]) for d, s in A.legs], sym=(2,))
    assert A.blocks == sorted(set(U.blocks) & set(Z.blocks))


@pytest.mark.parametrize("sym", [(2,), (3,), (4,), (0, 2), (0, 3), (2, 2)])
def test_symmetric_contraction_equals_einsum(sym):
    rng = np.random.default_rng(7 + len(sym) * 10 + sym[-1])
    for _ in range(12):
        ra, rb = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        nc = min(int(rng.integers(0, 4)), ra, rb)
        A, B = _random_sym_pair(rng, ra, rb, nc, sym)
        C = orc.contract(A, B)
        assert C.sym == tuple(sym)
        dense = _einsum_reference(A, B)
        got = orc.embed(C)
        assert np.allclose(got, dense, rtol=1e-13, atol=1e-13 * max(1.0, np.abs(dense).max(initial=0)))
        # symmetry-violating entries of the dense product are exactly zero
        mask = np.ones(dense.shape, dtype=bool)
        so = C.sector_offsets()
        for b, t in enumerate(C.blocks):
            mask[tuple(slice(so[i][k], so[i][k] + C.shapes[b][i]) for i, k in enumerate(t))] = False
        assert np.all(dense[mask] == 0.0)


def test_zn_combine_rule():
    z = (1, [(0, 1), (1, 1), (2, 1)])
    assert orc.combine_bonds(z, z, sym=(3,)) == (1, [(0, 3), (1, 3), (2, 3)])
    # U(1) x Z_2: components combine separately
    a = (1, [((0, 1), 1), ((1, 0), 2)])
    b = (1, [((1, 1), 1)])
    assert orc.combine_bonds(a, b, sym=(0, 2)) == (1, [((1, 0), 1), ((2, 1), 2)])


def test_symmetry_errors():
    with pytest.raises(orc.QnumError):
        orc.BlockTensor(["a"], [(1, [(3, 1)])], sym=(3,))
    with pytest.raises(orc.OracleError):
        orc.BlockTensor(["a"], [(1, [(0, 1)])], sym=(1,))
    A = orc.BlockTensor(["a", "x"], [(1, [(0, 1), (1, 1)]), (-1, [(0, 1), (1, 1)])], sym=(2,))
    B = orc.BlockTensor(["x", "b"], [(1, [(0, 1), (1, 1)]), (-1, [(0, 1), (1, 1)])], sym=(3,))
    with pytest.raises(orc.QnumError):
        orc.contract(A, B)


def tfim_closed_form(nsites: int, h: float, J: float = 1.0) -> float:
    """Open transverse-field Ising chain (Jordan-Wigner free fermions): the
    ground energy is -1/2 the sum of the singular values of the bidiagonal
    matrix with 2h on the diagonal and 2J above it."""
    T = np.diag([2.0 * h] * nsites) + np.diag([2.0 * J] * (nsites - 1), 1)
    return -0.5 * float(np.linalg.svd(T, compute_uv=False).sum())


@pytest.mark.parametrize("nsites", [2, 3, 4, 6, 8, 9])
@pytest.mark.parametrize("h", [0.3, 1.0, 1.7])
def test_tfim_exact_diagonalisation_closed_form(nsites, h):
    """The even-parity ground energy of the oracle's dense TFIM equals the
    free-fermion closed form."""
    assert abs(orc.tfim_chain_ground(nsites, h, parity=0) - tfim_closed_form(nsites, h)) < 1e-12


@pytest.mark.parametrize("h", [0.0, 0.6])
def test_tfim_mpo_bond_term(h):
    """sum_w W[start, w] (x) W[w, end] is the two-site TFIM Hamiltonian, and
    W conserves Z_2 parity on its grouped legs."""
    from paper_2401_01921_amd import workloads as wl
    W = wl.tfim_mpo_dense(h)
    a, b = wl.tfim_grouped_index(2), wl.tfim_grouped_index(0)
    acc = sum(np.kron(W[a, :, :, w], W[w, :, :, b]) for w in range(3))
    assert np.array_equal(acc, orc.tfim_chain_hamiltonian(2, h))
    orc.from_dense(*wl.tfim_heff_specs([(0, 1)], [(0, 1)])["W1"], W, sym=(2,))


@pytest.mark.parametrize("nsites,h", [(4, 0.5), (6, 1.0), (8, 1.3)])
def test_tfim_heff_with_z2_environments(nsites, h):
    """Z_2-symmetric two-site H_eff with exact environments: its lowest
    eigenvalue (dense, and by the oracle's Lanczos) is the chain's ground
    energy."""
    from tests import chain_env
    from paper_2401_01921_amd import workloads as wl
    Ld, Rd, Wd, specs = chain_env.tfim_chain_heff_dense(nsites, h)
    sym = wl.TFIM_SYM
    L = orc.from_dense(*specs["L"], Ld, sym=sym)
    R = orc.from_dense(*specs["R"], Rd, sym=sym)
    W = orc.from_dense(*specs["W1"], Wd, sym=sym)
    psi = orc.BlockTensor(*specs["psi"], sym=sym)
    n = psi.numel
    H = np.zeros((n, n))
    for i in range(n):
        e = orc.BlockTensor(psi.labels, psi.legs, sym=sym)
        e.data[i] = 1.0
        H[:, i] = orc.heff_apply(L, W, W, R, e).data
    E0 = tfim_closed_form(nsites, h)
    assert np.allclose(H, H.T, atol=1e-13)
    assert abs(np.linalg.eigvalsh(H)[0] - E0) < 1e-10
    mv = lambda v: orc.heff_apply(L, W, W, R, orc.BlockTensor(psi.labels, psi.legs, v, sym=sym)).data
    res = orc.lanczos_ground(mv, np.random.default_rng(nsites).standard_normal(n), n)
    assert abs(res["energy"] - E0) < 1e-10
