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
