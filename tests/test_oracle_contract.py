"""Pins of the oracle's contraction: closed forms of the paper's ones-tensor
examples, brute-force einsum of dense embeddings, exact zeros outside valid
blocks, the legality checks, and the paper's two-site operator built densely
and from charge-carrying symmetric pieces."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import oracle as orc
from paper_2401_01921_amd import workloads as wl
from tests.test_oracle_structure import _paper_examples
from tests.helpers import _random_pair, _einsum_reference


def dense_leg(n):
    return (orc.IN, [(0, n)])


def dense_out(n):
    return (orc.OUT, [(0, n)])


def ones(labels, legs):
    T = orc.BlockTensor(labels, legs)
    T.data[:] = 1.0
    return T


def test_ones_closed_forms():
    ex = _paper_examples()
    # Sec. "Sneak preview": A(alpha,beta,gamma) B(beta,delta) C(gamma), all ones, dims 2
    A = ones(["alpha", "beta", "gamma"], [dense_leg(2), dense_out(2), dense_out(2)])
    B = ones(["beta", "delta"], [dense_leg(2), dense_out(2)])
    C = ones(["gamma"], [dense_leg(2)])
    D = orc.contract(orc.contract(A, B), C)
    assert D.labels == ["alpha", "delta"]
    assert np.all(D.data == float(ex["ones_chain_value"]))
    # Sec. "Tensor contraction": A[2,3,5](i,j,l) . B[3,1,5,4](j,k,l,m)
    A = ones(["i", "j", "l"], [dense_leg(2), dense_out(3), dense_out(5)])
    B = ones(["j", "k", "l", "m"], [dense_leg(3), dense_out(1), dense_leg(5), dense_out(4)])
    AB = orc.contract(A, B)
    assert AB.labels == ex["contract_ones_labels"].split()
    assert list(AB.shapes[0]) == [int(v) for v in ex["contract_ones_shape"].split()]
    assert np.all(AB.data == float(ex["contract_ones_value"]))
    # Sec. "Network": matmul of 2x2 ones
    M1 = ones(["i", "j"], [dense_leg(2), dense_out(2)])
    M2 = ones(["j", "k"], [dense_leg(2), dense_out(2)])
    assert np.all(orc.contract(M1, M2).data == float(ex["network_matmul_value"]))


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 10_000), st.integers(1, 4), st.integers(1, 4), st.integers(0, 3))
def test_contract_matches_dense_einsum(seed, ra, rb, nc):
    nc = min(nc, ra, rb)
    rng = np.random.default_rng(seed)
    A, B = _random_pair(rng, ra, rb, nc)
    C = orc.contract(A, B)
    ref = _einsum_reference(A, B)
    dense = orc.embed(C)
    scale = max(1.0, float(np.max(np.abs(ref))) if ref.size else 1.0)
    assert np.max(np.abs(dense - ref), initial=0.0) <= 1e-13 * scale
    # charge conservation: the reference is exactly zero outside valid blocks
    mask = np.zeros(dense.shape, dtype=bool)
    so = C.sector_offsets()
    for b, t in enumerate(C.blocks):
        sl = tuple(slice(so[i][k], so[i][k] + C.shapes[b][i]) for i, k in enumerate(t))
        mask[sl] = True
    assert np.all(ref[~mask] == 0.0)


def test_pairwise_workload_counts():
    """Pairwise workload: A has 8 blocks / 392 elements, the result has all 16
    zero-flux blocks (718 elements), 2 of which receive no contribution."""
    specs = wl.pairwise_specs()
    A = orc.BlockTensor(*specs["A"])
    B = orc.BlockTensor(*specs["B"])
    A.data[:] = wl.normal(wl.seed_for(1, "A"), A.numel)
    B.data[:] = wl.normal(wl.seed_for(1, "B"), B.numel)
    C = orc.contract(A, B)
    assert (len(A.blocks), A.numel) == (8, 392)
    assert (len(C.blocks), C.numel) == (16, 718)
    zero_blocks = sum(1 for b in range(len(C.blocks)) if not np.any(C.block(b)))
    assert zero_blocks == 2
    assert C.labels == ["l", "s", "t", "r"]
    ref = _einsum_reference(A, B)
    assert np.max(np.abs(orc.embed(C) - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_legality_checks():
    a = (orc.IN, [(0, 2), (1, 3)])
    A = orc.BlockTensor(["x", "y"], [a, (orc.OUT, [(0, 2), (1, 3)])])
    same_dir = orc.BlockTensor(["y", "z"], [(orc.OUT, [(0, 2), (1, 3)]), (orc.OUT, [(0, 2)])])
    with pytest.raises(orc.DirectionError):
        orc.contract(A, same_dir)
    bad_q = orc.BlockTensor(["y", "z"], [(orc.IN, [(0, 2), (2, 3)]), (orc.OUT, [(0, 2)])])
    with pytest.raises(orc.QnumError):
        orc.contract(A, bad_q)
    bad_g = orc.BlockTensor(["y", "z"], [(orc.IN, [(0, 2), (1, 4)]), (orc.OUT, [(0, 2)])])
    with pytest.raises(orc.DimError):
        orc.contract(A, bad_g)
    reordered = orc.BlockTensor(["y", "z"], [(orc.IN, [(1, 3), (0, 2)]), (orc.OUT, [(0, 2)])])
    with pytest.raises(orc.QnumError):
        orc.contract(A, reordered)


def test_two_site_operator_dense_equals_symmetric():
    """Sec. "Conversion between UniTensor with and without symmetries": the
    two-site operator s+s- + s-s+ + szsz built from symmetric pieces with a
    charge-carrying dim-1 bond equals the dense Kronecker construction."""
    sp = np.array([[0.0, 1.0], [0.0, 0.0]])
    sm = sp.T
    sz = np.diag([1.0, -1.0])
    H = np.kron(sp, sm) + np.kron(sm, sp) + np.kron(sz, sz)
    bi = (orc.IN, [(1, 1), (-1, 1)])
    bo = (orc.OUT, [(1, 1), (-1, 1)])
    bqo = (orc.OUT, [(2, 1)])
    bqi = (orc.IN, [(2, 1)])

    def sym(labels, legs, entries):
        T = orc.BlockTensor(labels, legs)
        dense = np.zeros(T.dims())
        for idx, v in entries:
            dense[idx] = v
        return orc.from_dense(labels, legs, dense)

    def term(op1, op2):
        return orc.permute(orc.contract(op1, op2), ["i1", "i2", "j1", "j2"])

    Sp1 = sym(["i1", "j1", "q"], [bi, bo, bqo], [((0, 1, 0), 1.0)])
    Sp2 = sym(["i2", "j2", "q"], [bi, bo, bqo], [((0, 1, 0), 1.0)])
    Sm1 = sym(["q", "i1", "j1"], [bqi, bi, bo], [((0, 1, 0), 1.0)])
    Sm2 = sym(["q", "i2", "j2"], [bqi, bi, bo], [((0, 1, 0), 1.0)])
    Sz1 = sym(["i1", "j1"], [bi, bo], [((0, 0), 1.0), ((1, 1), -1.0)])
    Sz2 = sym(["i2", "j2"], [bi, bo], [((0, 0), 1.0), ((1, 1), -1.0)])
    t1, t2, t3 = term(Sp1, Sm2), term(Sm1, Sp2), term(Sz1, Sz2)
    assert t1.blocks == t2.blocks == t3.blocks
    total = orc.BlockTensor(t1.labels, t1.legs, t1.data + t2.data + t3.data)
    assert np.array_equal(orc.embed(total).reshape(4, 4), H)


def test_planted_mistake_is_caught():
    """A contraction that drops the transpose of B (a plausible slip) must fail
    the dense pin; the pin is not vacuous."""
    rng = np.random.default_rng(5)
    v = [(-1, 2), (0, 3), (1, 2)]
    A = orc.BlockTensor(["x", "c0", "c1"], [(orc.IN, v), (orc.OUT, v), (orc.IN, v)])
    B = orc.BlockTensor(["y", "c1", "c0"], [(orc.IN, v), (orc.OUT, v), (orc.IN, v)])
    A.data[:] = rng.standard_normal(A.numel)
    B.data[:] = rng.standard_normal(B.numel)

    def broken_contract(A, B):
        C = orc.BlockTensor(*orc._contract_meta(A, B))
        ac, bc = [1, 2], [2, 1]
        for a, ta in enumerate(A.blocks):
            for b, tb in enumerate(B.blocks):
                if (ta[1], ta[2]) != (tb[2], tb[1]):
                    continue
                am = A.block(a).reshape(A.shapes[a][0], -1)
                bm = B.block(b).reshape(-1, B.shapes[b][0])  # transpose of B forgotten
                cb = C.index[(ta[0], tb[0])]
                C.block(cb)[...] += am @ bm
        return C

    ref = _einsum_reference(A, B)
    good = orc.embed(orc.contract(A, B))
    bad = orc.embed(broken_contract(A, B))
    assert np.allclose(good, ref, atol=1e-13)
    assert not np.allclose(bad, ref, atol=1e-6)
