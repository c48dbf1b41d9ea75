"""Pins of the oracle's block structure, permute and bond combination against
what the paper prints and against brute force."""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as orc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper_examples():
    vals = {}
    with open(os.path.join(GOLD, "paper_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    return vals


def _parse_bond(tok):
    d = orc.IN if tok[0] == "IN" else orc.OUT
    secs = []
    for s in tok[1:]:
        q, g = s.split(":")
        secs.append((int(q), int(g)))
    return (d, secs)


def test_block_order_matches_paper_listing():
    """Sec. "Symmetric UniTensor": 4 valid blocks, in the printed order."""
    legs, labels, blocks, exists = [], [], [], []
    with open(os.path.join(GOLD, "symm_tensor_blocks.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "bond":
                labels.append(t[1])
                legs.append(_parse_bond(t[2:]))
            elif t[0] == "block":
                blocks.append((int(t[1]), tuple(map(int, t[3].split(","))), tuple(map(int, t[5].split(",")))))
            elif t[0] == "exists":
                exists.append((tuple(map(int, t[1].split(","))), t[2] == "true"))
    T = orc.BlockTensor(labels, legs)
    assert len(T.blocks) == len(blocks) == 4
    for b, qn, shape in blocks:
        assert T.blocks[b] == qn
        assert T.shapes[b] == shape
        assert T.find_block(qn) == b
    for el, ex in exists:
        assert T.exists(el) == ex
    with pytest.raises(orc.NoBlockError):
        T.find_block((0, 0, 1))


def test_flux_rule_brute_force():
    """Every element of a valid block has zero flux and every zero-flux element
    is inside a valid block (brute force over the dense index space)."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        rank = int(rng.integers(1, 5))
        legs = []
        for _ in range(rank):
            ns = int(rng.integers(1, 4))
            qs = sorted(rng.choice(np.arange(-3, 4), ns, replace=False).tolist())
            legs.append((int(rng.choice([1, -1])), [(q, int(rng.integers(1, 3))) for q in qs]))
        T = orc.BlockTensor([f"l{i}" for i in range(rank)], legs)
        charges = [[q for q, g in secs for _ in range(g)] for _, secs in legs]
        for el in itertools.product(*[range(len(c)) for c in charges]):
            flux = sum(d * charges[i][e] for i, ((d, _), e) in enumerate(zip(legs, el)))
            assert T.exists(el) == (flux == 0)
        assert T.numel == sum(int(np.prod(s)) for s in T.shapes)
        # blocks sorted lexicographically, offsets contiguous
        assert T.blocks == sorted(T.blocks)


def test_combine_bonds_matches_paper():
    ex = _paper_examples()
    b = orc.combine_bonds((orc.IN, [(0, 1), (1, 1)]), (orc.IN, [(2, 1), (3, 1)]))
    want = [(int(s.split(":")[0]), int(s.split(":")[1])) for s in ex["combine_bonds"].split()]
    assert b == (orc.IN, want)
    ug = orc.combine_bonds((orc.IN, [(0, 1), (1, 1)]), (orc.IN, [(2, 1), (3, 1)]), grouped=False)
    assert ug[1] == [(2, 1), (3, 1), (3, 1), (4, 1)]


def test_permute_storage_matches_paper():
    ex = _paper_examples()
    legs = [(orc.IN, [(0, 2)]), (orc.IN, [(0, 2)]), (orc.OUT, [(0, 2)])]
    T = orc.BlockTensor(["x", "y", "z"], legs, np.arange(8.0))
    P = orc.permute(T, [0, 2, 1])
    assert P.data.tolist() == [float(v) for v in ex["permute_storage"].split()]


def test_permute_labels_and_shapes_match_paper():
    ex = _paper_examples()
    legs = [(orc.IN, [(0, 2)]), (orc.IN, [(0, 3)]), (orc.OUT, [(0, 4)])]
    T = orc.BlockTensor(["a", "b", "c"], legs, np.arange(24.0))
    P = orc.permute(T, ["b", "c", "a"])
    assert P.labels == ["b", "c", "a"]
    assert list(P.shapes[0]) == [int(v) for v in ex["permute_labels_bca_shape"].split()]
    Q = orc.permute(T, [2, 0, 1])
    assert Q.labels == ex["permute_201_labels"].split()
    assert list(Q.shapes[0]) == [int(v) for v in ex["permute_201_shape"].split()]


def test_permute_is_transpose_of_embedding_bitwise():
    rng = np.random.default_rng(1)
    for _ in range(30):
        rank = int(rng.integers(2, 6))
        legs = []
        for _ in range(rank):
            ns = int(rng.integers(1, 4))
            qs = sorted(rng.choice(np.arange(-2, 3), ns, replace=False).tolist())
            legs.append((int(rng.choice([1, -1])), [(q, int(rng.integers(1, 4))) for q in qs]))
        T = orc.BlockTensor([f"l{i}" for i in range(rank)], legs)
        T.data[:] = rng.standard_normal(T.numel)
        perm = [int(p) for p in rng.permutation(rank)]
        P = orc.permute(T, perm)
        assert np.array_equal(orc.embed(P), np.transpose(orc.embed(T), perm))
        inv = [perm.index(i) for i in range(rank)]
        assert np.array_equal(orc.permute(P, inv).data, T.data)


def test_dense_round_trip_and_force():
    legs = [(orc.IN, [(1, 1), (-1, 1)]), (orc.IN, [(1, 1), (-1, 1)]), (orc.OUT, [(2, 1), (0, 2), (-2, 1)])]
    T = orc.BlockTensor(["a", "b", "c"], legs, np.arange(1.0, 7.0))
    D = orc.embed(T)
    assert np.count_nonzero(D) == 6
    T2 = orc.from_dense(["a", "b", "c"], legs, D)
    assert np.array_equal(T2.data, T.data)
    D[0, 0, 1] = 5.0  # a symmetry-violating element
    with pytest.raises(orc.StructureError):
        orc.from_dense(["a", "b", "c"], legs, D)
    T3 = orc.from_dense(["a", "b", "c"], legs, D, force=True)
    assert np.array_equal(T3.data, T.data)


def test_invalid_inputs_raise():
    with pytest.raises(orc.OracleError):
        orc.BlockTensor(["a"], [(orc.IN, [(0, 0)])])
    with pytest.raises(orc.LabelError):
        orc.BlockTensor(["a", "a"], [(orc.IN, [(0, 1)]), (orc.OUT, [(0, 1)])])
    T = orc.BlockTensor(["a", "b"], [(orc.IN, [(0, 2)]), (orc.OUT, [(1, 2)])])
    assert T.numel == 0 and T.blocks == []
