"""Network (Sec. "Network"): the library's contraction-order optimizer
(dynamic programming with cost capping) against the matrix-chain closed form
and against the oracle's exhaustive search over every binary tree; network
definitions, explicit orders and the order string; the oracle's network
contraction against one dense einsum of the whole network."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2401_01921_amd import bst
from paper_2401_01921_amd.network import Network, _order_string


def _lib_order(indices, dims):
    net = Network([f"{n}: {', '.join(ix)}" for n, ix in indices.items()] +
                  ["TOUT: " + ", ".join(_open(indices))])
    for n, ix in indices.items():
        legs = [(1, [(0, dims[l])]) for l in ix]
        net.put(n, bst.Tensor([f"x{k}" for k in range(len(ix))], legs), [f"x{k}" for k in range(len(ix))])
    cost = net.optimize()
    return cost, net.order


def _open(indices):
    count = {}
    for ix in indices.values():
        for l in ix:
            count[l] = count.get(l, 0) + 1
    return sorted(l for l, c in count.items() if c == 1)


def _tree_cost(tree, indices, dims):
    """Total cost of a given tree (the sum of its step costs)."""
    count = {}
    for ix in indices.values():
        for l in ix:
            count[l] = count.get(l, 0) + 1

    def run(node):
        if isinstance(node, str):
            return 0, list(indices[node]), [node]
        ca, ia, ga = run(node[0])
        cb, ib, gb = run(node[1])
        group = ga + gb
        inside = {}
        for n in group:
            for l in indices[n]:
                inside[l] = inside.get(l, 0) + 1
        op = [l for l in inside if inside[l] < count[l] or count[l] == 1]
        return ca + cb + orc.network_step_cost(ia, ib, dims), op, group

    return run(tree)[0]


def test_matrix_chain_closed_form():
    """(2x100)(100x3)(3x50): ((M1,M2),M3) costs 2*100*3 + 2*3*50 = 900,
    (M1,(M2,M3)) costs 100*3*50 + 2*100*50 = 25000."""
    idx = {"M1": ["i", "j"], "M2": ["j", "k"], "M3": ["k", "l"]}
    dims = {"i": 2, "j": 100, "k": 3, "l": 50}
    cost, tree = _lib_order(idx, dims)
    assert cost == 900 and _order_string(tree) == "((M1,M2),M3)"
    assert _tree_cost(("M1", ("M2", "M3")), idx, dims) == 25000


def _random_network(rng, n):
    names = [f"T{i}" for i in range(n)]
    indices = {t: [] for t in names}
    dims = {}
    k = 0
    # a spanning chain keeps it connected, then random extra bonds and legs
    for i in range(1, n):
        j = int(rng.integers(0, i))
        l = f"b{k}"; k += 1
        indices[names[i]].append(l); indices[names[j]].append(l)
        dims[l] = int(rng.integers(2, 12))
    for _ in range(int(rng.integers(0, n))):
        a, b = rng.choice(n, 2, replace=False)
        l = f"b{k}"; k += 1
        indices[names[a]].append(l); indices[names[b]].append(l)
        dims[l] = int(rng.integers(2, 12))
    for _ in range(int(rng.integers(0, 3))):
        a = int(rng.integers(0, n))
        l = f"o{k}"; k += 1
        indices[names[a]].append(l)
        dims[l] = int(rng.integers(2, 12))
    return indices, dims


@pytest.mark.parametrize("seed", range(40))
def test_optimizer_matches_exhaustive_search(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    indices, dims = _random_network(rng, n)
    cost, tree = _lib_order(indices, dims)
    ref_cost, _ = orc.network_optimal_bruteforce(indices, dims)
    assert cost == ref_cost
    # the returned tree really costs that much
    assert _tree_cost(tree, indices, dims) == cost


def test_definition_and_order_strings():
    net = Network(["M1: i, j", "M2: j, k", "M3: k, l", "TOUT: i ; l", "ORDER: ((M1,M2),M3)"])
    assert net.names == ["M1", "M2", "M3"] and net.tout == ["i", "l"]
    assert net.get_order() == "((M1,M2),M3)" and not net.optimal
    net.set_order(optimal=False, order="(M2,(M1,M3))")
    assert net.get_order() == "(M2,(M1,M3))"
    with pytest.raises(ValueError):
        Network(["M1: i, j", "M2: j, k", "TOUT: i"])        # k is open too
    with pytest.raises(ValueError):
        Network(["A: i", "B: i", "C: i", "TOUT:"])          # i joins three tensors


def test_optimizer_errors():
    lib = bst.lib()
    import ctypes as C
    nl = (C.c_int32 * 3)(1, 1, 1)
    lg = (C.c_int32 * 3)(0, 0, 0)
    dm = (C.c_int64 * 1)(2)
    assert lib.bst_network_order(3, nl, lg, 1, dm, None, None) != 0   # an index on three tensors
    assert lib.bst_network_order(17, nl, lg, 1, dm, None, None) != 0


@pytest.mark.parametrize("seed", range(6))
def test_oracle_network_contract_equals_einsum(seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(2, 5))
    indices, dims = _random_network(rng, n)
    # U(1) legs: every index gets sectors {-1, 0, 1}; bonds opposite directions
    tensors, dense, letters = {}, {}, {}
    seen = {}
    for l in dims:
        letters[l] = chr(ord("a") + len(letters))
    for t, ix in indices.items():
        legs = []
        for l in ix:
            g = [max(1, dims[l] // 3), max(1, dims[l] // 3), max(1, dims[l] - 2 * max(1, dims[l] // 3))]
            d = 1 if l not in seen else -seen[l]
            seen[l] = d
            legs.append((d, [(-1, g[0]), (0, g[1]), (1, g[2])]))
        T = orc.BlockTensor(ix, legs)
        T.data[:] = rng.standard_normal(T.numel)
        tensors[t] = T
        dense[t] = orc.embed(T)
    out = _open(indices)
    _, tree = orc.network_optimal_bruteforce(indices, {l: dims[l] for l in dims})
    got = orc.network_contract(tensors, tree, out)
    spec = ",".join("".join(letters[l] for l in indices[t]) for t in indices) + "->" + \
        "".join(letters[l] for l in out)
    ref = np.einsum(spec, *[dense[t] for t in indices])
    assert np.allclose(orc.embed(got), ref, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(ref).max(initial=0)))
