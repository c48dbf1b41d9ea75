"""Network contractions on the GPU (Sec. "Network"): the paper's
three-matrix example with ones (closed form), random U(1) networks with the
optimized and with explicit orders, and a DMRG left-environment update
L'[b, w', b'] = L[a, w, a'] A[a', s', b'] W[w, s, s', w'] Abar[a, s, b] as a
four-tensor network, each against the oracle."""
import numpy as np
import pytest

from tests.gpu_common import DEV, TOL, check, dev, host, rel_err, require_gpu, torch
from tests.test_network import _open, _random_network
from oracle import oracle as orc
from paper_2401_01921_amd import bst, workloads as wl
from paper_2401_01921_amd.network import Network

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _print(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("order", ["((M1,M2),M3)", "(M2,(M1,M3))", None])
def test_paper_example_three_ones_matrices(order):
    """Three 2x2 ones matrices, every one labelled (a, b): M1 M2 M3 = 4 ones."""
    legs = [(1, [(0, 2)]), (-1, [(0, 2)])]
    T = bst.Tensor(["a", "b"], legs)
    net = Network(["M1: i, j", "M2: j, k", "M3: k, l", "TOUT: i ; l"])
    for n in ("M1", "M2", "M3"):
        net.put(n, T, ["a", "b"])
    if order is not None:
        net.set_order(optimal=False, order=order)
    ones = torch.ones(4, dtype=torch.float64, device=DEV)
    out_t, out = net.launch({"M1": ones, "M2": ones, "M3": ones})
    torch.cuda.synchronize()
    assert out_t.labels == ["i", "l"]
    assert np.array_equal(host(out), np.full(4, 4.0))
    if order is not None:
        assert net.get_order() == order


def _u1_network(rng, n):
    indices, dims = _random_network(rng, n)
    seen, tensors = {}, {}
    for t, ix in indices.items():
        legs = []
        for l in ix:
            g1 = max(1, dims[l] // 3)
            g = [g1, g1, max(1, dims[l] - 2 * g1)]
            d = 1 if l not in seen else -seen[l]
            seen[l] = d
            legs.append((d, [(-1, 3 * g[0]), (0, 3 * g[1]), (1, 3 * g[2])]))
        T = orc.BlockTensor(ix, legs)
        T.data[:] = rng.standard_normal(T.numel)
        tensors[t] = T
    return indices, tensors


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_random_u1_networks(prec):
    rng = np.random.default_rng(11)
    for case in range(8):
        n = int(rng.integers(2, 6))
        indices, O = _u1_network(rng, n)
        out_labels = _open(indices)
        net = Network([f"{k}: {', '.join(ix)}" for k, ix in indices.items()] +
                      ["TOUT: " + ", ".join(out_labels)])
        for k, T in O.items():
            # the loaded tensor has labels of its own: x0, x1, ...
            own = [f"x{i}" for i in range(T.rank)]
            net.put(k, bst.Tensor(own, T.legs), own)
        bufs = {k: dev(T.data) for k, T in O.items()}
        for explicit in (False, True):
            if explicit:   # the optimizer's tree, mirrored at the root
                t = net.order
                net.set_order(optimal=False, order=net.get_order() if isinstance(t, str) else
                              f"({_s(t[1])},{_s(t[0])})")
            out_t, out = net.launch(bufs, prec)
            torch.cuda.synchronize()
            ref = orc.network_contract(O, net.order, out_labels)
            assert out_t.labels == out_labels and out_t.numel == ref.numel
            if ref.numel == 0:
                continue
            check(host(out), ref.data, prec, f"network {case} {net.get_order()}",
                  steps=max(1, len(O) - 1))


def _s(t):
    return t if isinstance(t, str) else f"({_s(t[0])},{_s(t[1])})"


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_environment_update_network(prec):
    """Left-environment update of a two-site DMRG step, spin 1/2, chi 128 -> 96."""
    va = wl.gaussian_sector_dims(128, 6)
    vb = wl.gaussian_sector_dims(96, 6)
    ph = wl.physical_sectors("1/2")
    L = orc.BlockTensor(*wl.heff_specs("1/2", va, va)["L"])           # a IN, w OUT, a' OUT
    W = orc.from_dense(*wl.heff_specs("1/2", va, va)["W1"], wl.heisenberg_mpo_dense("1/2"))
    A = orc.BlockTensor(["a", "s", "b"], [(1, va), (1, ph), (-1, vb)])
    Ab = orc.BlockTensor(["a", "s", "b"], [(-1, va), (-1, ph), (1, vb)])
    rng = np.random.default_rng(3)
    for T in (L, A, Ab):
        T.data[:] = rng.standard_normal(T.numel)
    net = Network(["L: a, w, ap", "A: ap, sp, bp", "W: w, s, sp, wp", "Abar: a, s, b",
                   "TOUT: b, wp, bp"])
    tens = {"L": (L, ["a", "w", "ap"]), "A": (A, ["a", "s", "b"]),
            "W": (W, ["wl", "s", "sp", "wr"]), "Abar": (Ab, ["a", "s", "b"])}
    for k, (T, own) in tens.items():
        net.put(k, bst.Tensor(T.labels, T.legs), own)
    cost = net.optimize()
    out_t, out = net.launch({k: dev(T.data) for k, (T, _) in tens.items()}, prec)
    torch.cuda.synchronize()
    named = {"L": orc.relabel(L, ["a", "w", "ap"]), "A": orc.relabel(A, ["ap", "sp", "bp"]),
             "W": orc.relabel(W, ["w", "s", "sp", "wp"]), "Abar": orc.relabel(Ab, ["a", "s", "b"])}
    ref = orc.network_contract(named, net.order, ["b", "wp", "bp"])
    assert out_t.labels == ["b", "wp", "bp"]
    check(host(out), ref.data, prec, f"env update {net.get_order()} {cost} {ref.numel}", steps=3)
