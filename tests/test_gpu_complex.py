"""GPU parity of complex128 tensors through the C ABI: permute bit for bit
and contraction against the oracle's complex contraction in every form
(Sec. "Creating a non-symmetric UniTensor", paragraph "Complex elements
and data types"), and a statevector simulation of a Trotterised
transverse-field Ising circuit with a longitudinal field (App. "Quantum
Circuit Simulation": J = h_x = 1, h_z = 3, dt = 0.1) against a dense
numpy statevector run of the same gates."""
import numpy as np
import pytest

from tests.gpu_common import DEV, TOL, TOL_MAX, host, rel_err, require_gpu, torch
from tests.helpers import _random_sym_pair
from oracle import oracle as orc
from paper_2401_01921_amd import bst

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def cdev(x: np.ndarray):
    """A complex host array as the interleaved float64 device buffer."""
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to(DEV)
    return torch.view_as_real(t).reshape(-1)


def chost(t) -> np.ndarray:
    a = host(t).reshape(-1, 2)
    return a[:, 0] + 1j * a[:, 1]


def _sym(O):
    return None if O.sym == orc.U1 else list(O.sym)


def _complexify(T, rng):
    return orc.BlockTensor(T.labels, T.legs, rng.standard_normal(T.numel) + 1j * rng.standard_normal(T.numel),
                           sym=T.sym)


@pytest.mark.parametrize("sym", [(0,), (3,), (0, 2)])
def test_complex_permute_bit_exact(sym):
    rng = np.random.default_rng(3 + sum(sym))
    for case in range(10):
        A, _ = _random_sym_pair(rng, int(rng.integers(1, 6)), 1, 0, sym, dmax=9)
        if A.numel == 0:
            continue
        A = _complexify(A, rng)
        order = [A.labels[i] for i in rng.permutation(A.rank)]
        P = orc.permute(A, order)
        T = bst.Tensor(A.labels, A.legs, sym=_sym(A))
        out_t, plan = bst.permute_plan(T, order, dtype="c128")
        y = torch.full((2 * out_t.numel,), np.nan, dtype=torch.float64, device=DEV)
        plan.execute([cdev(A.data)], [y], bst.workspace(plan.workspace_bytes))
        torch.cuda.synchronize()
        assert out_t.table() == [(tuple(t), tuple(s), o) for t, s, o in P.table()]
        assert np.array_equal(chost(y), P.data)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("sym", [(0,), (2,), (0, 2)])
def test_complex_contractions(sym, prec):
    rng = np.random.default_rng(40 + sum(sym) + 3 * len(sym))
    done = 0
    for case in range(60):
        ra, rb = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        nc = min(int(rng.integers(0, 4)), ra, rb)
        if ra + rb - 2 * nc > 7:   # the complex output is limited to rank 7
            continue
        A, B = _random_sym_pair(rng, ra, rb, nc, sym, dmax=7)
        free = [i for i, l in enumerate(A.labels) if l not in B.labels]
        if free:
            scale = int(rng.integers(1, 12))
            A = orc.BlockTensor(A.labels, [(d, [(q, g * scale if i == free[0] else g) for q, g in s])
                                           for i, (d, s) in enumerate(A.legs)], sym=sym)
        if A.numel == 0 or B.numel == 0:
            continue
        drng = np.random.default_rng(1000 + case)
        A, B = _complexify(A, drng), _complexify(B, drng)
        C = orc.contract(A, B)
        tA, tB = bst.Tensor(A.labels, A.legs, sym=_sym(A)), bst.Tensor(B.labels, B.legs, sym=_sym(B))
        tC, plan = bst.contract_plan(tA, tB, prec, dtype="c128")
        assert tC.table() == [(tuple(t), tuple(s), o) for t, s, o in C.table()]
        out = torch.full((2 * tC.numel,), np.nan, dtype=torch.float64, device=DEV)
        plan.execute([cdev(A.data), cdev(B.data)], [out], bst.workspace(plan.workspace_bytes))
        torch.cuda.synchronize()
        got = chost(out)
        if C.numel == 0:
            continue
        nrm, mx = rel_err(got, C.data)
        print("complex", sym, prec, case, A.labels, B.labels, "normwise", nrm, "max", mx, flush=True)
        assert nrm <= TOL[prec] and mx <= TOL_MAX[prec], (nrm, mx)
        done += 1
    assert done >= 5


def _tfim_gate(J=1.0, hx=1.0, hz=3.0, dt=0.1):
    """exp(-i dt h) of the two-site term of the appendix's Hamiltonian,
    as G[out1, out2, in1, in2] (host input, built with scipy)."""
    from scipy.linalg import expm
    sz = np.diag([1.0, -1.0])
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    I = np.eye(2)
    h = J * np.kron(sz, sz) + 0.5 * hz * (np.kron(sz, I) + np.kron(I, sz)) + \
        0.5 * hx * (np.kron(sx, I) + np.kron(I, sx))
    return expm(-1j * dt * h).reshape(2, 2, 2, 2)


def test_trotter_circuit_statevector():
    """Brickwork Trotter steps of the appendix's TFIM on its 11 qubits from
    |up up down x7 up up>: the state is a rank-4 tensor [left, q_i, q_i+1,
    right] (no symmetry, so grouping qubits is free), each gate a complex
    contraction with the state followed by a permute back, all on the GPU;
    the state and <sigma^z> of the centre qubit (site 6) equal a dense numpy
    run of the same gates."""
    n, steps = 11, 4
    G = _tfim_gate()
    init = [0, 0, 1, 1, 1, 1, 1, 1, 1, 0, 0]     # up up down ... down up up (0 = up)
    psi0 = np.zeros([2] * n, dtype=complex)
    psi0[tuple(init)] = 1.0
    x = cdev(psi0.ravel())
    dense = psi0.copy()
    tg = bst.Tensor(["o1", "o2", "a", "b"], [(1, [(0, 2)]), (1, [(0, 2)]), (-1, [(0, 2)]), (-1, [(0, 2)])])
    gdev = cdev(G.ravel())
    for step in range(steps):
        for start in (0, 1):
            for i in range(start, n - 1, 2):
                dl, dr = 2 ** i, 2 ** (n - i - 2)
                ts = bst.Tensor(["l", "a", "b", "r"], [(1, [(0, dl)]), (1, [(0, 2)]), (1, [(0, 2)]), (1, [(0, dr)])])
                tc, plan = bst.contract_plan(ts, tg, "fp64", dtype="c128")     # l, r, o1, o2
                y = torch.empty(2 * tc.numel, dtype=torch.float64, device=DEV)
                plan.execute([x, gdev], [y], bst.workspace(plan.workspace_bytes))
                tp, pplan = bst.permute_plan(tc, ["l", "o1", "o2", "r"], dtype="c128")
                z = torch.empty_like(y)
                pplan.execute([y], [z], bst.workspace(pplan.workspace_bytes))
                x = z
                dense = np.moveaxis(np.tensordot(G, dense, axes=([2, 3], [i, i + 1])), [0, 1], [i, i + 1])
    torch.cuda.synchronize()
    got = chost(x).reshape([2] * n)
    assert np.max(np.abs(got - dense)) <= 1e-13
    assert abs(np.linalg.norm(got) - 1.0) <= 1e-12
    w = np.array([1.0, -1.0]).reshape([2 if k == n // 2 else 1 for k in range(n)])
    mz, mz_d = float(np.sum(np.abs(got) ** 2 * w)), float(np.sum(np.abs(dense) ** 2 * w))
    print("trotter <sz_6>", mz, mz_d, flush=True)
    assert abs(mz - mz_d) <= 1e-13
