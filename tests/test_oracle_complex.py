"""Pins of the oracle's complex128 tensors (Sec. "Creating a non-symmetric
UniTensor", paragraph "Complex elements and data types"): contraction
against the dense einsum of the complex embeddings, against the four real
contractions of the real and imaginary parts, norm preservation by a
unitary, and permute against numpy's transpose, bitwise."""
import numpy as np
import pytest

from oracle import oracle as orc
from tests.helpers import _random_sym_pair


def _complexify(T, rng):
    return orc.BlockTensor(T.labels, T.legs, rng.standard_normal(T.numel) + 1j * rng.standard_normal(T.numel),
                           sym=T.sym)


def _pairs():
    rng = np.random.default_rng(77)
    out = []
    for sym in [(0,), (3,), (0, 2)]:
        for case in range(8):
            ra, rb = int(rng.integers(1, 5)), int(rng.integers(1, 5))
            nc = min(int(rng.integers(0, 4)), ra, rb)
            A, B = _random_sym_pair(rng, ra, rb, nc, sym, dmax=4)
            out.append((_complexify(A, rng), _complexify(B, rng)))
    return out


def _einsum(A, B):
    letters = "abcdefghijklmnopqrstuvwxyz"
    labs = {l: letters[i] for i, l in enumerate(dict.fromkeys(A.labels + B.labels))}
    out = [l for l in A.labels if l not in B.labels] + [l for l in B.labels if l not in A.labels]
    spec = "".join(labs[l] for l in A.labels) + "," + "".join(labs[l] for l in B.labels) + "->" + \
        "".join(labs[l] for l in out)
    return np.einsum(spec, orc.embed(A), orc.embed(B))


@pytest.mark.parametrize("k", range(24))
def test_complex_contract_equals_dense_einsum(k):
    A, B = _pairs()[k]
    C = orc.contract(A, B)
    assert C.data.dtype == np.complex128
    ref = _einsum(A, B)
    assert np.allclose(orc.embed(C), ref, rtol=0, atol=1e-12 * max(1.0, np.max(np.abs(ref), initial=0)))


def test_complex_contract_equals_real_parts():
    for A, B in _pairs():
        def part(T, f):
            return orc.BlockTensor(T.labels, T.legs, f(T.data).copy(), sym=T.sym)
        Ar, Ai, Br, Bi = part(A, np.real), part(A, np.imag), part(B, np.real), part(B, np.imag)
        C = orc.contract(A, B)
        re = orc.contract(Ar, Br).data - orc.contract(Ai, Bi).data
        im = orc.contract(Ar, Bi).data + orc.contract(Ai, Br).data
        assert np.allclose(C.data, re + 1j * im, atol=1e-12)


def test_unitary_preserves_norm():
    rng = np.random.default_rng(5)
    psi = orc.BlockTensor(["a", "s", "b"], [(1, [(0, 3), (1, 4)]), (1, [(0, 5), (1, 2)]), (-1, [(1, 6), (2, 3)])])
    psi.data[:] = 0
    psi = _complexify(psi, rng)
    z = rng.standard_normal((7, 7)) + 1j * rng.standard_normal((7, 7))
    # U[t, s] acting on leg s: block diagonal in the charge of s
    legs = [(1, [(0, 5), (1, 2)]), (-1, [(0, 5), (1, 2)])]
    U = orc.BlockTensor(["t", "s"], legs, dtype=np.complex128)
    qb = np.zeros((7, 7), dtype=complex)
    qb[:5, :5] = np.linalg.qr(z[:5, :5])[0]
    qb[5:, 5:] = np.linalg.qr(z[5:, 5:])[0]
    U.block(0)[...] = qb[:5, :5]
    U.block(1)[...] = qb[5:, 5:]
    out = orc.contract(U, psi)
    assert abs(np.linalg.norm(out.data) - np.linalg.norm(psi.data)) <= 1e-12 * np.linalg.norm(psi.data)


def test_complex_permute_equals_transpose():
    for A, _ in _pairs():
        order = list(reversed(A.labels))
        P = orc.permute(A, order)
        perm = [A.labels.index(l) for l in order]
        assert np.array_equal(orc.embed(P), np.transpose(orc.embed(A), perm))
