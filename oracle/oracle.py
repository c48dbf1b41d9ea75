"""Plain FP64 CPU oracle for U(1) block-sparse contraction and H_eff.psi.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never
does, and this module imports nothing from the library.

It is written to be read against the paper (arXiv:2401.01921, "The Cytnx
Library for Tensor Networks"):

* U(1), Z_n and product symmetries .... Sec. "Symmetry and quantum numbers"
  (combine rules: sum, sum modulo n; reverse rule: negation)
* block structure and zero flux ........ Sec. "UniTensor with Symmetries",
  Sec. "Bond with quantum numbers", Sec. "Symmetric UniTensor" (the printed
  block list of the rank-3 example fixes the lexicographic block order)
* row-major data, permute semantics .... Sec. "Permute", App. "Contiguous"
* contraction over common labels ....... Sec. "Tensor contraction" (checks of
  direction, quantum numbers and per-sector dims)
* combining bonds ...................... Sec. "Combining bonds with quantum
  numbers" (equal charges grouped, ascending)
* dense <-> symmetric conversion ....... Sec. "Conversion between UniTensor
  with and without symmetries"
* H_eff.psi ............................ Sec. "Benchmarks", Fig. Hpsi_fig
  (L, two-site MPO, R, two-site wavefunction)
* Heisenberg and XX chains (dense, for . Sec. "Benchmarks" (the DMRG benchmark
  exact diagonalisation in tests)        is the XX chain)
* network contraction and its optimal . Sec. "Network" (exhaustive search
  order                                  over binary trees, dense cost)
* SVD of a symmetric tensor and its .... Sec. "Singular value decomposition"
  truncation (keepdim, err,              (the printed block values of the
  min_blockdim)                          symmetric example fix the rule)
* two-site DMRG sweep .................. Sec. "Benchmarks" (DMRG of the XX
                                         chain)
* Lanczos on a linear operator ......... Sec. "Eigenvalue decomposition"
  (LinOp + Lanczos; the paper gives no algorithmic detail, so this is the
  textbook method with full classical Gram-Schmidt reorthogonalisation done
  twice, a Sturm-bisection tridiagonal eigensolve and inverse iteration)

Everything is float64 (complex128 where a tensor holds complex elements,
Sec. "Creating a non-symmetric UniTensor", paragraph "Complex elements and
data types").  numpy matmul is used as the per-block product; there is no
blocking, fusion or reordering beyond the definitions.
"""
from __future__ import annotations

import itertools
import math
from typing import Callable, Dict, List, Sequence, Tuple

import numpy as np

IN, OUT = +1, -1


class OracleError(Exception):
    status = "E_INVALID"


class DirectionError(OracleError):
    status = "E_DIRECTION"


class QnumError(OracleError):
    status = "E_QNUM"


class DimError(OracleError):
    status = "E_DIM"


class LabelError(OracleError):
    status = "E_LABEL"


class NoBlockError(OracleError):
    status = "E_NOBLOCK"


class StructureError(OracleError):
    status = "E_STRUCTURE"


Leg = Tuple[int, List[Tuple[int, int]]]


# --------------------------------------------------------------------------
# Structure (Sec. "UniTensor with Symmetries"; block order from the printed
# block list of the rank-3 example in Sec. "Symmetric UniTensor")
# --------------------------------------------------------------------------
def check_legs(legs: Sequence[Leg]) -> None:
    for d, secs in legs:
        if d not in (IN, OUT):
            raise OracleError("direction must be +1 (in) or -1 (out)")
        if len(secs) == 0:
            raise OracleError("a leg needs at least one sector")
        for _, g in secs:
            if g < 1:
                raise OracleError("sector dims must be >= 1")


U1 = (0,)   # the default symmetry list: one U(1)


def _components(q, nsym: int) -> Tuple[int, ...]:
    return tuple(int(c) for c in q) if nsym > 1 else (int(q),)


def valid_blocks(legs: Sequence[Leg], sym: Sequence[int] = U1) -> List[Tuple[int, ...]]:
    """All sector-index tuples whose flux (sum of in charges minus sum of out
    charges) vanishes, in lexicographic order with leg 0 most significant.
    Sec. "Symmetry and quantum numbers": each symmetry combines charges by its
    rule (U(1): the sum; Z_n: the sum modulo n) and reverses those of
    outgoing legs (negation); `sym` lists the moduli, 0 for U(1)."""
    out = []
    for t in itertools.product(*[range(len(secs)) for _, secs in legs]):
        ok = True
        for c, n in enumerate(sym):
            flux = sum(d * _components(secs[k][0], len(sym))[c] for (d, secs), k in zip(legs, t))
            ok = ok and (flux == 0 if n == 0 else flux % n == 0)
        if ok:
            out.append(t)
    return out


class BlockTensor:
    """Labels, legs, canonical block list, and one flat float64 buffer with the
    blocks stored one after another in block order, each row-major."""

    def __init__(self, labels: Sequence[str], legs: Sequence[Leg], data: np.ndarray | None = None,
                 sym: Sequence[int] = U1, dtype=None):
        if len(labels) != len(legs):
            raise LabelError("one label per leg")
        if len(set(labels)) != len(labels):
            raise LabelError("labels must be unique")
        check_legs(legs)
        self.sym = tuple(int(n) for n in sym)
        if not self.sym or any(n < 0 or n == 1 for n in self.sym):
            raise OracleError("a symmetry is U(1) (0) or Z_n with n >= 2")
        ns = len(self.sym)

        def charge(q):
            c = _components(q, ns)
            if len(c) != ns:
                raise OracleError("one charge per symmetry")
            for v, n in zip(c, self.sym):
                if n >= 2 and not 0 <= v < n:
                    raise QnumError("a Z_n charge must lie in [0, n)")
            return c if ns > 1 else c[0]

        self.labels = list(labels)
        self.legs = [(int(d), [(charge(q), int(g)) for q, g in secs]) for d, secs in legs]
        self.blocks = valid_blocks(self.legs, self.sym)
        self.shapes = [tuple(self.legs[i][1][k][1] for i, k in enumerate(t)) for t in self.blocks]
        self.offsets = []
        off = 0
        for sh in self.shapes:
            self.offsets.append(off)
            off += int(np.prod(sh)) if sh else 1
        self.numel = off
        self.index = {t: b for b, t in enumerate(self.blocks)}
        # float64, or complex128 (two float64 per element, as the paper's
        # ComplexDouble UniTensors): given, or taken from complex data
        if dtype is None:
            dtype = np.complex128 if data is not None and np.iscomplexobj(data) else np.float64
        if np.dtype(dtype) not in (np.dtype(np.float64), np.dtype(np.complex128)):
            raise OracleError("element type is float64 or complex128")
        if data is None:
            data = np.zeros(self.numel, dtype=dtype)
        data = np.asarray(data, dtype=dtype)
        if data.shape != (self.numel,):
            raise OracleError("data length does not match the block structure")
        self.data = data

    @property
    def rank(self) -> int:
        return len(self.legs)

    def block(self, b: int) -> np.ndarray:
        sh = self.shapes[b]
        n = int(np.prod(sh))
        return self.data[self.offsets[b]:self.offsets[b] + n].reshape(sh)

    def find_block(self, qn_idx: Sequence[int]) -> int:
        t = tuple(int(k) for k in qn_idx)
        if t not in self.index:
            raise NoBlockError("no valid block with these Qn indices")
        return self.index[t]

    def table(self):
        return [(t, sh, off) for t, sh, off in zip(self.blocks, self.shapes, self.offsets)]

    def sector_offsets(self) -> List[List[int]]:
        """Start of each sector inside the full (dense) range of each leg."""
        return [list(np.cumsum([0] + [g for _, g in secs])[:-1]) for _, secs in self.legs]

    def dims(self) -> List[int]:
        return [sum(g for _, g in secs) for _, secs in self.legs]

    def exists(self, element: Sequence[int]) -> bool:
        """Whether a dense element index lies inside a valid block."""
        t = []
        for (_, secs), e in zip(self.legs, element):
            acc = 0
            for k, (_, g) in enumerate(secs):
                if e < acc + g:
                    t.append(k)
                    break
                acc += g
            else:
                raise IndexError("element index out of range")
        return tuple(t) in self.index


# --------------------------------------------------------------------------
# Dense embedding and extraction (Sec. "Conversion between UniTensor with and
# without symmetries": convert_from, with and without force)
# --------------------------------------------------------------------------
def embed(T: BlockTensor) -> np.ndarray:
    dense = np.zeros(T.dims(), dtype=T.data.dtype)
    so = T.sector_offsets()
    for b, t in enumerate(T.blocks):
        sl = tuple(slice(so[i][k], so[i][k] + T.shapes[b][i]) for i, k in enumerate(t))
        dense[sl] = T.block(b)
    return dense


def from_dense(labels, legs, dense: np.ndarray, force: bool = False,
               sym: Sequence[int] = U1) -> BlockTensor:
    T = BlockTensor(labels, legs, sym=sym)
    dense = np.asarray(dense, dtype=np.float64)
    if list(dense.shape) != T.dims():
        raise DimError("dense shape does not match the bonds")
    so = T.sector_offsets()
    kept = np.zeros(dense.shape, dtype=bool)
    for b, t in enumerate(T.blocks):
        sl = tuple(slice(so[i][k], so[i][k] + T.shapes[b][i]) for i, k in enumerate(t))
        T.block(b)[...] = dense[sl]
        kept[sl] = True
    if not force and np.any(dense[~kept] != 0.0):
        raise StructureError("nonzero elements in symmetry-violating blocks")
    return T


# --------------------------------------------------------------------------
# Combining bonds (Sec. "Combining bonds with quantum numbers")
# --------------------------------------------------------------------------
def combine_bonds(a: Leg, b: Leg, grouped: bool = True, sym: Sequence[int] = U1) -> Leg:
    """Charges combine by each symmetry's rule (U(1): the sum; Z_n: the sum
    modulo n).  Ungrouped: pairs in row-major order (a slow).  Grouped:
    equal charges merged, ascending charge."""
    da, sa = a
    db, sb = b
    if da != db:
        raise DirectionError("combined bonds must have the same direction")
    ns = len(sym)

    def comb(qa, qb):
        c = tuple(x + y if n == 0 else (x + y) % n
                  for x, y, n in zip(_components(qa, ns), _components(qb, ns), sym))
        return c if ns > 1 else c[0]

    pairs = [(comb(qa, qb), ga * gb) for qa, ga in sa for qb, gb in sb]
    if not grouped:
        return (da, pairs)
    acc: Dict[int, int] = {}
    for q, g in pairs:
        acc[q] = acc.get(q, 0) + g
    return (da, sorted(acc.items()))


# --------------------------------------------------------------------------
# Permute (Sec. "Permute": new leg i is the old leg with label order[i];
# App. "Contiguous": data is moved into the new row-major order)
# --------------------------------------------------------------------------
def permute(T: BlockTensor, order: Sequence) -> BlockTensor:
    if all(isinstance(o, (int, np.integer)) for o in order):
        perm = [int(o) for o in order]
    else:
        try:
            perm = [T.labels.index(o) for o in order]
        except ValueError:
            raise LabelError("unknown label in permutation")
    if sorted(perm) != list(range(T.rank)):
        raise LabelError("not a permutation of the legs")
    out = BlockTensor([T.labels[p] for p in perm], [T.legs[p] for p in perm], sym=T.sym, dtype=T.data.dtype)
    for b, t in enumerate(T.blocks):
        nt = tuple(t[p] for p in perm)
        out.block(out.index[nt])[...] = np.transpose(T.block(b), perm)
    return out


# --------------------------------------------------------------------------
# Contract (Sec. "Tensor contraction")
# --------------------------------------------------------------------------
def contract(A: BlockTensor, B: BlockTensor) -> BlockTensor:
    """Sum over all labels common to A and B.

    Each common leg must have opposite directions and the same (charge, dim)
    sector list in the same order.  The result has A's free legs (A order)
    then B's free legs (B order) and holds every zero-flux block, zero-filled
    where nothing contributes.  Output block (fa, fb) is the sum, over the
    contracted sector tuples kc in lexicographic order (A's leg order), of
    A[fa, kc] . B[kc, fb] with the contracted multi-index row-major in A's
    contracted-leg order.
    """
    common = [l for l in A.labels if l in B.labels]
    ac = [A.labels.index(l) for l in common]
    bc = [B.labels.index(l) for l in common]
    if A.sym != B.sym:
        raise QnumError("the tensors carry different symmetries")
    for i, j in zip(ac, bc):
        (da, sa), (db, sb) = A.legs[i], B.legs[j]
        if da == db:
            raise DirectionError(f"leg '{A.labels[i]}' has the same direction on both tensors")
        if [q for q, _ in sa] != [q for q, _ in sb]:
            raise QnumError(f"leg '{A.labels[i]}' has different quantum numbers")
        if [g for _, g in sa] != [g for _, g in sb]:
            raise DimError(f"leg '{A.labels[i]}' has different sector dims")
    af = [i for i in range(A.rank) if i not in ac]
    bf = [j for j in range(B.rank) if j not in bc]
    C = BlockTensor([A.labels[i] for i in af] + [B.labels[j] for j in bf],
                    [A.legs[i] for i in af] + [B.legs[j] for j in bf], sym=A.sym,
                    dtype=np.result_type(A.data, B.data))
    by_kc: Dict[Tuple[int, ...], List[int]] = {}
    for b, t in enumerate(B.blocks):
        by_kc.setdefault(tuple(t[j] for j in bc), []).append(b)
    for a, ta in enumerate(A.blocks):
        kc = tuple(ta[i] for i in ac)
        fa = tuple(ta[i] for i in af)
        ablk = A.block(a)
        m = int(np.prod([ablk.shape[i] for i in af])) if af else 1
        k = int(np.prod([ablk.shape[i] for i in ac])) if ac else 1
        amat = np.transpose(ablk, af + ac).reshape(m, k)
        for b in by_kc.get(kc, []):
            tb = B.blocks[b]
            fb = tuple(tb[j] for j in bf)
            bblk = B.block(b)
            n = int(np.prod([bblk.shape[j] for j in bf])) if bf else 1
            bmat = np.transpose(bblk, bc + bf).reshape(k, n)
            cb = C.index[fa + fb]
            C.block(cb)[...] += (amat @ bmat).reshape(C.shapes[cb])
    return C


# --------------------------------------------------------------------------
# Network (Sec. "Network"): contraction along a binary tree of tensor names,
# and the optimal tree by exhaustive search (every binary tree is tried).
# Cost of one pairwise step: the product of the dims of every index it
# involves, each once.
# --------------------------------------------------------------------------
def network_step_cost(a_idx: Sequence[str], b_idx: Sequence[str], dims: Dict[str, int]) -> int:
    return int(np.prod([dims[l] for l in dict.fromkeys(list(a_idx) + list(b_idx))], dtype=object))


def network_optimal_bruteforce(indices: Dict[str, Sequence[str]], dims: Dict[str, int]):
    """(minimal total cost, tree) over every binary contraction tree of the
    named tensors; indices[name] = its index names, an index on two tensors
    is summed.  Exponential: for small networks only."""
    names = list(indices)
    count: Dict[str, int] = {}
    for n in names:
        for l in indices[n]:
            count[l] = count.get(l, 0) + 1

    def open_indices(group):
        inside: Dict[str, int] = {}
        for n in group:
            for l in indices[n]:
                inside[l] = inside.get(l, 0) + 1
        return [l for l in inside if inside[l] < count[l] or count[l] == 1]

    def best(group):
        if len(group) == 1:
            return 0, group[0]
        first, rest = group[0], group[1:]
        out = None
        # every split into two non-empty parts; the first tensor stays left
        for r in range(len(rest)):
            for right in itertools.combinations(rest, r + 1):
                left = [first] + [n for n in rest if n not in right]
                right = list(right)
                cl, tl = best(left)
                cr, tr = best(right)
                c = cl + cr + network_step_cost(open_indices(left), open_indices(right), dims)
                if out is None or c < out[0]:
                    out = (c, (tl, tr))
        return out

    return best(names)


def network_contract(tensors: Dict[str, BlockTensor], tree, out_labels: Sequence[str]) -> BlockTensor:
    """Contract along `tree` (nested pairs of names) and permute to out_labels."""
    def run(node):
        if isinstance(node, str):
            return tensors[node]
        return contract(run(node[0]), run(node[1]))

    return permute(run(tree), list(out_labels))


# --------------------------------------------------------------------------
# H_eff.psi (Sec. "Benchmarks", Fig. Hpsi_fig), pairwise in the order
# L -> psi -> W1 -> W2 -> R.
# --------------------------------------------------------------------------
def relabel(T: BlockTensor, labels: Sequence[str]) -> BlockTensor:
    return BlockTensor(labels, T.legs, T.data, sym=T.sym, dtype=T.data.dtype)


def heff_apply(L: BlockTensor, W1: BlockTensor, W2: BlockTensor, R: BlockTensor,
               psi: BlockTensor) -> BlockTensor:
    """out[a,s1,s2,b] = sum L[a,w1,a'] psi[a',t1,t2,b'] W1[w1,s1,t1,w2]
    W2[w2,s2,t2,w3] R[b,w3,b'], legs as in the workload specs:
    L[a,w,a'], W[wl,s(ket),s'(bra),wr], R[b,w,b'], psi[a,s1,s2,b]."""
    Lr = relabel(L, ["a", "w1", "x"])
    Pr = relabel(psi, ["x", "t1", "t2", "y"])
    W1r = relabel(W1, ["w1", "s1", "t1", "w2"])
    W2r = relabel(W2, ["w2", "s2", "t2", "w3"])
    Rr = relabel(R, ["b", "w3", "y"])
    T1 = contract(Lr, Pr)        # a, w1, t1, t2, y
    T2 = contract(T1, W1r)       # a, t2, y, s1, w2
    T3 = contract(T2, W2r)       # a, y, s1, s2, w3
    out = contract(T3, Rr)       # a, s1, s2, b
    out = permute(out, ["a", "s1", "s2", "b"])
    return relabel(out, psi.labels)


def heff_flops(L: BlockTensor, W1: BlockTensor, W2: BlockTensor, R: BlockTensor,
               psi: BlockTensor) -> List[int]:
    """Algorithmic flops (2 m n k over valid block products) of the four steps."""
    Lr = relabel(L, ["a", "w1", "x"])
    Pr = relabel(psi, ["x", "t1", "t2", "y"])
    W1r = relabel(W1, ["w1", "s1", "t1", "w2"])
    W2r = relabel(W2, ["w2", "s2", "t2", "w3"])
    Rr = relabel(R, ["b", "w3", "y"])
    f = []
    T1 = BlockTensor(*_contract_meta(Lr, Pr), sym=L.sym); f.append(_contract_flops(Lr, Pr))
    T2 = BlockTensor(*_contract_meta(T1, W1r), sym=L.sym); f.append(_contract_flops(T1, W1r))
    T3 = BlockTensor(*_contract_meta(T2, W2r), sym=L.sym); f.append(_contract_flops(T2, W2r))
    f.append(_contract_flops(T3, Rr))
    return f


def _contract_meta(A, B):
    common = [l for l in A.labels if l in B.labels]
    af = [i for i, l in enumerate(A.labels) if l not in common]
    bf = [j for j, l in enumerate(B.labels) if l not in common]
    return ([A.labels[i] for i in af] + [B.labels[j] for j in bf],
            [A.legs[i] for i in af] + [B.legs[j] for j in bf])


def _contract_flops(A, B) -> int:
    common = [l for l in A.labels if l in B.labels]
    ac = [A.labels.index(l) for l in common]
    bc = [B.labels.index(l) for l in common]
    bf = [j for j in range(B.rank) if j not in bc]
    by_kc: Dict[Tuple[int, ...], List[int]] = {}
    for b, t in enumerate(B.blocks):
        by_kc.setdefault(tuple(t[j] for j in bc), []).append(b)
    total = 0
    for a, ta in enumerate(A.blocks):
        size_a = int(np.prod(A.shapes[a]))
        for b in by_kc.get(tuple(ta[i] for i in ac), []):
            n = int(np.prod([B.shapes[b][j] for j in bf])) if bf else 1
            total += 2 * size_a * n
    return total


# --------------------------------------------------------------------------
# Lanczos (Sec. "Eigenvalue decomposition": lowest eigenpair of a Hermitian
# LinOp).  Textbook Lanczos with CGS2 full reorthogonalisation.
# --------------------------------------------------------------------------
def sturm_count(alpha: np.ndarray, beta: np.ndarray, x: float) -> int:
    """Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x
    (negative pivots of the LDL^T factorisation of T - x I)."""
    count = 0
    d = 1.0
    tiny = np.finfo(np.float64).tiny
    for i in range(len(alpha)):
        b2 = beta[i - 1] ** 2 if i > 0 else 0.0
        d = (alpha[i] - x) - b2 / d
        if d == 0.0:
            d = -tiny
        if d < 0.0:
            count += 1
    return count


def tridiag_lowest(alpha: Sequence[float], beta: Sequence[float]):
    """Lowest eigenpair of the symmetric tridiagonal matrix with diagonal alpha
    and off-diagonal beta: Sturm bisection to full precision for the value,
    inverse iteration for the vector (largest component made positive)."""
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    n = len(a)
    if n == 1:
        return float(a[0]), np.ones(1)
    radius = np.zeros(n)
    radius[:-1] += np.abs(b)
    radius[1:] += np.abs(b)
    lo = float(np.min(a - radius))
    hi = float(np.max(a + radius))
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if sturm_count(a, b, mid) >= 1:
            hi = mid
        else:
            lo = mid
    theta = hi
    # inverse iteration on T - theta I with a tridiagonal LU (partial pivoting)
    shift = theta - 4.0 * np.finfo(np.float64).eps * max(1.0, abs(theta))
    s = np.ones(n) / math.sqrt(n)
    T = np.diag(a - shift) + np.diag(b, 1) + np.diag(b, -1)
    for _ in range(3):
        s = np.linalg.solve(T, s)
        s /= np.linalg.norm(s)
    if s[np.argmax(np.abs(s))] < 0:
        s = -s
    return theta, s


def lanczos_ground(matvec: Callable[[np.ndarray], np.ndarray], psi0: np.ndarray, nsteps: int,
                   refine_matvec: Callable[[np.ndarray], np.ndarray] | None = None,
                   breakdown: float = 1e-12):
    """Lowest eigenpair of a symmetric operator by nsteps Lanczos steps.

    v1 = psi0/|psi0|; for each j: w = H v_j; c = V^T w; w -= V c; d = V^T w;
    w -= V d; alpha_j = c_j + d_j; beta_j = |w|; stop if beta_j is below
    breakdown * max(|alpha|, beta_j); v_{j+1} = w / beta_j.  The Ritz pair
    (theta, y = V s) comes from the tridiagonal (alpha, beta); the refined
    energy is the Rayleigh quotient y.Hy / y.y with one more (FP64) apply.
    """
    x = np.asarray(psi0, dtype=np.float64)
    n = x.size
    V = np.empty((nsteps, n))
    V[0] = x / np.linalg.norm(x)
    alpha: List[float] = []
    beta: List[float] = []
    for j in range(nsteps):
        w = matvec(V[j])
        Vj = V[:j + 1]
        c = Vj @ w
        w = w - Vj.T @ c
        d = Vj @ w
        w = w - Vj.T @ d
        alpha.append(float(c[j] + d[j]))
        bj = float(np.linalg.norm(w))
        if bj <= breakdown * max(max(abs(v) for v in alpha), bj):
            break
        if j + 1 == nsteps:
            beta.append(bj)
            break
        beta.append(bj)
        V[j + 1] = w / bj
    m = len(alpha)
    theta, s = tridiag_lowest(alpha, beta[:m - 1])
    y = s @ V[:m]
    hm = refine_matvec if refine_matvec is not None else matvec
    hy = hm(y)
    yy = float(y @ y)
    E = float(y @ hy) / yy
    resid = float(np.linalg.norm(hy - E * y))
    return dict(theta=theta, energy=E, y=y, residual=resid, alpha=np.array(alpha),
                beta=np.array(beta), steps=m, V=V[:m])


# --------------------------------------------------------------------------
# Exact diagonalisation of open Heisenberg chains (dense, Kronecker products)
# --------------------------------------------------------------------------
def _spin_ops(spin: str):
    if spin == "1/2":
        sp = np.array([[0.0, 1.0], [0.0, 0.0]])
        sz = np.diag([0.5, -0.5])
        q = np.array([1, -1])
    elif spin == "1":
        sp = np.sqrt(2.0) * np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0]])
        sz = np.diag([1.0, 0.0, -1.0])
        q = np.array([1, 0, -1])
    else:
        raise ValueError(spin)
    return sp, sp.T, sz, q


def spin_chain_hamiltonian(nsites: int, spin: str, J: float = 1.0, Jz: float = 1.0) -> np.ndarray:
    """H = sum_i [J (Sx Sx + Sy Sy) + Jz Sz Sz] over the bonds of an open
    chain, dense, basis highest Sz first; J (Sx Sx + Sy Sy) is written as
    (J/2)(S+ S- + S- S+)."""
    sp, sm, sz, _ = _spin_ops(spin)
    d = sp.shape[0]
    H = np.zeros((d ** nsites, d ** nsites))
    for i in range(nsites - 1):
        left = np.eye(d ** i)
        right = np.eye(d ** (nsites - i - 2))
        bond = 0.5 * J * (np.kron(sp, sm) + np.kron(sm, sp)) + Jz * np.kron(sz, sz)
        H += np.kron(np.kron(left, bond), right)
    return H


def heisenberg_chain_hamiltonian(nsites: int, spin: str, J: float = 1.0) -> np.ndarray:
    """H = J sum_i S_i.S_{i+1} (open chain)."""
    return spin_chain_hamiltonian(nsites, spin, J, J)


def xx_chain_hamiltonian(nsites: int, spin: str, J: float = 1.0) -> np.ndarray:
    """H = J sum_i (Sx_i Sx_{i+1} + Sy_i Sy_{i+1}) (open chain): the XX model
    of the paper's DMRG benchmark (Sec. "Benchmarks")."""
    return spin_chain_hamiltonian(nsites, spin, J, 0.0)


def chain_ground(nsites: int, spin: str, model: str = "heisenberg", J: float = 1.0,
                 charge: int | None = 0) -> float:
    """Lowest eigenvalue of the Heisenberg or XX chain, optionally restricted
    to one total-charge sector."""
    if model == "heisenberg":
        H = heisenberg_chain_hamiltonian(nsites, spin, J)
    elif model == "xx":
        H = xx_chain_hamiltonian(nsites, spin, J)
    else:
        raise ValueError(model)
    return _lowest_in_sector(H, nsites, spin, charge)


def heisenberg_chain_ground(nsites: int, spin: str, J: float = 1.0, charge: int | None = 0) -> float:
    """Lowest eigenvalue, optionally restricted to one total-charge sector."""
    return chain_ground(nsites, spin, "heisenberg", J, charge)


def tfim_chain_hamiltonian(nsites: int, h: float, J: float = 1.0) -> np.ndarray:
    """H = -J sum_i sx_i sx_{i+1} - h sum_i sz_i (open chain), dense, basis
    sz = +1 first: the transverse-field Ising model of the paper's MPO
    example (Sec. "Conversion from/to NumPy") without the longitudinal field."""
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    sz = np.diag([1.0, -1.0])
    H = np.zeros((2 ** nsites, 2 ** nsites))
    for i in range(nsites):
        H -= h * np.kron(np.kron(np.eye(2 ** i), sz), np.eye(2 ** (nsites - i - 1)))
    for i in range(nsites - 1):
        H -= J * np.kron(np.kron(np.eye(2 ** i), np.kron(sx, sx)), np.eye(2 ** (nsites - i - 2)))
    return H


def tfim_chain_ground(nsites: int, h: float, J: float = 1.0, parity: int | None = 0) -> float:
    """Lowest eigenvalue, optionally in one parity sector (number of
    sz = -1 sites mod 2)."""
    H = tfim_chain_hamiltonian(nsites, h, J)
    if parity is not None:
        down = np.array([bin(i).count("1") % 2 for i in range(2 ** nsites)])
        keep = np.nonzero(down == parity)[0]
        H = H[np.ix_(keep, keep)]
    return float(np.linalg.eigvalsh(H)[0])


def _lowest_in_sector(H: np.ndarray, nsites: int, spin: str, charge: int | None) -> float:
    if charge is not None:
        _, _, _, q = _spin_ops(spin)
        tot = np.zeros(1, dtype=int)
        for _ in range(nsites):
            tot = (tot[:, None] + q[None, :]).ravel()
        keep = np.nonzero(tot == charge)[0]
        H = H[np.ix_(keep, keep)]
    return float(np.linalg.eigvalsh(H)[0])


# --------------------------------------------------------------------------
# Singular value decomposition of a symmetric tensor (Sec. "Tensor
# decomposition and linear algebra": "Matrix form of a UniTensor" and
# "Singular value decomposition", paragraphs "With truncation" and "SVD for
# symmetric UniTensor").  The first rowrank legs are the rows, the others the
# columns.  Every charge q of the new bond has one block matrix M_q: its rows
# are the row-leg sector tuples whose combined flux (sum of dir * charge) is q,
# its columns the column-leg tuples of combined flux -q, so that each (row
# tuple, column tuple) pair is exactly one valid block of T.  The SVD of T is
# the SVD of every M_q; the new bond leaves U outgoing and enters V^dagger.
#
# Readings where the paper is silent (listed in the design notes):
#   * the sectors of the new bond are ordered as their charges first appear
#     when the column tuples are enumerated lexicographically (for a single
#     outgoing column leg this is that leg's sector order, as in the paper's
#     printed rank-3 example); rows and columns inside M_q are the tuples in
#     lexicographic order, each tuple's elements row-major;
#   * truncation: the min_blockdim[q] largest values of each sector are kept
#     first; the remaining room up to keepdim goes to the largest other values
#     not below err, ties going to the earlier sector and then the earlier
#     value; a sector left with no value is dropped from the new bond; s_err
#     is the largest value not kept (0 when nothing is dropped).
# --------------------------------------------------------------------------
def _group_flux(T: BlockTensor, legs_idx: Sequence[int], t: Sequence[int]):
    comps = []
    for c, n in enumerate(T.sym):
        f = sum(T.legs[i][0] * _components(T.legs[i][1][t[i]][0], len(T.sym))[c] for i in legs_idx)
        comps.append(f % n if n >= 2 else f)
    return tuple(comps)


def _neg_charge(q: Tuple[int, ...], sym: Sequence[int]) -> Tuple[int, ...]:
    return tuple((-v) % n if n >= 2 else -v for v, n in zip(q, sym))


def svd_sectors(T: BlockTensor, rowrank: int):
    """The block matrices of T seen as a matrix with the first rowrank legs as
    rows: a list, in new-bond order, of dicts with the bond charge q, the row
    and column tuples ((sector tuple, first row or column, extent), ...) and M."""
    if not 0 < rowrank < T.rank:
        raise OracleError("rowrank must leave at least one row and one column leg")
    ri = list(range(rowrank))
    ci = list(range(rowrank, T.rank))
    rtup = list(itertools.product(*[range(len(T.legs[i][1])) for i in ri]))
    ctup = list(itertools.product(*[range(len(T.legs[i][1])) for i in ci]))
    order: List[Tuple[int, ...]] = []
    for c in ctup:
        full = tuple([0] * rowrank) + tuple(c)
        q = _neg_charge(_group_flux(T, ci, full), T.sym)
        if q not in order:
            order.append(q)
    out = []
    for q in order:
        rows, cols = [], []
        nr = nc = 0
        for r in rtup:
            full = tuple(r) + tuple([0] * len(ci))
            if _group_flux(T, ri, full) == q:
                ext = int(np.prod([T.legs[i][1][k][1] for i, k in zip(ri, r)]))
                rows.append((tuple(r), nr, ext))
                nr += ext
        for c in ctup:
            full = tuple([0] * rowrank) + tuple(c)
            if _neg_charge(_group_flux(T, ci, full), T.sym) == q:
                ext = int(np.prod([T.legs[i][1][k][1] for i, k in zip(ci, c)]))
                cols.append((tuple(c), nc, ext))
                nc += ext
        if nr == 0 or nc == 0:
            continue
        M = np.zeros((nr, nc))
        for r, r0, re in rows:
            for c, c0, ce in cols:
                b = T.index[r + c]
                M[r0:r0 + re, c0:c0 + ce] = T.block(b).reshape(re, ce)
        out.append(dict(q=q if len(T.sym) > 1 else q[0], rows=rows, cols=cols, M=M))
    return out


def svd(T: BlockTensor, rowrank: int):
    """Full SVD of every sector matrix (numpy's LAPACK SVD as the per-block
    step): a list of (q, U_q, s_q descending, Vt_q) in new-bond order."""
    res = []
    for sec in svd_sectors(T, rowrank):
        U, s, Vt = np.linalg.svd(sec["M"], full_matrices=False)
        res.append((sec["q"], U, s, Vt))
    return res


def truncation_counts(svals: Sequence[np.ndarray], keepdim: int, err: float = 0.0,
                      min_blockdim: Sequence[int] | None = None):
    """Values kept per sector and the largest value not kept, for per-sector
    singular values given in descending order (the truncation rule above)."""
    ns = len(svals)
    mb = [0] * ns if min_blockdim is None else [int(x) for x in min_blockdim]
    if len(mb) != ns:
        raise OracleError("one min_blockdim entry per sector")
    kept = [min(mb[q], len(svals[q])) for q in range(ns)]
    room = keepdim - sum(kept)
    cand = [(float(svals[q][i]), q, i) for q in range(ns) for i in range(kept[q], len(svals[q]))
            if float(svals[q][i]) >= err]
    # descending value, then earlier sector, then earlier position
    cand.sort(key=lambda x: (-x[0], x[1], x[2]))
    for v, q, i in cand[:max(room, 0)]:
        kept[q] += 1
    s_err = 0.0
    for q in range(ns):
        if kept[q] < len(svals[q]):
            s_err = max(s_err, float(svals[q][kept[q]]))
    return kept, s_err


def svd_truncate(T: BlockTensor, rowrank: int, keepdim: int, err: float = 0.0,
                 min_blockdim: Sequence[int] | None = None, bond: str = "_m", absorb: str | None = None):
    """Svd_truncate of a symmetric tensor: U[rows..., bond] (bond outgoing),
    the kept singular values per kept sector, V^dagger[bond, cols...] (bond
    incoming) and s_err.  absorb = "u" or "v" multiplies the singular values
    into that factor."""
    secs = svd_sectors(T, rowrank)
    full = svd(T, rowrank)
    kept, s_err = truncation_counts([s for _, _, s, _ in full], keepdim, err, min_blockdim)
    keep_idx = [i for i in range(len(secs)) if kept[i] > 0]
    bond_secs = [(secs[i]["q"], kept[i]) for i in keep_idx]
    rlegs = T.legs[:rowrank]
    clegs = T.legs[rowrank:]
    U = BlockTensor(T.labels[:rowrank] + [bond], list(rlegs) + [(OUT, bond_secs)], sym=T.sym)
    Vd = BlockTensor([bond] + T.labels[rowrank:], [(IN, bond_secs)] + list(clegs), sym=T.sym)
    S = []
    for pos, i in enumerate(keep_idx):
        q, Uq, sq, Vtq = full[i]
        k = kept[i]
        u, s, vt = Uq[:, :k], sq[:k], Vtq[:k, :]
        if absorb == "u":
            u = u * s[None, :]
        elif absorb == "v":
            vt = vt * s[:, None]
        S.append(s.copy())
        for r, r0, re in secs[i]["rows"]:
            b = U.index[r + (pos,)]
            U.block(b)[...] = u[r0:r0 + re, :].reshape(U.shapes[b])
        for c, c0, ce in secs[i]["cols"]:
            b = Vd.index[(pos,) + c]
            Vd.block(b)[...] = vt[:, c0:c0 + ce].reshape(Vd.shapes[b])
    return U, S, Vd, s_err


# --------------------------------------------------------------------------
# Two-site DMRG of an open chain (Sec. "Benchmarks": the DMRG iteration of the
# XX chain; Fig. Hpsi_fig for the effective Hamiltonian).  MPS tensors
# A[a, s, b] (in, in, out); environments L[a, w, a'] (in, out, out) and
# R[b, w, b'] (out, in, in) as in heff_apply.  Textbook procedure: bring the
# MPS to right-canonical form with SVDs from the right, then sweep: at each
# bond, the ground state of H_eff (Lanczos) is split by a truncated SVD; the
# orthonormal factor stays, the singular values move with the centre, and the
# environment grows by one site.
# --------------------------------------------------------------------------
def dagger(T: BlockTensor) -> BlockTensor:
    """Every leg's direction reversed and the elements complex-conjugated
    (UniTensor.Dagger, Sec. "Change the bond direction")."""
    return BlockTensor(T.labels, [(-d, secs) for d, secs in T.legs], np.conj(T.data), sym=T.sym,
                       dtype=T.data.dtype)


def left_env_update(L: BlockTensor, A: BlockTensor, W: BlockTensor) -> BlockTensor:
    """L'[b, w', b'] = sum A*[a, s, b] L[a, w, a'] W[w, s, s', w'] A[a', s', b']."""
    X = contract(relabel(L, ["a", "w", "ap"]), relabel(A, ["ap", "sp", "bp"]))
    Y = contract(X, relabel(W, ["w", "s", "sp", "wp"]))
    Z = contract(Y, relabel(dagger(A), ["a", "s", "b"]))
    return relabel(permute(Z, ["b", "wp", "bp"]), ["a", "w", "ap"])


def right_env_update(R: BlockTensor, B: BlockTensor, W: BlockTensor) -> BlockTensor:
    """R'[a, w, a'] = sum B*[a, s, b] W[w, s, s', w'] R[b, w', b'] B[a', s', b']."""
    X = contract(relabel(R, ["b", "wp", "bp"]), relabel(B, ["ap", "sp", "bp"]))
    Y = contract(X, relabel(W, ["w", "s", "sp", "wp"]))
    Z = contract(Y, relabel(dagger(B), ["a", "s", "b"]))
    return relabel(permute(Z, ["a", "w", "ap"]), ["b", "w", "bp"])


def _two_site(A: BlockTensor, B: BlockTensor) -> BlockTensor:
    return contract(relabel(A, ["a", "s1", "m"]), relabel(B, ["m", "s2", "b"]))


def dmrg_two_site(mps: Sequence[BlockTensor], W: BlockTensor, Lb: BlockTensor, Rb: BlockTensor,
                  nsweeps: int, keepdim: int, err: float = 1e-12, lanczos_steps: int = 40):
    """Right-canonicalise, then nsweeps left-to-right-to-left sweeps.  Returns
    the refined Lanczos energy of every bond update in order and the final MPS
    (centre on site 0)."""
    A = [relabel(t, ["a", "s", "b"]) for t in mps]
    N = len(A)
    if N < 2:
        raise OracleError("two-site DMRG needs at least two sites")
    # right-canonical form: A_j = V^dagger, U S moves left
    for j in range(N - 1, 0, -1):
        U, S, Vd, _ = svd_truncate(A[j], 1, 1 << 30, 0.0, bond="m", absorb="u")
        A[j] = relabel(Vd, ["a", "s", "b"])
        A[j - 1] = relabel(contract(relabel(A[j - 1], ["a", "s", "x"]), relabel(U, ["x", "m"])),
                           ["a", "s", "b"])
    Rs = [None] * (N + 1)
    Rs[N] = Rb
    for j in range(N - 1, 1, -1):
        Rs[j] = right_env_update(Rs[j + 1], A[j], W)
    Ls = [None] * (N + 1)
    Ls[0] = Lb
    energies = []

    def solve(i):
        psi = _two_site(A[i], A[i + 1])
        Lr, Rr = Ls[i], Rs[i + 2]

        def mv(x):
            return heff_apply(Lr, W, W, Rr, BlockTensor(psi.labels, psi.legs, x, sym=psi.sym)).data
        steps = min(lanczos_steps, psi.numel)
        r = lanczos_ground(mv, psi.data, steps)
        energies.append(r["energy"])
        y = r["y"] / np.linalg.norm(r["y"])
        return BlockTensor(psi.labels, psi.legs, y, sym=psi.sym)

    for _ in range(nsweeps):
        for i in range(N - 1):                  # left to right
            psi = solve(i)
            U, S, Vd, _ = svd_truncate(psi, 2, keepdim, err, bond="m", absorb="v")
            A[i] = relabel(U, ["a", "s", "b"])
            A[i + 1] = relabel(Vd, ["a", "s", "b"])
            if i + 1 < N - 1:
                Ls[i + 1] = left_env_update(Ls[i], A[i], W)
        for i in range(N - 2, -1, -1):          # right to left
            psi = solve(i)
            U, S, Vd, _ = svd_truncate(psi, 2, keepdim, err, bond="m", absorb="u")
            A[i] = relabel(U, ["a", "s", "b"])
            A[i + 1] = relabel(Vd, ["a", "s", "b"])
            if i > 0:
                Rs[i + 1] = right_env_update(Rs[i + 2], A[i + 1], W)
    return energies, A
