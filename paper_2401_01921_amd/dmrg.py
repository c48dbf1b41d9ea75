"""Two-site DMRG of an open chain on the GPU (Sec. "Benchmarks": the DMRG
iteration of the XX chain; Fig. Hpsi_fig for the effective Hamiltonian;
Sec. "Singular value decomposition" for the truncation).

Orchestration only: every numeric step runs in the library's kernels --
the two-site contraction and the environment updates as block-sparse
contraction plans, the ground state of H_eff as bst_lanczos_ground, the
split of the two-site state as the symmetric truncated SVD.  This module
decides the order of the calls, keeps the device buffers and builds the
descriptors (labels, directions) of their inputs.

Conventions (those of bst_heff_plan): MPS tensors A[a, s, b] with legs
(in, in, out); environments L[a, w, a'] (in, out, out) and R[b, w, b']
(out, in, in); MPO W[wl, s, s', wr] (in, in, out, out).  The procedure is
the textbook one: the MPS is brought to right-canonical form with SVDs
from the right, then every sweep visits the bonds left to right and back;
at each bond the Lanczos ground state of H_eff is split by a truncated SVD,
the orthonormal factor stays, the singular values move with the centre and
the environment grows by one site.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

from . import bst


@dataclass
class DevTensor:
    """A descriptor and its float64 device data (canonical block layout)."""
    t: bst.Tensor
    data: object   # torch tensor

    @property
    def labels(self) -> List[str]:
        return self.t.labels


def legs_full(T: bst.Tensor):
    sym = T.symmetry()
    labels, legs = T.legs()
    if sym == [0]:
        return labels, legs, None
    full = []
    for i, (d, secs) in enumerate(legs):
        qs = T.leg_charges(i)
        full.append((d, [(q if len(sym) > 1 else q[0], g) for q, (_, g) in zip(qs, secs)]))
    return labels, full, sym


def relabel(T: bst.Tensor, labels: Sequence[str]) -> bst.Tensor:
    """The same legs under new labels (descriptor only)."""
    _, legs, sym = legs_full(T)
    return bst.Tensor(list(labels), legs, sym=sym)


def dagger(T: bst.Tensor, labels: Sequence[str] | None = None) -> bst.Tensor:
    """Every leg's direction reversed: the descriptor of the conjugate of a
    real tensor, whose data (valid blocks, order, layout) is unchanged."""
    old, legs, sym = legs_full(T)
    return bst.Tensor(list(labels or old), [(-d, s) for d, s in legs], sym=sym)


def contract(A: DevTensor, a_labels, B: DevTensor, b_labels, prec="fp64") -> DevTensor:
    import torch
    ta, tb = relabel(A.t, a_labels), relabel(B.t, b_labels)
    tc, plan = bst.contract_plan(ta, tb, prec)
    out = torch.empty(tc.numel, dtype=torch.float64, device=A.data.device)
    plan.execute([A.data, B.data], [out], bst.workspace(plan.workspace_bytes, A.data.device))
    return DevTensor(tc, out)


def contract_desc(ta: bst.Tensor, A, tb: bst.Tensor, B, prec="fp64") -> DevTensor:
    """Contraction of device data A, B under the given descriptors."""
    import torch
    tc, plan = bst.contract_plan(ta, tb, prec)
    out = torch.empty(tc.numel, dtype=torch.float64, device=A.device)
    plan.execute([A, B], [out], bst.workspace(plan.workspace_bytes, A.device))
    return DevTensor(tc, out)


def permute(T: DevTensor, order: Sequence[str]) -> DevTensor:
    import torch
    tp, plan = bst.permute_plan(T.t, list(order))
    out = torch.empty(tp.numel, dtype=torch.float64, device=T.data.device)
    plan.execute([T.data], [out], bst.workspace(plan.workspace_bytes, T.data.device))
    return DevTensor(tp, out)


def left_env_update(L: DevTensor, A: DevTensor, W: DevTensor, prec="fp64") -> DevTensor:
    """L'[b, w', b'] = sum A*[a, s, b] L[a, w, a'] W[w, s, s', w'] A[a', s', b']."""
    X = contract(L, ["a", "w", "ap"], A, ["ap", "sp", "bp"], prec)          # a, w, sp, bp
    Y = contract(X, X.labels, W, ["w", "s", "sp", "wp"], prec)              # a, bp, s, wp
    Z = contract_desc(relabel(Y.t, Y.labels), Y.data, dagger(A.t, ["a", "s", "b"]), A.data, prec)
    Z = permute(Z, ["b", "wp", "bp"])
    return DevTensor(relabel(Z.t, ["a", "w", "ap"]), Z.data)


def right_env_update(R: DevTensor, B: DevTensor, W: DevTensor, prec="fp64") -> DevTensor:
    """R'[a, w, a'] = sum B*[a, s, b] W[w, s, s', w'] R[b, w', b'] B[a', s', b']."""
    X = contract(R, ["b", "wp", "bp"], B, ["ap", "sp", "bp"], prec)         # b, wp, ap, sp
    Y = contract(X, X.labels, W, ["w", "s", "sp", "wp"], prec)              # b, ap, w, s
    Z = contract_desc(relabel(Y.t, Y.labels), Y.data, dagger(B.t, ["a", "s", "b"]), B.data, prec)
    Z = permute(Z, ["a", "w", "ap"])
    return DevTensor(relabel(Z.t, ["b", "w", "bp"]), Z.data)


def svd_split(T: DevTensor, rowrank: int, keepdim: int, err: float, absorb, bond="m"):
    """(U, V^dagger) as device tensors after Svd_truncate, the singular
    values absorbed as asked, and s_err."""
    Ut, U, S, Vt, Vd, s_err, kept = bst.svd_truncate(T.t, T.data, rowrank, keepdim, err, None, bond, absorb,
                                                     device=T.data.device)
    return DevTensor(Ut, U), DevTensor(Vt, Vd), s_err


def two_site(A: DevTensor, B: DevTensor, prec="fp64") -> DevTensor:
    return contract(A, ["a", "s1", "m"], B, ["m", "s2", "b"], prec)


def dmrg_two_site(mps: Sequence[DevTensor], W: DevTensor, Lb: DevTensor, Rb: DevTensor, nsweeps: int,
                  keepdim: int, err: float = 1e-12, lanczos_steps: int = 40, prec="fp64",
                  contract_prec="fp64"):
    """Right-canonicalise, then nsweeps left-to-right-to-left sweeps.  Returns
    the refined Lanczos energy of every bond update, the truncation error
    (s_err) of every split, and the final MPS (centre on site 0).  prec is
    the form of the H_eff matvecs inside Lanczos (the refinement apply is
    float64); contract_prec that of the other contractions."""
    import torch
    A = [DevTensor(relabel(t.t, ["a", "s", "b"]), t.data) for t in mps]
    N = len(A)
    if N < 2:
        raise ValueError("two-site DMRG needs at least two sites")
    for j in range(N - 1, 0, -1):
        U, Vd, _ = svd_split(A[j], 1, 1 << 40, 0.0, "u")
        A[j] = DevTensor(relabel(Vd.t, ["a", "s", "b"]), Vd.data)
        C = contract(A[j - 1], ["a", "s", "x"], U, ["x", "m"], contract_prec)
        A[j - 1] = DevTensor(relabel(C.t, ["a", "s", "b"]), C.data)
    Rs = [None] * (N + 1)
    Rs[N] = Rb
    for j in range(N - 1, 1, -1):
        Rs[j] = right_env_update(Rs[j + 1], A[j], W, contract_prec)
    Ls = [None] * (N + 1)
    Ls[0] = Lb
    energies, errs = [], []
    Wd = relabel(W.t, ["wl", "s", "sp", "wr"])

    def solve(i):
        psi = two_site(A[i], A[i + 1], contract_prec)
        pt = relabel(psi.t, ["a", "s1", "s2", "b"])
        Lt = relabel(Ls[i].t, ["a", "w", "ap"])
        Rt = relabel(Rs[i + 2].t, ["b", "w", "bp"])
        plan = bst.heff_plan(Lt, Wd, Wd, Rt, pt, prec)
        steps = min(lanczos_steps, pt.numel)
        r = bst.lanczos_ground(plan, [Ls[i].data, W.data, W.data, Rs[i + 2].data], psi.data, steps, prec,
                               True)
        energies.append(r["energy"])
        return DevTensor(pt, r["psi"])

    for _ in range(nsweeps):
        for i in range(N - 1):
            psi = solve(i)
            U, Vd, se = svd_split(psi, 2, keepdim, err, "v")
            errs.append(se)
            A[i] = DevTensor(relabel(U.t, ["a", "s", "b"]), U.data)
            A[i + 1] = DevTensor(relabel(Vd.t, ["a", "s", "b"]), Vd.data)
            if i + 1 < N - 1:
                Ls[i + 1] = left_env_update(Ls[i], A[i], W, contract_prec)
        for i in range(N - 2, -1, -1):
            psi = solve(i)
            U, Vd, se = svd_split(psi, 2, keepdim, err, "u")
            errs.append(se)
            A[i] = DevTensor(relabel(U.t, ["a", "s", "b"]), U.data)
            A[i + 1] = DevTensor(relabel(Vd.t, ["a", "s", "b"]), Vd.data)
            if i > 0:
                Rs[i + 1] = right_env_update(Rs[i + 2], A[i + 1], W, contract_prec)
    torch.cuda.synchronize()
    return energies, errs, A
