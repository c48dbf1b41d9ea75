"""Seeded synthetic workloads for the block-sparse H_eff.psi path.

This module is the only code shared by the GPU library's callers and the
CPU oracle's callers.  It produces *inputs* only:

* a counter-based pseudo-random stream (SplitMix64 -> Box-Muller normals),
* the per-leg sector lists (charge, dim) of every workload,
* the dense closed-form Heisenberg MPO tensor W[wl, s, s', wr],
* value recipes for the environments L and R, which take a block table
  (block sector tuples, shapes, flat offsets) computed by the caller.

It performs no charge matching, no block enumeration and no contraction:
block tables always come from the caller, so the structure arithmetic of the
method lives only in the library and in the oracle.

Leg conventions (Sec. "UniTensor with Symmetries", flux rule "in minus out is
zero"): a leg is ``(dir, [(q, g), ...])`` with dir = +1 for an incoming and
-1 for an outgoing bond, q the U(1) charge of a sector and g its dimension.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

IN, OUT = +1, -1
Leg = Tuple[int, List[Tuple[int, int]]]

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


# --------------------------------------------------------------------------
# Counter-based random numbers (SplitMix64, Steele/Lea/Flood 2014)
# --------------------------------------------------------------------------
def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream of ``seed``.

    Output i is the SplitMix64 finaliser applied to ``seed + (i+1)*gamma``
    (mod 2**64), i.e. exactly what the sequential generator returns on its
    (i+1)-th call.
    """
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def normal(seed: int, n: int) -> np.ndarray:
    """n standard-normal float64 values (Box-Muller on SplitMix64 pairs)."""
    if n == 0:
        return np.zeros(0, dtype=np.float64)
    u = splitmix64(seed, 0, 2 * n)
    scale = 1.0 / float(1 << 53)
    u1 = ((u[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * scale  # (0, 1]
    u2 = (u[1::2] >> np.uint64(11)).astype(np.float64) * scale          # [0, 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def uniform_ints(seed: int, start: int, lo: int, hi: int, count: int) -> np.ndarray:
    """count integers in [lo, hi] from positions start.. of the stream."""
    u = splitmix64(seed, start, count)
    return (lo + (u % np.uint64(hi - lo + 1)).astype(np.int64)).astype(np.int64)


# --------------------------------------------------------------------------
# Seeds: workload k uses base 20240101 + k; each tensor has its own stream.
# --------------------------------------------------------------------------
TENSOR_SLOT = {"L": 1, "psi": 2, "R": 3, "A": 4, "B": 5, "psi0": 6, "draws": 7}


def seed_for(workload: int, tensor: str, instance: int = 0) -> int:
    base = 20240101 + workload
    return (base * 16 + TENSOR_SLOT[tensor]) * 1024 + instance


# --------------------------------------------------------------------------
# Sector lists
# --------------------------------------------------------------------------
def gaussian_sector_dims(chi: int, qmax: int) -> List[Tuple[int, int]]:
    """Sectors q = -qmax..qmax (ascending) with a Gaussian dim profile.

    sigma = qmax/2; g(q) = max(1, round_half_up(chi*exp(-q^2/2 sigma^2)/Z))
    for q != 0 (symmetric in q) and g(0) takes the remainder so that the
    dims add up to chi exactly.
    """
    if qmax == 0:
        return [(0, chi)]
    sigma = qmax / 2.0
    w = {q: math.exp(-q * q / (2.0 * sigma * sigma)) for q in range(-qmax, qmax + 1)}
    z = sum(w.values())
    g = {}
    for q in range(1, qmax + 1):
        v = max(1, int(math.floor(chi * w[q] / z + 0.5)))
        g[q] = g[-q] = v
    g[0] = chi - sum(v for q, v in g.items() if q != 0)
    if g[0] < 1:
        raise ValueError("chi too small for qmax")
    return [(q, g[q]) for q in range(-qmax, qmax + 1)]


def physical_sectors(spin: str) -> List[Tuple[int, int]]:
    """Physical sectors, highest Sz first, each of dim 1.

    spin-1/2 uses q = 2 Sz (charges +1, -1); spin-1 uses q = Sz (+1, 0, -1).
    """
    if spin == "1/2":
        return [(+1, 1), (-1, 1)]
    if spin == "1":
        return [(+1, 1), (0, 1), (-1, 1)]
    raise ValueError(spin)


def mpo_charge_step(spin: str) -> int:
    """Charge carried by a spin-raising MPO channel (2 for q = 2Sz, 1 for q = Sz)."""
    return 2 if spin == "1/2" else 1


def spin_matrices(spin: str):
    """(S+, S-, Sz, I) in the physical basis ordered highest Sz first."""
    if spin == "1/2":
        sp = np.array([[0.0, 1.0], [0.0, 0.0]])
        sz = np.diag([0.5, -0.5])
    elif spin == "1":
        r2 = math.sqrt(2.0)
        sp = np.array([[0.0, r2, 0.0], [0.0, 0.0, r2], [0.0, 0.0, 0.0]])
        sz = np.diag([1.0, 0.0, -1.0])
    else:
        raise ValueError(spin)
    return sp, sp.T.copy(), sz, np.eye(sp.shape[0])


# MPO channels in the lower-triangular convention (the transverse-field Ising
# MPO example of the paper puts the identity in the first and last diagonal
# slots the same way): channel 4 starts a term (left boundary), channel 0 ends
# it (right boundary), channels 1, 2, 3 carry S+, S-, Sz across the bond.
# Channel charges are (0, -delta, +delta, 0, 0).  Grouped by ascending charge
# the bond reads [-delta: ch1], [0: ch0, ch3, ch4], [+delta: ch2].
MPO_GROUPED_ORDER = (1, 0, 3, 4, 2)
# The XX chain (the paper's DMRG benchmark model) has no Sz-Sz coupling: the
# same MPO without channel 3, a bond of dimension 4.
MPO_GROUPED_ORDER_XX = (1, 0, 4, 2)
MODELS = ("heisenberg", "xx")


def _grouped_order(model: str):
    if model not in MODELS:
        raise ValueError(model)
    return MPO_GROUPED_ORDER if model == "heisenberg" else MPO_GROUPED_ORDER_XX


def mpo_bond(spin: str, model: str = "heisenberg") -> List[Tuple[int, int]]:
    d = mpo_charge_step(spin)
    return [(-d, 1), (0, len(_grouped_order(model)) - 2), (+d, 1)]


def grouped_index(ch: int, model: str = "heisenberg") -> int:
    """Position of an MPO channel on the grouped (dense) MPO bond."""
    return _grouped_order(model).index(ch)


def channel_position(ch: int) -> Tuple[int, int]:
    """(sector index, index inside the sector) of an MPO channel in the grouped bond."""
    return {1: (0, 0), 0: (1, 0), 3: (1, 1), 4: (1, 2), 2: (2, 0)}[ch]


def mpo_dense(spin: str, model: str = "heisenberg", J: float = 1.0) -> np.ndarray:
    """Dense W of the chosen model: J S.S (Heisenberg, bond 5) or
    J (Sx Sx + Sy Sy) = (J/2)(S+ S- + S- S+) (XX, bond 4)."""
    w = heisenberg_mpo_dense(spin, J)
    if model == "heisenberg":
        return w
    keep = [MPO_GROUPED_ORDER.index(ch) for ch in _grouped_order(model)]
    return np.ascontiguousarray(w[keep][:, :, :, keep])


def heisenberg_mpo_dense(spin: str, J: float = 1.0) -> np.ndarray:
    """Dense W[wl, s, s', wr] of H = J sum_i S_i.S_{i+1}, channels grouped.

    s is the ket (output) index and s' the bra (input) index; summing
    W[4, w] (x) W[w, 0] over w gives J S.S for one bond.
    """
    sp, sm, sz, eye = spin_matrices(spin)
    d = eye.shape[0]
    w = np.zeros((5, d, d, 5))
    w[0, :, :, 0] = eye
    w[1, :, :, 0] = sp
    w[2, :, :, 0] = sm
    w[3, :, :, 0] = sz
    w[4, :, :, 1] = 0.5 * J * sm
    w[4, :, :, 2] = 0.5 * J * sp
    w[4, :, :, 3] = J * sz
    w[4, :, :, 4] = eye
    p = list(MPO_GROUPED_ORDER)
    return np.ascontiguousarray(w[p][:, :, :, p])


def mpo_legs(spin: str, model: str = "heisenberg") -> List[Leg]:
    """W legs (wl IN, s IN, s' OUT, wr OUT): q_wl + q_s = q_s' + q_wr."""
    b = mpo_bond(spin, model)
    ph = physical_sectors(spin)
    return [(IN, b), (IN, ph), (OUT, ph), (OUT, b)]


# --------------------------------------------------------------------------
# Tensor specs of the workloads: (labels, legs)
# --------------------------------------------------------------------------
def heff_specs(spin: str, virt_a: List[Tuple[int, int]], virt_b: List[Tuple[int, int]],
               model: str = "heisenberg"):
    """Leg specs of L, W1, W2, R and psi for a two-site H_eff.

    psi[a, s1, s2, b] (IN, IN, IN, OUT); L[a, w, a'] (IN, OUT, OUT);
    R[b, w, b'] (OUT, IN, IN); W as in mpo_legs.
    """
    ph = physical_sectors(spin)
    mb = mpo_bond(spin, model)
    psi = (["a", "s1", "s2", "b"], [(IN, virt_a), (IN, ph), (IN, ph), (OUT, virt_b)])
    L = (["a", "w", "ap"], [(IN, virt_a), (OUT, mb), (OUT, virt_a)])
    R = (["b", "w", "bp"], [(OUT, virt_b), (IN, mb), (IN, virt_b)])
    W = (["wl", "s", "sp", "wr"], mpo_legs(spin, model))
    return {"L": L, "W1": W, "W2": W, "R": R, "psi": psi}


def pairwise_specs():
    """Pairwise workload: A[l,s,m] . B[m,s',r], chi = 32 in 5 sectors."""
    v = [(-2, 4), (-1, 7), (0, 10), (1, 7), (2, 4)]
    ph = physical_sectors("1/2")
    A = (["l", "s", "m"], [(IN, v), (IN, ph), (OUT, v)])
    B = (["m", "t", "r"], [(IN, v), (IN, ph), (OUT, v)])
    return {"A": A, "B": B}


WORKLOADS = {
    1: dict(name="pairwise-chi32-fp64"),
    2: dict(name="heff-spin1/2-chi512", spin="1/2", chi=512, qmax=8),
    3: dict(name="heff-spin1/2-chi2048", spin="1/2", chi=2048, qmax=16),
    4: dict(name="heff-batch64-spin1/2-chi128..1024", spin="1/2", n=64, chi_lo=128, chi_hi=1024,
            qmax_lo=4, qmax_hi=16),
    5: dict(name="lanczos40-spin1-chi4096", spin="1", chi=4096, qmax=20, steps=40),
}


def heff_workload_specs(k: int):
    wl = WORKLOADS[k]
    v = gaussian_sector_dims(wl["chi"], wl["qmax"])
    return heff_specs(wl["spin"], v, v)


def batch_draws(k: int = 4) -> List[Tuple[int, int]]:
    """(chi_i, qmax_i) of the batched workload, one SplitMix64 stream."""
    wl = WORKLOADS[k]
    s = seed_for(k, "draws")
    n = wl["n"]
    chis = uniform_ints(s, 0, wl["chi_lo"], wl["chi_hi"], n)
    qs = uniform_ints(s, n, wl["qmax_lo"], wl["qmax_hi"], n)
    out = []
    for c, q in zip(chis.tolist(), qs.tolist()):
        # every sector needs at least one state
        q = min(q, (c - 1) // 2)
        out.append((c, q))
    return out


# --------------------------------------------------------------------------
# Environment value recipes (take a block table from the caller)
# --------------------------------------------------------------------------
BlockTable = Sequence[Tuple[Tuple[int, ...], Tuple[int, ...], int]]


def _by_idx(table: BlockTable) -> Dict[Tuple[int, ...], Tuple[Tuple[int, ...], int]]:
    return {tuple(qi): (tuple(sh), off) for qi, sh, off in table}


def symmetrized_env(table: BlockTable, numel: int, seed: int) -> np.ndarray:
    """X[x, w, x'] -> (X[x,w,x'] + X[x', pi(w), x]) / sqrt(2) with N(0,1) X.

    pi swaps the S+ and S- channels (grouped sectors 0 and 2) and fixes the
    charge-0 channels.  With the MPO above this makes H_eff real-symmetric.
    """
    x = normal(seed, numel)
    out = np.empty_like(x)
    blocks = _by_idx(table)
    for qi, (sh, off) in blocks.items():
        n = int(np.prod(sh))
        ka, kw, kb = qi
        pshape, poff = blocks[(kb, 2 - kw, ka)]
        mine = x[off:off + n].reshape(sh)
        part = x[poff:poff + int(np.prod(pshape))].reshape(pshape)
        out[off:off + n] = ((mine + part.transpose(2, 1, 0)) / math.sqrt(2.0)).ravel()
    return out


def dmrg_like_env(table: BlockTable, numel: int, seed: int, side: str, virt: List[Tuple[int, int]],
                  coupling: float = 0.15) -> np.ndarray:
    """Environment with the structure of a converged DMRG block.

    For L (side "L") the left-boundary channel (ch4) is the identity and ch0
    holds a block Hamiltonian; for R (side "R") ch0 is the identity and ch4
    the block Hamiltonian.  The block Hamiltonian of charge q is diagonal
    with levels e_{q,0} = min(|q|, 1) and e_{q,i} = 1 + 2 i/g (i >= 1) plus a
    small symmetric N(0,1) perturbation; the S+/S-/Sz channels are N(0,1)
    boundary operators scaled by coupling/sqrt(g), with S- the transpose of
    S+ so that H_eff is real-symmetric.  The gapped, narrow spectrum is what
    lets a 40-step Lanczos solve converge from a random start.
    """
    x = normal(seed, numel)
    out = np.zeros_like(x)
    blocks = _by_idx(table)
    ident_pos = 2 if side == "L" else 0   # position inside the charge-0 MPO sector
    ham_pos = 0 if side == "L" else 2
    # first pass: everything except the transposed S- (sector 2) blocks
    for qi, (sh, off) in blocks.items():
        ka, kw, kb = qi
        ga, gw, gb = sh
        n = ga * gw * gb
        xb = x[off:off + n].reshape(sh)
        ob = np.zeros(sh)
        if kw == 1:
            if ka != kb or ga != gb:
                raise ValueError("charge-0 environment block must be square")
            q = virt[ka][0]
            levels = np.array([min(abs(q), 1)] + [1.0 + 2.0 * i / ga for i in range(1, ga)])
            pert = xb[:, ham_pos, :]
            ob[:, ident_pos, :] = np.eye(ga)
            ob[:, ham_pos, :] = np.diag(levels) + 0.02 * (pert + pert.T) / math.sqrt(2.0 * ga)
            sz = xb[:, 1, :]
            ob[:, 1, :] = coupling * (sz + sz.T) / math.sqrt(2.0 * ga)
        elif kw == 0:
            ob[:] = coupling * xb / math.sqrt(max(ga, gb))
        out[off:off + n] = ob.ravel()
    for qi, (sh, off) in blocks.items():
        ka, kw, kb = qi
        if kw != 2:
            continue
        psh, poff = blocks[(kb, 0, ka)]
        part = out[poff:poff + int(np.prod(psh))].reshape(psh)
        out[off:off + int(np.prod(sh))] = part.transpose(2, 1, 0).ravel()
    return out


# --------------------------------------------------------------------------
# Transverse-field Ising chain with Z_2 parity (the paper's MPO example in
# Sec. "Conversion from/to NumPy", without its longitudinal field, so that
# the parity prod_i sigma^z_i is conserved): H = -J sum sx sx - h sum sz.
# Basis sigma^z = +1, -1 with Z_2 charges 0, 1; sigma^x carries charge 1.
# Channels as in the Heisenberg MPO (start 2, end 0, 1 carries sigma^x),
# grouped by charge: [0: ch0, ch2], [1: ch1].
# --------------------------------------------------------------------------
TFIM_GROUPED_ORDER = (0, 2, 1)
TFIM_SYM = (2,)


def tfim_physical_sectors() -> List[Tuple[int, int]]:
    return [(0, 1), (1, 1)]


def tfim_mpo_bond() -> List[Tuple[int, int]]:
    return [(0, 2), (1, 1)]


def tfim_grouped_index(ch: int) -> int:
    return TFIM_GROUPED_ORDER.index(ch)


def tfim_mpo_dense(h: float, J: float = 1.0) -> np.ndarray:
    """Dense W[wl, s, s', wr] (channels grouped) of H = -J sum sx sx - h sum sz."""
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    sz = np.diag([1.0, -1.0])
    w = np.zeros((3, 2, 2, 3))
    w[0, :, :, 0] = np.eye(2)
    w[2, :, :, 2] = np.eye(2)
    w[1, :, :, 0] = sx
    w[2, :, :, 1] = -J * sx
    w[2, :, :, 0] = -h * sz
    p = list(TFIM_GROUPED_ORDER)
    return np.ascontiguousarray(w[p][:, :, :, p])


def tfim_heff_specs(virt_a: List[Tuple[int, int]], virt_b: List[Tuple[int, int]]):
    """Leg specs (Z_2 charges) of L, W1, W2, R and psi, as heff_specs."""
    ph = tfim_physical_sectors()
    mb = tfim_mpo_bond()
    psi = (["a", "s1", "s2", "b"], [(IN, virt_a), (IN, ph), (IN, ph), (OUT, virt_b)])
    L = (["a", "w", "ap"], [(IN, virt_a), (OUT, mb), (OUT, virt_a)])
    R = (["b", "w", "bp"], [(OUT, virt_b), (IN, mb), (IN, virt_b)])
    W = (["wl", "s", "sp", "wr"], [(IN, mb), (IN, ph), (OUT, ph), (OUT, mb)])
    return {"L": L, "W1": W, "W2": W, "R": R, "psi": psi}


# --------------------------------------------------------------------------
# Open-chain MPS inputs (structure and seeded values only)
# --------------------------------------------------------------------------
def _charge_counts(nsites: int, spin: str) -> Dict[int, int]:
    """Number of product states of nsites sites per total charge."""
    qs = [q for q, _ in physical_sectors(spin)]
    c = {0: 1}
    for _ in range(nsites):
        n: Dict[int, int] = {}
        for t, m in c.items():
            for q in qs:
                n[t + q] = n.get(t + q, 0) + m
        c = n
    return c


def mps_bonds(nsites: int, spin: str, charge: int = 0, cap: int | None = None) -> List[List[Tuple[int, int]]]:
    """Sector lists of the nsites + 1 virtual bonds of an open-chain MPS in the
    total-charge sector `charge`: bond i carries the charge of sites 0..i-1,
    with the number of left-block states of that charge as its dim, capped by
    the number of right-block states completing it to `charge` (and by cap)."""
    bonds = []
    for i in range(nsites + 1):
        left, right = _charge_counts(i, spin), _charge_counts(nsites - i, spin)
        secs = []
        for q in sorted(left):
            d = min(left[q], right.get(charge - q, 0))
            if cap is not None:
                d = min(d, cap)
            if d > 0:
                secs.append((q, d))
        bonds.append(secs)
    return bonds


def mps_specs(nsites: int, spin: str, charge: int = 0, cap: int | None = None):
    """(labels, legs) of the site tensors A_i[a, s, b] (in, in, out)."""
    bonds = mps_bonds(nsites, spin, charge, cap)
    ph = physical_sectors(spin)
    return [(["a", "s", "b"], [(IN, bonds[i]), (IN, ph), (OUT, bonds[i + 1])]) for i in range(nsites)]


def boundary_env_specs(spin: str, model: str = "heisenberg", charge: int = 0):
    """(labels, legs) of the trivial boundary environments L[1, D_W, 1] and
    R[1, D_W, 1], and the dense position of their single 1.0 (the left
    boundary channel 4 in L, the right boundary channel 0 in R)."""
    mb = mpo_bond(spin, model)
    L = (["a", "w", "ap"], [(IN, [(0, 1)]), (OUT, mb), (OUT, [(0, 1)])])
    R = (["b", "w", "bp"], [(OUT, [(charge, 1)]), (IN, mb), (IN, [(charge, 1)])])
    return L, (0, grouped_index(4, model), 0), R, (0, grouped_index(0, model), 0)
