"""Shared test helpers (random block-sparse operand pairs, dense references)."""
import numpy as np

from oracle import oracle as orc


def _random_pair(rng, rank_a, rank_b, ncommon):
    def leg(d):
        ns = int(rng.integers(1, 4))
        qs = sorted(rng.choice(np.arange(-2, 3), ns, replace=False).tolist())
        return (d, [(q, int(rng.integers(1, 4))) for q in qs])
    la = [leg(int(rng.choice([1, -1]))) for _ in range(rank_a)]
    lb = [leg(int(rng.choice([1, -1]))) for _ in range(rank_b)]
    la_lab = [f"a{i}" for i in range(rank_a)]
    lb_lab = [f"b{i}" for i in range(rank_b)]
    ia = rng.choice(rank_a, ncommon, replace=False)
    ib = rng.choice(rank_b, ncommon, replace=False)
    for n, (i, j) in enumerate(zip(ia, ib)):
        la_lab[i] = lb_lab[j] = f"c{n}"
        lb[j] = (-la[i][0], list(la[i][1]))
    A = orc.BlockTensor(la_lab, la)
    B = orc.BlockTensor(lb_lab, lb)
    A.data[:] = rng.standard_normal(A.numel)
    B.data[:] = rng.standard_normal(B.numel)
    return A, B


def _einsum_reference(A, B):
    letters = "abcdefghijklmnopqrstuvwxyz"
    labs = {l: letters[i] for i, l in enumerate(dict.fromkeys(A.labels + B.labels))}
    sa = "".join(labs[l] for l in A.labels)
    sb = "".join(labs[l] for l in B.labels)
    out = [l for l in A.labels if l not in B.labels] + [l for l in B.labels if l not in A.labels]
    so = "".join(labs[l] for l in out)
    return np.einsum(f"{sa},{sb}->{so}", orc.embed(A), orc.embed(B))


def _random_sym_pair(rng, rank_a, rank_b, ncommon, sym, dmax=4):
    """A random pair under the symmetry list `sym` (0 = U(1) with charges in
    [-2, 2], n = Z_n with charges in [0, n)); charges are tuples when there
    are several symmetries."""
    def charge_set(ns):
        pool = set()
        while len(pool) < ns:
            c = tuple(int(rng.integers(-2, 3)) if n == 0 else int(rng.integers(0, n)) for n in sym)
            pool.add(c)
        return sorted(pool)

    distinct = int(np.prod([5 if n == 0 else n for n in sym]))

    def leg(d):
        ns = min(int(rng.integers(1, 4)), distinct)
        cs = charge_set(ns)
        return (d, [(c if len(sym) > 1 else c[0], int(rng.integers(1, dmax))) for c in cs])
    la = [leg(int(rng.choice([1, -1]))) for _ in range(rank_a)]
    lb = [leg(int(rng.choice([1, -1]))) for _ in range(rank_b)]
    la_lab = [f"a{i}" for i in range(rank_a)]
    lb_lab = [f"b{i}" for i in range(rank_b)]
    ia = rng.choice(rank_a, ncommon, replace=False)
    ib = rng.choice(rank_b, ncommon, replace=False)
    for n, (i, j) in enumerate(zip(ia, ib)):
        la_lab[i] = lb_lab[j] = f"c{n}"
        lb[j] = (-la[i][0], list(la[i][1]))
    A = orc.BlockTensor(la_lab, la, sym=sym)
    B = orc.BlockTensor(lb_lab, lb, sym=sym)
    A.data[:] = rng.standard_normal(A.numel)
    B.data[:] = rng.standard_normal(B.numel)
    return A, B
