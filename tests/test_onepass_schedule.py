"""The one-pass Lanczos schedule the GPU runs, restated in numpy and held
against the oracle's textbook two-pass classical Gram-Schmidt Lanczos (Sec.
"Eigenvalue decomposition"): the basis rows keep the residuals as the pass
writes them, a lower-triangular C maps them to the orthonormal vectors, and
the step's scalars (the lagged projection d, alpha, beta, the next
coefficients) are formed from the pass's sums u_m . w through C.  In exact
arithmetic alpha and beta equal the textbook ones; in float64 they agree to
rounding.  CPU only: it pins the algebra of the schedule, not the kernels."""
import numpy as np
import pytest

from oracle import oracle as orc


def onepass_lanczos(H, psi0, m):
    """The schedule step by step, in the order the kernels evaluate it."""
    n = psi0.size
    U = np.zeros((m, n))
    C = np.zeros((m, m))
    alpha = np.zeros(m)
    beta = np.zeros(m)
    U[0] = psi0 / np.linalg.norm(psi0)
    aest = 0.0
    sums = None                     # u_m . w (m <= j) and w . w of the last pass
    for j in range(m):
        z = H @ U[j]
        g = U[j] @ z
        d = np.zeros(j)
        if j > 0:
            d = np.array([C[k, :k + 1] @ sums[:k + 1] for k in range(j)])   # V^T u_j
            alpha[j - 1] = aest + d[j - 1]
            beta[j - 1] = np.sqrt(max(sums[j] - d @ d, 0.0))
        bp = beta[j - 1] if j > 0 else 1.0
        rb = 1.0 / bp
        C[j, :j + 1] = -rb * (d @ C[:j, :j + 1]) if j > 0 else 0.0
        C[j, j] += rb
        # coefficients of v_0..v_j in w = z rb - sum coef_k v_k
        f = np.zeros(j)
        for k in range(j):
            yn = d[k + 1] if k + 1 < j else bp
            f[k] = alpha[k] * d[k] + beta[k] * yn + (beta[k - 1] * d[k - 1] if k > 0 else 0.0)
        vz = rb * (g - d @ f)
        cf = np.zeros(j + 1)
        for i in range(j):
            e = alpha[i] * d[i] + (beta[i - 1] * d[i - 1] if i > 0 else 0.0) + \
                (beta[i] * d[i + 1] if i + 1 < j else 0.0)
            cf[i] = rb * e + (bp if i == j - 1 else 0.0)
        ej = beta[j - 1] * d[j - 1] if j > 0 else 0.0
        aest = rb * (vz - ej)
        cf[j] = rb * ej + aest
        coef = cf @ C[:j + 1, :j + 1]          # in the stored rows
        w = z * rb - coef @ U[:j + 1]
        if j + 1 < m:
            U[j + 1] = w
        sums = np.concatenate([U[:j + 1] @ w, [w @ w]])
    j = m - 1
    d = np.array([C[k, :k + 1] @ sums[:k + 1] for k in range(j + 1)])
    alpha[j] = aest + d[j]
    beta[j] = np.sqrt(max(sums[j + 1] - d @ d, 0.0))
    return alpha, beta, C, U


@pytest.mark.parametrize("n,m,shift,seed", [(300, 40, 0.0, 1), (300, 40, 30.0, 2), (400, 80, -50.0, 3),
                                            (200, 60, 5.0, 4)])
def test_onepass_matches_textbook(n, m, shift, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    H = (A + A.T) / 2 + shift * np.eye(n)
    psi0 = rng.standard_normal(n)
    ref = orc.lanczos_ground(lambda v: H @ v, psi0, m)
    alpha, beta, C, U = onepass_lanczos(H, psi0, m)
    scale = np.max(np.abs(np.linalg.eigvalsh(H)))
    assert np.max(np.abs(alpha - ref["alpha"])) <= 1e-12 * scale
    assert np.max(np.abs(beta[:m - 1] - ref["beta"][:m - 1])) <= 1e-12 * scale
    V = C @ U                                   # the orthonormal vectors
    assert np.max(np.abs(V @ V.T - np.eye(m))) <= 1e-13
    # the Ritz vector through C^T s, and its Rayleigh quotient
    theta, s = orc.tridiag_lowest(alpha, beta[:m - 1])
    y = (s @ C) @ U
    E = y @ (H @ y) / (y @ y)
    assert abs(theta - ref["theta"]) <= 1e-12 * scale
    assert abs(E - ref["energy"]) <= 1e-12 * scale


def test_onepass_rows_are_the_written_residuals():
    """Row m + 1 is w of step m as formed: v_{m+1} = (u_{m+1} - V_m d) / beta_m,
    i.e. C's diagonal is 1 / beta and the basis is never rewritten."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((120, 120))
    H = (A + A.T) / 2
    alpha, beta, C, U = onepass_lanczos(H, rng.standard_normal(120), 20)
    assert C[0, 0] == 1.0
    assert np.allclose(np.diag(C)[1:], 1.0 / beta[:19], rtol=1e-14, atol=0)
    assert np.all(np.triu(C, 1) == 0.0)
