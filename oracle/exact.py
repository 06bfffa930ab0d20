"""Exact squared biharmonic distance in binary64 -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

  * ``beta_dense``: Definition 2.1 with the pseudoinverse of section 2.1,
    L^+ = (L + 11^T/n)^{-1} - 11^T/n, evaluated two of the ways Eq. (1) lists:
    ||L^+ b||^2 and (L^+)^2_ss + (L^+)^2_tt - 2 (L^+)^2_st.
  * ``beta_cg``: the Laplacian-solver route of section 2.3: conjugate
    gradients on the nonsingular system (L + 11^T/n) x = b (b is orthogonal to
    1, so x = L^+ b); beta = ||x||^2 from the first solve and
    beta = b^T y with (L + 11^T/n) y = x from a second solve.
  * ``h_truncated`` / ``beta_truncated``: the truncated series of Lemma 2.3,
    h^(L) = sum_{i=0..L} P^i D^{-1} b, beta^(L) = ||h||^2 - (1^T h)^2 / n.
  * ``mixing_factor``: lambda = max(|lambda_2|, |lambda_n|) of P (section 2.1)
    from the dense spectrum of D^{-1/2} A D^{-1/2}, which P is similar to.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def laplacian(g) -> sp.csr_matrix:
    A = g.scipy()
    return (sp.diags(g.deg.astype(np.float64)) - A).tocsr()


def pinv_dense(g) -> np.ndarray:
    n = g.n
    Lm = laplacian(g).toarray()
    J = np.full((n, n), 1.0 / n)
    return np.linalg.inv(Lm + J) - J


def beta_dense(g, s: int, t: int, Lp: np.ndarray | None = None):
    """(||L^+ b||^2, (L^+)^2_ss + (L^+)^2_tt - 2 (L^+)^2_st)."""
    if Lp is None:
        Lp = pinv_dense(g)
    x = Lp[:, s] - Lp[:, t]
    b1 = float(x @ x)
    L2 = Lp @ Lp
    b2 = float(L2[s, s] + L2[t, t] - 2.0 * L2[s, t])
    return b1, b2


def beta_dense_all(g, s, t):
    """||L^+ b_st||^2 for many pairs from one dense pseudoinverse."""
    Lp = pinv_dense(g)
    s = np.asarray(s)
    t = np.asarray(t)
    X = Lp[:, s] - Lp[:, t]
    return np.einsum("ij,ij->j", X, X)


def _pcg(g, rhs: np.ndarray, tol: float, maxit: int):
    Lm = laplacian(g)
    n = g.n
    diag = g.deg.astype(np.float64) + 1.0 / n

    def apply(v):
        return Lm @ v + v.sum() / n

    x = np.zeros(n)
    r = rhs.copy()
    zv = r / diag
    p = zv.copy()
    rz = r @ zv
    bnorm = np.sqrt(rhs @ rhs)
    it = 0
    while it < maxit:
        Ap = apply(p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        it += 1
        if np.sqrt(r @ r) <= tol * bnorm:
            break
        zv = r / diag
        rz_new = r @ zv
        p = zv + (rz_new / rz) * p
        rz = rz_new
    return x, it


def beta_cg(g, s: int, t: int, tol: float = 1e-12, maxit: int = 100000):
    """(||x||^2, b^T y, iterations) with x = L^+ b and y = L^+ x."""
    b = np.zeros(g.n)
    b[s] = 1.0
    b[t] = -1.0
    x, it1 = _pcg(g, b, tol, maxit)
    y, it2 = _pcg(g, x, tol, maxit)
    return float(x @ x), float(y[s] - y[t]), it1 + it2


def h_truncated(g, s: int, t: int, L: int) -> np.ndarray:
    """h^(L) = sum_{i=0..L} P^i D^{-1} b_st with P = D^{-1} A."""
    A = g.scipy()
    dinv = 1.0 / g.deg.astype(np.float64)
    v = np.zeros(g.n)
    v[s] = dinv[s]
    v[t] = -dinv[t]
    h = v.copy()
    for _ in range(L):
        v = dinv * (A @ v)
        h += v
    return h


def beta_truncated(g, s: int, t: int, L: int) -> float:
    h = h_truncated(g, s, t, L)
    return float(h @ h - h.sum() ** 2 / g.n)


def beta_truncated_multi(g, s, t, Ls) -> np.ndarray:
    """beta^(L)(s_j, t_j) for every pair j and every L in ``Ls``: out[i, j] for Ls[i].

    The same series as ``h_truncated``, run once for all pairs as columns of one
    matrix; h^(L) for a smaller L is a partial sum of the series for a larger L.
    """
    s = np.asarray(s, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    Ls = [int(x) for x in Ls]
    A = g.scipy().astype(np.float64)
    dinv = 1.0 / g.deg.astype(np.float64)
    m = s.size
    cols = np.arange(m)
    V = np.zeros((g.n, m))
    V[s, cols] += dinv[s]
    V[t, cols] -= dinv[t]
    H = V.copy()
    out = np.zeros((len(Ls), m))

    def record(step):
        for i, L in enumerate(Ls):
            if L == step:
                out[i] = (H * H).sum(axis=0) - H.sum(axis=0) ** 2 / g.n

    record(0)
    for step in range(1, max(Ls) + 1):
        V = dinv[:, None] * (A @ V)
        H += V
        record(step)
    return out


def phi(g, s: int, t: int, L: int, z: np.ndarray) -> float:
    """phi(z) = z^T h^(L) (Lemma 3.3)."""
    return float(np.asarray(z, dtype=np.float64) @ h_truncated(g, s, t, L))


def mixing_factor(g) -> float:
    """max(|lambda_2|, |lambda_n|) over the eigenvalues of P (dense; small graphs)."""
    A = g.scipy().toarray()
    r = 1.0 / np.sqrt(g.deg.astype(np.float64))
    ev = np.sort(np.linalg.eigvalsh(A * r[:, None] * r[None, :]))
    return float(max(abs(ev[-2]), abs(ev[0])))
