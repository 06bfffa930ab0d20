"""Exact squared biharmonic distance by conjugate gradients in binary64, in
plain torch on a torch device -- oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). It shares nothing with
the HIP library: the Laplacian is applied with torch's own sparse CSR product.

The route is the one of ``exact.beta_cg`` (the Laplacian-solver formulation
of section 2.3), written for many right-hand sides at once so that graphs
with 10^7 - 10^9 adjacency entries can be solved on a GPU:

  * M = L + 11^T/n is nonsingular and symmetric positive definite; b_st is
    orthogonal to 1, so M x = b_st gives x = L^+ b_st, and
    beta(s, t) = ||L^+ b_st||^2 = ||x||^2 (Definition 2.1, Eq. (1)).
  * A second solve M y = x gives y = (L^+)^2 b_st (x is orthogonal to 1 as
    well), hence beta = b_st^T y = y_s - y_t. The two values come from
    different computations; their agreement is the acceptance check.
  * Jacobi preconditioning, diag(M) = d + 1/n.
  * Each column of the n x Q right-hand side runs its own conjugate-gradient
    recurrence (its own step sizes) until ||r|| <= tol ||rhs||; a finished
    column is frozen while the others continue.
"""

from __future__ import annotations

import numpy as np
import torch


class Laplacian:
    """v -> (L + 11^T/n) v for an n x Q block, L = D - A of a canonical CSR."""

    def __init__(self, g, device):
        self.n = int(g.n)
        self.device = torch.device(device)
        idx = torch.int32 if g.nnz < 2 ** 31 else torch.int64
        crow = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(idx)
        col = torch.from_numpy(np.ascontiguousarray(g.col)).to(idx)
        ones = torch.ones(int(g.nnz), dtype=torch.float64)
        self.A = torch.sparse_csr_tensor(crow, col, ones, size=(self.n, self.n)).to(self.device)
        self.deg = torch.from_numpy(np.ascontiguousarray(g.deg, dtype=np.float64)).to(self.device)
        self.diag = (self.deg + 1.0 / self.n).unsqueeze(1)

    def __call__(self, V: torch.Tensor) -> torch.Tensor:
        Y = torch.sparse.mm(self.A, V)  # A V
        Y.neg_()
        Y.addcmul_(self.deg.unsqueeze(1), V)  # D V - A V
        Y.add_(V.sum(dim=0, keepdim=True) / self.n)  # + 1 (1^T V) / n
        return Y


def pcg(op: Laplacian, rhs: torch.Tensor, tol: float, maxit: int, log=None, log_every: int = 50):
    """Column-wise Jacobi-preconditioned CG for op X = rhs. Returns (X, iterations
    per column, final relative residual per column)."""
    Q = rhs.shape[1]
    X = torch.zeros_like(rhs)
    R = rhs.clone()
    Z = R / op.diag
    P = Z.clone()
    rz = (R * Z).sum(dim=0)
    bn = torch.linalg.vector_norm(rhs, dim=0)
    active = torch.ones(Q, dtype=torch.bool, device=rhs.device)
    iters = torch.zeros(Q, dtype=torch.int64, device=rhs.device)
    rel = torch.ones(Q, dtype=torch.float64, device=rhs.device)
    for _ in range(maxit):
        AP = op(P)
        pAp = (P * AP).sum(dim=0)
        alpha = torch.where(active, rz / pAp, torch.zeros_like(rz))
        X.addcmul_(P, alpha.unsqueeze(0))
        R.addcmul_(AP, alpha.unsqueeze(0), value=-1.0)
        del AP
        iters += active.to(torch.int64)
        rn = torch.linalg.vector_norm(R, dim=0)
        rel = torch.where(active, rn / bn, rel)
        active = active & (rn > tol * bn)
        if not bool(active.any()):
            break
        if log is not None and int(iters.max()) % log_every == 0:
            log(f"  cg iteration {int(iters.max())}: {int(active.sum())} columns left, "
                f"largest relative residual {float(rel.max()):.2e}")
        Z = R / op.diag
        rz_new = (R * Z).sum(dim=0)
        beta = torch.where(active, rz_new / rz, torch.zeros_like(rz))
        P.mul_(beta.unsqueeze(0)).add_(Z)
        rz = torch.where(active, rz_new, rz)
        del Z
    return X, iters, rel


def beta_cg_many(g, s, t, device="cuda", tol: float = 1e-12, maxit: int = 20000, chunk: int = 32,
                 op: Laplacian | None = None, log=None):
    """(||x||^2, y_s - y_t, CG iterations of both solves, final relative
    residuals) for each pair, x = L^+ b_st and y = L^+ x; ``chunk`` pairs share
    one block solve."""
    s = np.asarray(s, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    if op is None:
        op = Laplacian(g, device)
    m = s.size
    b1 = np.zeros(m)
    b2 = np.zeros(m)
    its = np.zeros(m, dtype=np.int64)
    res = np.zeros(m)
    for c0 in range(0, m, chunk):
        sc, tc = s[c0:c0 + chunk], t[c0:c0 + chunk]
        Q = sc.size
        cols = torch.arange(Q, device=op.device)
        rhs = torch.zeros((op.n, Q), dtype=torch.float64, device=op.device)
        rhs[torch.from_numpy(sc).to(op.device), cols] = 1.0
        rhs[torch.from_numpy(tc).to(op.device), cols] = -1.0
        X, it1, r1 = pcg(op, rhs, tol, maxit, log)
        del rhs
        Y, it2, r2 = pcg(op, X, tol, maxit, log)
        b1[c0:c0 + Q] = (X * X).sum(dim=0).cpu().numpy()
        ys = Y[torch.from_numpy(sc).to(op.device), cols]
        yt = Y[torch.from_numpy(tc).to(op.device), cols]
        b2[c0:c0 + Q] = (ys - yt).cpu().numpy()
        its[c0:c0 + Q] = (it1 + it2).cpu().numpy()
        res[c0:c0 + Q] = torch.maximum(r1, r2).cpu().numpy()
        del X, Y
        if log is not None:
            log(f"cg pairs {c0}..{c0 + Q - 1}: iterations {int(it1.max())} + {int(it2.max())}")
    return b1, b2, its, res


def beta_truncated_many(g, s, t, L: int, device="cuda", op: Laplacian | None = None):
    """beta^(L)(s_j, t_j) = ||h||^2 - (1^T h)^2 / n with h = sum_{i=0..L} P^i D^{-1} b
    (Lemma 2.3), P = D^{-1} A, for every pair as the columns of one block."""
    s = np.asarray(s, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    if op is None:
        op = Laplacian(g, device)
    Q = s.size
    cols = torch.arange(Q, device=op.device)
    dinv = (1.0 / op.deg).unsqueeze(1)
    si = torch.from_numpy(s).to(op.device)
    ti = torch.from_numpy(t).to(op.device)
    V = torch.zeros((op.n, Q), dtype=torch.float64, device=op.device)
    V[si, cols] = dinv[si, 0]
    V[ti, cols] = -dinv[ti, 0]
    H = V.clone()
    for _ in range(L):
        V = torch.sparse.mm(op.A, V).mul_(dinv)
        H.add_(V)
    out = (H * H).sum(dim=0) - H.sum(dim=0) ** 2 / op.n
    return out.cpu().numpy()
