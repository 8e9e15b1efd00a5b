"""Conjugate-gradient solve of the normal equations (oracle; test infrastructure only).

Sec. 2.3 ("Matrix inversion") of the paper: the system (Sigma + lambda M^* M) theta = b is
Hermitian positive definite, and each product with Sigma costs O(m^d log m) through its
multilevel Toeplitz structure, so the system is solved with conjugate gradients.  The paper
fixes neither a preconditioner nor a stopping rule; the reading taken here is the Jacobi
preconditioner diag(Sigma) + lambda diag(P) and the stop ||b - A theta_k|| <= tol ||b||
on the recursively updated residual.

What CG computes is the solution A^-1 b, whose plain definition is `solve.solve_system`;
`pcg` below is the textbook preconditioned iteration in float64 (no blocking, no batching,
one system at a time), kept for its iteration counts and residual history.  The product
with Sigma is the definition Sigma[k, l] = M[l - k] written as a dense matrix
(`fourier.toeplitz_matrix`), not an FFT.
"""
from __future__ import annotations

import numpy as np

from .fourier import modes, toeplitz_matrix


def toeplitz_apply(M: np.ndarray, x: np.ndarray, m: int) -> np.ndarray:
    """y = Sigma x for Sigma[k, l] = M[l - k] (Sec. 2.3, covariance matrix).

    x is [N] or [V, N] (rows are vectors); returns the same shape, complex128."""
    S = toeplitz_matrix(M, m)
    x = np.asarray(x, dtype=np.complex128)
    return x @ S.T if x.ndim == 2 else S @ x


def toeplitz_apply_rows(M: np.ndarray, x: np.ndarray, m: int, rows) -> np.ndarray:
    """Selected entries y[k] = sum_l M[l - k] x[l] of Sigma x, one row at a time, for inputs
    too large for the dense matrix.  rows are flat mode indices; x is [N]."""
    d = M.ndim
    ks = modes(m, d)
    x = np.asarray(x, dtype=np.complex128)
    out = np.empty(len(rows), dtype=np.complex128)
    for i, r in enumerate(rows):
        diff = ks - ks[r] + 2 * m                       # l - k, shifted to 0..4m
        out[i] = np.sum(M[tuple(diff[:, a] for a in range(d))] * x)
    return out


def pcg(A: np.ndarray, b: np.ndarray, dg: np.ndarray, tol: float, maxit: int):
    """Preconditioned conjugate gradients for the Hermitian positive definite A
    (preconditioner diag(dg)), started from theta = 0.

    Returns (theta, iterations, history) where history[k] = ||r_k|| / ||b|| of the
    recursively updated residual after k iterations (history[0] = 1).  Stops at the first
    k with history[k] <= tol, or after maxit iterations."""
    b = np.asarray(b, dtype=np.complex128)
    theta = np.zeros_like(b)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return theta, 0, [0.0]
    r = b.copy()
    z = r / dg
    p = z.copy()
    rho = np.real(np.vdot(r, z))
    hist = [1.0]
    it = 0
    while it < maxit:
        q = A @ p
        alpha = rho / np.real(np.vdot(p, q))
        theta = theta + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol:
            break
        z = r / dg
        rho_new = np.real(np.vdot(r, z))
        p = z + (rho_new / rho) * p
        rho = rho_new
    return theta, it, hist
