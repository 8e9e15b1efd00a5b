"""Kernel ridge regression in its n x n kernel form (oracle; test infrastructure only).

Sec. 2.1 gives the classical closed form f(x) = k(x)^T (K_n + lambda I)^-1 Y.  With
the empirical risk scaled by 1/n (as in R(theta) of the same section) the ridge
term becomes n * lambda; this is the reading used here.  For the truncated
Fourier kernel K(x, y) = sum_k exp(i k.(x - y)) / p_k the two forms meet through
the push-through identity (Phi^* Phi + n lambda P)^-1 Phi^* = P^-1 Phi^* (Phi P^-1
Phi^* + n lambda I)^-1, so theta = P^-1 Phi^* alpha with alpha = (K + n lambda I)^-1 Y.
This route solves an n x n system instead of the N x N normal equations.
"""
from __future__ import annotations

import numpy as np

from .fourier import design_matrix


def krr_theta(X: np.ndarray, Y: np.ndarray, m: int, lam: float, p: np.ndarray) -> np.ndarray:
    """theta through the kernel form; X [d, n] with small n, Y [n] or [T, n], p [N]."""
    Phi = design_matrix(X, m)                                  # [n, N]
    n = Phi.shape[0]
    K = (Phi / p[None, :]) @ np.conj(Phi).T                    # sum_k e^{ik(Xi-Xj)}/p_k
    K = 0.5 * (K + np.conj(K).T)
    Yt = np.atleast_2d(Y).astype(np.float64).T                 # [n, T]
    alpha = np.linalg.solve(K + n * lam * np.eye(n), Yt)       # [n, T]
    theta = (np.conj(Phi).T @ alpha) / p[:, None]              # [N, T]
    return theta.T if np.ndim(Y) == 2 else theta[:, 0]
