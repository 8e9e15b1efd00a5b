"""Held-out MSE of the fitted estimator and its gradients (oracle; test infrastructure only).

Not in the paper: the differentiable path fits theta(lambda, p) = A^-1 b with
A = Sigma + lambda diag(p) on the training sample and scores it on a held-out
sample (Xv, Yv).  With the held-out Gram Sigma_v = [M_v[l - k]] and right-hand
side b_v (the same direct sums as in ``fourier``):

  L = n_v^-1 sum_j |f_theta(Xv_j) - Yv_j|^2
    = theta^* Sigma_v theta - 2 Re(b_v^* theta) + n_v^-1 sum_j Yv_j^2.

With g = Sigma_v theta - b_v and u = A^-1 g (A is Hermitian):
  dL/d log(lambda) = -2 lambda Re(u^* diag(p) theta),
  dL/d p_k        = -2 lambda Re(conj(u_k) theta_k),
  dL/d conj(theta) = g  (Wirtinger derivative; 2 Re(conj(g)^T d theta) = dL).
"""
from __future__ import annotations

import numpy as np

from .predict import predict
from .fourier import toeplitz_matrix


def heldout_mse(theta: np.ndarray, Xv: np.ndarray, Yv: np.ndarray, m: int) -> np.ndarray:
    """n_v^-1 sum |f_theta(Xv) - Yv|^2 by direct evaluation. theta [T, N], Yv [T, n_v]."""
    f = predict(np.atleast_2d(theta), Xv, m)
    r = f - np.atleast_2d(Yv).astype(np.float64)
    return (np.abs(r) ** 2).mean(axis=1)


def heldout_mse_quadratic(theta: np.ndarray, Mv: np.ndarray, bv: np.ndarray, yv2: np.ndarray,
                          m: int) -> np.ndarray:
    """The same loss from held-out Gram / RHS: theta^* Sigma_v theta - 2 Re(b_v^* theta) + mean(Yv^2)."""
    Tv = toeplitz_matrix(Mv, m)
    th = np.atleast_2d(theta)
    quad = np.einsum("tk,kl,tl->t", np.conj(th), Tv, th).real
    lin = (np.conj(np.atleast_2d(bv)) * th).sum(axis=1).real
    return quad - 2.0 * lin + np.asarray(yv2, dtype=np.float64)


def theta_path_gradients(A: np.ndarray, theta: np.ndarray, p: np.ndarray, lam: float, G: np.ndarray):
    """Gradients through theta = A^-1 b, A = Sigma + lambda diag(p), of a loss whose Wirtinger
    gradient with respect to conj(theta) is G (dLoss = 2 Re(G^* dtheta)).

    d theta / d lambda = -A^-1 diag(p) theta and d theta / d p_k = -lambda A^-1 e_k theta_k, so with
    u = A^-1 G (A Hermitian): returns (dLoss/dlog lambda = -2 lambda Re(u^* diag(p) theta),
    dLoss/dp [N] = -2 lambda Re(conj(u) theta))."""
    u = np.linalg.solve(A, G)
    return float(-2.0 * lam * np.real(np.conj(u) @ (p * theta))), -2.0 * lam * np.real(np.conj(u) * theta)


def mse_gradients(A: np.ndarray, theta: np.ndarray, p: np.ndarray, lam: float,
                  Mv: np.ndarray, bv: np.ndarray, m: int):
    """Gradients of the held-out MSE for one lambda and one target.

    Returns (dL/dlog lambda, dL/dp [N], dL/dconj(theta) [N])."""
    Tv = toeplitz_matrix(Mv, m)
    g = Tv @ theta - bv
    u = np.linalg.solve(A, g)
    dloglam = -2.0 * lam * np.real(np.conj(u) @ (p * theta))
    dp = -2.0 * lam * np.real(np.conj(u) * theta)
    return float(dloglam), dp, g
