"""Evaluation of the fitted trigonometric polynomial (oracle; test infrastructure only)."""
from __future__ import annotations

import numpy as np

from .fourier import _powers, CHUNK


def predict(theta: np.ndarray, Xq: np.ndarray, m: int) -> np.ndarray:
    """f_theta(x) = sum_k theta_k exp(+i k.x) by direct sum (Sec. 2.1, estimator).

    theta is [T, (2m+1)^d] (or [N]); returns complex128 [T, nq].  For real data the
    imaginary part is at rounding level."""
    Xq = np.atleast_2d(Xq)
    d, nq = Xq.shape
    th = np.atleast_2d(theta)
    T = th.shape[0]
    L = 2 * m + 1
    th = th.reshape((T,) + (L,) * d)
    out = np.empty((T, nq), dtype=np.complex128)
    for s in range(0, nq, CHUNK):
        e = min(nq, s + CHUNK)
        tabs = [_powers(Xq[a, s:e], m) for a in range(d)]
        for t in range(T):
            # contract one axis at a time: sum over k_1, then k_2, ... (pointwise in j)
            v = tabs[0] @ th[t].reshape(L, -1)                 # [c, L^(d-1)]
            for a in range(1, d):
                v = np.einsum("jkr,jk->jr", v.reshape(e - s, L, -1), tabs[a])
            out[t, s:e] = v.reshape(-1)
    return out if theta.ndim == 2 else out[0]


def predict_additive(theta: np.ndarray, Xq: np.ndarray, m: int) -> np.ndarray:
    """Additive model: f(x) = sum_a sum_k theta_{a,k} exp(+i k x_a) (Sec. 5)."""
    Xq = np.atleast_2d(Xq)
    d = Xq.shape[0]
    L = 2 * m + 1
    th = np.atleast_2d(theta)
    out = 0
    for a in range(d):
        out = out + predict(th[:, a * L:(a + 1) * L], Xq[a:a + 1], m)
    return out if theta.ndim == 2 else out[0]
