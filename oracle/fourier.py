"""Direct Fourier sums (oracle; test infrastructure only).

Sec. 2.3 of the paper: the right-hand side n^-1 Phi^* Y and the Gram
n^-1 Phi^* Phi are sums over the sample of complex exponentials.  Here they are
computed by their definition in float64: per chunk of points the powers
exp(i q x) for q = 0..K are built by repeated multiplication of exp(i x)
(accumulated rounding ~ K * 1e-16), negative frequencies are their conjugates,
and the multi-dimensional sum over points is a matrix product of the per-axis
tables (no reordering beyond the sum over points).
"""
from __future__ import annotations

import numpy as np

CHUNK = 1 << 15


def modes(m: int, d: int) -> np.ndarray:
    """All multi-indices k in {-m..m}^d, row-major (k_d fastest), shape [N, d]."""
    axes = [np.arange(-m, m + 1)] * d
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel() for g in grid], axis=1)


def _powers(x: np.ndarray, K: int) -> np.ndarray:
    """E[j, K + q] = exp(i q x_j) for q = -K..K (float64 complex)."""
    z = np.exp(1j * x.astype(np.float64))
    pos = np.empty((x.shape[0], K + 1), dtype=np.complex128)
    pos[:, 0] = 1.0
    for q in range(1, K + 1):
        pos[:, q] = pos[:, q - 1] * z
    return np.concatenate([np.conj(pos[:, :0:-1]), pos], axis=1)


def _weighted_sum(X: np.ndarray, W: np.ndarray, K: int, sign: int) -> np.ndarray:
    """S_c[q] = sum_j W[c, j] exp(sign * i q.X_j) for q in {-K..K}^d, shape [C, (2K+1)^d]."""
    d, n = X.shape
    C = W.shape[0]
    L = 2 * K + 1
    acc = np.zeros((C,) + (L,) * d, dtype=np.complex128)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        tabs = [_powers(X[a, s:e], K) for a in range(d)]
        if sign < 0:
            tabs = [np.conj(t) for t in tabs]
        w = W[:, s:e].astype(np.float64)
        if d == 1:
            acc += w @ tabs[0]
        elif d == 2:
            for c in range(C):
                acc[c] += (tabs[0] * w[c][:, None]).T @ tabs[1]
        else:
            for c in range(C):
                prod = tabs[0] * w[c][:, None]
                for a in range(1, d):
                    prod = (prod[:, :, None] * tabs[a][:, None, :]).reshape(e - s, -1)
                acc[c] += prod.sum(axis=0).reshape((L,) * d)
    return acc.reshape(C, -1)


def gram_generator(X: np.ndarray, m: int) -> np.ndarray:
    """M[q] = n^-1 sum_j exp(+i q.X_j), q in {-2m..2m}^d (Sec. 2.3, covariance matrix).

    The first row of the empirical covariance n^-1 Phi^* Phi, extended to all
    differences of modes, with Sigma[k, l] = M[l - k].  Returns a complex128
    array of shape (4m+1,)*d.
    """
    X = np.atleast_2d(X)
    d, n = X.shape
    ones = np.ones((1, n))
    S = _weighted_sum(X, ones, 2 * m, +1)[0] / n
    return S.reshape((4 * m + 1,) * d)


def rhs(X: np.ndarray, Y: np.ndarray, m: int) -> np.ndarray:
    """b_k = n^-1 sum_j Y_j exp(-i k.X_j), k in {-m..m}^d (Sec. 2.3, covariance vector).

    The sign is the one of n^-1 Phi^* Y with Phi[j, k] = exp(+i k.X_j); the paper
    prints the opposite sign in the displayed formula.  Y is [T, n]; returns
    complex128 [T, (2m+1)^d].
    """
    X = np.atleast_2d(X)
    Y = np.atleast_2d(Y)
    n = X.shape[1]
    return _weighted_sum(X, Y, m, -1) / n


def fourier_entry(X: np.ndarray, w, q, sign: int, chunk: int = 1 << 22) -> complex:
    """One entry n^-1 sum_j w_j exp(sign * i q.X_j) of the sums above, for a single frequency
    vector q (w = None for weight 1), by direct evaluation of the exponential per point in
    float64 (Sec. 2.3).  For checking sampled entries of large inputs one at a time."""
    X = np.atleast_2d(X)
    d, n = X.shape
    q = np.asarray(q, dtype=np.float64).reshape(d)
    acc = 0.0 + 0.0j
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        phase = np.zeros(e - s)
        for a in range(d):
            phase += q[a] * X[a, s:e].astype(np.float64)
        z = np.exp(sign * 1j * phase)
        acc += z.sum() if w is None else (np.asarray(w[s:e], dtype=np.float64) * z).sum()
    return acc / n


def toeplitz_matrix(M: np.ndarray, m: int) -> np.ndarray:
    """The multilevel Toeplitz matrix Sigma[k, l] = M[l - k] over k, l in {-m..m}^d."""
    d = M.ndim
    ks = modes(m, d)
    diff = ks[None, :, :] - ks[:, None, :] + 2 * m      # l - k, shifted
    return M[tuple(diff[..., a] for a in range(d))]


def design_matrix(X: np.ndarray, m: int) -> np.ndarray:
    """Phi[j, k] = exp(+i k.X_j): the rows are phi(X_j)^* (Sec. 2.1). Small n only."""
    X = np.atleast_2d(X).astype(np.float64)
    ks = modes(m, X.shape[0])
    return np.exp(1j * (X.T @ ks.T))


def additive_blocks(X: np.ndarray, m: int) -> np.ndarray:
    """Block Gram of the additive model (Sec. 5): B[a, b][k, l] = n^-1 sum_j
    exp(-i k X_ja) exp(+i l X_jb), k, l in -m..m.  Returns [d(2m+1), d(2m+1)]."""
    X = np.atleast_2d(X)
    d, n = X.shape
    L = 2 * m + 1
    B = np.zeros((d * L, d * L), dtype=np.complex128)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        E = np.concatenate([_powers(X[a, s:e], m) for a in range(d)], axis=1)  # [c, d*L]
        B += np.conj(E).T @ E
    return B / n


def additive_rhs(X: np.ndarray, Y: np.ndarray, m: int) -> np.ndarray:
    """Stacked right-hand side (n^-1 Phi_a^* Y)_a of the additive model, [T, d(2m+1)]."""
    X = np.atleast_2d(X)
    Y = np.atleast_2d(Y)
    d, n = X.shape
    return np.concatenate([_weighted_sum(X[a:a + 1], Y, m, -1) / n for a in range(d)], axis=1)
