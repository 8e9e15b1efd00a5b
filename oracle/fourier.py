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

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1 << 14


def _threads() -> int:
    """Worker threads: FK_ORACLE_THREADS, else OMP_NUM_THREADS, else the core count (at most 16)."""
    v = os.environ.get("FK_ORACLE_THREADS") or os.environ.get("OMP_NUM_THREADS")
    return max(1, int(v) if v else min(16, os.cpu_count() or 1))


def _chunk_sum(fn, n: int, chunk: int, out: np.ndarray) -> np.ndarray:
    """out += fn(s, e) over the chunks [s, e) of range(n), added in chunk order.

    The chunks are evaluated by a pool of threads (numpy releases the GIL in its kernels; each
    chunk's arithmetic is the same as in a serial loop) with BLAS held to one thread each; the
    partial sums are added in the order of the chunks, so the result does not depend on the
    number of threads."""
    starts = list(range(0, n, chunk))
    nt = min(_threads(), len(starts))
    if nt <= 1:
        for s in starts:
            out += fn(s, min(n, s + chunk))
        return out
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1, user_api="blas"), ThreadPoolExecutor(nt) as pool:
        for w in range(0, len(starts), 4 * nt):
            for part in pool.map(lambda s: fn(s, min(n, s + chunk)), starts[w:w + 4 * nt]):
                out += part
    return out


def modes(m: int, d: int) -> np.ndarray:
    """All multi-indices k in {-m..m}^d, row-major (k_d fastest), shape [N, d]."""
    axes = [np.arange(-m, m + 1)] * d
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel() for g in grid], axis=1)


def _powers(x: np.ndarray, K: int) -> np.ndarray:
    """E[j, K + q] = exp(i q x_j) for q = -K..K (float64 complex).

    Built one power at a time (E[., q] = E[., q - 1] exp(i x)) in rows of contiguous memory and
    returned as the transposed view, so that each step streams through memory."""
    z = np.exp(1j * x.astype(np.float64))
    pos = np.empty((K + 1, x.shape[0]), dtype=np.complex128)
    pos[0] = 1.0
    for q in range(1, K + 1):
        pos[q] = pos[q - 1] * z
    return np.concatenate([np.conj(pos[:0:-1]), pos], axis=0).T


def _weighted_sum(X: np.ndarray, W: np.ndarray, K: int, sign: int) -> np.ndarray:
    """S_c[q] = sum_j W[c, j] exp(sign * i q.X_j) for q in {-K..K}^d, shape [C, (2K+1)^d]."""
    d, n = X.shape
    C = W.shape[0]
    L = 2 * K + 1

    def part(s, e):
        tabs = [_powers(X[a, s:e], K) for a in range(d)]
        if sign < 0:
            tabs = [np.conj(t) for t in tabs]
        w = W[:, s:e].astype(np.float64)
        acc = np.zeros((C,) + (L,) * d, dtype=np.complex128)
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
        return acc

    acc = _chunk_sum(part, n, CHUNK, np.zeros((C,) + (L,) * d, dtype=np.complex128))
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


def fourier_entries(X: np.ndarray, W, qs, sign: int, chunk: int = 1 << 20) -> np.ndarray:
    """Entries S[t, f] = n^-1 sum_j W[t, j] exp(sign * i qs[f].X_j) for a few frequency vectors qs
    [F, d] and weight rows W [T, n] (W = None: one row of ones), by direct evaluation of each
    exponential in float64 (Sec. 2.3).  The exponentials of a chunk are shared by all weight rows.
    For sampled entries of very large inputs; returns complex128 [T, F]."""
    X = np.atleast_2d(X)
    d, n = X.shape
    qs = np.asarray(qs, dtype=np.float64).reshape(-1, d)
    T = 1 if W is None else np.atleast_2d(W).shape[0]
    Wr = None if W is None else np.atleast_2d(W)

    def part(s, e):
        phase = qs @ X[:, s:e].astype(np.float64)          # [F, c]
        z = np.exp(sign * 1j * phase)
        if Wr is None:
            return z.sum(axis=1)[None, :]
        return Wr[:, s:e].astype(np.float64) @ z.T         # [T, F]

    acc = _chunk_sum(part, n, chunk, np.zeros((T, qs.shape[0]), dtype=np.complex128))
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

    def part(s, e):
        E = np.concatenate([_powers(X[a, s:e], m) for a in range(d)], axis=1)  # [c, d*L]
        return np.conj(E).T @ E

    B = _chunk_sum(part, n, CHUNK, np.zeros((d * L, d * L), dtype=np.complex128))
    return B / n


def additive_rhs(X: np.ndarray, Y: np.ndarray, m: int) -> np.ndarray:
    """Stacked right-hand side (n^-1 Phi_a^* Y)_a of the additive model, [T, d(2m+1)]."""
    X = np.atleast_2d(X)
    Y = np.atleast_2d(Y)
    d, n = X.shape
    return np.concatenate([_weighted_sum(X[a:a + 1], Y, m, -1) / n for a in range(d)], axis=1)
