"""Penalty matrices lambda M^* M (oracle; test infrastructure only)."""
from __future__ import annotations

import numpy as np

from .fourier import modes


def sobolev_weights(m: int, d: int, s: float) -> np.ndarray:
    """S^2 diagonal of Sec. 3.1: p_k = 1 + ||k||_2^(2s) over k in {-m..m}^d."""
    k = modes(m, d).astype(np.float64)
    r2 = (k * k).sum(axis=1)
    return 1.0 + r2 ** s


def sobolev_bessel_weights(m: int, d: int, s: float) -> np.ndarray:
    """The equivalent Sobolev norm (1 + ||k||^2)^s (Sec. 3.1 notes the norms are equivalent)."""
    k = modes(m, d).astype(np.float64)
    return (1.0 + (k * k).sum(axis=1)) ** s


def _box_integral(q: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """int_lo^hi exp(i q x) dx for integer q (closed form)."""
    q = np.asarray(q, dtype=np.float64)
    out = np.empty(q.shape, dtype=np.complex128)
    z = q == 0
    out[z] = hi - lo
    qq = q[~z]
    out[~z] = (np.exp(1j * qq * hi) - np.exp(1j * qq * lo)) / (1j * qq)
    return out


def piml_box_fourier_matrix(m: int, lo, hi, L: float) -> np.ndarray:
    """Fourier matrix C of a box domain (Sec. 4, tractable domains), the matrix with
    theta^* C theta = (4L)^-d int_Omega |f_theta(x)|^2 dx for f_theta = sum_k theta_k exp(i k.x):
    C[k1, k2] = (4L)^-d int_Omega exp(i <k2 - k1, x> pi / (2L)) dx, in torus radians
    u = pi x / (2L), i.e. (2 pi)^-d int_{Omega'} exp(i <k2 - k1, u>) du over the box Omega' in radians.
    (The paper prints k1 - k2, the transpose; the two agree for boxes symmetric about 0.)
    lo, hi are the box corners in radians."""
    lo = np.atleast_1d(np.asarray(lo, dtype=np.float64))
    hi = np.atleast_1d(np.asarray(hi, dtype=np.float64))
    d = lo.shape[0]
    ks = modes(m, d)
    diff = ks[None, :, :] - ks[:, None, :]          # k2 - k1
    C = np.ones(diff.shape[:2], dtype=np.complex128)
    for a in range(d):
        C *= _box_integral(diff[..., a], lo[a], hi[a])
    del L
    return C / (2.0 * np.pi) ** d


def pde_symbol(m: int, d: int, alphas, coefs) -> np.ndarray:
    """Diagonal D of a linear constant-coefficient operator sum_t a_t d^alpha_t (Sec. 4) on the
    basis exp(i k.x): D_k = sum_t a_t prod_l (i k_l)^alpha_t[l].

    The derivative of exp(i k.x) along axis l is (+i k_l) exp(i k.x); the paper prints
    (-i pi / 2L)^|alpha|, which would be the symbol for the conjugate basis (radians:
    pi / 2L = 1).  alphas: [nterms, d] non-negative integers, coefs: [nterms] reals."""
    alphas = np.asarray(alphas, dtype=np.int64).reshape(-1, d)
    coefs = np.asarray(coefs, dtype=np.float64).reshape(-1)
    ik = 1j * modes(m, d).astype(np.float64)
    D = np.zeros(ik.shape[0], dtype=np.complex128)
    for a, c in zip(alphas, coefs):
        term = np.full(ik.shape[0], c, dtype=np.complex128)
        for ax in range(d):
            term = term * ik[:, ax] ** int(a[ax])
        D += term
    return D


def piml_box_penalty(m: int, d: int, lam: float, mu: float, D: np.ndarray, lo, hi, s: float = 1.0) -> np.ndarray:
    """lambda S^2 + mu D^* C D (Sec. 4, tractable domains): the Sobolev weights 1 + ||k||^(2s) of
    Sec. 3.1 and the Fourier matrix C of the box [lo, hi] (radians) around the operator symbol D."""
    p = sobolev_weights(m, d, s)
    C = piml_box_fourier_matrix(m, lo, hi, L=np.pi / 2)
    return lam * np.diag(p).astype(np.complex128) + mu * (np.conj(D)[:, None] * C * D[None, :])


def heat_symbol(m: int) -> np.ndarray:
    """Diagonal D of the heat operator d_t - d_xx on the basis exp(i (k_t t + k_x x)).

    The derivative of exp(i k.x) is (+i k) exp(i k.x); the paper prints
    (-i pi / 2L)^|alpha|, which would be the symbol for the conjugate basis.
    Modes are ordered (k_t, k_x).  D_k = i k_t - (i k_x)^2 = i k_t + k_x^2."""
    k = modes(m, 2).astype(np.float64)
    return 1j * k[:, 0] + k[:, 1] ** 2


def piml_heat_penalty(m: int, lam: float, mu: float, lo=(-np.pi / 2, -np.pi / 2),
                      hi=(np.pi / 2, np.pi / 2)) -> np.ndarray:
    """lambda S^2 + mu D^* C D (Sec. 4) with s = 1 (S^2 = 1 + ||k||^2) and the
    heat operator on the box [lo, hi] (radians)."""
    p = sobolev_weights(m, 2, 1.0)
    C = piml_box_fourier_matrix(m, lo, hi, L=np.pi / 2)
    D = heat_symbol(m)
    return lam * np.diag(p).astype(np.complex128) + mu * (np.conj(D)[:, None] * C * D[None, :])


def additive_penalty(m: int, d: int, s: float) -> np.ndarray:
    """Block-diagonal Sobolev weights for the additive model, [d(2m+1)]."""
    return np.concatenate([sobolev_weights(m, 1, s)] * d)


def collocation_penalty(Xr: np.ndarray, m: int, mu: float, D: np.ndarray) -> np.ndarray:
    """mu n_r^-1 D^* (Phi_r^* Phi_r) D (Sec. 4, domains without a closed-form Fourier matrix):
    the physics term sampled at the n_r collocation points Xr [d, n_r], for the operator whose
    symbol on exp(i k.x) is the diagonal D [N].  Phi_r^* Phi_r / n_r is the multilevel Toeplitz
    matrix of the collocation points' own generator."""
    from .fourier import gram_generator, toeplitz_matrix
    C = toeplitz_matrix(gram_generator(np.atleast_2d(Xr), m), m)
    return mu * (np.conj(D)[:, None] * C * D[None, :])
