"""Normal-equation solve of eq. (kenrel_reg) (oracle; test infrastructure only)."""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fourier import gram_generator, rhs, toeplitz_matrix


def system_matrix(M: np.ndarray, m: int, lam: float, P: np.ndarray) -> np.ndarray:
    """A = Sigma + lambda P with Sigma[k, l] = M[l - k] (Sec. 2.3).

    P is either the diagonal weights [N] (Sobolev / low-bias) or a dense
    Hermitian matrix [N, N] that already includes its own scale (PIML)."""
    A = toeplitz_matrix(M, m).astype(np.complex128)
    if P.ndim == 1:
        A[np.diag_indices_from(A)] += lam * P
    else:
        A += P
    return A


def solve_system(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """theta = A^-1 b by FP64 LAPACK Cholesky (zpotrf/zpotrs). b is [T, N] or [N]."""
    c = sla.cho_factor(A, lower=True, check_finite=True)
    rhs_ = np.atleast_2d(b).T
    x = sla.cho_solve(c, rhs_)
    return x.T if b.ndim == 2 else x[:, 0]


def condition_number(A: np.ndarray) -> float:
    """2-norm condition number of the Hermitian matrix A."""
    ev = np.linalg.eigvalsh(A)
    return float(ev[-1] / ev[0])


def fit(X: np.ndarray, Y: np.ndarray, m: int, lam: float, P: np.ndarray):
    """theta-hat of eq. (kenrel_reg) from data: returns (theta [T, N], M, b)."""
    M = gram_generator(X, m)
    b = rhs(X, Y, m)
    A = system_matrix(M, m, lam, P)
    return solve_system(A, b), M, b
