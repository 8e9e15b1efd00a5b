"""Pins for the oracle's Toeplitz product and conjugate-gradient iteration."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("d,m,n", [(1, 4, 37), (2, 2, 23), (3, 1, 11)])
def test_toeplitz_apply_is_design_matrix_product(d, m, n):
    # Sigma x = n^-1 Phi^* (Phi x), with Phi[j, k] = exp(+i k.X_j) built directly from the
    # points: a route that never forms the generator M or indexes differences of modes.
    rng = np.random.default_rng(10 + d)
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    N = (2 * m + 1) ** d
    x = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    Phi = oracle.design_matrix(X, m)
    want = (np.conj(Phi).T @ (Phi @ x.T)).T / n
    M = oracle.gram_generator(X, m)
    np.testing.assert_allclose(oracle.toeplitz_apply(M, x, m), want, atol=1e-12)
    np.testing.assert_allclose(oracle.toeplitz_apply(M, x[1], m), want[1], atol=1e-12)


def test_toeplitz_rows_match_dense_product():
    rng = np.random.default_rng(11)
    for d, m in [(1, 6), (2, 3), (3, 2)]:
        X = rng.uniform(-np.pi, np.pi, size=(d, 17))
        M = oracle.gram_generator(X, m)
        N = (2 * m + 1) ** d
        x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        rows = rng.choice(N, 5, replace=False)
        np.testing.assert_allclose(oracle.toeplitz_apply_rows(M, x, m, rows),
                                   oracle.toeplitz_apply(M, x, m)[rows], atol=1e-13)


def test_toeplitz_apply_planted_transpose_is_caught():
    # Sigma[k, l] = M[l - k]; the transposed reading M[k - l] gives the conjugate matrix,
    # which the design-matrix route tells apart for a non-symmetric sample.
    rng = np.random.default_rng(3)
    X = rng.uniform(0.2, 1.4, size=(2, 9))
    m = 2
    M = oracle.gram_generator(X, m)
    x = rng.standard_normal(25) + 1j * rng.standard_normal(25)
    Phi = oracle.design_matrix(X, m)
    want = np.conj(Phi).T @ (Phi @ x) / 9
    wrong = oracle.toeplitz_matrix(M, m).T @ x
    assert np.abs(wrong - want).max() > 1e-3
    assert np.abs(oracle.toeplitz_apply(M, x, m) - want).max() < 1e-12


def _hpd(N, kappa, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    ev = np.geomspace(1.0, kappa, N)
    return (Q * ev) @ np.conj(Q).T


def test_pcg_reaches_the_direct_solution():
    rng = np.random.default_rng(4)
    N = 40
    A = _hpd(N, 1e4, rng)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    th, it, hist = oracle.pcg(A, b, np.real(np.diag(A)), 1e-13, 400)
    ref = np.linalg.solve(A, b)
    assert hist[-1] <= 1e-13 and it == len(hist) - 1
    assert np.linalg.norm(th - ref) / np.linalg.norm(ref) < 1e-13 * 1e4 * 10


def test_pcg_a_norm_error_decreases_and_residuals_orthogonal():
    # CG minimises the A-norm of the error over growing Krylov spaces: it never increases,
    # and the preconditioned residuals are mutually orthogonal (z_i^* r_j = 0, i != j).
    # A wrong sign in alpha or beta, or a dropped preconditioner, breaks both.
    rng = np.random.default_rng(5)
    N = 30
    A = _hpd(N, 1e3, rng)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ref = np.linalg.solve(A, b)
    dg = np.real(np.diag(A)) * rng.uniform(0.5, 2.0, N)
    errs, rs = [], []
    for k in range(1, 12):
        th, it, _ = oracle.pcg(A, b, dg, 0.0, k)
        e = th - ref
        errs.append(np.real(np.vdot(e, A @ e)))
        rs.append(b - A @ th)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    for i in range(4):
        for j in range(i + 1, 5):
            zi = rs[i] / dg
            assert abs(np.vdot(zi, rs[j])) < 1e-8 * np.linalg.norm(rs[i]) * np.linalg.norm(rs[j]) * 1e3


def test_pcg_special_cases():
    rng = np.random.default_rng(6)
    # diagonal system with the exact Jacobi preconditioner: one iteration
    dgv = rng.uniform(1, 100, 20)
    b = rng.standard_normal(20) + 0j
    th, it, _ = oracle.pcg(np.diag(dgv).astype(complex), b, dgv, 1e-14, 5)
    assert it == 1 and np.allclose(th, b / dgv, rtol=1e-15)
    # identity plus a rank-2 term: the Krylov space is exhausted in at most 3 steps
    U = rng.standard_normal((20, 2)) + 1j * rng.standard_normal((20, 2))
    A = np.eye(20) + U @ np.conj(U).T
    th, it, _ = oracle.pcg(A, b, np.ones(20), 1e-12, 50)
    assert it <= 3 and np.allclose(A @ th, b, atol=1e-11)
    # zero right-hand side: zero solution, no iteration
    th, it, _ = oracle.pcg(A, np.zeros(20, complex), np.ones(20), 1e-12, 50)
    assert it == 0 and not th.any()


def test_collocation_penalty_is_the_sampled_operator_energy():
    # theta^* P theta = mu n_r^-1 sum_l |(d_t - d_xx) f_theta(X_r,l)|^2 for the heat operator, with the
    # derivatives of the oracle's predictor taken by central finite differences at each collocation
    # point (no symbol, no Toeplitz matrix).  Pins the placement D^* C D (not D C D^*) and the sign of
    # the derivative symbol.
    m, nr, mu = 3, 40, 0.7
    rng = np.random.default_rng(12)
    r = np.sqrt(rng.uniform(0, 1, nr)) * 1.2
    a = rng.uniform(0, 2 * np.pi, nr)
    Xr = np.stack([r * np.cos(a), r * np.sin(a)])            # a disk: no closed-form Fourier matrix used
    N = (2 * m + 1) ** 2
    th = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    th = 0.5 * (th + np.conj(th[::-1]))                      # real-valued f
    P = oracle.collocation_penalty(Xr, m, mu, oracle.heat_symbol(m))
    quad = np.real(np.conj(th) @ P @ th)
    f = lambda t, x: oracle.predict(th, np.stack([t, x]), m).real
    h1, h2 = 1e-5, 1e-3
    t, x = Xr
    ft = (f(t + h1, x) - f(t - h1, x)) / (2 * h1)
    fxx = (f(t, x + h2) - 2 * f(t, x) + f(t, x - h2)) / h2 ** 2
    want = mu * np.mean((ft - fxx) ** 2)
    assert abs(quad - want) / want < 1e-5
    # the conjugate placement D C D^* gives a different value for this sample
    D = oracle.heat_symbol(m)
    wrong = np.real(np.conj(th) @ (mu * D[:, None] * oracle.toeplitz_matrix(oracle.gram_generator(Xr, m), m)
                                   * np.conj(D)[None, :]) @ th)
    assert abs(wrong - want) / want > 1e-3


def test_predict_3d_small_is_the_explicit_sum():
    # the oracle's axis-by-axis contraction against a plain loop over the 27 modes of m = 1
    rng = np.random.default_rng(13)
    th = rng.standard_normal(27) + 1j * rng.standard_normal(27)
    Xq = rng.uniform(-np.pi, np.pi, (3, 5))
    want = np.zeros(5, complex)
    for i, k in enumerate(oracle.modes(1, 3)):
        want += th[i] * np.exp(1j * (k @ Xq))
    np.testing.assert_allclose(oracle.predict(th, Xq, 1), want, atol=1e-13)
