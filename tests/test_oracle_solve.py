"""Pins for the oracle's penalties, solve, prediction and gradients."""
import numpy as np
import pytest
from scipy import integrate

import oracle


# ---------------------------------------------------------------- penalties

def test_sobolev_weights_closed_form():
    p = oracle.sobolev_weights(2, 2, 2.0).reshape(5, 5)
    # k = (1, 1): 1 + (sqrt 2)^4 = 5 ; k = (2, 0): 1 + 2^4 = 17 ; k = (0, 0): 1
    assert p[3, 3] == 5.0 and p[4, 2] == 17.0 and p[2, 2] == 1.0
    pb = oracle.sobolev_bessel_weights(2, 2, 2.0).reshape(5, 5)
    assert pb[3, 3] == 9.0 and pb[4, 2] == 25.0
    # s = 1: the two forms agree
    np.testing.assert_array_equal(oracle.sobolev_weights(3, 2, 1.0), oracle.sobolev_bessel_weights(3, 2, 1.0))


def test_box_fourier_matrix_against_quadrature():
    m = 2
    lo, hi = (-np.pi / 2, -np.pi / 2), (np.pi / 2, np.pi / 2)
    C = oracle.piml_box_fourier_matrix(m, lo, hi, L=np.pi / 2)
    ks = oracle.modes(m, 2)
    rng = np.random.default_rng(0)
    for _ in range(6):
        i, j = rng.integers(0, ks.shape[0], 2)
        q = ks[i] - ks[j]
        re = integrate.dblquad(lambda y, x: np.cos(q[0] * x + q[1] * y), lo[0], hi[0], lo[1], hi[1])[0]
        im = integrate.dblquad(lambda y, x: np.sin(q[0] * x + q[1] * y), lo[0], hi[0], lo[1], hi[1])[0]
        assert abs(C[i, j] - (re + 1j * im) / (2 * np.pi) ** 2) < 1e-10
    # the symmetric box gives a real symmetric matrix with the sinc closed form
    q = ks[:, None, :] - ks[None, :, :]
    sinc = lambda t: np.where(t == 0, np.pi, 2 * np.sin(t * np.pi / 2) / np.where(t == 0, 1, t))
    np.testing.assert_allclose(C, sinc(q[..., 0]) * sinc(q[..., 1]) / (2 * np.pi) ** 2, atol=1e-14)


def test_heat_penalty_quadratic_form_against_quadrature():
    # theta^* (D^* C D) theta = (2 pi)^-2 int_box |d_t f - d_xx f|^2 for f = f_theta,
    # with the derivatives taken by finite differences of the oracle's predictor.
    # This pins the sign of the derivative symbol (+i k).
    m = 2
    rng = np.random.default_rng(1)
    N = (2 * m + 1) ** 2
    th = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    th = 0.5 * (th + np.conj(th[::-1]))      # real-valued f
    P = oracle.piml_heat_penalty(m, lam=0.0, mu=1.0)
    quad_form = np.real(np.conj(th) @ P @ th)
    xg, wg = np.polynomial.legendre.leggauss(40)
    t = xg * np.pi / 2
    x = xg * np.pi / 2
    T, Xx = np.meshgrid(t, x, indexing="ij")
    W = np.outer(wg, wg) * (np.pi / 2) ** 2
    f = lambda tt, xx: oracle.predict(th, np.stack([tt.ravel(), xx.ravel()]), m).real.reshape(tt.shape)
    h1, h2 = 1e-4, 1e-3
    ft = (f(T + h1, Xx) - f(T - h1, Xx)) / (2 * h1)
    fxx = (f(T, Xx + h2) - 2 * f(T, Xx) + f(T, Xx - h2)) / h2 ** 2
    integral = np.sum(W * (ft - fxx) ** 2) / (2 * np.pi) ** 2
    assert abs(integral - quad_form) / quad_form < 1e-5
    # the conjugate symbol (-i k), as printed, gives the backward heat operator instead
    Dbad = -1j * oracle.modes(m, 2)[:, 0] + oracle.modes(m, 2)[:, 1] ** 2
    C = oracle.piml_box_fourier_matrix(m, (-np.pi / 2,) * 2, (np.pi / 2,) * 2, L=np.pi / 2)
    bad = np.real(np.conj(th) @ (np.conj(Dbad)[:, None] * C * Dbad[None, :]) @ th)
    assert abs(bad - integral) / integral > 1e-3


# ---------------------------------------------------------------- solve

@pytest.mark.parametrize("d,m,n", [(1, 6, 120), (2, 2, 150)])
def test_normal_equations_match_kernel_ridge_regression(d, m, n):
    rng = np.random.default_rng(2 + d)
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    Y = np.sin(X[0]) + 0.3 * rng.standard_normal(n)
    p = oracle.sobolev_weights(m, d, 1.5)
    lam = 1e-3
    theta, M, b = oracle.fit(X, Y[None, :], m, lam, p)
    theta_krr = oracle.krr_theta(X, Y, m, lam, p)
    np.testing.assert_allclose(theta[0], theta_krr, rtol=0, atol=1e-10 * np.abs(theta_krr).max())


def test_exact_recovery_of_trigonometric_polynomial():
    rng = np.random.default_rng(4)
    m, n = 10, 400
    X = rng.uniform(-np.pi, np.pi, size=(1, n))
    Y = np.sin(3 * X[0]) + 0.5 * np.cos(7 * X[0])
    p = oracle.sobolev_weights(m, 1, 1.0)
    theta, _, _ = oracle.fit(X, Y[None, :], m, 1e-13, p)
    ref = np.zeros(2 * m + 1, dtype=complex)
    ref[m + 3], ref[m - 3] = -0.5j, 0.5j
    ref[m + 7], ref[m - 7] = 0.25, 0.25
    np.testing.assert_allclose(theta[0], ref, atol=1e-8)


def test_solution_is_hermitian_and_residual_small():
    rng = np.random.default_rng(5)
    m, d, n = 4, 2, 2000
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    Y = np.exp(-(X ** 2).sum(0)) + 0.1 * rng.standard_normal(n)
    p = oracle.sobolev_weights(m, d, 2.0)
    theta, M, b = oracle.fit(X, Y[None, :], m, 1e-3, p)
    np.testing.assert_allclose(theta[0][::-1], np.conj(theta[0]), atol=1e-12)
    A = oracle.system_matrix(M, m, 1e-3, p)
    assert np.abs(A @ theta[0] - b[0]).max() < 1e-13
    assert oracle.condition_number(A) > 1.0


def test_piml_system_matches_direct_minimization():
    # The PIML estimator minimises n^-1 |Phi th - Y|^2 + th^* Q th; check the
    # normal-equation solution against a least-squares solve of the stacked system.
    rng = np.random.default_rng(6)
    m, n = 2, 300
    X = rng.uniform(-np.pi / 2, np.pi / 2, size=(2, n))
    Y = np.exp(-X[0]) * np.sin(X[1])
    Q = oracle.piml_heat_penalty(m, lam=1e-3, mu=1e-2)
    theta, M, b = oracle.fit(X, Y[None, :], m, 0.0, Q)
    Phi = oracle.design_matrix(X, m)
    Lq = np.linalg.cholesky(Q)
    stacked = np.concatenate([Phi / np.sqrt(n), np.conj(Lq).T])
    rhs_ = np.concatenate([Y / np.sqrt(n), np.zeros(Q.shape[0])])
    th_ls = np.linalg.lstsq(stacked, rhs_, rcond=None)[0]
    np.testing.assert_allclose(theta[0], th_ls, atol=1e-9)


# ---------------------------------------------------------------- predict

@pytest.mark.parametrize("d,m", [(1, 5), (2, 3), (3, 2)])
def test_predict_matches_design_matrix(d, m):
    rng = np.random.default_rng(10 + d)
    N = (2 * m + 1) ** d
    th = rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))
    Xq = rng.uniform(-np.pi, np.pi, size=(d, 77))
    f = oracle.predict(th, Xq, m)
    ref = (oracle.design_matrix(Xq, m) @ th.T).T
    np.testing.assert_allclose(f, ref, atol=1e-12)


def test_predict_type2_type1_energy_identities():
    rng = np.random.default_rng(12)
    m, d, n = 3, 2, 500
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    Y = rng.standard_normal(n)
    N = (2 * m + 1) ** d
    th = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    th = 0.5 * (th + np.conj(th[::-1]))
    f = oracle.predict(th, X, m)
    M = oracle.gram_generator(X, m)
    b = oracle.rhs(X, Y[None, :], m)[0]
    T = oracle.toeplitz_matrix(M, m)
    assert abs(np.mean(np.abs(f) ** 2) - np.real(np.conj(th) @ T @ th)) < 1e-12
    assert abs(np.mean(Y * f.real) - np.real(np.conj(b) @ th)) < 1e-12
    assert np.abs(f.imag).max() < 1e-12


def test_predict_additive():
    rng = np.random.default_rng(13)
    d, m = 3, 2
    L = 2 * m + 1
    th = rng.standard_normal(d * L) + 1j * rng.standard_normal(d * L)
    Xq = rng.uniform(-np.pi, np.pi, size=(d, 50))
    Phi = np.concatenate([oracle.design_matrix(Xq[a:a + 1], m) for a in range(d)], axis=1)
    np.testing.assert_allclose(oracle.predict_additive(th, Xq, m), Phi @ th, atol=1e-12)


# ---------------------------------------------------------------- gradients

def _setup(seed=20):
    rng = np.random.default_rng(seed)
    m, d, n, nv = 3, 2, 600, 400
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    Xv = rng.uniform(-np.pi, np.pi, size=(d, nv))
    f = lambda x: np.sin(2 * x[0]) * np.cos(x[1])
    Y = f(X) + 0.1 * rng.standard_normal(n)
    Yv = f(Xv) + 0.1 * rng.standard_normal(nv)
    M = oracle.gram_generator(X, m)
    b = oracle.rhs(X, Y[None, :], m)[0]
    Mv = oracle.gram_generator(Xv, m)
    bv = oracle.rhs(Xv, Yv[None, :], m)[0]
    p = oracle.sobolev_weights(m, d, 2.0)
    return m, Xv, Yv, M, b, Mv, bv, p


def _loss(m, M, b, Mv, bv, yv2, lam, p):
    A = oracle.system_matrix(M, m, lam, p)
    th = oracle.solve_system(A, b)
    return oracle.heldout_mse_quadratic(th[None, :], Mv, bv[None, :], yv2, m)[0]


def test_two_mse_routes_agree():
    m, Xv, Yv, M, b, Mv, bv, p = _setup()
    A = oracle.system_matrix(M, m, 1e-2, p)
    th = oracle.solve_system(A, b)
    l1 = oracle.heldout_mse(th[None, :], Xv, Yv[None, :], m)[0]
    l2 = oracle.heldout_mse_quadratic(th[None, :], Mv, bv[None, :], np.mean(Yv ** 2), m)[0]
    assert abs(l1 - l2) < 1e-12


def test_gradients_against_central_differences():
    m, Xv, Yv, M, b, Mv, bv, p = _setup()
    yv2 = np.mean(Yv ** 2)
    lam = 3e-2
    A = oracle.system_matrix(M, m, lam, p)
    th = oracle.solve_system(A, b)
    dll, dp, g = oracle.mse_gradients(A, th, p, lam, Mv, bv, m)
    h = 1e-3
    fd = (_loss(m, M, b, Mv, bv, yv2, lam * np.exp(h), p) -
          _loss(m, M, b, Mv, bv, yv2, lam * np.exp(-h), p)) / (2 * h)
    assert abs(fd - dll) <= 1e-5 * abs(dll) + 1e-12
    for k in [0, 5, 24, 30]:
        e = np.zeros_like(p)
        e[k] = 1e-4 * p[k]
        fdp = (_loss(m, M, b, Mv, bv, yv2, lam, p + e) - _loss(m, M, b, Mv, bv, yv2, lam, p - e)) / (2e-4 * p[k])
        assert abs(fdp - dp[k]) <= 1e-5 * np.abs(dp).max()
    # Wirtinger: dL = 2 Re(g^* dtheta) for an arbitrary complex direction
    rng = np.random.default_rng(3)
    dth = rng.standard_normal(th.size) + 1j * rng.standard_normal(th.size)
    Lq = lambda t: oracle.heldout_mse_quadratic(t[None, :], Mv, bv[None, :], yv2, m)[0]
    eps = 1e-6
    fdt = (Lq(th + eps * dth) - Lq(th - eps * dth)) / (2 * eps)
    assert abs(fdt - 2 * np.real(np.conj(g) @ dth)) < 1e-7 * max(1.0, abs(fdt))
