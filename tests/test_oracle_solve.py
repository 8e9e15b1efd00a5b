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
    ks = oracle.modes(m, 2)
    rng = np.random.default_rng(0)
    # entries: (2 pi)^-2 int_box exp(i <l - k, x>) dx, on the centred box and on an off-centre one
    for lo, hi in [((-np.pi / 2, -np.pi / 2), (np.pi / 2, np.pi / 2)), ((-0.4, 0.1), (1.3, 2.0))]:
        C = oracle.piml_box_fourier_matrix(m, lo, hi, L=np.pi / 2)
        for _ in range(6):
            i, j = rng.integers(0, ks.shape[0], 2)
            q = ks[j] - ks[i]
            re = integrate.dblquad(lambda y, x: np.cos(q[0] * x + q[1] * y), lo[0], hi[0], lo[1], hi[1])[0]
            im = integrate.dblquad(lambda y, x: np.sin(q[0] * x + q[1] * y), lo[0], hi[0], lo[1], hi[1])[0]
            assert abs(C[i, j] - (re + 1j * im) / (2 * np.pi) ** 2) < 1e-10
    # theta^* C theta is the box integral of |f_theta|^2 (the identity the estimator of Sec. 4 needs),
    # by Gauss-Legendre quadrature of the oracle's predictor on the off-centre box
    th = rng.standard_normal(ks.shape[0]) + 1j * rng.standard_normal(ks.shape[0])
    lo, hi = (-0.4, 0.1), (1.3, 2.0)
    C = oracle.piml_box_fourier_matrix(m, lo, hi, L=np.pi / 2)
    xg, wg = np.polynomial.legendre.leggauss(30)
    a = [0.5 * (hi[i] - lo[i]) * xg + 0.5 * (hi[i] + lo[i]) for i in range(2)]
    W = np.outer(0.5 * (hi[0] - lo[0]) * wg, 0.5 * (hi[1] - lo[1]) * wg)
    T, Xx = np.meshgrid(a[0], a[1], indexing="ij")
    f = oracle.predict(th, np.stack([T.ravel(), Xx.ravel()]), m).reshape(T.shape)
    assert abs(np.sum(W * np.abs(f) ** 2) / (2 * np.pi) ** 2 - np.real(np.conj(th) @ C @ th)) < 1e-12
    # the symmetric box gives a real symmetric matrix with the sinc closed form
    C = oracle.piml_box_fourier_matrix(m, (-np.pi / 2, -np.pi / 2), (np.pi / 2, np.pi / 2), L=np.pi / 2)
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


# ---------------------------------------------------------------- condition number and additive penalty

def _unitary(n, seed):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    return Q * (np.diag(R) / np.abs(np.diag(R)))[None, :]


def test_condition_number_of_known_spectrum():
    # diagonal: the ratio of the extreme entries, whatever their order
    assert oracle.condition_number(np.diag([3.0, 0.5, 12.0, 2.0])) == pytest.approx(24.0, rel=1e-14)
    # Q diag(ev) Q^* with the spectrum 10^linspace(0, 4): kappa = 1e4 exactly, and no diagonal
    # entry or Gershgorin bound gives it (a ratio of diagonal entries would read far less)
    ev = 10.0 ** np.linspace(0.0, 4.0, 24)
    Q = _unitary(24, 7)
    A = (Q * ev[None, :]) @ np.conj(Q).T
    A = 0.5 * (A + np.conj(A).T)
    assert oracle.condition_number(A) == pytest.approx(1e4, rel=1e-9)
    dg = np.real(np.diag(A))
    assert dg.max() / dg.min() < 1e3
    # scaling leaves it unchanged; the inverse has the same condition number
    assert oracle.condition_number(5.0 * A) == pytest.approx(1e4, rel=1e-9)
    assert oracle.condition_number(np.linalg.inv(A)) == pytest.approx(1e4, rel=1e-8)


def test_condition_number_of_the_2d_sobolev_system_brackets_the_weights():
    # Sigma of equispaced points on the torus is the identity (M = delta), so
    # kappa(I + lambda diag(p)) = (1 + lambda p_max) / (1 + lambda p_min) exactly
    m, d, s, lam = 3, 2, 2.0, 1e-2
    g = np.arange(16) * (2 * np.pi / 16) - np.pi
    X = np.stack([np.repeat(g, 16), np.tile(g, 16)])
    M = oracle.gram_generator(X, m)
    p = oracle.sobolev_weights(m, d, s)
    A = oracle.system_matrix(M, m, lam, p)
    assert oracle.condition_number(A) == pytest.approx((1 + lam * p.max()) / (1 + lam * p.min()), rel=1e-10)


def test_additive_penalty_closed_form_in_block_order():
    # one block of Sobolev weights 1 + |k|^(2s), k = -m..m, per component, components in order
    np.testing.assert_array_equal(oracle.additive_penalty(2, 3, 1.5), np.array([9.0, 2.0, 1.0, 2.0, 9.0] * 3))
    np.testing.assert_array_equal(oracle.additive_penalty(2, 2, 1.0), np.array([5.0, 2.0, 1.0, 2.0, 5.0] * 2))
    np.testing.assert_array_equal(oracle.additive_penalty(1, 4, 0.0), np.full(12, 2.0))


def test_additive_penalty_is_the_sum_of_component_sobolev_norms():
    # theta^* diag(p) theta = sum_a (2 pi)^-1 int |f_a|^2 + |f_a'|^2 dx (s = 1), for
    # f_a(x) = sum_k theta_{a,k} exp(i k x); the derivative is taken by central differences
    rng = np.random.default_rng(8)
    d, m = 3, 4
    L = 2 * m + 1
    th = rng.standard_normal(d * L) + 1j * rng.standard_normal(d * L)
    quad = np.real(np.conj(th) @ (oracle.additive_penalty(m, d, 1.0) * th))
    xg, wg = np.polynomial.legendre.leggauss(64)
    x = np.pi * xg
    h = 1e-5
    total = 0.0
    for a in range(d):
        f = lambda u: oracle.predict(th[a * L:(a + 1) * L], u[None, :], m)
        fp = (f(x + h) - f(x - h)) / (2 * h)
        total += np.sum(np.pi * wg * (np.abs(f(x)) ** 2 + np.abs(fp) ** 2)) / (2 * np.pi)
    assert abs(total - quad) / quad < 1e-8


# ---------------------------------------------------------------- general operators on a box

def _box_integral_of_operator(th, m, d, lo, hi, apply_op, npts=48):
    """(2 pi)^-d int_box |op f_theta|^2 by Gauss-Legendre quadrature, op applied by finite differences."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    axes = [0.5 * (hi[a] - lo[a]) * xg + 0.5 * (hi[a] + lo[a]) for a in range(d)]
    wts = [0.5 * (hi[a] - lo[a]) * wg for a in range(d)]
    grid = np.meshgrid(*axes, indexing="ij")
    W = wts[0] if d == 1 else np.outer(wts[0], wts[1])
    f = lambda *u: oracle.predict(th, np.stack([g.ravel() for g in u]), m).reshape(u[0].shape)
    v = apply_op(f, *grid)
    return np.sum(W * np.abs(v) ** 2) / (2 * np.pi) ** d


def test_pde_symbol_reduces_to_the_heat_symbol():
    np.testing.assert_array_equal(oracle.pde_symbol(3, 2, [[1, 0], [0, 2]], [1.0, -1.0]), oracle.heat_symbol(3))


@pytest.mark.parametrize("case", ["1d_paper", "2d_mixed"])
def test_pde_box_penalty_quadratic_form_against_quadrature(case):
    rng = np.random.default_rng(30)
    if case == "1d_paper":
        # the paper's one-dimensional constraint f' - f = 0 on Omega = ]0, 1[ (L = pi/2: radians = x)
        d, m, lo, hi = 1, 6, (0.0,), (1.0,)
        alphas, coefs = [[1], [0]], [1.0, -1.0]
        h = 1e-5
        op = lambda f, x: (f(x + h) - f(x - h)) / (2 * h) - f(x)
    else:
        # d_t d_x + 0.5 d_xx + d_t - 2 on an off-centre box
        d, m, lo, hi = 2, 3, (-1.0, -0.3), (0.5, 1.2)
        alphas, coefs = [[1, 1], [0, 2], [1, 0], [0, 0]], [1.0, 0.5, 1.0, -2.0]
        h = 1e-3
        op = lambda f, t, x: ((f(t + h, x + h) - f(t + h, x - h) - f(t - h, x + h) + f(t - h, x - h)) / (4 * h * h)
                              + 0.5 * (f(t, x + h) - 2 * f(t, x) + f(t, x - h)) / (h * h)
                              + (f(t + h, x) - f(t - h, x)) / (2 * h) - 2 * f(t, x))
    N = (2 * m + 1) ** d
    th = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    th = 0.5 * (th + np.conj(th[::-1]))          # a real function
    D = oracle.pde_symbol(m, d, alphas, coefs)
    P = oracle.piml_box_penalty(m, d, 0.0, 1.0, D, lo, hi)
    quad_form = np.real(np.conj(th) @ P @ th)
    integral = _box_integral_of_operator(th, m, d, lo, hi, op)
    assert abs(integral - quad_form) / quad_form < 2e-5
    # the printed sign of the symbol (-i k) gives another operator (odd derivatives flip)
    Dbad = oracle.pde_symbol(m, d, alphas, [c * (-1) ** int(np.sum(a)) for a, c in zip(alphas, coefs)])
    bad = np.real(np.conj(th) @ oracle.piml_box_penalty(m, d, 0.0, 1.0, Dbad, lo, hi) @ th)
    assert abs(bad - integral) / integral > 1e-3


def test_pde_box_system_matches_direct_minimization():
    # Sec. 4: theta-hat minimises n^-1 |Phi th - Y|^2 + lambda |S th|^2 + mu int_Omega |D f|^2 (scaled
    # by (2 pi)^-d); compare the normal equations with a least-squares solve of the stacked system.
    rng = np.random.default_rng(31)
    m, n, lam, mu = 5, 400, 1e-3, 1.0
    X = rng.uniform(0.0, 1.0, size=(1, n))
    Y = np.exp(X[0]) + rng.standard_normal(n)
    D = oracle.pde_symbol(m, 1, [[1], [0]], [1.0, -1.0])
    Q = oracle.piml_box_penalty(m, 1, lam, mu, D, (0.0,), (1.0,), s=1.0)
    theta, M, b = oracle.fit(X, Y[None, :], m, 0.0, Q)
    Phi = oracle.design_matrix(X, m)
    Lq = np.linalg.cholesky(Q)
    stacked = np.concatenate([Phi / np.sqrt(n), np.conj(Lq).T])
    rhs_ = np.concatenate([Y / np.sqrt(n), np.zeros(Q.shape[0])])
    th_ls = np.linalg.lstsq(stacked, rhs_, rcond=None)[0]
    np.testing.assert_allclose(theta[0], th_ls, atol=1e-9 * np.abs(th_ls).max())


def test_theta_path_gradients_against_central_differences():
    # a loss of theta alone, E(theta) = Re(c^* theta) + |theta_j|^2, through theta(lambda, p) = A^-1 b
    m, Xv, Yv, M, b, Mv, bv, p = _setup(24)
    rng = np.random.default_rng(25)
    N = p.size
    c = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    j = 7
    E = lambda th: np.real(np.conj(c) @ th) + abs(th[j]) ** 2
    lam = 2e-2
    A = oracle.system_matrix(M, m, lam, p)
    th = oracle.solve_system(A, b)
    G = 0.5 * c
    G[j] += th[j]                        # Wirtinger gradient of E with respect to conj(theta)
    dll, dp = oracle.theta_path_gradients(A, th, p, lam, G)
    th_at = lambda lm, pp: oracle.solve_system(oracle.system_matrix(M, m, lm, pp), b)
    h = 1e-4
    fd = (E(th_at(lam * np.exp(h), p)) - E(th_at(lam * np.exp(-h), p))) / (2 * h)
    assert abs(fd - dll) <= 1e-7 * max(1.0, abs(dll))
    for k in [0, 11, 24, 40]:
        e = np.zeros_like(p)
        e[k] = 1e-5 * p[k]
        fdp = (E(th_at(lam, p + e)) - E(th_at(lam, p - e))) / (2e-5 * p[k])
        assert abs(fdp - dp[k]) <= 1e-6 * np.abs(dp).max()
    # the mse gradients are the special case G = g (held-out Wirtinger gradient)
    dll2, dp2, g = oracle.mse_gradients(A, th, p, lam, Mv, bv, m)
    a, bb = oracle.theta_path_gradients(A, th, p, lam, g)
    assert a == pytest.approx(dll2, rel=1e-12) and np.allclose(bb, dp2, rtol=1e-12, atol=0)


def test_mse_theta_gradient_along_hermitian_directions():
    # the library reports dL/dconj(theta) = g; along Hermitian-symmetric directions (the only ones a
    # real fit moves in) the directional derivative of the held-out loss is 2 Re(g^* dtheta)
    m, Xv, Yv, M, b, Mv, bv, p = _setup(26)
    A = oracle.system_matrix(M, m, 1e-2, p)
    th = oracle.solve_system(A, b)
    _, _, g = oracle.mse_gradients(A, th, p, 1e-2, Mv, bv, m)
    rng = np.random.default_rng(27)
    yv2 = np.mean(Yv ** 2)
    for _ in range(3):
        dth = rng.standard_normal(th.size) + 1j * rng.standard_normal(th.size)
        dth = 0.5 * (dth + np.conj(dth[::-1]))
        eps = 1e-5
        Lp = oracle.heldout_mse(th + eps * dth, Xv, Yv[None, :], m)[0]
        Lm = oracle.heldout_mse(th - eps * dth, Xv, Yv[None, :], m)[0]
        assert abs((Lp - Lm) / (2 * eps) - 2 * np.real(np.conj(g) @ dth)) < 1e-7
    del yv2
