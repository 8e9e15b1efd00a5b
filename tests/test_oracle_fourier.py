"""Pins for the oracle's direct Fourier sums (Sec. 2.3): closed forms, a different
library routine (numpy.fft), a 40-digit mpmath sum, invariants and statistics."""
import mpmath
import numpy as np
import pytest

import oracle
from oracle import fourier


def _q(m, d):
    return oracle.modes(2 * m, d)


def test_single_point_closed_forms_1d():
    m = 5
    q = np.arange(-2 * m, 2 * m + 1)
    # x0 = 0: all ones
    M = oracle.gram_generator(np.zeros((1, 1)), m)
    np.testing.assert_allclose(M, np.ones_like(M), atol=1e-15)
    # x0 = -pi: (-1)^q
    M = oracle.gram_generator(np.full((1, 1), -np.pi), m)
    np.testing.assert_allclose(M, (-1.0) ** q, atol=1e-13)
    # x0 = pi/2: i^q (pins the + sign of the generator)
    M = oracle.gram_generator(np.full((1, 1), np.pi / 2), m)
    np.testing.assert_allclose(M, 1j ** q, atol=1e-13)


def test_single_point_closed_forms_2d():
    m = 3
    X = np.array([[np.pi / 2], [-np.pi]])
    M = oracle.gram_generator(X, m)
    q1, q2 = np.meshgrid(np.arange(-2 * m, 2 * m + 1), np.arange(-2 * m, 2 * m + 1), indexing="ij")
    np.testing.assert_allclose(M, (1j ** q1) * (-1.0) ** q2, atol=1e-13)
    # b with Y = 1 at x0 = pi/2 (dim 0): exp(-i k pi/2) = (-i)^k1 * (-1)^k2 (pins the - sign)
    b = oracle.rhs(X, np.ones((1, 1)), m)[0].reshape(2 * m + 1, 2 * m + 1)
    k1, k2 = np.meshgrid(np.arange(-m, m + 1), np.arange(-m, m + 1), indexing="ij")
    np.testing.assert_allclose(b, ((-1j) ** k1) * (-1.0) ** k2, atol=1e-13)


def test_equispaced_points_give_delta_and_fft():
    # x_j = -pi + 2 pi j / n with n > 4m: M = delta_{q,0}; b = (-1)^k FFT(Y)[k mod n] / n
    m, n = 6, 37
    x = -np.pi + 2 * np.pi * np.arange(n) / n
    M = oracle.gram_generator(x[None, :], m)
    delta = np.zeros(4 * m + 1)
    delta[2 * m] = 1.0
    np.testing.assert_allclose(M, delta, atol=1e-13)
    rng = np.random.default_rng(0)
    Y = rng.standard_normal(n)
    b = oracle.rhs(x[None, :], Y[None, :], m)[0]
    F = np.fft.fft(Y)
    k = np.arange(-m, m + 1)
    np.testing.assert_allclose(b, (-1.0) ** k * F[k % n] / n, atol=1e-13)


def test_equispaced_tensor_grid_2d_fft2():
    m, n1 = 3, 13
    g = -np.pi + 2 * np.pi * np.arange(n1) / n1
    G1, G2 = np.meshgrid(g, g, indexing="ij")
    X = np.stack([G1.ravel(), G2.ravel()])
    M = oracle.gram_generator(X, m)
    ref = np.zeros_like(M)
    ref[2 * m, 2 * m] = 1.0
    np.testing.assert_allclose(M, ref, atol=1e-13)
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((n1, n1))
    b = oracle.rhs(X, Y.ravel()[None, :], m)[0].reshape(2 * m + 1, 2 * m + 1)
    F = np.fft.fft2(Y)
    k = np.arange(-m, m + 1)
    K1, K2 = np.meshgrid(k, k, indexing="ij")
    np.testing.assert_allclose(b, (-1.0) ** (K1 + K2) * F[K1 % n1, K2 % n1] / n1 ** 2, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2])
def test_mpmath_40_digit_sum(d):
    mpmath.mp.dps = 40
    rng = np.random.default_rng(2 + d)
    n, m = 7, 3
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    Y = rng.standard_normal(n)
    M = oracle.gram_generator(X, m).ravel()
    b = oracle.rhs(X, Y[None, :], m)[0]
    for qi, q in enumerate(oracle.modes(2 * m, d)):
        s = mpmath.fsum(mpmath.expj(sum(int(q[a]) * mpmath.mpf(float(X[a, j])) for a in range(d)))
                        for j in range(n)) / n
        assert abs(complex(s) - M[qi]) < 1e-14
    for ki, k in enumerate(oracle.modes(m, d)):
        s = mpmath.fsum(mpmath.mpf(float(Y[j])) *
                        mpmath.expj(-sum(int(k[a]) * mpmath.mpf(float(X[a, j])) for a in range(d)))
                        for j in range(n)) / n
        assert abs(complex(s) - b[ki]) < 1e-14


def test_invariants_hermitian_bounded_psd_rank():
    rng = np.random.default_rng(5)
    m, d, n = 3, 2, 20                        # N = 49 > n
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    M = oracle.gram_generator(X, m)
    assert abs(M[2 * m, 2 * m] - 1.0) < 1e-15
    np.testing.assert_allclose(M[::-1, ::-1], np.conj(M), atol=1e-15)
    assert np.abs(M).max() <= 1.0 + 1e-14
    T = oracle.toeplitz_matrix(M, m)
    np.testing.assert_allclose(T, np.conj(T).T, atol=1e-15)
    ev = np.linalg.eigvalsh(T)
    assert ev.min() > -1e-12
    assert (ev > 1e-10).sum() == n            # rank = n exactly for n < N generic points
    # T equals Phi^* Phi / n from the explicit design matrix
    Phi = oracle.design_matrix(X, m)
    np.testing.assert_allclose(T, np.conj(Phi).T @ Phi / n, atol=1e-13)


def test_rhs_of_ones_is_reflected_generator_and_linear():
    rng = np.random.default_rng(6)
    m, d, n = 4, 2, 300
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    M = oracle.gram_generator(X, m)
    b1 = oracle.rhs(X, np.ones((1, n)), m)[0].reshape(2 * m + 1, 2 * m + 1)
    # b(Y = 1)_k = M[-k]
    Mk = M[m:3 * m + 1, m:3 * m + 1]
    np.testing.assert_allclose(b1, Mk[::-1, ::-1], atol=1e-14)
    Y = rng.standard_normal((2, n))
    b = oracle.rhs(X, Y, m)
    bl = oracle.rhs(X, (2.0 * Y[0] - 3.0 * Y[1])[None, :], m)[0]
    np.testing.assert_allclose(bl, 2.0 * b[0] - 3.0 * b[1], atol=1e-13)
    # real Y: b_{-k} = conj b_k
    np.testing.assert_allclose(b[0][::-1], np.conj(b[0]), atol=1e-14)


def test_uniform_sample_statistics():
    # For U[-pi, pi)^d and q != 0: E M[q] = 0 and n E|M[q]|^2 = 1 exactly.
    rng = np.random.default_rng(7)
    m, d, n, reps = 4, 2, 400, 30
    vals = []
    for _ in range(reps):
        X = rng.uniform(-np.pi, np.pi, size=(d, n))
        M = oracle.gram_generator(X, m).ravel()
        M = np.delete(M, M.size // 2)
        vals.append(n * np.abs(M) ** 2)
    v = np.mean(vals)
    assert abs(v - 1.0) < 0.05


def test_planted_sign_error_is_caught():
    # The '+' sign in the right-hand side (the sign printed in the paper's display)
    # is conj(b) for real Y; the FFT pin above rejects it.
    m, n = 6, 37
    x = -np.pi + 2 * np.pi * np.arange(n) / n
    Y = np.random.default_rng(8).standard_normal(n)
    b_plus = np.conj(oracle.rhs(x[None, :], Y[None, :], m)[0])
    F = np.fft.fft(Y)
    k = np.arange(-m, m + 1)
    assert np.abs(b_plus - (-1.0) ** k * F[k % n] / n).max() > 1e-2


def test_powers_recurrence_matches_direct_exp():
    x = np.random.default_rng(9).uniform(-2 * np.pi, 2 * np.pi, 1000)
    E = fourier._powers(x, 64)
    q = np.arange(-64, 65)
    np.testing.assert_allclose(E, np.exp(1j * np.outer(x, q)), atol=1e-13)


def test_additive_blocks_match_stacked_design_matrix():
    rng = np.random.default_rng(10)
    d, m, n = 4, 3, 150
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    Y = rng.standard_normal(n)
    Phi = np.concatenate([oracle.design_matrix(X[a:a + 1], m) for a in range(d)], axis=1)
    B = oracle.additive_blocks(X, m)
    np.testing.assert_allclose(B, np.conj(Phi).T @ Phi / n, atol=1e-13)
    r = oracle.additive_rhs(X, Y[None, :], m)[0]
    np.testing.assert_allclose(r, np.conj(Phi).T @ Y / n, atol=1e-13)
    # diagonal blocks are the 1-D Toeplitz matrices of each coordinate
    L = 2 * m + 1
    for a in range(d):
        Ma = oracle.gram_generator(X[a:a + 1], m)
        np.testing.assert_allclose(B[a * L:(a + 1) * L, a * L:(a + 1) * L],
                                   oracle.toeplitz_matrix(Ma, m), atol=1e-13)
    # the constant function is shared by all components: the Gram has a null
    # space of dimension exactly d - 1 (for n large enough)
    ev = np.linalg.eigvalsh(B)
    assert (ev < 1e-10).sum() == d - 1


def test_fourier_entry_closed_forms_and_tables():
    # single point: exp(sign i q.x0) exactly; x0 = (-pi, pi/2) gives (-1)^q1 i^q2 for sign +
    x0 = np.array([[-np.pi], [np.pi / 2]])
    for q in [(0, 0), (1, 0), (3, 2), (-5, 7), (64, -64)]:
        want = (-1.0) ** q[0] * (1j) ** (q[1] % 4)
        assert abs(oracle.fourier_entry(x0, None, q, +1) - want) < 1e-12
        assert abs(oracle.fourier_entry(x0, None, q, -1) - np.conj(want)) < 1e-12
    # equispaced points: zero for 0 < |q| < n, weights linear
    n = 1000
    xe = (-np.pi + 2 * np.pi * np.arange(n) / n)[None, :]
    for q in [1, 17, 499]:
        assert abs(oracle.fourier_entry(xe, None, [q], +1)) < 1e-12
    # chunked sum equals the tabulated sums of gram_generator / rhs entry by entry
    rng = np.random.default_rng(3)
    X = rng.uniform(-np.pi, np.pi, size=(2, 3001))
    Y = rng.standard_normal((1, 3001))
    M = oracle.gram_generator(X, 3)
    b = oracle.rhs(X, Y, 3)[0].reshape(7, 7)
    for (q1, q2) in [(0, 0), (6, -6), (-2, 5)]:
        assert abs(oracle.fourier_entry(X, None, (q1, q2), +1, chunk=1000) - M[q1 + 6, q2 + 6]) < 1e-13
    for (k1, k2) in [(1, 2), (-3, 3)]:
        assert abs(oracle.fourier_entry(X, Y[0], (k1, k2), -1, chunk=777) - b[k1 + 3, k2 + 3]) < 1e-13


@pytest.mark.parametrize("d", [1, 2, 3])
def test_sampled_entries_match_the_table_sums(d):
    # fourier_entries (one exp per point and frequency) against gram_generator / rhs (power
    # recurrences and matrix products): two routes to the same sums; chunks smaller than n so the
    # ordered accumulation over chunks and threads is exercised
    rng = np.random.default_rng(40 + d)
    m, n = 4, 20_011
    X = rng.uniform(-2 * np.pi, 2 * np.pi, size=(d, n))
    Y = rng.standard_normal((3, n))
    M = oracle.gram_generator(X, m)
    b = oracle.rhs(X, Y, m).reshape((3,) + (2 * m + 1,) * d)
    qs = rng.integers(-2 * m, 2 * m + 1, size=(6, d))
    ks = rng.integers(-m, m + 1, size=(5, d))
    eM = oracle.fourier_entries(X, None, qs, +1, chunk=4096)
    eb = oracle.fourier_entries(X, Y, ks, -1, chunk=4096)
    assert eM.shape == (1, 6) and eb.shape == (3, 5)
    for f, q in enumerate(qs):
        assert abs(eM[0, f] - M[tuple(q + 2 * m)]) <= 1e-13
        assert abs(eM[0, f] - oracle.fourier_entry(X, None, q, +1)) <= 1e-13
    for f, k in enumerate(ks):
        for t in range(3):
            assert abs(eb[t, f] - b[(t,) + tuple(k + m)]) <= 1e-13
    # the sign matters: the + sign gives the conjugate of the - sign's weighted sum
    assert np.abs(oracle.fourier_entries(X, Y, ks, +1) - np.conj(eb)).max() <= 1e-13
    assert np.abs(oracle.fourier_entries(X, Y, ks, +1) - eb).max() > 1e-3


def test_chunk_sums_do_not_depend_on_the_thread_count(monkeypatch):
    rng = np.random.default_rng(7)
    X = rng.uniform(-np.pi, np.pi, size=(2, 50_000))
    monkeypatch.setenv("FK_ORACLE_THREADS", "1")
    a = oracle.gram_generator(X, 3)
    monkeypatch.setenv("FK_ORACLE_THREADS", "5")
    b = oracle.gram_generator(X, 3)
    assert np.array_equal(a, b)
