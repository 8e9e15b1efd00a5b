"""Parity of the type-2 prediction and of the held-out-MSE gradients with the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fk():
    import paper_2509_02649_amd as fk
    return fk


def _herm(rng, N, scale=1.0):
    th = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * scale
    return 0.5 * (th + np.conj(th[::-1]))


@pytest.mark.parametrize("d,m,nq", [(1, 50, 10_000), (2, 32, 100_003), (2, 5, 17)])
def test_predict_matches_direct_sum(fk, d, m, nq):
    rng = np.random.default_rng(d + m)
    N = (2 * m + 1) ** d
    k = oracle.modes(m, d)
    decay = 1.0 / (1.0 + (k ** 2).sum(1))
    th = np.stack([_herm(rng, N) * decay, _herm(rng, N) * decay])
    Xq = rng.uniform(-np.pi, np.pi, size=(d, nq)).astype(np.float32)
    f = fk.predict(torch.from_numpy(th).cuda(), torch.from_numpy(Xq).cuda(), m).cpu().numpy()
    fo = oracle.predict(th, Xq.astype(np.float64), m).real
    # type-2 error bound: eps * ||theta||_1 (FP32 interpolation)
    bound = 2e-6 * np.abs(th).sum(axis=1, keepdims=True)
    err = np.abs(f - fo)
    print(f"predict d={d} m={m}: max err {err.max():.2e}, bound {bound.min():.2e}")
    assert (err <= bound).all()


def test_predict_type1_type2_identity(fk):
    # n^-1 sum |f(X_j)|^2 = theta^* T theta with T from the GPU type-1 on the same points
    rng = np.random.default_rng(3)
    m, n = 16, 200_000
    X = synth.uniform_points(8, 2, n)
    N = (2 * m + 1) ** 2
    th = _herm(rng, N) / N
    Xd = torch.from_numpy(X).cuda()
    f = fk.predict(torch.from_numpy(th[None]).cuda(), Xd, m).cpu().numpy()[0].astype(np.float64)
    M, _ = fk.gram(Xd, None, m)
    T = oracle.toeplitz_matrix(M.cpu().numpy(), m)
    lhs = np.mean(f ** 2)
    rhs = np.real(np.conj(th) @ T @ th)
    assert abs(lhs - rhs) / rhs < 1e-5


def test_heldout_mse_and_gradients(fk):
    m, n, nv, T = 8, 100_000, 50_000, 3
    X = synth.uniform_points(21, 2, n)
    Y = synth.batched_targets(X, 21, ntgt=T)
    Xv = synth.uniform_points(22, 2, nv)
    Yv = synth.batched_targets(Xv, 22, ntgt=T)
    lams = [1e-4, 1e-2]
    p = oracle.sobolev_weights(m, 2, 2.0)
    loglam = torch.tensor(np.log(lams), dtype=torch.float64, device="cuda", requires_grad=True)
    pt = torch.tensor(p, dtype=torch.float64, device="cuda", requires_grad=True)
    mse = fk.KernelRidgeGridLoss.apply(loglam, pt, torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                                       torch.from_numpy(Xv).cuda(), torch.from_numpy(Yv).cuda(), m)
    w = torch.tensor(np.random.default_rng(0).uniform(0.5, 1.5, size=(len(lams), T)), device="cuda")
    (mse * w).sum().backward()
    mse = mse.detach().cpu().numpy()
    # oracle
    X64, Y64, Xv64, Yv64 = (a.astype(np.float64) for a in (X, Y, Xv, Yv))
    M = oracle.gram_generator(X64, m)
    b = oracle.rhs(X64, Y64, m)
    Mv = oracle.gram_generator(Xv64, m)
    bv = oracle.rhs(Xv64, Yv64, m)
    wn = w.cpu().numpy()
    g_ll = np.zeros(len(lams))
    g_p = np.zeros_like(p)
    for i, lam in enumerate(lams):
        A = oracle.system_matrix(M, m, lam, p)
        th = oracle.solve_system(A, b)
        mo = oracle.heldout_mse(th, Xv64, Yv64, m)
        # the loss inherits the type-1 error: |d mse| <= eps_T ||theta||_1^2 + 2 eps_b mean|Yv| ||theta||_1
        l1 = np.abs(th).sum(axis=1)
        bound = 1e-6 * (l1 ** 2 + 2 * np.abs(Yv64).mean(axis=1) * l1)
        assert (np.abs(mse[i] - mo) <= bound).all()
        for t in range(T):
            dll, dp, _ = oracle.mse_gradients(A, th[t], p, lam, Mv, bv[t], m)
            g_ll[i] += wn[i, t] * dll
            g_p += wn[i, t] * dp
    gl = loglam.grad.cpu().numpy()
    gp = pt.grad.cpu().numpy()
    print("dlog lambda gpu", gl, "oracle", g_ll)
    assert np.abs(gl - g_ll).max() <= 1e-4 * np.abs(g_ll).max()
    assert np.abs(gp - g_p).max() <= 1e-4 * np.abs(g_p).max()


@pytest.mark.parametrize("T,n,dt", [(16, 1_000_003, np.float32), (3, 1, np.float64), (1, 70_000, np.float64)])
def test_mean_square(fk, T, n, dt):
    # the constant term of the held-out loss: exact FP64 sums of squares of the stored values
    rng = np.random.default_rng(T * 7 + n)
    Y = (rng.standard_normal((T, n)) * 3.0).astype(dt)
    got = fk.mean_square(torch.from_numpy(Y).cuda()).cpu().numpy()
    want = np.array([np.sum(Y[t].astype(np.float64) ** 2) / n for t in range(T)])
    assert np.allclose(got, want, rtol=1e-12, atol=0)
