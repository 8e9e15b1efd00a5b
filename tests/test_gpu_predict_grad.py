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


# (2, 41): the largest m whose grid fits LDS, with 40 coefficient sets; (2, 45): the global-memory
# path beyond it
@pytest.mark.parametrize("d,m,nq", [(1, 50, 10_000), (2, 32, 100_003), (2, 5, 17), (2, 41, 5_001), (2, 45, 5_001)])
def test_predict_matches_direct_sum(fk, d, m, nq):
    rng = np.random.default_rng(d + m)
    N = (2 * m + 1) ** d
    k = oracle.modes(m, d)
    decay = 1.0 / (1.0 + (k ** 2).sum(1))
    th = np.stack([_herm(rng, N) * decay for _ in range(40 if (d, m) == (2, 41) else 2)])
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


def _grad_problem(seed, m=8, n=100_000, nv=50_000, T=3):
    X = synth.uniform_points(seed, 2, n)
    Y = synth.batched_targets(X, seed, ntgt=T)
    Xv = synth.uniform_points(seed + 1, 2, nv)
    Yv = synth.batched_targets(Xv, seed + 1, ntgt=T)
    X64, Y64, Xv64, Yv64 = (a.astype(np.float64) for a in (X, Y, Xv, Yv))
    o = dict(M=oracle.gram_generator(X64, m), b=oracle.rhs(X64, Y64, m), Mv=oracle.gram_generator(Xv64, m),
             bv=oracle.rhs(Xv64, Yv64, m), Xv64=Xv64, Yv64=Yv64)
    dev = [torch.from_numpy(a).cuda() for a in (X, Y, Xv, Yv)]
    return dev, o


def test_heldout_mse_and_gradients(fk):
    m, T = 8, 3
    (X, Y, Xv, Yv), o = _grad_problem(21, m=m, T=T)
    lams = [1e-4, 1e-2]
    p = oracle.sobolev_weights(m, 2, 2.0)
    N = p.size
    loglam = torch.tensor(np.log(lams), dtype=torch.float64, device="cuda", requires_grad=True)
    pt = torch.tensor(p, dtype=torch.float64, device="cuda", requires_grad=True)
    mse, theta = fk.KernelRidgeGridLoss.apply(loglam, pt, X, Y, Xv, Yv, m)
    rng = np.random.default_rng(0)
    w = torch.tensor(rng.uniform(0.5, 1.5, size=(len(lams), T)), device="cuda")
    # a second use of theta: E = sum Re(conj(c) theta), so dE/dconj(theta) = c / 2
    c = rng.standard_normal((len(lams), T, N)) + 1j * rng.standard_normal((len(lams), T, N))
    ct = torch.from_numpy(c).cuda()
    ((mse * w).sum() + (torch.conj(ct) * theta).real.sum()).backward()
    mse = mse.detach().cpu().numpy()
    wn = w.cpu().numpy()
    g_ll = np.zeros(len(lams))
    g_p = np.zeros_like(p)
    for i, lam in enumerate(lams):
        A = oracle.system_matrix(o["M"], m, lam, p)
        th = oracle.solve_system(A, o["b"])
        tg = theta[i].detach().cpu().numpy()
        assert _rel_herm(tg, th) <= 1e-4
        # the loss at the library's own theta: the held-out Gram and right-hand sides carry the
        # type-1 errors, so |d mse| <= eps_T ||theta||_1^2 + 2 eps_b mean|Yv| ||theta||_1 (theta's own
        # error is the check above)
        mo = oracle.heldout_mse(tg, o["Xv64"], o["Yv64"], m)
        l1 = np.abs(tg).sum(axis=1)
        bound = 1e-6 * (l1 ** 2 + 2 * np.abs(o["Yv64"]).mean(axis=1) * l1)
        assert (np.abs(mse[i] - mo) <= bound).all()
        for t in range(T):
            _, _, g = oracle.mse_gradients(A, th[t], p, lam, o["Mv"], o["bv"][t], m)
            dll, dp = oracle.theta_path_gradients(A, th[t], p, lam, wn[i, t] * g + 0.5 * c[i, t])
            g_ll[i] += dll
            g_p += dp
    gl = loglam.grad.cpu().numpy()
    gp = pt.grad.cpu().numpy()
    # the weights are tied, p_{-k} = p_k (the real form requires it and the library rejects any other
    # p), so the gradient with respect to p is the oracle's projected onto symmetric vectors; the
    # random c has an anti-Hermitian part, which moves dp_k and dp_{-k} in opposite directions
    g_p = 0.5 * (g_p + g_p[::-1])
    print("dlog lambda gpu", gl, "oracle", g_ll)
    assert np.abs(gl - g_ll).max() <= 1e-4 * np.abs(g_ll).max()
    assert np.abs(gp - g_p).max() <= 1e-4 * np.abs(g_p).max()


def _rel_herm(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_theta_gradient_of_the_heldout_loss(fk):
    # fit_backward(want_theta): dL/dconj(theta) = grad_mse * (Sigma_v theta - b_v), the Wirtinger
    # convention of the header (PyTorch's .grad would be twice this)
    m, T = 6, 2
    (X, Y, Xv, Yv), o = _grad_problem(41, m=m, T=T)
    lams = [3e-3]
    p = oracle.sobolev_weights(m, 2, 1.0)
    ctx = fk.Context(0)
    theta = fk.fit(X, Y, m, lams, penalty="sobolev", s=1.0, ctx=ctx)
    vctx = fk.Context(0)
    Mv, bv = fk.gram(Xv, Yv, m, ctx=vctx)
    mse = fk.heldout_mse(Mv, bv, fk.mean_square(Yv, ctx=vctx), m, len(lams), ctx)
    gm = torch.tensor([[0.7, -1.3]], dtype=torch.float64, device="cuda")
    _, _, gt = fk.fit_backward(gm, m, 2, ctx, want_theta=True)
    A = oracle.system_matrix(o["M"], m, lams[0], p)
    th = oracle.solve_system(A, o["b"])
    for t in range(T):
        _, _, g = oracle.mse_gradients(A, th[t], p, lams[0], o["Mv"], o["bv"][t], m)
        want = gm[0, t].item() * g
        got = gt[0, t].cpu().numpy()
        assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want)
    del mse, theta


def test_two_applies_alive_in_one_graph(fk):
    # two folds with different data summed into one loss: each apply keeps its own factors
    m, T = 6, 2
    lams = [1e-3, 1e-1]
    p = oracle.sobolev_weights(m, 2, 2.0)
    loglam = torch.tensor(np.log(lams), dtype=torch.float64, device="cuda", requires_grad=True)
    pt = torch.tensor(p, dtype=torch.float64, device="cuda", requires_grad=True)
    total = 0
    folds = []
    for seed in (51, 61):
        (X, Y, Xv, Yv), o = _grad_problem(seed, m=m, n=60_000, nv=30_000, T=T)
        mse, _ = fk.KernelRidgeGridLoss.apply(loglam, pt, X, Y, Xv, Yv, m)
        total = total + mse.sum()
        folds.append(o)
    total.backward()
    g_ll = np.zeros(len(lams))
    g_p = np.zeros_like(p)
    for o in folds:
        for i, lam in enumerate(lams):
            A = oracle.system_matrix(o["M"], m, lam, p)
            th = oracle.solve_system(A, o["b"])
            for t in range(T):
                dll, dp, _ = oracle.mse_gradients(A, th[t], p, lam, o["Mv"], o["bv"][t], m)
                g_ll[i] += dll
                g_p += dp
    gl = loglam.grad.cpu().numpy()
    assert np.abs(gl - g_ll).max() <= 1e-4 * np.abs(g_ll).max()
    assert np.abs(pt.grad.cpu().numpy() - g_p).max() <= 1e-4 * np.abs(g_p).max()


def test_kept_factors_are_guarded(fk):
    # a call that writes the workspace holding the factors makes the gradient calls refuse (FK_EINVAL)
    m, T = 6, 1
    (X, Y, Xv, Yv), _ = _grad_problem(71, m=m, n=20_000, nv=10_000, T=T)
    ctx, vctx = fk.Context(0), fk.Context(0)
    Mv, bv = fk.gram(Xv, Yv, m, ctx=vctx)
    yv2 = fk.mean_square(Yv, ctx=vctx)
    gm = torch.ones((1, T), dtype=torch.float64, device="cuda")
    fk.fit(X, Y, m, [1e-3], ctx=ctx)
    fk.gram(X, Y, m, ctx=ctx)                      # overwrites the factors (same workspace)
    with pytest.raises(fk.FkError) as e:
        fk.heldout_mse(Mv, bv, yv2, m, 1, ctx)
    assert e.value.code == 1
    fk.fit(X, Y, m, [1e-3], ctx=ctx)
    fk.heldout_mse(Mv, bv, yv2, m, 1, ctx)
    fk.predict(torch.zeros((1, (2 * m + 1) ** 2), dtype=torch.complex128, device="cuda"), Xv, m, ctx=ctx)
    with pytest.raises(fk.FkError) as e:
        fk.fit_backward(gm, m, 2, ctx)
    assert e.value.code == 1
    # backward before any held-out loss, and a shape mismatch, are refused too
    fk.fit(X, Y, m, [1e-3], ctx=ctx)
    with pytest.raises(fk.FkError) as e:
        fk.fit_backward(gm, m, 2, ctx)
    assert e.value.code == 1
    with pytest.raises(fk.FkError) as e:
        fk.heldout_mse(Mv, bv, yv2, m, 2, ctx)
    assert e.value.code == 1
    fk.heldout_mse(Mv, bv, yv2, m, 1, ctx)
    gl, _, _ = fk.fit_backward(gm, m, 2, ctx)
    assert torch.isfinite(gl).all()
    # a NaN loss weight reaches the adjoint solve: FK_ENAN, not a stalled refinement
    with pytest.raises(fk.FkError) as e:
        fk.fit_backward(torch.full((1, T), float("nan"), dtype=torch.float64, device="cuda"), m, 2, ctx)
    assert e.value.code == 3


def test_fit_kept_matches_fit_and_keeps_factors(fk):
    # fk_fit_kept: the same theta as fk_fit (the type-1 stage's atomics only reorder additions, and both
    # refinements stop at a 1e-10 relative residual, so the two thetas agree to about kappa 1e-10), its
    # factors kept in the caller's buffer for the held-out loss, and overlapping buffers refused
    m, T, lams = 6, 2, [1e-2, 1e-3]
    (X, Y, Xv, Yv), _ = _grad_problem(73, m=m, n=50_000, nv=10_000, T=T)
    ctx, vctx = fk.Context(0), fk.Context(0)
    th_ref = fk.fit(X, Y, m, lams, ctx=ctx)
    sb, tb = fk.fit_kept_workspace_size(2, X.shape[1], T, m, len(lams), ctx)
    kept = torch.empty(sb, dtype=torch.uint8, device="cuda")
    th = fk.fit(X, Y, m, lams, ctx=ctx, ws=kept)
    e = (torch.linalg.vector_norm(th - th_ref) / torch.linalg.vector_norm(th_ref)).item()
    print(f"fit_kept vs fit: {e:.2e}")
    assert e <= 1e-6
    Mv, bv = fk.gram(Xv, Yv, m, ctx=vctx)
    yv2 = fk.mean_square(Yv, ctx=vctx)
    mse_k = fk.heldout_mse(Mv, bv, yv2, m, len(lams), ctx, ws=kept)
    fk.fit(X, Y, m, lams, ctx=ctx)   # the context's own workspace: the kept buffer is untouched
    mse_r = fk.heldout_mse(Mv, bv, yv2, m, len(lams), ctx)
    print(f"held-out mse, kept buffer vs context workspace: {((mse_k - mse_r).abs() / mse_r.abs()).max().item():.2e}")
    assert torch.allclose(mse_k, mse_r, rtol=1e-6, atol=0)
    big = torch.empty(sb + tb, dtype=torch.uint8, device="cuda")
    L = ctx.lib
    out = torch.empty((len(lams), T, (2 * m + 1) ** 2, 2), dtype=torch.float64, device="cuda")
    lam_c = (fk.C.c_double * 2)(*lams)
    pen = fk.fk_penalty()
    code = L.fk_fit_kept(ctx.h, 2, X.shape[1], 0, fk._ptr(X), T, fk._ptr(Y), m, lam_c, 2, fk.C.byref(pen),
                         fk._ptr(out), fk._ptr(big), sb, fk.C.c_void_p(big.data_ptr() + sb // 2), tb, None)
    assert code == 1   # FK_EINVAL: the two workspaces overlap


@pytest.mark.parametrize("T,n,dt", [(16, 1_000_003, np.float32), (3, 1, np.float64), (1, 70_000, np.float64)])
def test_mean_square(fk, T, n, dt):
    # the constant term of the held-out loss: exact FP64 sums of squares of the stored values
    rng = np.random.default_rng(T * 7 + n)
    Y = (rng.standard_normal((T, n)) * 3.0).astype(dt)
    got = fk.mean_square(torch.from_numpy(Y).cuda()).cpu().numpy()
    want = np.array([np.sum(Y[t].astype(np.float64) ** 2) / n for t in range(T)])
    assert np.allclose(got, want, rtol=1e-12, atol=0)
