"""Parity of the FFT Toeplitz product and of the conjugate-gradient solve with the FP64 oracle.

Bars: the product to 1e-12 of its largest entry (FP64 FFTs of length <= 1024); theta within
max(1e-10, 10 kappa tol) of the oracle's Cholesky solution, and the iteration count within 2
of the oracle's textbook PCG with the same preconditioner and stopping rule."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fk():
    import paper_2509_02649_amd as fk
    return fk


def _cplx(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gen(d, m, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    return rng, X, oracle.gram_generator(X, m)


@pytest.mark.parametrize("d,m,n,dense", [(1, 5, 300, True), (1, 40, 300, True), (1, 255, 200, True),
                                         (2, 3, 300, True), (2, 32, 200, True), (2, 100, 40, False),
                                         (3, 2, 300, True), (3, 8, 150, False), (3, 40, 6, False)])
def test_toeplitz_apply_parity(fk, d, m, n, dense):
    print(f"toeplitz d={d} m={m}", flush=True)
    rng, X, M = _gen(d, m, n, 100 * d + m)
    N = (2 * m + 1) ** d
    V = 3
    x = rng.standard_normal((V, N)) + 1j * rng.standard_normal((V, N))
    y = fk.toeplitz_apply(_cplx(M), _cplx(x), m).cpu().numpy()
    if dense:
        ref = oracle.toeplitz_apply(M, x, m)
        np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    else:
        rows = np.concatenate([[0, N // 2, N - 1], rng.choice(N, 13, replace=False)])
        for v in range(V):
            ref = oracle.toeplitz_apply_rows(M, x[v], m, rows)
            np.testing.assert_allclose(y[v, rows], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def _problem(d, m, n, ntgt, s, seed):
    rng, X, M = _gen(d, m, n, seed)
    Y = np.stack([np.sin(X[0] + t) * np.cos(X[-1]) + 0.1 * rng.standard_normal(n) for t in range(ntgt)])
    b = oracle.rhs(X, Y, m)
    p = oracle.sobolev_weights(m, d, s)
    return M, b, p


@pytest.mark.parametrize("d,m,n,lams", [(1, 50, 10_000, [1e-2, 1e-5]), (2, 16, 20_000, [1e-2, 1e-4, 1e-6]),
                                        (3, 4, 5_000, [1e-3, 1e-6])])
def test_solve_cg_parity(fk, d, m, n, lams):
    print(f"cg d={d} m={m}", flush=True)
    s, tol, ntgt = 2.0, 1e-12, 2
    M, b, p = _problem(d, m, n, ntgt, s, 7 + d)
    th, inf = fk.solve_cg(_cplx(M), _cplx(b), m, lams, penalty="sobolev", s=s, tol=tol, maxit=2000, info=True)
    th = th.cpu().numpy()
    m0 = M[(2 * m,) * d].real
    it_ref = 0
    for l, lam in enumerate(lams):
        A = oracle.system_matrix(M, m, lam, p)
        ref = oracle.solve_system(A, b)
        kappa = oracle.condition_number(A)
        bar = max(1e-10, 10 * kappa * tol)
        for t in range(ntgt):
            err = np.linalg.norm(th[l, t] - ref[t]) / np.linalg.norm(ref[t])
            assert err <= bar, (lam, t, err, kappa)
            assert inf["relres"][l][t] <= 10 * tol
            _, it, _ = oracle.pcg(A, b[t], m0 + lam * p, tol, 2000)
            it_ref = max(it_ref, it)
    assert abs(inf["iters"] - it_ref) <= 2, (inf["iters"], it_ref)


def test_solve_cg_edge_cases(fk):
    d, m = 2, 6
    M, b, p = _problem(d, m, 3_000, 3, 1.0, 21)
    b[1] = 0.0                                          # a zero right-hand side
    th, inf = fk.solve_cg(_cplx(M), _cplx(b), m, [1e-3], penalty="sobolev", s=1.0, tol=1e-11, info=True)
    th = th.cpu().numpy()
    assert not th[0, 1].any() and inf["relres"][0][1] == 0.0
    ref = oracle.solve_system(oracle.system_matrix(M, m, 1e-3, p), b)
    for t in (0, 2):
        assert np.linalg.norm(th[0, t] - ref[t]) / np.linalg.norm(ref[t]) < 1e-9
    # identity penalty (the low-bias estimator) and a caller-given diagonal
    pd = oracle.sobolev_bessel_weights(m, d, 1.5)
    th2 = fk.solve_cg(_cplx(M), _cplx(b), m, [1e-2], penalty="diag", p=torch.from_numpy(pd), tol=1e-11)
    ref2 = oracle.solve_system(oracle.system_matrix(M, m, 1e-2, pd), b)
    assert np.linalg.norm(th2.cpu().numpy()[0, 0] - ref2[0]) / np.linalg.norm(ref2[0]) < 1e-9
    th3 = fk.solve_cg(_cplx(M), _cplx(b), m, [1e-2], penalty="identity", tol=1e-11)
    ref3 = oracle.solve_system(oracle.system_matrix(M, m, 1e-2, np.ones_like(p)), b)
    assert np.linalg.norm(th3.cpu().numpy()[0, 2] - ref3[2]) / np.linalg.norm(ref3[2]) < 1e-9
    # too few iterations: FK_ENOCONV; a dense penalty or lambda <= 0: FK_EINVAL
    with pytest.raises(fk.FkError) as e:
        fk.solve_cg(_cplx(M), _cplx(b), m, [1e-8], penalty="sobolev", s=3.0, tol=1e-14, maxit=1)
    assert e.value.code == 5
    with pytest.raises(fk.FkError) as e:
        fk.solve_cg(_cplx(M), _cplx(b), m, [1e-3], penalty="heat_box", mu=1e-3)
    assert e.value.code == 1
    with pytest.raises(fk.FkError) as e:
        fk.solve_cg(_cplx(M), _cplx(b), m, [0.0])
    assert e.value.code == 1
    # a NaN in b, or in an off-centre entry of M: FK_ENAN, not a silent zero or a pivot error
    bn = b.copy()
    bn[2, 5] = np.nan
    with pytest.raises(fk.FkError) as e:
        fk.solve_cg(_cplx(M), _cplx(bn), m, [1e-3])
    assert e.value.code == 3
    Mn = M.copy()
    Mn[0, 3] = np.nan
    with pytest.raises(fk.FkError) as e:
        fk.solve_cg(_cplx(Mn), _cplx(b), m, [1e-3])
    assert e.value.code == 3


def test_solve_cg_batched_shape_against_dense_path(fk):
    # 2-D, m = 32, 16 targets x 64 log-spaced lambdas in [1e-8, 1e-1] with the s = 2 Sobolev
    # weights, from a 1e7-point Gram on the device: CG against the FP32-Cholesky + FP64
    # refinement path on every system, and against the oracle's Cholesky on two of them.
    print("cg batched shape", flush=True)
    m, ntgt, nlam, n = 32, 16, 64, 10_000_000
    ctx = fk.Context(0)
    X = fk.generate_uniform(2509026495, 2, n, ctx=ctx)
    Y = fk.generate_targets(2509026495, X, ntgt, ctx=ctx)
    M, b = fk.gram(X, Y, m, ctx=ctx)
    del X, Y
    lams = [10.0 ** (-8.0 + 7.0 * i / (nlam - 1)) for i in range(nlam)]
    th_cg, inf = fk.solve_cg(M, b, m, lams, penalty="sobolev", s=2.0, tol=1e-12, ctx=ctx, info=True)
    th_d = fk.solve(M, b, m, lams, penalty="sobolev", s=2.0, ctx=ctx)
    num = torch.linalg.vector_norm(th_cg - th_d, dim=-1)
    den = torch.linalg.vector_norm(th_d, dim=-1)
    assert float((num / den).max()) < 1e-8
    assert max(max(r) for r in inf["relres"]) <= 1e-11
    Mh, bh = M.cpu().numpy(), b.cpu().numpy()
    p = oracle.sobolev_weights(m, 2, 2.0)
    for l, t in [(0, 3), (nlam - 1, 11)]:
        ref = oracle.solve_system(oracle.system_matrix(Mh, m, lams[l], p), bh[t])
        got = th_cg[l, t].cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9


def _disk(n, radius, rng):
    r = np.sqrt(rng.uniform(0, 1, n)) * radius
    a = rng.uniform(0, 2 * np.pi, n)
    return np.stack([r * np.cos(a), r * np.sin(a)])


@pytest.mark.parametrize("m,mu", [(6, 1e-3), (10, 1e-4)])
def test_solve_cg_collocation_parity(fk, m, mu):
    # Sec. 4, intractable domains: heat operator d_t - d_xx sampled at n_r collocation points in a disk;
    # data in the same disk.  Generators from the oracle (solver parity), then from the device Gram
    # (end to end).
    print(f"cg collocation m={m} mu={mu}", flush=True)
    rng = np.random.default_rng(40 + m)
    n, nr, lams, tol = 20_000, 15_000, [1e-2, 1e-4], 1e-12
    X = _disk(n, 1.3, rng)
    Y = np.stack([np.exp(-X[0]) * np.sin(X[1]) + 0.05 * rng.standard_normal(n) for _ in range(2)])
    Xr = _disk(nr, 1.3, rng)
    M, Mr = oracle.gram_generator(X, m), oracle.gram_generator(Xr, m)
    b = oracle.rhs(X, Y, m)
    D = oracle.heat_symbol(m)
    p = oracle.sobolev_weights(m, 2, 1.0)
    P = oracle.collocation_penalty(Xr, m, mu, D)
    th, inf = fk.solve_cg(_cplx(M), _cplx(b), m, lams, penalty="sobolev", s=1.0, tol=tol, maxit=5000, info=True,
                          collocation=(mu, _cplx(Mr), _cplx(D)))
    th = th.cpu().numpy()
    dg = M[2 * m, 2 * m].real + mu * np.abs(D) ** 2 * Mr[2 * m, 2 * m].real
    it_ref = 0
    for l, lam in enumerate(lams):
        A = oracle.system_matrix(M, m, lam, p) + P
        ref = oracle.solve_system(A, b)
        kappa = oracle.condition_number(A)
        for t in range(2):
            err = np.linalg.norm(th[l, t] - ref[t]) / np.linalg.norm(ref[t])
            assert err <= max(1e-10, 10 * kappa * tol), (lam, t, err, kappa)
            _, it, _ = oracle.pcg(A, b[t], dg + lam * p, tol, 5000)
            it_ref = max(it_ref, it)
    # hundreds of iterations: rounding (FFT against dense products) may shift the count a little
    assert abs(inf["iters"] - it_ref) <= 2 + 0.1 * it_ref, (inf["iters"], it_ref)
    # end to end: both generators and b from the device type-1 stage (Gram error <= 1e-6 relative,
    # so theta moves by up to about kappa times that)
    Xd = torch.from_numpy(X).cuda()
    Md, bd = fk.gram(Xd, torch.from_numpy(Y).cuda(), m)
    Mrd, _ = fk.gram(torch.from_numpy(Xr).cuda(), None, m)
    th2 = fk.solve_cg(Md, bd, m, lams, penalty="sobolev", s=1.0, tol=1e-11,
                      collocation=(mu, Mrd, _cplx(D))).cpu().numpy()
    for l, lam in enumerate(lams):
        A = oracle.system_matrix(M, m, lam, p) + P
        ref = oracle.solve_system(A, b)
        bar = max(1e-4, 1e-6 * oracle.condition_number(A))
        assert np.linalg.norm(th2[l] - ref) / np.linalg.norm(ref) < bar
    # mu = 0 is the plain iteration
    th0 = fk.solve_cg(_cplx(M), _cplx(b), m, lams, penalty="sobolev", s=1.0, tol=1e-12,
                      collocation=(0.0, _cplx(Mr), _cplx(D))).cpu().numpy()
    th1 = fk.solve_cg(_cplx(M), _cplx(b), m, lams, penalty="sobolev", s=1.0, tol=1e-12).cpu().numpy()
    assert np.abs(th0 - th1).max() <= 1e-12 * np.abs(th1).max()


def test_restrict_serves_a_sweep_over_s(fk):
    # One type-1 stage at the largest m of a sweep serves every smaller m (M[q] and b_k do not depend
    # on m).  The sweep ties m and lambda to s as in the Sobolev rates, m = n^(1/(2s+d)),
    # lambda = n^(-2s/(2s+d)), and solves each s by conjugate gradients.
    print("restrict / s sweep", flush=True)
    rng = np.random.default_rng(77)
    n, d = 30_000, 2
    X = rng.uniform(-np.pi, np.pi, (d, n))
    Y = (np.sin(X[0]) * np.cos(2 * X[1]) + 0.1 * rng.standard_normal(n))[None, :]
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    sweep = [(s, int(round(n ** (1 / (2 * s + d)))), n ** (-2 * s / (2 * s + d))) for s in (1.0, 1.5, 2.0, 3.0)]
    mmax = max(m for _, m, _ in sweep)
    Mbig, bbig = fk.gram(Xd, Yd, mmax)
    scale_b = np.abs(Y).mean()
    for s, m, lam in sweep:
        Mm, bm = fk.restrict(Mbig, bbig, mmax, m)
        o, ob = 2 * (mmax - m), mmax - m
        assert torch.equal(Mm, Mbig[o:o + 4 * m + 1, o:o + 4 * m + 1])
        bb = bbig.reshape(1, 2 * mmax + 1, 2 * mmax + 1)[:, ob:ob + 2 * m + 1, ob:ob + 2 * m + 1].reshape(1, -1)
        assert torch.equal(bm, bb)
        Mref, bref = oracle.gram_generator(X, m), oracle.rhs(X, Y, m)
        assert np.abs(Mm.cpu().numpy() - Mref).max() / Mref[2 * m, 2 * m].real <= 1e-6
        assert np.abs(bm.cpu().numpy() - bref).max() / scale_b <= 1e-6
        th = fk.solve_cg(Mm, bm, m, [lam], penalty="sobolev", s=s, tol=1e-12).cpu().numpy()
        A = oracle.system_matrix(Mref, m, lam, oracle.sobolev_weights(m, d, s))
        ref = oracle.solve_system(A, bref)
        assert np.linalg.norm(th[0] - ref) / np.linalg.norm(ref) <= max(1e-4, 1e-6 * oracle.condition_number(A))
    with pytest.raises(fk.FkError):
        fk.restrict(Mbig, bbig, mmax, mmax + 1)


@pytest.mark.parametrize("m,n,ntgt", [(4, 50_001, 1), (6, 150_000, 2)])
def test_gram_3d_and_cg_fit(fk, m, n, ntgt):
    # 3-D type-1 stage (FP64-atomic spread, three pruned transforms) against the oracle's direct sums,
    # then a 3-D fit by conjugate gradients against the oracle's Cholesky solve.
    print(f"gram 3-D m={m} n={n}", flush=True)
    rng = np.random.default_rng(300 + m)
    X = rng.uniform(-np.pi, np.pi, (3, n))
    Y = np.stack([np.cos(X[0] - t) * np.sin(X[1]) * np.cos(X[2]) + 0.1 * rng.standard_normal(n) for t in range(ntgt)])
    for dt in (torch.float64, torch.float32):
        Xd, Yd = torch.from_numpy(X).to(dt).cuda(), torch.from_numpy(Y).to(dt).cuda()
        M, b = fk.gram(Xd, Yd, m)
        Xh, Yh = Xd.double().cpu().numpy(), Yd.double().cpu().numpy()
        Mref, bref = oracle.gram_generator(Xh, m), oracle.rhs(Xh, Yh, m)
        eps_T = np.abs(M.cpu().numpy() - Mref).max() / Mref[(2 * m,) * 3].real
        eps_b = np.abs(b.cpu().numpy() - bref).max() / np.abs(Yh).mean()
        assert eps_T <= 1e-6 and eps_b <= 1e-6, (dt, eps_T, eps_b)
    lam = 1e-3
    th = fk.solve_cg(M, b, m, [lam], penalty="sobolev", s=1.5, tol=1e-12).cpu().numpy()
    A = oracle.system_matrix(Mref, m, lam, oracle.sobolev_weights(m, 3, 1.5))
    ref = oracle.solve_system(A, bref)
    assert np.linalg.norm(th[0] - ref) / np.linalg.norm(ref) <= max(1e-4, 1e-6 * oracle.condition_number(A))


@pytest.mark.parametrize("m,nq", [(3, 1001), (12, 20_000)])
def test_predict_3d_matches_direct_sum(fk, m, nq):
    # 3-D type-2: f(x) = Re sum_k theta_k exp(+i k.x) against the oracle's direct sum; bound as in
    # 1-D / 2-D: eps ||theta||_1 with the FP32 interpolation.
    print(f"predict 3-D m={m}", flush=True)
    rng = np.random.default_rng(500 + m)
    N = (2 * m + 1) ** 3
    k = oracle.modes(m, 3)
    decay = 1.0 / (1.0 + (k ** 2).sum(1))
    th = []
    for _ in range(2):
        z = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * decay
        th.append(0.5 * (z + np.conj(z[::-1])))
    th = np.stack(th)
    Xq = rng.uniform(-np.pi, np.pi, size=(3, nq)).astype(np.float32)
    f = fk.predict(torch.from_numpy(th).cuda(), torch.from_numpy(Xq).cuda(), m).cpu().numpy()
    fo = oracle.predict(th, Xq.astype(np.float64), m).real
    bound = 2e-6 * np.abs(th).sum(axis=1, keepdims=True)
    err = np.abs(f - fo)
    print(f"predict 3-D m={m}: max err {err.max():.2e}, bound {bound.min():.2e}")
    assert (err <= bound).all()
