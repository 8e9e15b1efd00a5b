"""Parity of the dense stage (real-form FP32 MFMA Cholesky + FP64 refinement) and of the
end-to-end fit with the FP64 oracle.  Bar: ||theta_gpu - theta|| / ||theta|| <= 1e-4 where
the oracle's condition number is <= 1e6 (both solver-only and end-to-end)."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-4
TOL_GRAM = 1e-6


@pytest.fixture(scope="module")
def fk():
    import paper_2509_02649_amd as fk
    return fk


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _cplx(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("d,m,n,s,lam", [(1, 50, 10_000, 1.0, 1e4 ** (-2 / 3)), (2, 8, 50_000, 2.0, 1e-3),
                                         (2, 16, 60_000, 2.0, 1e-3), (2, 32, 100_000, 2.0, 1e-3)])
def test_solver_only_parity(fk, d, m, n, s, lam):
    rng = np.random.default_rng(d * 100 + m)
    X = rng.uniform(-np.pi, np.pi, size=(d, n))
    Y = np.sin(X[0]) + 0.1 * rng.standard_normal(n)
    M = oracle.gram_generator(X, m)
    b = oracle.rhs(X, Y[None, :], m)
    p = oracle.sobolev_weights(m, d, s)
    A = oracle.system_matrix(M, m, lam, p)
    th = oracle.solve_system(A, b)
    kappa = oracle.condition_number(A)
    tg, info = fk.solve(_cplx(M), _cplx(b), m, [lam], penalty="sobolev", s=s, info=True)
    e = _rel(tg[0].cpu().numpy(), th)
    print(f"solver-only d={d} m={m}: rel={e:.2e} kappa={kappa:.2e} iters={info['refine_iters']} "
          f"resid={info['resid_rel']:.1e} factor={info['t_factor_ms']:.2f} ms")
    assert kappa <= 1e6
    assert e <= TOL


def test_unrefined_solve_is_fp32_class(fk):
    # The factorization keeps its finished panels as FP16 pairs (about 22 significant bits) and
    # accumulates their products in FP32.  Without the FP64 refinement (max_refine = 0, any residual
    # accepted) its solution must be as accurate as an FP32 LAPACK Cholesky solve of the same
    # equilibrated system: the FP32 accumulation over 2432-long dot products, not the operands'
    # representation, sets the factor's error.
    import scipy.linalg as sl
    m, n = 24, 200_000
    X = synth.uniform_points(4242, 2, n)
    Y = synth.batched_targets(X, 4242, ntgt=2)
    M, b = fk.gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m)
    Mh, bh = M.cpu().numpy(), b.cpu().numpy()
    p = oracle.sobolev_weights(m, 2, 2.0)
    lams = [1e-2, 1e-4, 1e-6]
    ctx0 = fk.Context(0, max_refine=0, refine_tol=1e30)
    th0 = fk.solve(M, b, m, lams, penalty="sobolev", s=2.0, ctx=ctx0).cpu().numpy()
    for i, lam in enumerate(lams):
        A = oracle.system_matrix(Mh, m, lam, p)
        ref = oracle.solve_system(A, bh)
        dg = 1.0 / np.sqrt(np.diag(A).real)
        A32 = (dg[:, None] * A * dg[None, :]).astype(np.complex64)
        c = sl.cho_factor(A32, lower=True)
        th32 = np.stack([dg * sl.cho_solve(c, (dg * bt).astype(np.complex64)) for bt in bh])
        e32 = _rel(th32, ref)
        e0 = _rel(th0[i], ref)
        print(f"lambda={lam:.0e}: unrefined GPU solve {e0:.2e}, FP32 LAPACK {e32:.2e}")
        assert e0 <= 2.0 * e32 + 1e-7


def test_fit_1d_small_config(fk):
    w = synth.workload_1d()
    X, Y, m = w["X"], w["Y"], w["m"]
    p = oracle.sobolev_weights(m, 1, 1.0)
    th, M, b = oracle.fit(X, Y, m, w["lam"], p)
    tg = fk.fit(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m, w["lam"], penalty="sobolev", s=1.0)
    e = _rel(tg[0].cpu().numpy(), th)
    print(f"fit 1-D: rel={e:.2e}")
    assert e <= TOL
    # the sin 3x + cos(7x)/2 target is recovered: theta_{+-3} ~ -+ i/2, theta_{+-7} ~ 1/4
    t = tg[0, 0].cpu().numpy()
    assert abs(t[m + 3] + 0.5j) < 0.05 and abs(t[m - 3] - 0.5j) < 0.05 and abs(t[m + 7] - 0.25) < 0.05


def test_fit_2d_medium(fk):
    w = synth.workload_2d(n=1_000_000)
    X, Y, m = w["X"], w["Y"], w["m"]
    lam = 1e7 ** (-4 / 5)
    p = oracle.sobolev_weights(m, 2, 2.0)
    th, M, b = oracle.fit(X.astype(np.float64), Y.astype(np.float64), m, lam, p)
    A = oracle.system_matrix(M, m, lam, p)
    kappa = oracle.condition_number(A)
    tg, info = fk.fit(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m, lam, penalty="sobolev", s=2.0,
                      info=True)
    e = _rel(tg[0].cpu().numpy(), th)
    print(f"fit 2-D n=1e6: rel={e:.2e} kappa={kappa:.2e} info={info}")
    assert kappa <= 1e6 and e <= TOL


def test_fit_many_lambdas_and_targets(fk):
    X = synth.uniform_points(99, 2, 200_000)
    Y = synth.batched_targets(X, 99, ntgt=4)
    m = 12
    lams = [1e-5, 1e-3, 1e-1]
    p = oracle.sobolev_weights(m, 2, 2.0)
    M = oracle.gram_generator(X.astype(np.float64), m)
    b = oracle.rhs(X.astype(np.float64), Y.astype(np.float64), m)
    tg = fk.fit(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m, lams, penalty="sobolev", s=2.0)
    tg = tg.cpu().numpy()
    for i, lam in enumerate(lams):
        A = oracle.system_matrix(M, m, lam, p)
        th = oracle.solve_system(A, b)
        for t in range(4):
            assert _rel(tg[i, t], th[t]) <= TOL


def test_solve_at_the_batched_benchmark_shape(fk):
    # the dense stage exactly as the benchmark runs it: N = 4225 unknowns (m = 32), 64 lambdas in
    # [1e-8, 1e-1], 16 targets (paired FP16-pair panel updates, FP32 diagonal blocks, two block columns
    # per triangular-solve launch), on a Gram from 2e6 device-generated points; three lambdas checked
    # against the oracle's FP64 solve of the same system
    m, T, nlam = 32, 16, 64
    ctx = fk.Context(0)
    X = fk.generate_uniform(2509026495, 2, 2_000_000, ctx=ctx)
    Y = fk.generate_targets(2509026495, X, T, ctx=ctx)
    M, b = fk.gram(X, Y, m, ctx=ctx)
    lams = [10.0 ** (-8.0 + 7.0 * i / (nlam - 1)) for i in range(nlam)]
    tg, info = fk.solve(M, b, m, lams, penalty="sobolev", s=2.0, ctx=ctx, info=True)
    print(f"benchmark shape: resid {info['resid_rel']:.1e}, {info['refine_iters']} refinement steps, "
          f"factor {info['t_factor_ms']:.2f} ms")
    assert info["resid_rel"] <= 1e-10
    # the dense stage has no atomics (the split updates' parts are added in a fixed order): a repeat
    # gives the same bits
    tg2 = fk.solve(M, b, m, lams, penalty="sobolev", s=2.0, ctx=ctx)
    assert torch.equal(tg, tg2)
    Mh, bh, th = M.cpu().numpy(), b.cpu().numpy(), tg.cpu().numpy()
    p = oracle.sobolev_weights(m, 2, 2.0)
    for i in (0, 31, 63):
        A = oracle.system_matrix(Mh, m, lams[i], p)
        ref = oracle.solve_system(A, bh)
        e = max(_rel(th[i, t], ref[t]) for t in range(T))
        print(f"lambda={lams[i]:.1e}: worst rel {e:.2e}")
        assert e <= TOL


def test_split_update_solve_is_deterministic(fk):
    # a few lambdas and targets at N = 4225: the paired updates' grids are small, so from the third
    # pair of block columns on their sums over the panels are split and the parts added in a fixed
    # order; two solves of the same system give the same bits, and theta matches the oracle
    m, T, lams = 32, 2, [1e-6, 1e-4, 1e-2]
    ctx = fk.Context(0)
    X = fk.generate_uniform(2509026496, 2, 1_000_000, ctx=ctx)
    Y = fk.generate_targets(2509026496, X, T, ctx=ctx)
    M, b = fk.gram(X, Y, m, ctx=ctx)
    t1 = fk.solve(M, b, m, lams, penalty="sobolev", s=2.0, ctx=ctx).cpu().numpy()
    t2 = fk.solve(M, b, m, lams, penalty="sobolev", s=2.0, ctx=ctx).cpu().numpy()
    assert np.array_equal(t1, t2)
    Mh, bh = M.cpu().numpy(), b.cpu().numpy()
    p = oracle.sobolev_weights(m, 2, 2.0)
    ref = oracle.solve_system(oracle.system_matrix(Mh, m, lams[1], p), bh)
    e = max(_rel(t1[1, t], ref[t]) for t in range(T))
    print(f"split updates, lambda={lams[1]:.0e}: worst rel {e:.2e}")
    assert e <= TOL


def test_solve_more_than_16_right_hand_sides(fk):
    # 20 right-hand sides: the triangular solves take 32-column blocks (two 16-column MFMA tiles)
    rng = np.random.default_rng(2020)
    m, n, T = 8, 30_000, 20
    X = rng.uniform(-np.pi, np.pi, size=(2, n))
    Y = rng.standard_normal((T, n))
    M = oracle.gram_generator(X, m)
    b = oracle.rhs(X, Y, m)
    p = oracle.sobolev_weights(m, 2, 2.0)
    lams = [1e-4, 1e-2]
    tg = fk.solve(_cplx(M), _cplx(b), m, lams, penalty="sobolev", s=2.0).cpu().numpy()
    for i, lam in enumerate(lams):
        th = oracle.solve_system(oracle.system_matrix(M, m, lam, p), b)
        e = max(_rel(tg[i, t], th[t]) for t in range(T))
        print(f"{T} right-hand sides, lambda={lam:.0e}: worst rel {e:.2e}")
        assert e <= TOL


def test_fit_low_bias_and_bessel_penalties(fk):
    X = synth.uniform_points(5, 2, 100_000)
    Y = synth.batched_targets(X, 5, ntgt=1)
    m = 10
    M = oracle.gram_generator(X.astype(np.float64), m)
    b = oracle.rhs(X.astype(np.float64), Y.astype(np.float64), m)
    for pen, p in [("identity", np.ones((2 * m + 1) ** 2)), ("sobolev_bessel", oracle.sobolev_bessel_weights(m, 2, 2.0))]:
        th = oracle.solve_system(oracle.system_matrix(M, m, 1e-4, p), b)
        tg = fk.fit(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m, 1e-4, penalty=pen, s=2.0)
        assert _rel(tg[0].cpu().numpy(), th) <= TOL


@pytest.mark.parametrize("mu", [1e-3, 1.0])
def test_fit_physics_informed_heat(fk, mu):
    w = synth.workload_piml(n=300_000)
    X, Y, m = w["X"], w["Y"], w["m"]
    lam = w["lam"]
    Q = oracle.piml_heat_penalty(m, lam, mu)
    M = oracle.gram_generator(X.astype(np.float64), m)
    b = oracle.rhs(X.astype(np.float64), Y.astype(np.float64), m)
    A = oracle.system_matrix(M, m, 0.0, Q)
    th = oracle.solve_system(A, b)
    kappa = oracle.condition_number(A)
    print(f"PIML mu={mu}: kappa={kappa:.2e}")
    if kappa > 1e7:
        # beyond FP32's reach even after equilibration: the documented outcome is a
        # status (FK_ENOTPD or FK_ENOCONV) naming the failing lambda, not a wrong theta
        try:
            tg = fk.fit(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m, lam, penalty="heat_box", mu=mu)
        except fk.FkError as e:
            assert e.code in (4, 5)
            return
        assert _rel(tg[0].cpu().numpy(), th) <= 1e-2
        return
    tg, info = fk.fit(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m, lam, penalty="heat_box", mu=mu,
                      info=True)
    e = _rel(tg[0].cpu().numpy(), th)
    print(f"PIML mu={mu}: rel={e:.2e} iters={info['refine_iters']}")
    assert e <= TOL


def test_fit_physics_informed_heat_full_size(fk):
    # The heat workload at full size: n = 1e8 points in [-pi/2, pi/2]^2, m = 20, lambda = 1e-4,
    # mu = 1e-3 (the pass/fail case).  Sampled entries of M and b against the oracle's direct sums
    # (all of M over 1e8 points would take the oracle minutes); theta against the oracle's FP64
    # solve of the same M and b; and the whole fit (type-1 stage + solve) against that.
    # inputs made on the device (the host generator would take minutes at 1e8 points): the
    # workload's Philox points, and Y = e^-t sin x + N(0, 0.05^2) with torch's seeded normal draws
    n, m, lam, mu = 100_000_000, 20, 1e-4, 1e-3
    Xd = fk.generate_uniform(synth.SEED_BASE + 3, 2, n, lo=(-np.pi / 2,) * 2, hi=(np.pi / 2,) * 2)
    g = torch.Generator(device="cuda").manual_seed(synth.SEED_BASE + 3)
    noise = torch.randn((1, n), generator=g, device="cuda", dtype=torch.float32)
    Yd = (torch.exp(-Xd[0:1].double()) * torch.sin(Xd[1:2].double()) + 0.05 * noise.double()).float()
    del noise
    X, Y = Xd.cpu().numpy(), Yd.cpu().numpy()
    M, b = fk.gram(Xd, Yd, m)
    M, b = M.cpu().numpy(), b.cpu().numpy()
    c = 2 * m
    qs = np.array([(0, 0), (1, 0), (0, 1), (40, -40), (-40, -40), (17, 3), (-9, 33)])
    mo = oracle.fourier_entries(X, None, qs, +1)[0]
    eT = max(abs(M[c + q[0], c + q[1]] - v) for q, v in zip(qs, mo))
    ks = np.array([(0, 0), (1, 0), (0, 1), (-20, 20), (13, -7)])
    bo = oracle.fourier_entries(X, Y, ks, -1)[0]
    sc = float(np.abs(Y).mean(dtype=np.float64))
    b2 = b[0].reshape(2 * m + 1, 2 * m + 1)
    eb = max(abs(b2[m + k[0], m + k[1]] - v) / sc for k, v in zip(ks, bo))
    print(f"PIML n=1e8 sampled: eps_T={eT:.2e} eps_b={eb:.2e}")
    assert eT <= TOL_GRAM and eb <= TOL_GRAM
    Q = oracle.piml_heat_penalty(m, lam, mu)
    A = oracle.system_matrix(M, m, 0.0, Q)
    th = oracle.solve_system(A, b)
    kappa = oracle.condition_number(A)
    ts = fk.solve(_cplx(M), _cplx(b), m, [lam], penalty="heat_box", mu=mu)[0].cpu().numpy()
    tg, info = fk.fit(Xd, Yd, m, lam, penalty="heat_box", mu=mu, info=True)
    e_s = _rel(ts, th)
    e = _rel(tg[0].cpu().numpy(), th)
    print(f"PIML n=1e8 mu=1e-3: kappa={kappa:.2e} solver-only {e_s:.2e} end-to-end {e:.2e} "
          f"iters={info['refine_iters']}")
    assert kappa <= 1e6 and e_s <= TOL and e <= TOL


def _pde_fit(fk, X, Y, m, lam, mu, alpha, coef, lo, hi, s=1.0):
    return fk.fit(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), m, lam, penalty="pde_box", s=s, mu=mu,
                  box_lo=lo, box_hi=hi, alpha=alpha, coef=coef, info=True)


@pytest.mark.parametrize("n", [27_000, 250_000])
def test_fit_pde_box_paper_1d_example(fk, n):
    # The one-dimensional example of Sec. 4: X ~ U(]0, 1[) with L = pi/2 (radians = x), Y = e^X + N(0, 1),
    # the constraint f' - f = 0 on ]0, 1[, s = d = 1, m = n^(1/3), lambda = n^(-2/3), mu = 1.
    m = min(64, int(round(n ** (1 / 3))))
    lam = n ** (-2 / 3)
    rng = np.random.default_rng(2025)
    X = rng.uniform(0.0, 1.0, size=(1, n))
    Y = (np.exp(X[0]) + rng.standard_normal(n))[None, :]
    alpha, coef = [[1], [0]], [1.0, -1.0]
    D = oracle.pde_symbol(m, 1, alpha, coef)
    Q = oracle.piml_box_penalty(m, 1, lam, 1.0, D, (0.0,), (1.0,), s=1.0)
    th, M, b = oracle.fit(X, Y, m, 0.0, Q)
    kappa = oracle.condition_number(oracle.system_matrix(M, m, 0.0, Q))
    # solver-only: the oracle's M and b through the library's assembly and solve
    ts = fk.solve(_cplx(M), _cplx(b), m, [lam], penalty="pde_box", s=1.0, mu=1.0, box_lo=(0.0,), box_hi=(1.0,),
                  alpha=alpha, coef=coef)
    e_s = _rel(ts[0].cpu().numpy(), th)
    tg, info = _pde_fit(fk, X, Y, m, lam, 1.0, alpha, coef, (0.0,), (1.0,))
    e = _rel(tg[0].cpu().numpy(), th)
    print(f"PDE box 1-D n={n} m={m}: kappa={kappa:.2e} solver-only {e_s:.2e} end-to-end {e:.2e} "
          f"iters={info['refine_iters']}")
    if kappa <= 1e6:
        assert e_s <= TOL and e <= TOL
    else:
        # reported, not bound: the bar applies where kappa <= 1e6
        assert e <= 1e-2


def test_fit_pde_box_2d_operator_off_centre_box(fk):
    # d_t d_x + 0.5 d_xx + d_t - 2 on the box [-1, 0.5] x [-0.3, 1.2] (radians), s = 1.5: an operator
    # with odd and even terms and a box whose Fourier matrix is complex (orientation matters)
    rng = np.random.default_rng(77)
    n, m, lam, mu = 200_000, 10, 1e-3, 1e-3
    X = np.stack([rng.uniform(-1.0, 0.5, n), rng.uniform(-0.3, 1.2, n)]).astype(np.float32)
    Y = (np.exp(-X[0]) * np.sin(X[1]) + 0.05 * rng.standard_normal(n)).astype(np.float32)[None, :]
    alpha, coef = [[1, 1], [0, 2], [1, 0], [0, 0]], [1.0, 0.5, 1.0, -2.0]
    lo, hi = (-1.0, -0.3), (0.5, 1.2)
    D = oracle.pde_symbol(m, 2, alpha, coef)
    Q = oracle.piml_box_penalty(m, 2, lam, mu, D, lo, hi, s=1.5)
    th, M, b = oracle.fit(X.astype(np.float64), Y.astype(np.float64), m, 0.0, Q)
    kappa = oracle.condition_number(oracle.system_matrix(M, m, 0.0, Q))
    tg, info = _pde_fit(fk, X, Y, m, lam, mu, alpha, coef, lo, hi, s=1.5)
    e = _rel(tg[0].cpu().numpy(), th)
    print(f"PDE box 2-D: kappa={kappa:.2e} rel={e:.2e}")
    assert kappa <= 1e6 and e <= TOL
    # the heat operator through the general kind equals the heat kind; both solve the same M and b
    # (two type-1 stages differ in the order of their atomic additions, so not bit for bit)
    w = synth.workload_piml(n=100_000)
    Xh, Yh, mh = w["X"], w["Y"], w["m"]
    Mh, bh = fk.gram(torch.from_numpy(Xh).cuda(), torch.from_numpy(Yh).cuda(), mh)
    a = fk.solve(Mh, bh, mh, [w["lam"]], penalty="heat_box", mu=1e-3)
    g = fk.solve(Mh, bh, mh, [w["lam"]], penalty="pde_box", s=1.0, mu=1e-3, alpha=[[1, 0], [0, 2]],
                 coef=[1.0, -1.0], box_lo=(-np.pi / 2,) * 2, box_hi=(np.pi / 2,) * 2)
    assert _rel(g.cpu().numpy(), a.cpu().numpy()) < 1e-12


def test_pde_box_arguments_are_checked(fk):
    M = _cplx(np.ones(81, dtype=np.complex128).reshape(9, 9))
    b = _cplx(np.ones((1, 25), dtype=np.complex128))
    bad = [dict(alpha=[[9, 0]], coef=[1.0]), dict(alpha=[[1, 0]], coef=[float("nan")]),
           dict(alpha=[[1, 0]] * 17, coef=[1.0] * 17), dict(alpha=[[1, 0]], coef=[1.0], box_lo=(0.0, 1.0),
                                                           box_hi=(1.0, 1.0))]
    for kw in bad:
        kw = dict(kw)
        kw.setdefault("box_lo", (-1.0, -1.0))
        kw.setdefault("box_hi", (1.0, 1.0))
        with pytest.raises(fk.FkError) as e:
            fk.solve(M, b, 2, [1e-2], penalty="pde_box", mu=1.0, **kw)
        assert e.value.code == 1
    # the iterative solver takes diagonal penalties only
    with pytest.raises(fk.FkError) as e:
        fk.solve_cg(M, b, 2, [1e-2], penalty="pde_box", mu=1.0, alpha=[[1, 0]], coef=[1.0], box_lo=(-1.0, -1.0),
                    box_hi=(1.0, 1.0))
    assert e.value.code == 1


def test_solve_reports_non_finite_right_hand_side(fk):
    rng = np.random.default_rng(8)
    X = rng.uniform(-np.pi, np.pi, size=(2, 5000))
    M = oracle.gram_generator(X, 4)
    b = oracle.rhs(X, np.sin(X[:1]), 4)
    # index 7 is the -k member of its pair (the real form reads the +k member), 40 is k = 0
    for v, i in [(np.nan, 7), (np.inf, 7), (np.nan, 40), (-np.inf, 80 - 7)]:
        bb = b.copy()
        bb[0, i] = v
        with pytest.raises(fk.FkError) as e:
            fk.solve(_cplx(M), _cplx(bb), 4, [1e-3, 1e-2])
        assert e.value.code == 3


def test_error_paths(fk):
    X = torch.from_numpy(synth.uniform_points(3, 2, 10_000)).cuda()
    Y = torch.ones((1, 10_000), dtype=torch.float32, device="cuda")
    with pytest.raises(fk.FkError) as e:
        fk.fit(X, Y, 8, -1.0)
    assert e.value.code == 1
    with pytest.raises(fk.FkError) as e:
        fk.fit(X, Y, 8, 1e-3, penalty="sobolev", s=-1.0)
    assert e.value.code == 1
    # refinement cap 0 with a tight tolerance cannot be met
    ctx = fk.Context(0, max_refine=0, refine_tol=1e-15)
    with pytest.raises(fk.FkError) as e:
        fk.fit(X, Y, 8, 1e-3, ctx=ctx)
    assert e.value.code == 5
