"""Parity of the type-1 stage (Gram generator M and right-hand side b) with the FP64 oracle.

Bars: eps_T = max_q |M_gpu - M| / M[0] <= 1e-6 (M[0] = 1 bounds every |M[q]|), and
eps_b = max_k |b_gpu - b| / (n^-1 sum_j |Y_j|) <= 1e-6 (the scale that bounds every |b_k|).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def fk():
    import paper_2509_02649_amd as fk
    return fk


def _errors(fk, X, Y, m, keep=None):
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    M, b, info = fk.gram(Xd, Yd, m, info=True)
    M = M.cpu().numpy()
    b = b.cpu().numpy()
    Mo = oracle.gram_generator(X.astype(np.float64), m)
    bo = oracle.rhs(X.astype(np.float64), Y.astype(np.float64), m)
    eT = np.abs(M - Mo).max() / abs(Mo.ravel()[Mo.size // 2])
    scale = np.abs(Y.astype(np.float64)).mean(axis=1, keepdims=True)
    eb = (np.abs(b - bo) / scale).max()
    if keep is not None:
        keep.update(Mo=Mo, bo=bo, Xd=Xd, Yd=Yd)
    return eT, eb, info


def test_gram_1d_small_config_fp64(fk):
    w = synth.workload_1d()
    eT, eb, info = _errors(fk, w["X"], w["Y"], w["m"])
    print(f"1-D n=1e4 m=50: eps_T={eT:.2e} eps_b={eb:.2e} w={info['w']} nf={info['nf']}")
    assert eT <= TOL and eb <= TOL


@pytest.mark.parametrize("m,ntgt", [(64, 32), (64, 19), (40, 32)])
def test_gram_1d_many_channels(fk, m, ntgt):
    # more channels than one workgroup's LDS holds as whole FP64 grids (C x nf x 8 B > 160 KB at
    # nf = 1024): the channels are spread in groups, the ones channel with the first
    rng = np.random.default_rng(m + ntgt)
    n = 30_001
    X = rng.uniform(-np.pi, np.pi, size=(1, n)).astype(np.float32)
    Y = rng.standard_normal((ntgt, n)).astype(np.float32)
    eT, eb, info = _errors(fk, X, Y, m)
    print(f"1-D m={m} T={ntgt}: eps_T={eT:.2e} eps_b={eb:.2e} nf={info['nf']}")
    assert eT <= TOL and eb <= TOL


@pytest.mark.parametrize("n", [1, 7, 1000, 65_537])
def test_gram_2d_sizes_and_ragged(fk, n):
    w = synth.workload_2d(n=n, seed=11 + n)
    eT, eb, info = _errors(fk, w["X"], w["Y"], 32)
    print(f"2-D n={n}: eps_T={eT:.2e} eps_b={eb:.2e} w={info['w']} nf={info['nf']} bin={info['bin']}")
    assert eT <= TOL and eb <= TOL


@pytest.mark.parametrize("m", [1, 5, 20])
def test_gram_2d_other_m(fk, m):
    w = synth.workload_2d(n=20_000, seed=40 + m)
    eT, eb, _ = _errors(fk, w["X"], w["Y"], m)
    assert eT <= TOL and eb <= TOL


@pytest.mark.parametrize("ntgt,n", [(16, 30_000), (8, 50_000), (7, 20_000), (17, 20_000), (16, 1_000_000),
                                    (2, 40_000), (3, 40_001), (16, 1), (16, 7), (3, 1), (2, 5)])
def test_gram_2d_multi_target(fk, ntgt, n):
    # 8..16 targets: channel-row MFMA spread (4 x 4-cell bins at these sizes), weights gathered
    # by position; 0..7 targets: outer-product MFMA spread over 8 x 8-cell bins with 1-, 2-, 4-
    # or 8-word records; 17 targets: the FP64 atomic spread.  n = 1, 5 and 7 leave most bins empty.
    X = synth.uniform_points(77 + ntgt, 2, n)
    Y = synth.batched_targets(X, 77 + ntgt, ntgt=ntgt)
    eT, eb, info = _errors(fk, X, Y, 32)
    print(f"2-D T={ntgt} n={n}: eps_T={eT:.2e} eps_b={eb:.2e} bin={info['bin']} spread={info['t_spread_ms']:.3f} ms")
    assert eT <= TOL and eb <= TOL


@pytest.mark.parametrize("ntgt,n,m", [(16, 5_000_000, 4), (9, 4_300_000, 4)])
def test_gram_2d_multi_target_dense_bins(fk, ntgt, n, m):
    # dense bins (>= 4096 points per 2 x 2-cell bin on the 64 x 64 grid of m = 4) take the
    # MFMA spread over 2 x 2-cell bins; the same path serves the 1e9-point workload (m = 32)
    X = synth.uniform_points(91 + ntgt, 2, n)
    Y = synth.batched_targets(X, 91 + ntgt, ntgt=ntgt)
    eT, eb, info = _errors(fk, X, Y, m)
    print(f"2-D T={ntgt} n={n} m={m}: eps_T={eT:.2e} eps_b={eb:.2e} bin={info['bin']} nf={info['nf']}")
    assert info["bin"] == -2
    assert eT <= TOL and eb <= TOL


@pytest.mark.parametrize("n", [3, 250_001])
def test_gram_only_no_targets(fk, n):
    # the Gram channel alone (Y = None): records without weight words, one MFMA per 4 points
    X = synth.uniform_points(63, 2, n)
    M, b = fk.gram(torch.from_numpy(X).cuda(), None, 24)
    Mo = oracle.gram_generator(X.astype(np.float64), 24)
    eT = np.abs(M.cpu().numpy() - Mo).max() / abs(Mo.ravel()[Mo.size // 2])
    print(f"2-D gram only n={n}: eps_T={eT:.2e}")
    assert b is None or b.numel() == 0
    assert eT <= TOL


@pytest.mark.parametrize("ntgt", [16, 1])
@pytest.mark.parametrize("shape", ["square", "line"])
def test_gram_clustered_points(fk, ntgt, shape):
    # skewed inputs for the two-pass sort and the binned spreads: every point in one small square
    # (one or a few bins take all 300k points, cut into slices; every other bin empty), or on the
    # line x1 = 0.3 (one bin row takes all points in the first pass)
    rng = np.random.default_rng(17 + ntgt)
    n = 300_000
    if shape == "square":
        X = rng.uniform(0.1, 0.112, size=(2, n))
    else:
        X = np.stack([np.full(n, 0.3), rng.uniform(-np.pi, np.pi, size=n)])
    X = X.astype(np.float32)
    Y = rng.standard_normal((ntgt, n)).astype(np.float32)
    eT, eb, info = _errors(fk, X, Y, 8)
    print(f"clustered ({shape}) T={ntgt}: eps_T={eT:.2e} eps_b={eb:.2e} bin={info['bin']}")
    assert eT <= TOL and eb <= TOL


def test_gram_boundary_points_fold(fk):
    # points on the seam: -pi, fp32(pi) > pi, values just inside [-2pi, 2pi) that fold
    pts = np.array([-np.pi, np.float32(np.pi), 0.0, -2 * np.pi + 1e-3, 2 * np.pi - 1e-3, 3.0, -3.0],
                   dtype=np.float32)
    X = np.stack([pts, pts[::-1].copy()]).astype(np.float32)
    Y = np.linspace(-1, 1, X.shape[1], dtype=np.float32)[None, :]
    eT, eb, _ = _errors(fk, X, Y, 16)
    assert eT <= TOL and eb <= TOL


def test_gram_half_box_points(fk):
    w = synth.workload_piml(n=50_000)
    eT, eb, _ = _errors(fk, w["X"], w["Y"], w["m"])
    assert eT <= TOL and eb <= TOL


def test_gram_full_size_2d_config(fk):
    # 2-D Sobolev configuration at full size: n = 1e7 fp32 points, m = 32, s = 2, lambda = n^-0.8;
    # the type-1 outputs element by element, then theta end to end (type-1 stage + solve)
    w = synth.workload_2d()
    o = {}
    eT, eb, info = _errors(fk, w["X"], w["Y"], w["m"], keep=o)
    print(f"2-D n=1e7 m=32: eps_T={eT:.2e} eps_b={eb:.2e} spread={info['t_spread_ms']:.3f} ms "
          f"sort={info['t_sort_ms']:.3f} ms total={info['t_total_ms']:.3f} ms")
    assert eT <= TOL and eb <= TOL
    m, lam = w["m"], w["lam"]
    p = oracle.sobolev_weights(m, 2, w["s"])
    A = oracle.system_matrix(o["Mo"], m, lam, p)
    th = oracle.solve_system(A, o["bo"])
    kappa = oracle.condition_number(A)
    tg = fk.fit(o["Xd"], o["Yd"], m, lam, penalty="sobolev", s=w["s"])[0].cpu().numpy()
    e = np.linalg.norm(tg - th) / np.linalg.norm(th)
    print(f"2-D n=1e7 theta end to end: rel={e:.2e} kappa={kappa:.2e}")
    assert kappa <= 1e6 and e <= 1e-4


def test_invalid_inputs_are_reported(fk):
    X = synth.uniform_points(5, 2, 1000)
    Y = np.ones((1, 1000), dtype=np.float32)
    Xn = X.copy()
    Xn[0, 17] = np.nan
    with pytest.raises(fk.FkError) as e:
        fk.gram(torch.from_numpy(Xn).cuda(), torch.from_numpy(Y).cuda(), 8)
    assert e.value.code == 3
    Xr = X.copy()
    Xr[1, 3] = 7.0
    with pytest.raises(fk.FkError) as e:
        fk.gram(torch.from_numpy(Xr).cuda(), torch.from_numpy(Y).cuda(), 8)
    assert e.value.code == 2
    Yn = Y.copy()
    Yn[0, 5] = np.inf
    with pytest.raises(fk.FkError) as e:
        fk.gram(torch.from_numpy(X).cuda(), torch.from_numpy(Yn).cuda(), 8)
    assert e.value.code == 3
    # the context recovers after an error
    M, b = fk.gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), 8)
    assert abs(M[16, 16].item() - 1.0) < 1e-6


def test_device_generator_matches_host_generator(fk):
    seed, n = 2509026495, 200_000
    Xd = fk.generate_uniform(seed, 2, n, start=123)
    Xh = synth.uniform_points(seed, 2, n, start=123)
    assert np.array_equal(Xd.cpu().numpy(), Xh)
    Yd = fk.generate_targets(seed, Xd, 16, start=123).cpu().numpy()
    Yh = synth.batched_targets(Xh, seed, 16, start=123)
    ulp = np.abs(Yd.view(np.int32).astype(np.int64) - Yh.view(np.int32).astype(np.int64))
    assert ulp.max() <= 1
    assert (ulp == 0).mean() > 0.999


def test_gram_full_size_batched_sampled(fk):
    # The batched workload at full size, in the configuration bench.py times: n = 1e9 points and
    # 16 targets generated on the device (seed of the benchmark), m = 32, two-pass sort into
    # 2 x 2-cell bins and the MFMA spread.  The oracle evaluates sampled entries one by one.
    import gc
    n, T, m, seed = 1_000_000_000, 16, 32, 2509026495
    gc.collect()
    torch.cuda.empty_cache()
    ctx = fk.Context(0)
    X = fk.generate_uniform(seed, 2, n, ctx=ctx)
    Y = fk.generate_targets(seed, X, T, ctx=ctx)
    M, b, info = fk.gram(X, Y, m, ctx=ctx, info=True)
    assert info["bin"] == -2
    M = M.cpu().numpy()
    b = b.cpu().numpy()
    Xh = X.cpu().numpy()
    del X, ctx
    gc.collect()
    torch.cuda.empty_cache()
    Yh = Y.cpu().numpy()                      # [16, 1e9] fp32, 64 GB of host memory
    del Y
    gc.collect()
    torch.cuda.empty_cache()
    c = 2 * m
    assert abs(M[c, c] - 1.0) <= 1e-6
    errs = []
    # M: q = 0, the four corners of the +-2m square, the axes' ends and two interior frequencies
    qs = np.array([(0, 0), (1, 0), (64, -64), (-64, 64), (64, 64), (-64, -1), (0, 64), (37, -5), (-12, 50)])
    mo = oracle.fourier_entries(Xh, None, qs, +1)[0]
    for q, v in zip(qs, mo):
        errs.append(abs(M[c + q[0], c + q[1]] - v))
    print(f"M at {len(qs)} frequencies: max error {max(errs):.2e}", flush=True)
    # b: every target at two frequencies (the exponentials shared by the 16 weight rows)
    ks = np.array([(-32, 31), (5, -17)])
    bo = oracle.fourier_entries(Xh, Yh, ks, -1)           # [16, 2]
    for t in range(T):
        sc = float(np.abs(Yh[t]).mean(dtype=np.float64))
        bt = b[t].reshape(2 * m + 1, 2 * m + 1)
        for f, k in enumerate(ks):
            errs.append(abs(bt[m + k[0], m + k[1]] - bo[t, f]) / sc)
    print(f"b of {T} targets at {len(ks)} frequencies: max error {max(errs[len(qs):]):.2e}", flush=True)
    print(f"n=1e9 T=16 sampled: errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= TOL
