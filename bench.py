"""Benchmark: Gram+RHS points/s and fit time (one MI355X).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched|sobolev2d] [--n N]

A step is one pass of the whole hot path over one batch of synthetic input
already resident in HBM:
  batched   (default) 2-D Sobolev, n = 1e9 fp32 points generated on the device from a
            seed, 16 targets, m = 32, 64 log-spaced lambdas in [1e-8, 1e-1]:
            type-1 Gram + 16 right-hand sides, assembly, 64 batched FP32 Cholesky
            factorizations with FP64 refinement, held-out (n_v = 1e7) Gram and MSE,
            and the backward pass (adjoint solves, d/dlog lambda and d/dp).
  sobolev2d 2-D Sobolev, n = 1e7, one target, one lambda: type-1 stage + solve.
  cg        the batched inputs (n = 1e9, 16 targets, m = 32, 64 lambdas, s = 2 Sobolev
            weights): type-1 Gram + right-hand sides, then all 1024 systems by
            Jacobi-preconditioned conjugate gradients with FFT Toeplitz products (tol 1e-10).
Prints one JSON line.  value = n / (seconds per step) = whole-step points/s.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3
MFMA_F16_PEAK_TFLOPS = 2500.0
SPLIT_TERMS = 3   # FP16 products per FP32-accurate product of two FP16-pair operands


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _blas_vendor() -> str:
    import numpy as np
    try:
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        return f"{b.get('name', '?')} {b.get('version', '')}".strip()
    except Exception:
        return "unknown"


def _cpu_baseline(Xd, Yd, m: int, lam: float):
    """Time the FP64 CPU oracle on a bounded prefix of the workload's own inputs (copied from the
    device): the direct Fourier sums for M and b (linear in n, so points/s extrapolates) and,
    separately, one FP64 LAPACK Cholesky solve of the (2m+1)^2 system (independent of n)."""
    import numpy as np
    import oracle
    from oracle.fourier import _threads
    threads = str(_threads())
    ntgt = Yd.shape[0]
    n = min(Xd.shape[1], 12_000_000 if ntgt > 1 else 4_000_000)   # about 10-20 s of host work
    X = Xd[:, :n].cpu().numpy()
    Y = Yd[:, :n].cpu().numpy()
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    t0 = time.perf_counter()
    M = oracle.gram_generator(X64, m)
    b = oracle.rhs(X64, Y64, m)
    dt = time.perf_counter() - t0
    p = oracle.sobolev_weights(m, 2, 2.0)
    t1 = time.perf_counter()
    oracle.solve_system(oracle.system_matrix(M, m, lam, p), b)
    ds = time.perf_counter() - t1
    return {"value": n / dt, "unit": "points/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": _cpu_model(), "blas": _blas_vendor(), "solve_s_per_lambda": ds,
            "sample": f"FP64 direct sums for M (|q|<=2m) and {ntgt} right-hand sides on the first {n} points "
                      f"({dt:.1f} s); one FP64 LAPACK Cholesky solve of the {(2 * m + 1) ** 2}-unknown complex "
                      f"system for the {ntgt} targets ({ds:.1f} s per lambda)"}


def _traffic(kernel: str, n: int):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was taken on the
    current source of the kernel (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_hbm_traffic.md")
    unit = {"k_spread_mfma": "spread_mfma.hip", "k_spread_op": "spread_op.hip"}.get(kernel)
    if unit is None:
        return None
    src = os.path.join(ROOT, "paper_2509_02649_amd", "csrc", unit)
    if not os.path.exists(path) or not os.path.exists(src):
        return None
    text = open(path).read()
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    b = re.search(r"hbm_bytes_per_point:\s*([0-9.eE+-]+)", text)
    if not h or not b or h.group(1) != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return float(b.group(1)) * n


def _fft_roofline(fk, torch, M, m, nvec, ctx, reps=5):
    """FFT Toeplitz product over nvec vectors (the per-iteration product of the CG solve), timed
    with HIP events on the library's stream.  Algorithmic bytes per call (2-D): every vector read
    and written once (2 N complex), the two intermediates of Lf x (2m+1) entries written and read
    once each (4 Lf (2m+1)), and the Lf^2 spectrum read once."""
    N, n0 = (2 * m + 1) ** 2, 2 * m + 1
    Lf = 1
    while Lf < 4 * m + 1:
        Lf <<= 1
    x = torch.randn(nvec, N, dtype=torch.complex128, device=M.device)
    fk.toeplitz_apply(M, x, m, ctx=ctx)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fk.toeplitz_apply(M, x, m, ctx=ctx)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 16.0 * (nvec * (2 * N + 4 * Lf * n0) + Lf * Lf)
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": "k_line_fft256" if Lf == 256 else "k_line_fft", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": _traffic_fft(nvec, m), "ms_per_product": ms, "vectors": nvec}


def _traffic_fft(nvec: int, m: int):
    """HBM bytes of one product from the committed counter summary (measured for 1024 vectors at
    m = 32), if it was taken on the current source of the transform (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_line_fft256_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2509_02649_amd", "csrc", "cg.hip")
    if nvec != 1024 or m != 32 or not os.path.exists(path) or not os.path.exists(src):
        return None
    text = open(path).read()
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    b = re.search(r"hbm_bytes_per_product:\s*([0-9.eE+-]+)", text)
    if not h or not b or h.group(1) != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return float(b.group(1))


def _extra_batched(fk, torch, np, X, Y, m, ctx, theta, reps=3):
    """Further figures on the batched inputs (outside the timed steps):
    * the single-target type-1 stage on the same n points (the first target row, one lambda), HIP-event
      time; algorithmic HBM bytes 12 per point;
    * the type-2 prediction at n_q = 1e8 query points for 16 coefficient sets (one lambda's fits),
      timed with HIP events on the library's stream; algorithmic HBM bytes: 4d B of coordinates read
      and 4 B per set written per point."""
    n = X.shape[1]
    one = []
    for _ in range(reps + 1):
        _, inf = fk.fit(X, Y[:1], m, [float(n) ** -0.8], penalty="sobolev", s=2.0, ctx=ctx, info=True)
        one.append(inf)
    one = one[1:]
    gr1 = float(np.mean([i["t_sort_ms"] + i["t_spread_ms"] + i["t_fft_ms"] for i in one]))
    res = {"single_target": {"n": n, "gram_rhs_ms": gr1, "sort_ms": float(np.mean([i["t_sort_ms"] for i in one])),
                                  "spread_ms": float(np.mean([i["t_spread_ms"] for i in one])),
                                  "points_per_s": n / (gr1 * 1e-3),
                                  "hbm_frac": n * 12.0 / (gr1 * 1e-3) / (HBM_PEAK_GBS * 1e9)}}
    nq = 100_000_000
    Xq = fk.generate_uniform(2509026495 + 2000, 2, nq, ctx=ctx)
    th = theta[theta.shape[0] // 2].contiguous()          # [16, N]
    fk.predict(th, Xq, m, ctx=ctx)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fk.predict(th, Xq, m, ctx=ctx)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    T = th.shape[0]
    res["predict"] = {"nq": nq, "sets": T, "ms": ms, "points_per_s": nq / (ms * 1e-3),
                      "hbm_frac": nq * (8.0 + 4.0 * T) / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}
    del Xq
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched", choices=["batched", "sobolev2d", "cg"])
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="copy 1 GiB device to device before the steps (reference dispatch for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the point stream would shard "
              "by an all-reduce of the FP64 fine grids or of the extracted M and b)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2509_02649_amd as fk

    dev = torch.device("cuda:0")
    m = 32
    # the autograd Function and the plain fits share one context (one cached workspace)
    ctx = fk.default_context(0)
    vctx = fk.Context(0)
    if args.workload in ("batched", "cg"):
        n = args.n or 1_000_000_000
        nv = 10_000_000
        ntgt, nlam = 16, 64
        seed = 2509026495
        X = fk.generate_uniform(seed, 2, n, ctx=ctx)
        Y = fk.generate_targets(seed, X, ntgt, ctx=ctx)
        Xv = fk.generate_uniform(seed + 1000, 2, nv, ctx=ctx)
        Yv = fk.generate_targets(seed + 1000, Xv, ntgt, ctx=ctx)
        lams = [10.0 ** (-8.0 + 7.0 * i / (nlam - 1)) for i in range(nlam)]
        kk = np.stack(np.meshgrid(np.arange(-m, m + 1), np.arange(-m, m + 1), indexing="ij"), -1).reshape(-1, 2)
        p0 = torch.tensor(1.0 + ((kk ** 2).sum(1).astype(np.float64)) ** 2.0, device=dev)
        bytes_per_point = 4 * 2 + 4 * ntgt
    else:
        n = args.n or 10_000_000
        ntgt, nlam = 1, 1
        X = fk.generate_uniform(2509026492, 2, n, ctx=ctx)
        Y = fk.generate_targets(2509026492, X, 1, ctx=ctx)
        lams = [float(n) ** (-4.0 / 5.0)]
        bytes_per_point = 4 * 2 + 4
    torch.cuda.synchronize()
    if args.calibrate:
        # a plain copy of known size (1 GiB read, 1 GiB written) for scaling the HBM byte counters
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    infos = []
    cg_iters = []
    last = {}
    CG_TOL = 1e-10
    if args.workload in ("batched", "sobolev2d"):
        # size the shared workspace once, for the largest call (the plain fit)
        nb = C.c_size_t()
        fk._lib.check(ctx.lib.fk_fit_workspace_size(ctx.h, 2, n, ntgt, m, nlam, C.byref(nb)), "ws")
        ctx.workspace(nb.value)

    def plain_fit():
        pen = dict(penalty="diag", p=p0) if args.workload == "batched" else dict(penalty="sobolev", s=2.0)
        theta, info = fk.fit(X, Y, m, lams, ctx=ctx, info=True, **pen)
        infos.append(info)
        last["theta"] = theta

    def step():
        if args.workload == "cg":
            M, b, info = fk.gram(X, Y, m, ctx=ctx, info=True)
            theta, cinf = fk.solve_cg(M, b, m, lams, penalty="sobolev", s=2.0, tol=CG_TOL, ctx=ctx, info=True)
            last["M"] = M
            infos.append(info)
            cg_iters.append(cinf["iters"])
        elif args.workload == "batched":
            # the gradient path: the autograd Function's forward (fit, held-out Gram and MSE) and backward
            # (adjoint solves, d/dlog lambda and d/dp)
            loglam = torch.tensor(np.log(lams), dtype=torch.float64, device=dev, requires_grad=True)
            p = p0.clone().requires_grad_(True)
            mse, theta = fk.KernelRidgeGridLoss.apply(loglam, p, X, Y, Xv, Yv, m)
            mse.sum().backward()
            last["grad"] = loglam.grad
        else:
            plain_fit()

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    if args.workload == "batched":
        # plain fit (type-1 stage + 64 factorizations + refined solves), wall clock, with its stage times
        plain_fit()
        infos.clear()
        fit_s = timed(plain_fit, args.steps)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.workload != "batched":
        infos.clear()
    dt = timed(step, args.steps)

    spread_ms = float(np.mean([i["spread_kernel_ms"] for i in infos]))
    gr_ms = float(np.mean([i["t_sort_ms"] + i["t_spread_ms"] + i["t_fft_ms"] for i in infos]))
    if args.workload == "batched":
        fit_ms = fit_s * 1e3
    else:
        fit_ms = float(np.mean([i["t_total_ms"] for i in infos])) if args.workload != "cg" else dt * 1e3
    w = int(infos[-1]["w"])
    if args.workload in ("batched", "cg"):
        # dominant kernel: the MFMA spread; algorithmic work 2 w^2 (T + 1) flop per point
        # (every point adds its w x w kernel products to T target channels and the ones channel)
        kernel, bound, unit, peak = "k_spread_mfma", "mfma", "TFLOP/s", MFMA_F32_PEAK_TFLOPS
        work = n * 2.0 * w * w * (ntgt + 1)
        achieved = work / (spread_ms * 1e-3) / 1e12
    else:
        # dominant kernel: the outer-product MFMA spread; algorithmic bytes = inputs read once
        kernel, bound, unit, peak = "k_spread_op", "hbm", "GB/s", HBM_PEAK_GBS
        achieved = n * bytes_per_point / (spread_ms * 1e-3) / 1e9
    out = {
        "metric": "Gram+RHS points/s and fit time at 1e-6 Gram err; grad-path vs plain fit ratio",
        "value": n / dt,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 spread / f64 grid+FFT / f64 conjugate gradients with f64 FFT products"
                  if args.workload == "cg" else "f32 spread / f64 grid+FFT / f32 Cholesky with f16-pair panel products on MFMA + f64 refinement"),
        "data": "synthetic (Philox4x32-10 on device)",
        "config": {"workload": ("2-D Sobolev, n=%d fp32 ~U[-pi,pi)^2, %d targets sin(t x1)cos(x2)+N(0,0.01), "
                                "m=32, %d lambdas, held-out n=1e7 MSE + backward" % (n, ntgt, nlam))
                   if args.workload == "batched" else
                   ("2-D Sobolev, n=%d fp32 ~U[-pi,pi)^2, %d targets sin(t x1)cos(x2)+N(0,0.01), m=32, s=2, "
                    "%d lambdas, conjugate gradients to ||r|| <= 1e-10 ||b||" % (n, ntgt, nlam))
                   if args.workload == "cg" else
                   ("2-D Sobolev, n=%d fp32 ~U[-pi,pi)^2, Y=exp(-|x|^2)+N(0,0.01), m=32, s=2, lambda=n^-0.8"
                    % n),
                   "n": n, "m": m, "targets": ntgt, "lambdas": nlam},
        "gram_rhs_ms": gr_ms,
        "gram_rhs_points_per_s": n / (gr_ms * 1e-3),
        "fit_ms": fit_ms,
        "stage_ms": {k: float(np.mean([i[k] for i in infos])) for k in
                     ["t_sort_ms", "t_spread_ms", "t_fft_ms", "t_assemble_ms", "t_factor_ms", "t_solve_ms"]},
        "refine_iters": int(infos[-1]["refine_iters"]),
        "roofline": {"bound": bound, "kernel": kernel, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": _traffic(kernel, n)},
        "gram_rhs_hbm_frac": n * bytes_per_point / (gr_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
    }
    if args.workload in ("batched", "sobolev2d"):
        # the dense solve: nlam Cholesky factorizations of the N x N real form, N^3/3 flop each (one
        # real-form factor per lambda), nearly all of it in the panel updates, which run on the FP16
        # matrix cores with FP16-pair operands (three FP16 products per FP32-accurate product): the
        # peak is the FP16 dense peak over those three
        N = (2 * m + 1) ** 2
        fac_ms = out["stage_ms"]["t_factor_ms"]
        ach = nlam * N ** 3 / 3.0 / (fac_ms * 1e-3) / 1e12
        peak_s = MFMA_F16_PEAK_TFLOPS / SPLIT_TERMS
        out["roofline_solve"] = {"bound": "mfma", "kernel": "factorization (k_left_update2, k_left_update, "
                                 "k_potrf_diag, k_trsm_panel)", "achieved": ach, "peak": peak_s,
                                 "unit": "TFLOP/s", "frac": ach / peak_s, "factor_ms": fac_ms,
                                 "flop": nlam * N ** 3 / 3.0,
                                 "peak_basis": "f16 dense %.0f TFLOP/s / %d products per f32-accurate product"
                                               % (MFMA_F16_PEAK_TFLOPS, SPLIT_TERMS),
                                 "frac_of_f32_peak": ach / MFMA_F32_PEAK_TFLOPS}
    if args.workload == "batched":
        # grad path (autograd Function forward + backward) over the plain fit, both wall clock
        out["grad_vs_fit_ratio"] = dt * 1e3 / fit_ms
        out["grad_step_ms"] = dt * 1e3
        out.update(_extra_batched(fk, torch, np, X, Y, m, ctx, last["theta"]))
    if args.workload == "cg":
        out["cg_iters"] = int(max(cg_iters))
        out["cg_ms"] = dt * 1e3 - gr_ms
        out["roofline_fft"] = _fft_roofline(fk, torch, last["M"], m, nlam * ntgt, ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(X, Y, m, lams[nlam // 2])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
