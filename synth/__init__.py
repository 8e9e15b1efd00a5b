"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the CPU oracle, the tests and the benchmark.  It
holds no arithmetic of the fitting method: it only draws points and targets.

Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), a counter-based
generator.  The device-side generator in the HIP library implements the same
published definition, so a prefix drawn here is bit-identical to the device
draw for the integer stream and for the uniform coordinates.

Counter layout (one 128-bit counter per point j and stream s):
    counter = (j mod 2^32, j >> 32, s, 0), key = (seed mod 2^32, seed >> 32)
Stream 0 gives the coordinates (word 0 -> dim 0, word 1 -> dim 1, ...; for
d > 4 the stream index s = 16 + d//4 continues), streams 1 + t give the noise
of target t by Box-Muller on words (0, 1).
"""
from __future__ import annotations

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
MASK32 = np.uint64(0xFFFFFFFF)

TWO_PI = 2.0 * np.pi


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on uint32 arrays (SC'11, Sec. 4)."""
    c0 = np.asarray(c0, dtype=np.uint32)
    c1 = np.asarray(c1, dtype=np.uint32)
    c2 = np.asarray(c2, dtype=np.uint32)
    c3 = np.asarray(c3, dtype=np.uint32)
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    with np.errstate(over="ignore"):
        for _ in range(10):
            p0 = PHILOX_M0 * c0.astype(np.uint64)
            p1 = PHILOX_M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint32(k0), lo1, hi0 ^ c3 ^ np.uint32(k1), lo0
            k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
            k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
    return c0, c1, c2, c3


def _words(seed: int, stream: int, start: int, n: int):
    j = np.arange(start, start + n, dtype=np.uint64)
    c0 = (j & MASK32).astype(np.uint32)
    c1 = (j >> np.uint64(32)).astype(np.uint32)
    c2 = np.full(n, stream, dtype=np.uint32)
    c3 = np.zeros(n, dtype=np.uint32)
    return philox4x32_10(c0, c1, c2, c3, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def u01(word):
    """Top 24 bits of a uint32 word as a float in [0, 1), exact in float32."""
    return (np.asarray(word, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * (2.0 ** -24)


def uniform_points(seed: int, d: int, n: int, lo: float = -np.pi, hi: float = np.pi,
                   start: int = 0, dtype=np.float32) -> np.ndarray:
    """Points ~ U[lo, hi)^d as a [d, n] array (structure of arrays).

    The coordinate is lo + (hi - lo) * u computed in float64 (one multiply, one
    add, no fused operation) and then rounded to `dtype`.
    """
    out = np.empty((d, n), dtype=dtype)
    for g in range((d + 3) // 4):
        stream = 0 if g == 0 else 16 + g
        w = _words(seed, stream, start, n)
        for r in range(4):
            dim = 4 * g + r
            if dim >= d:
                break
            u = u01(w[r])
            out[dim] = (np.float64(lo) + np.float64(hi - lo) * u).astype(dtype)
    return out


def normal_noise(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Standard normals by Box-Muller on Philox words 0 and 1 (float64)."""
    w = _words(seed, stream, start, n)
    u1 = (w[0].astype(np.float64) + 1.0) * (2.0 ** -32)   # (0, 1]
    u2 = w[1].astype(np.float64) * (2.0 ** -32)           # [0, 1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(TWO_PI * u2)


# ---------------------------------------------------------------------------
# The five workload shapes.  Each returns a dict with X [d, n], Y [T, n] and the
# method parameters.  None of them computes anything of the fitting method.
# ---------------------------------------------------------------------------

SEED_BASE = 2509026490


def workload_1d(n: int = 10_000, seed: int = SEED_BASE + 1, start: int = 0):
    """1-D Sobolev regression: X ~ U[-pi, pi) fp64, Y = sin 3X + cos(7X)/2 + N(0, 0.1^2)."""
    X = uniform_points(seed, 1, n, start=start, dtype=np.float64)
    x = X[0]
    Y = np.sin(3.0 * x) + 0.5 * np.cos(7.0 * x) + 0.1 * normal_noise(seed, 1, n, start)
    return dict(X=X, Y=Y[None, :].astype(np.float64), m=50, s=1.0,
                lam=float(n) ** (-2.0 / 3.0), penalty="sobolev")


def workload_2d(n: int = 10_000_000, seed: int = SEED_BASE + 2, start: int = 0):
    """2-D Sobolev regression: X ~ U[-pi, pi)^2 fp32, Y = exp(-|x|^2) + N(0, 0.1^2)."""
    X = uniform_points(seed, 2, n, start=start)
    x = X.astype(np.float64)
    Y = np.exp(-(x[0] ** 2 + x[1] ** 2)) + 0.1 * normal_noise(seed, 1, n, start)
    return dict(X=X, Y=Y[None, :].astype(np.float32), m=32, s=2.0,
                lam=float(n) ** (-4.0 / 5.0), penalty="sobolev")


def workload_piml(n: int = 100_000_000, seed: int = SEED_BASE + 3, start: int = 0):
    """Heat-equation PIML: (t, x) ~ U[-pi/2, pi/2]^2 fp32, Y = exp(-t) sin x + N(0, 0.05^2)."""
    X = uniform_points(seed, 2, n, lo=-np.pi / 2, hi=np.pi / 2, start=start)
    x = X.astype(np.float64)
    Y = np.exp(-x[0]) * np.sin(x[1]) + 0.05 * normal_noise(seed, 1, n, start)
    return dict(X=X, Y=Y[None, :].astype(np.float32), m=20, s=1.0,
                lam=1e-4, mu=1.0, penalty="piml_heat")


def workload_additive(n: int = 100_000_000, d: int = 10, seed: int = SEED_BASE + 4, start: int = 0):
    """Additive model: X ~ U[-pi, pi)^10 fp32, Y = sum_a sin((a+1) X_a)/(a+1) + N(0, 0.1^2)."""
    X = uniform_points(seed, d, n, start=start)
    x = X.astype(np.float64)
    Y = sum(np.sin((a + 1) * x[a]) / (a + 1) for a in range(d)) + 0.1 * normal_noise(seed, 1, n, start)
    return dict(X=X, Y=Y[None, :].astype(np.float32), m=32, s=1.0,
                lam=float(n) ** (-2.0 / 3.0), penalty="additive")


def batched_targets(X: np.ndarray, seed: int, ntgt: int = 16, start: int = 0) -> np.ndarray:
    """Targets Y_t = sin(t x1) cos(x2) + N(0, 0.1^2), t = 1..ntgt, as fp32 [ntgt, n]."""
    x = X.astype(np.float64)
    n = X.shape[1]
    Y = np.empty((ntgt, n), dtype=np.float32)
    c2 = np.cos(x[1])
    for t in range(1, ntgt + 1):
        Y[t - 1] = (np.sin(t * x[0]) * c2 + 0.1 * normal_noise(seed, t, n, start)).astype(np.float32)
    return Y


def workload_batched(n: int = 1_000_000_000, n_val: int = 10_000_000, seed: int = SEED_BASE + 5,
                     start: int = 0, val_start: int = 0, ntgt: int = 16, nlam: int = 64):
    """Differentiable batched 2-D Sobolev: training and validation draws from
    independent seeds, 16 targets, 64 log-spaced lambdas in [1e-8, 1e-1]."""
    X = uniform_points(seed, 2, n, start=start)
    Y = batched_targets(X, seed, ntgt, start)
    vseed = seed + 1000
    Xv = uniform_points(vseed, 2, n_val, start=val_start)
    Yv = batched_targets(Xv, vseed, ntgt, val_start)
    lams = 10.0 ** (-8.0 + 7.0 * np.arange(nlam) / (nlam - 1))
    return dict(X=X, Y=Y, Xv=Xv, Yv=Yv, m=32, s=2.0, lams=lams, penalty="sobolev")
