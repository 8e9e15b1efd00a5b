// Conjugate-gradient solve of (Sigma + lambda P) theta = b with the multilevel-Toeplitz
// product done by FFT (Sec. 2.3, "Matrix inversion" and "Covariance matrix").
//
// Product.  Sigma[k, l] = M[l - k] over k, l in {-m..m}^d.  With mode k stored at
// position k + m (0..2m) per axis, (Sigma x)[k] = sum_l c[(k + m) - (l + m)] x[l] with
// c[r] = M[-r], r in [-2m, 2m]^d: a d-dimensional linear convolution, exact as a cyclic one
// of length Lf >= 4m + 1 per axis (Lf a power of two).  The spectrum FFT(c) / Lf^d is built
// once per generator.  A product then runs axis by axis over a batch of vectors:
//   axes 0..d-2 forward (n0 = 2m+1 inputs zero-padded to Lf, all Lf outputs kept),
//   axis d-1 forward, times the spectrum, inverse (n0 in, n0 out),
//   axes d-2..0 inverse (Lf in, the n0 outputs at positions 0..2m kept).
// Forward transforms are decimation in frequency (natural order in, bit-reversed out) and
// inverse ones decimation in time (bit-reversed in, natural out), so no pass reorders: the
// spectrum and every intermediate hold frequencies in bit-reversed order.
//
// One wave transforms one line in LDS (FP64, radix 4 with a radix-2 level when log2 Lf is
// odd; the twiddle table is computed once per call and copied to LDS by each workgroup).
//
// CG.  All nlam x ntgt systems iterate together, one workgroup per system for the vector
// updates; a system leaves the iteration (its lines and updates are skipped) once its
// recursive residual meets the tolerance.
#include "fk_internal.h"

#include <algorithm>
#include <cmath>

namespace fk {
namespace {

constexpr int FT = 256;          // threads per line-FFT workgroup
constexpr int FLINES = FT / 64;  // lines per workgroup, one wave each
constexpr int FMAX = 1024;       // longest line
constexpr int CT = 256;          // threads per CG system workgroup

enum LineMode { kForward = 0, kInverse = 1, kConvolve = 2 };

// One pass over one axis of a batch of row-major arrays.  Line li of a system covers
// elements o * (n * inner) + i + t * inner, t < n, for o = li / inner, i = li % inner
// (n = nin on input, nout on output).
struct LinePass {
  const double2* in;
  double2* out;
  int64_t in_sys, out_sys;   // complex elements per system
  int64_t lines_per_sys;
  int64_t inner;
  int nin, nout;
  int mode;
  const double2* spec;       // kConvolve: spectrum lines of Lf entries, line o at o * Lf
  double spec_scale;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Decimation in frequency, natural order in, bit-reversed order out, e^{-2 pi i / L}; tw[k] =
// e^{-2 pi i k / L}, k < L / 2.  Two radix-2 levels per LDS round trip (lengths len and len / 2
// over the four points pos, pos + len/4, pos + len/2, pos + 3 len/4 of a block), then a last
// radix-2 level when log2 L is odd.
__device__ __forceinline__ void dif_forward(double2* B, const double2* tw, int L, int lane) {
  int len = L, step = 1;
  for (; len >= 4; len >>= 2, step <<= 2) {
    const int q = len >> 2;
    for (int t = lane; t < L / 4; t += 64) {
      const int grp = t / q, pos = t - grp * q;
      const int i0 = grp * len + pos, i1 = i0 + q, i2 = i1 + q, i3 = i2 + q;
      const double2 a0 = B[i0], a1 = B[i1], a2 = B[i2], a3 = B[i3];
      const double2 b0 = cadd(a0, a2), b2 = cmul(csub(a0, a2), tw[pos * step]);
      const double2 b1 = cadd(a1, a3), b3 = cmul(csub(a1, a3), tw[(pos + q) * step]);
      const double2 w = tw[pos * step * 2];
      B[i0] = cadd(b0, b1);
      B[i1] = cmul(csub(b0, b1), w);
      B[i2] = cadd(b2, b3);
      B[i3] = cmul(csub(b2, b3), w);
    }
    __syncthreads();
  }
  if (len == 2) {
    for (int t = lane; t < L / 2; t += 64) {
      const double2 u = B[2 * t], v = B[2 * t + 1];
      B[2 * t] = cadd(u, v);
      B[2 * t + 1] = csub(u, v);
    }
    __syncthreads();
  }
}

// Decimation in time, bit-reversed order in, natural order out, e^{+2 pi i / L} (unnormalised
// inverse): a first radix-2 level when log2 L is odd, then two levels per LDS round trip
// (lengths len and 2 len over the points pos, pos + len/2, pos + len, pos + 3 len/2).
__device__ __forceinline__ void dit_inverse(double2* B, const double2* tw, int L, int lane) {
  int len = 2, step = L / 2;
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  if (lg & 1) {
    for (int t = lane; t < L / 2; t += 64) {
      const double2 u = B[2 * t], v = B[2 * t + 1];
      B[2 * t] = cadd(u, v);
      B[2 * t + 1] = csub(u, v);
    }
    __syncthreads();
    len = 4;
    step = L / 4;
  }
  for (; len <= L / 2; len <<= 2, step >>= 2) {
    const int h = len >> 1;
    for (int t = lane; t < L / 4; t += 64) {
      const int grp = t / h, pos = t - grp * h;
      const int i0 = grp * 2 * len + pos, i1 = i0 + h, i2 = i0 + len, i3 = i2 + h;
      const double2 w = cconj(tw[pos * step]);
      const double2 c1 = cmul(B[i1], w), c3 = cmul(B[i3], w);
      const double2 a0 = B[i0], a2 = B[i2];
      const double2 b0 = cadd(a0, c1), b1 = csub(a0, c1), b2 = cadd(a2, c3), b3 = csub(a2, c3);
      const double2 v2 = cmul(b2, cconj(tw[pos * (step >> 1)]));
      const double2 v3 = cmul(b3, cconj(tw[(pos + h) * (step >> 1)]));
      B[i0] = cadd(b0, v2);
      B[i2] = csub(b0, v2);
      B[i1] = cadd(b1, v3);
      B[i3] = csub(b1, v3);
    }
    __syncthreads();
  }
}

// Dynamic LDS: FLINES lines of L entries, then the L / 2 twiddles (copied from tw_g).
__global__ __launch_bounds__(FT) void k_line_fft(LinePass a, int L, int64_t nlines, const int* __restrict__ active,
                                                 const double2* __restrict__ tw_g) {
  extern __shared__ __align__(16) double2 lds[];
  double2* tw = lds + FLINES * L;
  for (int k = threadIdx.x; k < L / 2; k += FT) tw[k] = tw_g[k];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t line = (int64_t)blockIdx.x * FLINES + wv;
  bool live = line < nlines;
  int64_t sys = 0, li = 0;
  if (live) {
    sys = line / a.lines_per_sys;
    li = line - sys * a.lines_per_sys;
    if (active && !active[sys]) live = false;
  }
  const int64_t o = li / a.inner, i = li - o * a.inner;
  const double2* src = a.in + sys * a.in_sys + o * (a.nin * a.inner) + i;
  double2* dst = a.out + sys * a.out_sys + o * (a.nout * a.inner) + i;
  double2* B = lds + wv * L;
  for (int t = lane; t < L; t += 64) B[t] = (live && t < a.nin) ? src[t * a.inner] : make_double2(0.0, 0.0);
  __syncthreads();
  if (a.mode != kInverse) dif_forward(B, tw, L, lane);
  if (a.mode == kConvolve) {
    const double2* S = a.spec + o * L;
    for (int t = lane; t < L; t += 64) {
      const double2 s = S[t];
      B[t] = cmul(B[t], make_double2(s.x * a.spec_scale, s.y * a.spec_scale));
    }
    __syncthreads();
  }
  if (a.mode != kForward) dit_inverse(B, tw, L, lane);
  if (live)
    for (int t = lane; t < a.nout; t += 64) dst[t * a.inner] = B[t];
}

// ---- Lf = 256: four-step transform, 16 lanes per line, 16 points per lane in registers.
// A line's point t lives in lane t % 16, register t / 16, before and after each transform
// (natural order in and out), so forward, spectrum product and inverse chain in registers with
// one LDS transpose per transform.  All passes of a call with Lf = 256 take this kernel, the
// spectrum included, so its natural order is consistent.
constexpr int R16_LINES = FT / 16;   // lines per workgroup
constexpr int R16_ROW = 17;          // padded row of the 16 x 16 transpose (no bank conflicts)

__device__ __forceinline__ double2 w256(const double2* tw, int e, bool inv) {
  e &= 255;
  const double2 v = e >= 128 ? make_double2(-tw[e - 128].x, -tw[e - 128].y) : tw[e];
  return inv ? cconj(v) : v;
}

// In place: (a, b, c, d) -> the 4-point DFT with W4 = -i (forward) or +i (inverse).
__device__ __forceinline__ void dft4(double2& a, double2& b, double2& c, double2& d, bool inv) {
  const double2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = csub(b, d);
  const double2 jd1 = inv ? make_double2(-d1.y, d1.x) : make_double2(d1.y, -d1.x);
  a = cadd(s0, s1);
  c = csub(s0, s1);
  b = cadd(d0, jd1);
  d = csub(d0, jd1);
}

// v[k] <- sum_n v[n] W16^{nk}: 4 x 4 with twiddles W16^{n_a k_b}, n = n_a + 4 n_b, k = k_b + 4 k_a.
__device__ __forceinline__ void dft16(double2 v[16], const double2* tw, bool inv) {
  double2 A[16];
#pragma unroll
  for (int na = 0; na < 4; ++na) {
    double2 a = v[na], b = v[na + 4], c = v[na + 8], d = v[na + 12];
    dft4(a, b, c, d, inv);
    A[na * 4 + 0] = a;
    A[na * 4 + 1] = na ? cmul(b, w256(tw, 16 * na, inv)) : b;
    A[na * 4 + 2] = na ? cmul(c, w256(tw, 32 * na, inv)) : c;
    A[na * 4 + 3] = na ? cmul(d, w256(tw, 48 * na, inv)) : d;
  }
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    double2 a = A[kb], b = A[4 + kb], c = A[8 + kb], d = A[12 + kb];
    dft4(a, b, c, d, inv);
    v[kb] = a;
    v[kb + 4] = b;
    v[kb + 8] = c;
    v[kb + 12] = d;
  }
}

// 256-point DFT of the line held by 16 lanes (lane l16 holds points l16 + 16 r in v[r]); X is the
// line's 16 x R16_ROW LDS transpose buffer.  Every thread of the workgroup calls it together.
__device__ __forceinline__ void fft256(double2 v[16], double2* X, const double2* tw, int l16, bool inv) {
  dft16(v, tw, inv);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) X[k1 * R16_ROW + l16] = cmul(v[k1], w256(tw, l16 * k1, inv));
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = X[l16 * R16_ROW + n2];
  __syncthreads();
  dft16(v, tw, inv);
}

// Dynamic LDS: R16_LINES transpose buffers of 16 x R16_ROW entries, then 128 twiddles.
__global__ __launch_bounds__(FT) void k_line_fft256(LinePass a, int64_t nlines, const int* __restrict__ active,
                                                    const double2* __restrict__ tw_g) {
  extern __shared__ __align__(16) double2 lds[];
  double2* tw = lds + R16_LINES * 16 * R16_ROW;
  for (int k = threadIdx.x; k < 128; k += FT) tw[k] = tw_g[k];
  const int ls = threadIdx.x >> 4, l16 = threadIdx.x & 15;
  const int64_t line = (int64_t)blockIdx.x * R16_LINES + ls;
  bool live = line < nlines;
  int64_t sys = 0, li = 0;
  if (live) {
    if (a.mode == kConvolve) {
      // systems fastest: the lines of a workgroup share one spectrum line
      const int64_t nsys = nlines / a.lines_per_sys;
      li = line / nsys;
      sys = line - li * nsys;
    } else {
      sys = line / a.lines_per_sys;
      li = line - sys * a.lines_per_sys;
    }
    if (active && !active[sys]) live = false;
  }
  const int64_t o = li / a.inner, i = li - o * a.inner;
  const double2* src = a.in + sys * a.in_sys + o * (a.nin * a.inner) + i;
  double2* dst = a.out + sys * a.out_sys + o * (a.nout * a.inner) + i;
  double2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int t = l16 + 16 * r;
    v[r] = (live && t < a.nin) ? src[t * a.inner] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  double2* X = lds + ls * 16 * R16_ROW;
  if (a.mode != kInverse) fft256(v, X, tw, l16, false);
  if (a.mode == kConvolve) {
    const double2* S = a.spec + o * 256;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const double2 sp = live ? S[l16 + 16 * r] : make_double2(0.0, 0.0);
      v[r] = cmul(v[r], make_double2(sp.x * a.spec_scale, sp.y * a.spec_scale));
    }
  }
  if (a.mode != kForward) fft256(v, X, tw, l16, true);
  if (live) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int t = l16 + 16 * r;
      if (t < a.nout) dst[t * a.inner] = v[r];
    }
  }
}

// tw[k] = e^{-2 pi i k / L}, k < L / 2.
__global__ void k_twiddles(int L, double2* __restrict__ tw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L / 2) return;
  double s, c;
  sincospi(-2.0 * k / L, &s, &c);
  tw[k] = make_double2(c, s);
}

// c[j] = M[-r] at cyclic position j = r mod Lf, r in [-2m, 2m]^d; zero elsewhere.
__global__ void k_embed(const double2* __restrict__ M, int d, int m, int L, int64_t total, double2* __restrict__ c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int K = 4 * m + 1;
  int64_t rem = e, midx = 0;
  bool in = true;
  for (int a = d - 1, mul = 1; a >= 0; --a) {
    const int j = (int)(rem % L);
    rem /= L;
    const int r = j <= 2 * m ? j : (j >= L - 2 * m ? j - L : 1 << 30);
    if (r == 1 << 30) in = false;
    midx += (int64_t)(2 * m - r) * mul;   // index of M[-r]
    mul *= K;
  }
  c[e] = in ? M[midx] : make_double2(0.0, 0.0);
}

// ------------------------------------------------------------------ CG vector updates

__global__ void k_zero_int(int* __restrict__ v, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = 0;
}

// Optional physics term mu D^* Sigma_r D of the collocation form (Sec. 4): the operator symbol D
// (N complex), v = Sigma_r (D x) for the vector x of the current step (nsys x N), mu, and
// mu Re M_r[0] for the diagonal.  D == nullptr: no such term.
struct Colloc {
  const double2* D = nullptr;
  const double2* v = nullptr;
  double mu = 0.0, mu_m0r = 0.0;
};

__device__ __forceinline__ double colloc_diag(const Colloc& c, int64_t k) {
  if (!c.D) return 0.0;
  const double2 d = c.D[k];
  return c.mu_m0r * (d.x * d.x + d.y * d.y);
}

// mu conj(D_k) v[s][k]
__device__ __forceinline__ double2 colloc_term(const Colloc& c, int64_t s, int64_t N, int64_t k) {
  if (!c.D) return make_double2(0.0, 0.0);
  const double2 d = c.D[k], w = c.v[s * N + k];
  return make_double2(c.mu * (d.x * w.x + d.y * w.y), c.mu * (d.x * w.y - d.y * w.x));
}

// u[s][k] = D_k x[s][k]
__global__ void k_diag_mul(const double2* __restrict__ D, const double2* __restrict__ x, int64_t N, int64_t total,
                           double2* __restrict__ u) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    u[e] = cmul(D[e % N], x[e]);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < CT / 64; ++k) s += red[k];
  return s;
}

// theta = 0, r = b, z = r / dg, p = z, rho = <r, z>, bb = ||b||^2.  System s = l ntgt + t.
__global__ __launch_bounds__(CT) void k_cg_init(const double2* __restrict__ b, int ntgt, int64_t N,
                                                const double* __restrict__ lams, const double* __restrict__ pw,
                                                double m0, Colloc cl, double2* __restrict__ theta,
                                                double2* __restrict__ r, double2* __restrict__ p,
                                                double* __restrict__ rho, double* __restrict__ bb,
                                                int* __restrict__ active, int* __restrict__ iters,
                                                int* __restrict__ nactive, int* flags) {
  __shared__ double red[CT / 64];
  const int s = blockIdx.x;
  const double lam = lams[s / ntgt];
  const double2* bt = b + (int64_t)(s % ntgt) * N;
  double2* th = theta + (int64_t)s * N;
  double2* rs = r + (int64_t)s * N;
  double2* ps = p + (int64_t)s * N;
  double rz = 0.0, b2 = 0.0;
  for (int64_t k = threadIdx.x; k < N; k += CT) {
    const double2 v = bt[k];
    const double inv = 1.0 / (m0 + lam * pw[k] + colloc_diag(cl, k));
    th[k] = make_double2(0.0, 0.0);
    rs[k] = v;
    ps[k] = make_double2(v.x * inv, v.y * inv);
    const double a = v.x * v.x + v.y * v.y;
    b2 += a;
    rz += a * inv;
  }
  rz = block_sum(rz, red);
  b2 = block_sum(b2, red);
  if (threadIdx.x == 0) {
    rho[s] = rz;
    bb[s] = b2;
    iters[s] = 0;
    if (!(b2 == b2) || isinf(b2)) atomicOr(&flags[kFlagNaN], 1);   // a NaN or Inf right-hand side
    const int on = b2 > 0.0 && !isinf(b2);
    active[s] = on;
    if (on) atomicAdd(nactive, 1);
  }
}

// One iteration for every active system, given qraw = Sigma p:
//   q = qraw + lambda P p, alpha = rho / <p, q>, theta += alpha p, r -= alpha q,
//   stop if ||r||^2 <= tol2 ||b||^2, else z = r / dg, beta = <r, z> / rho, p = z + beta p.
// A non-positive <p, q> (the matrix is not positive definite in FP64) stops the system
// and raises the not-positive-definite flag.
__global__ __launch_bounds__(CT) void k_cg_step(const double2* __restrict__ qraw, int ntgt, int64_t N,
                                                const double* __restrict__ lams, const double* __restrict__ pw,
                                                double m0, Colloc cl, double tol2, double2* __restrict__ theta,
                                                double2* __restrict__ r, double2* __restrict__ p,
                                                double* __restrict__ rho, const double* __restrict__ bb,
                                                int* __restrict__ active, int* __restrict__ iters,
                                                int* __restrict__ nactive, int* flags) {
  __shared__ double red[CT / 64];
  const int s = blockIdx.x;
  if (!active[s]) return;
  const double lam = lams[s / ntgt];
  const double2* qs = qraw + (int64_t)s * N;
  double2* th = theta + (int64_t)s * N;
  double2* rs = r + (int64_t)s * N;
  double2* ps = p + (int64_t)s * N;
  const double rho0 = rho[s];
  double pq = 0.0;
  for (int64_t k = threadIdx.x; k < N; k += CT) {
    const double2 pk = ps[k], qk = qs[k], ck = colloc_term(cl, s, N, k);
    const double lp = lam * pw[k];
    pq += pk.x * (qk.x + lp * pk.x + ck.x) + pk.y * (qk.y + lp * pk.y + ck.y);
  }
  pq = block_sum(pq, red);
  if (!(pq > 0.0)) {
    if (threadIdx.x == 0) {
      active[s] = 0;
      atomicSub(nactive, 1);
      atomicOr(&flags[pq == pq ? kFlagNotPD : kFlagNaN], 1);   // NaN: a NaN in M or b reached the product
    }
    return;
  }
  const double alpha = rho0 / pq;
  double rr = 0.0, rz = 0.0;
  for (int64_t k = threadIdx.x; k < N; k += CT) {
    const double2 pk = ps[k], qk = qs[k], ck = colloc_term(cl, s, N, k);
    const double lp = lam * pw[k];
    double2 t = th[k], rk = rs[k];
    t.x += alpha * pk.x;
    t.y += alpha * pk.y;
    rk.x -= alpha * (qk.x + lp * pk.x + ck.x);
    rk.y -= alpha * (qk.y + lp * pk.y + ck.y);
    th[k] = t;
    rs[k] = rk;
    const double a = rk.x * rk.x + rk.y * rk.y;
    rr += a;
    rz += a / (m0 + lp + colloc_diag(cl, k));
  }
  rr = block_sum(rr, red);
  rz = block_sum(rz, red);
  const int it = iters[s] + 1;
  if (rr <= tol2 * bb[s]) {
    if (threadIdx.x == 0) {
      iters[s] = it;
      active[s] = 0;
      atomicSub(nactive, 1);
    }
    return;
  }
  const double beta = rz / rho0;
  for (int64_t k = threadIdx.x; k < N; k += CT) {
    const double inv = 1.0 / (m0 + lam * pw[k] + colloc_diag(cl, k));
    const double2 rk = rs[k], pk = ps[k];
    ps[k] = make_double2(rk.x * inv + beta * pk.x, rk.y * inv + beta * pk.y);
  }
  if (threadIdx.x == 0) {
    rho[s] = rz;
    iters[s] = it;
  }
}

// relres[s] = ||b - (Sigma theta + lambda P theta)|| / ||b|| (0 when b = 0), from qraw = Sigma theta.
__global__ __launch_bounds__(CT) void k_cg_resid(const double2* __restrict__ b, const double2* __restrict__ qraw,
                                                 const double2* __restrict__ theta, int ntgt, int64_t N,
                                                 const double* __restrict__ lams, const double* __restrict__ pw,
                                                 Colloc cl, const double* __restrict__ bb,
                                                 double* __restrict__ relres) {
  __shared__ double red[CT / 64];
  const int s = blockIdx.x;
  const double lam = lams[s / ntgt];
  const double2* bt = b + (int64_t)(s % ntgt) * N;
  const double2* qs = qraw + (int64_t)s * N;
  const double2* th = theta + (int64_t)s * N;
  double e = 0.0;
  for (int64_t k = threadIdx.x; k < N; k += CT) {
    const double lp = lam * pw[k];
    const double2 ck = colloc_term(cl, s, N, k);
    const double rx = bt[k].x - qs[k].x - lp * th[k].x - ck.x;
    const double ry = bt[k].y - qs[k].y - lp * th[k].y - ck.y;
    e += rx * rx + ry * ry;
  }
  e = block_sum(e, red);
  if (threadIdx.x == 0) relres[s] = bb[s] > 0.0 ? sqrt(e / bb[s]) : 0.0;
}

// ------------------------------------------------------------------ host side

struct ToepGeom {
  int d = 0, m = 0, n0 = 0, L = 0;
  int64_t N = 0, spec = 0, tmp = 0;   // complex elements: modes, spectrum, one intermediate
  double2* tw = nullptr;              // device twiddle table, L / 2 entries
};

ToepGeom toep_geom(int d, int m) {
  ToepGeom g;
  g.d = d;
  g.m = m;
  g.n0 = 2 * m + 1;
  g.L = 2;
  while (g.L < 4 * m + 1) g.L <<= 1;
  g.N = 1;
  g.spec = 1;
  for (int a = 0; a < d; ++a) {
    g.N *= g.n0;
    g.spec *= g.L;
  }
  g.tmp = g.spec / g.L * g.n0;
  return g;
}

fk_status run_pass(hipStream_t st, const ToepGeom& g, const int64_t* E, int axis, int nout, int mode,
                   const double2* in, double2* out, int nsys, const double2* spec, double scale, const int* active) {
  LinePass a;
  a.in = in;
  a.out = out;
  int64_t lines = 1, inner = 1, tot = 1;
  for (int b = 0; b < g.d; ++b) {
    tot *= E[b];
    if (b != axis) lines *= E[b];
    if (b > axis) inner *= E[b];
  }
  a.in_sys = tot;
  a.out_sys = tot / E[axis] * nout;
  a.lines_per_sys = lines;
  a.inner = inner;
  a.nin = (int)E[axis];
  a.nout = nout;
  a.mode = mode;
  a.spec = spec;
  a.spec_scale = scale;
  const int64_t nlines = lines * nsys;
  const int64_t blocks = (nlines + FLINES - 1) / FLINES;
  if (blocks > 0x7fffffff) return FK_EINVAL;
  if (g.L == 256) {
    const int64_t b256 = (nlines + R16_LINES - 1) / R16_LINES;
    if (b256 > 0x7fffffff) return FK_EINVAL;
    const size_t lds = sizeof(double2) * ((size_t)R16_LINES * 16 * R16_ROW + 128);
    hipLaunchKernelGGL(k_line_fft256, dim3((unsigned)b256), dim3(FT), lds, st, a, nlines, active, g.tw);
    return hipGetLastError() == hipSuccess ? FK_OK : FK_EHIP;
  }
  const size_t lds = sizeof(double2) * ((size_t)FLINES * g.L + g.L / 2);
  hipLaunchKernelGGL(k_line_fft, dim3((unsigned)blocks), dim3(FT), lds, st, a, g.L, nlines, active, g.tw);
  return hipGetLastError() == hipSuccess ? FK_OK : FK_EHIP;
}

// spec = FFT_d(c) over the Lf^d grid (bit-reversed frequencies).  The passes run in place:
// a line is read whole into LDS before any of it is written, and lines are disjoint.
fk_status build_spectrum(hipStream_t st, const ToepGeom& g, const double* M, double2* spec) {
  hipLaunchKernelGGL(k_twiddles, dim3((g.L / 2 + 255) / 256), dim3(256), 0, st, g.L, g.tw);
  const int64_t total = g.spec;
  hipLaunchKernelGGL(k_embed, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(M), g.d, g.m, g.L, total, spec);
  int64_t E[3] = {g.L, g.L, g.L};
  for (int a = 0; a < g.d; ++a) {
    fk_status s = run_pass(st, g, E, a, g.L, kForward, spec, spec, 1, nullptr, 1.0, nullptr);
    if (s != FK_OK) return s;
  }
  return FK_OK;
}

// y = Sigma x for nsys vectors (x, y: nsys x N), intermediates t0, t1 (nsys x g.tmp each).
fk_status toep_apply(hipStream_t st, const ToepGeom& g, const double2* spec, const double2* x, double2* y,
                     int nsys, double2* t0, double2* t1, const int* active) {
  const double scale = 1.0 / (double)g.spec;
  int64_t E[3] = {g.n0, g.n0, g.n0};
  const double2* cur = x;
  double2* bufs[2] = {t0, t1};
  int nb = 0;
  fk_status s = FK_OK;
  for (int a = 0; a < g.d - 1 && s == FK_OK; ++a) {
    s = run_pass(st, g, E, a, g.L, kForward, cur, bufs[nb], nsys, nullptr, 1.0, active);
    E[a] = g.L;
    cur = bufs[nb];
    nb ^= 1;
  }
  if (s != FK_OK) return s;
  double2* out = g.d == 1 ? y : bufs[nb];
  s = run_pass(st, g, E, g.d - 1, g.n0, kConvolve, cur, out, nsys, spec, scale, active);
  cur = out;
  nb ^= 1;
  for (int a = g.d - 2; a >= 0 && s == FK_OK; --a) {
    out = a == 0 ? y : bufs[nb];
    s = run_pass(st, g, E, a, g.n0, kInverse, cur, out, nsys, nullptr, 1.0, active);
    E[a] = g.n0;
    cur = out;
    nb ^= 1;
  }
  return s;
}

}  // namespace

bool toeplitz_fft_ok(int d, int m) {
  if (d < 1 || d > 3 || m < 1) return false;
  const int lim = d == 3 ? 63 : 255;   // Lf <= 256 in 3-D (a 268 MB spectrum), else <= 1024
  return m <= lim && toep_geom(d, m).L <= FMAX;
}

size_t toeplitz_apply_workspace(int d, int m, int nvec) {
  const ToepGeom g = toep_geom(d, m);
  Carve cv(nullptr, 0);
  cv.take<double2>((size_t)g.L / 2);
  cv.take<double2>((size_t)g.spec);
  cv.take<double2>((size_t)nvec * g.tmp);
  cv.take<double2>((size_t)nvec * g.tmp);
  return cv.off + 256;
}

fk_status toeplitz_apply_impl(fk_ctx* ctx, int d, int m, const double* M, int nvec, const double* x, double* y,
                              Carve& cv) {
  ToepGeom g = toep_geom(d, m);
  g.tw = cv.take<double2>((size_t)g.L / 2);
  double2* spec = cv.take<double2>((size_t)g.spec);
  double2* t0 = cv.take<double2>((size_t)nvec * g.tmp);
  double2* t1 = cv.take<double2>((size_t)nvec * g.tmp);
  if (!cv.ok()) return FK_ENOMEM;
  fk_status s = build_spectrum(ctx->stream, g, M, spec);
  if (s != FK_OK) return s;
  return toep_apply(ctx->stream, g, spec, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), nvec,
                    t0, t1, nullptr);
}

size_t cg_workspace(int d, int m, int nsys, int nlam, bool colloc) {
  const ToepGeom g = toep_geom(d, m);
  Carve cv(nullptr, 0);
  cv.take<double2>((size_t)g.L / 2);
  cv.take<double2>((size_t)g.spec);
  cv.take<double2>((size_t)nsys * g.tmp);
  cv.take<double2>((size_t)nsys * g.tmp);
  for (int k = 0; k < 3; ++k) cv.take<double2>((size_t)nsys * g.N);   // r, p, qraw
  cv.take<double>((size_t)g.N);                                          // penalty weights
  cv.take<double>((size_t)nlam);
  for (int k = 0; k < 3; ++k) cv.take<double>((size_t)nsys);            // rho, bb, relres
  for (int k = 0; k < 2; ++k) cv.take<int>((size_t)nsys);               // active, iters
  cv.take<int>(64);                                                      // counter
  if (colloc) {
    cv.take<double2>((size_t)g.spec);                                    // collocation spectrum
    cv.take<double2>((size_t)nsys * g.N);                                // D x
    cv.take<double2>((size_t)nsys * g.N);                                // Sigma_r D x
  }
  return cv.off + 256;
}

static double centre_of(hipStream_t st, const double* M, int d, int m, fk_status* err) {
  double2 c;
  int64_t centre = 0;
  for (int a = 0, mul = 1; a < d; ++a, mul *= 4 * m + 1) centre += (int64_t)(2 * m) * mul;
  if (hipMemcpyAsync(&c, M + 2 * centre, sizeof(double2), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    *err = FK_EHIP;
    return 0.0;
  }
  return c.x;
}

fk_status cg_solve_impl(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                        const std::vector<double>& lams, const std::vector<double>& pw, double mu, const double* Mr,
                        const double* Dsym, double tol, int maxit, double* theta_out, int* iters_out,
                        double* relres_out, Carve& cv) {
  ToepGeom g = toep_geom(d, m);
  const int nlam = (int)lams.size();
  const int nsys = nlam * ntgt;
  const bool colloc = Mr != nullptr;
  hipStream_t st = ctx->stream;
  g.tw = cv.take<double2>((size_t)g.L / 2);
  double2* spec = cv.take<double2>((size_t)g.spec);
  double2* t0 = cv.take<double2>((size_t)nsys * g.tmp);
  double2* t1 = cv.take<double2>((size_t)nsys * g.tmp);
  double2* r = cv.take<double2>((size_t)nsys * g.N);
  double2* p = cv.take<double2>((size_t)nsys * g.N);
  double2* q = cv.take<double2>((size_t)nsys * g.N);
  double* dpw = cv.take<double>((size_t)g.N);
  double* dlam = cv.take<double>((size_t)nlam);
  double* rho = cv.take<double>((size_t)nsys);
  double* bb = cv.take<double>((size_t)nsys);
  double* relres = cv.take<double>((size_t)nsys);
  int* active = cv.take<int>((size_t)nsys);
  int* iters = cv.take<int>((size_t)nsys);
  int* counter = cv.take<int>(64);
  double2 *spec_r = nullptr, *u = nullptr, *v = nullptr;
  if (colloc) {
    spec_r = cv.take<double2>((size_t)g.spec);
    u = cv.take<double2>((size_t)nsys * g.N);
    v = cv.take<double2>((size_t)nsys * g.N);
  }
  if (!cv.ok()) return FK_ENOMEM;
  double2* theta = reinterpret_cast<double2*>(theta_out);
  const double2* bv = reinterpret_cast<const double2*>(b);

  // the diagonal of Sigma is M[0] (the centre of the generator), real for a Hermitian Sigma
  fk_status s = FK_OK;
  const double m0 = centre_of(st, M, d, m, &s);
  if (s != FK_OK) return s;
  if (!(m0 > 0.0) || std::isinf(m0)) return FK_EINVAL;
  Colloc cl;
  if (colloc) {
    const double m0r = centre_of(st, Mr, d, m, &s);
    if (s != FK_OK) return s;
    if (!(m0r > 0.0) || std::isinf(m0r)) return FK_EINVAL;
    cl.D = reinterpret_cast<const double2*>(Dsym);
    cl.v = v;
    cl.mu = mu;
    cl.mu_m0r = mu * m0r;
  }
  s = stage_upload(ctx, dpw, pw.data(), sizeof(double) * g.N);
  if (s == FK_OK) s = stage_upload(ctx, dlam, lams.data(), sizeof(double) * nlam);
  if (s != FK_OK) return s;

  s = build_spectrum(st, g, M, spec);
  if (s == FK_OK && colloc) s = build_spectrum(st, g, Mr, spec_r);
  if (s != FK_OK) return s;
  const int64_t tot = (int64_t)nsys * g.N;
  const unsigned dblocks = (unsigned)std::min<int64_t>(4096, (tot + 255) / 256);
  // q = Sigma x, and with the physics term v = Sigma_r (D x)
  auto product = [&](const double2* x, const int* act) -> fk_status {
    fk_status e = toep_apply(st, g, spec, x, q, nsys, t0, t1, act);
    if (e != FK_OK || !colloc) return e;
    hipLaunchKernelGGL(k_diag_mul, dim3(dblocks), dim3(256), 0, st, cl.D, x, g.N, tot, u);
    return toep_apply(st, g, spec_r, u, v, nsys, t0, t1, act);
  };
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, counter, 64);
  hipLaunchKernelGGL(k_cg_init, dim3(nsys), dim3(CT), 0, st, bv, ntgt, g.N, dlam, dpw, m0, cl, theta, r, p, rho, bb,
                     active, iters, counter, ctx->flags);
  const double tol2 = tol * tol;
  int done_it = 0;
  int nact = 1;
  constexpr int kCheck = 4;   // iterations between reads of the active count
  while (done_it < maxit && nact > 0) {
    const int run = std::min(kCheck, maxit - done_it);
    for (int k = 0; k < run; ++k) {
      s = product(p, active);
      if (s != FK_OK) return s;
      hipLaunchKernelGGL(k_cg_step, dim3(nsys), dim3(CT), 0, st, q, ntgt, g.N, dlam, dpw, m0, cl, tol2, theta, r, p,
                         rho, bb, active, iters, counter, ctx->flags);
    }
    done_it += run;
    FK_HIP(hipMemcpyAsync(ctx->flags_host + kFlagCount, counter, sizeof(int), hipMemcpyDeviceToHost, st));
    FK_HIP(hipStreamSynchronize(st));
    nact = ctx->flags_host[kFlagCount];
  }
  // true residuals from one more product
  s = product(theta, nullptr);
  if (s != FK_OK) return s;
  hipLaunchKernelGGL(k_cg_resid, dim3(nsys), dim3(CT), 0, st, bv, q, theta, ntgt, g.N, dlam, dpw, cl, bb, relres);
  std::vector<int> it_h(nsys);
  FK_HIP(hipMemcpyAsync(it_h.data(), iters, sizeof(int) * nsys, hipMemcpyDeviceToHost, st));
  if (relres_out) FK_HIP(hipMemcpyAsync(relres_out, relres, sizeof(double) * nsys, hipMemcpyDeviceToHost, st));
  FK_HIP(hipStreamSynchronize(st));
  if (iters_out) {
    int mx = 0;
    for (int it : it_h) mx = std::max(mx, it);
    *iters_out = mx;
  }
  s = read_flags(ctx);
  if (s != FK_OK) return s;
  return nact > 0 ? FK_ENOCONV : FK_OK;
}

}  // namespace fk
