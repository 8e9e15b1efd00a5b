// Type-2 non-uniform FFT (prediction) and the on-device synthetic-input generator.
//
// Prediction evaluates the estimator f_theta(x) = sum_k theta_k exp(+i k.x)
// (Sec. 2.1) at new points: the coefficients are divided by the kernel's
// Fourier transform, placed on an oversampled grid, inverse-FFT'd in FP64, and
// each point gathers its w^d grid neighbours weighted by the same
// exponential-of-semicircle kernel as the type-1 spread.  Only the real part is
// kept (a real estimator has Hermitian-symmetric theta).
//   Re f(x) ~= sum_l Re(g_l) phi(l - u),  g_l = sum_q (-1)^q theta_q / Phihat(q h) e^{2 pi i q l / nf}.
#include "fk_internal.h"

#include <cmath>
#include <cstring>
#include <mutex>

namespace fk {

// Inverse DFT of one line with pruned input frequencies q = -K..K:
//   out[l] = sum_q in[q + K] * f(q) * e^{+2 pi i q l / nf},
// f(q) = (-1)^q / phihat[|q|] when phihat != nullptr, else 1.
// Input elements (complex) at in + line_in + (q+K)*istride; output complex (or
// real part only, when oreal) at out + line_out + l*ostride.
__global__ __launch_bounds__(256) void k_ifft_line(const double* __restrict__ in, int64_t istride,
                                                   int64_t in_outer, int64_t in_inner, int lines_inner, int K,
                                                   const double* __restrict__ phihat, int nf, int logn,
                                                   double* __restrict__ out, int oreal, int64_t ostride,
                                                   int64_t out_outer, int64_t out_inner) {
  __shared__ double re[1024], im[1024];
  const int line = blockIdx.x;
  const int lo = line / lines_inner, li = line - lo * lines_inner;
  const double* src = in + 2 * (lo * in_outer + li * in_inner);
  for (int i = threadIdx.x; i < nf; i += blockDim.x) {
    re[i] = 0.0;
    im[i] = 0.0;
  }
  __syncthreads();
  for (int q = -K + (int)threadIdx.x; q <= K; q += blockDim.x) {
    int l = q < 0 ? q + nf : q;
    int r = __brev((unsigned)l) >> (32 - logn);
    double f = 1.0;
    if (phihat) {
      int aq = q < 0 ? -q : q;
      f = 1.0 / phihat[aq];
      if (aq & 1) f = -f;
    }
    re[r] = src[2 * (q + K) * istride] * f;
    im[r] = src[2 * (q + K) * istride + 1] * f;
  }
  __syncthreads();
  for (int len = 2; len <= nf; len <<= 1) {
    const int half = len >> 1;
    for (int t = threadIdx.x; t < nf / 2; t += blockDim.x) {
      int grp = t / half, pos = t - grp * half;
      int i = grp * len + pos, j = i + half;
      double sn, cs;
      sincospi(2.0 * pos / len, &sn, &cs);
      double vr = re[j] * cs - im[j] * sn;
      double vi = re[j] * sn + im[j] * cs;
      double ur = re[i], ui = im[i];
      re[i] = ur + vr;
      im[i] = ui + vi;
      re[j] = ur - vr;
      im[j] = ui - vi;
    }
    __syncthreads();
  }
  double* dst = out + (lo * out_outer + li * out_inner) * (oreal ? 1 : 2);
  for (int l = threadIdx.x; l < nf; l += blockDim.x) {
    if (oreal) {
      dst[l * ostride] = re[l];
    } else {
      dst[2 * l * ostride] = re[l];
      dst[2 * l * ostride + 1] = im[l];
    }
  }
}

__global__ void k_d2f_grid(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ES kernel psi(s) = exp(beta (sqrt(1 - (2s/w)^2) - 1)) with beta pre-multiplied by log2 e, so that
// the hardware exp2 takes the exponent directly (it lies in [-beta log2 e, 0]: no range handling) and
// the hardware square root needs no denormal scaling (1 - z^2 below 2^-126 gives psi ~ e^-beta).
struct EsDev2 {
  float beta_log2e;
  float two_over_w;
};

__device__ __forceinline__ float es_eval2(float s, EsDev2 es) {
  const float z = s * es.two_over_w;
  const float r = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
  return __builtin_amdgcn_exp2f(fmaf(es.beta_log2e, __builtin_amdgcn_sqrtf(r), -es.beta_log2e));
}

// Grid coordinate in FP64 -> window start i0 = ceil(u - w/2) and offset s0 = i0 - u.
__device__ __forceinline__ bool window_of(double x, int nf, int w, int* i0, float* s0) {
  const double two_pi = 6.283185307179586476925;
  if (!(x == x) || x < -two_pi || x >= two_pi) return false;
  if (x < -3.14159265358979323846) x += two_pi;
  if (x >= 3.14159265358979323846) x -= two_pi;
  double u = (x + 3.14159265358979323846) * ((double)nf / two_pi);
  double c = ceil(u - 0.5 * w);
  *i0 = (int)c;
  *s0 = (float)(c - u);
  return true;
}

// window_of with the grid scale nf / 2 pi given (no division per point).
__device__ __forceinline__ bool window_at(double x, double scale, int w, int* i0, float* s0) {
  const double two_pi = 6.283185307179586476925;
  if (!(x == x) || x < -two_pi || x >= two_pi) return false;
  if (x < -3.14159265358979323846) x += two_pi;
  if (x >= 3.14159265358979323846) x -= two_pi;
  double u = (x + 3.14159265358979323846) * scale;
  double c = ceil(u - 0.5 * w);
  *i0 = (int)c;
  *s0 = (float)(c - u);
  return true;
}

template <int W>
__global__ __launch_bounds__(256) void k_interp(const float* __restrict__ grid, int d, int nf, int T,
                                                const void* __restrict__ Xq, fk_dtype dt, int64_t nq, EsDev2 es,
                                                float* __restrict__ out, int* flags) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nq) return;
  auto ld = [&](int64_t idx) -> double {
    return dt == FK_F64 ? static_cast<const double*>(Xq)[idx] : (double)static_cast<const float*>(Xq)[idx];
  };
  int i1, i2 = 0, i3 = 0;
  float s1, s2 = 0.f, s3 = 0.f;
  bool ok = window_of(ld(j), nf, W, &i1, &s1);
  if (d >= 2) ok = window_of(ld(nq + j), nf, W, &i2, &s2) && ok;
  if (d == 3) ok = window_of(ld(2 * nq + j), nf, W, &i3, &s3) && ok;
  if (!ok) {
    atomicOr(&flags[kFlagRange], 1);
    for (int t = 0; t < T; ++t) out[(int64_t)t * nq + j] = __int_as_float(0x7fc00000);
    return;
  }
  float k1[W], k2[W], k3[W];
#pragma unroll
  for (int a = 0; a < W; ++a) {
    k1[a] = es_eval2(s1 + (float)a, es);
    k2[a] = d >= 2 ? es_eval2(s2 + (float)a, es) : 1.f;
    k3[a] = d == 3 ? es_eval2(s3 + (float)a, es) : 1.f;
  }
  for (int t = 0; t < T; ++t) {
    float acc = 0.f;
    if (d == 1) {
      const float* g = grid + (int64_t)t * nf;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        int l = i1 + a;
        l = l < 0 ? l + nf : (l >= nf ? l - nf : l);
        acc += g[l] * k1[a];
      }
    } else if (d == 3) {
      const float* g = grid + (int64_t)t * nf * nf * nf;
      for (int a = 0; a < W; ++a) {
        int l1 = i1 + a;
        l1 = l1 < 0 ? l1 + nf : (l1 >= nf ? l1 - nf : l1);
        float ra = 0.f;
        for (int b = 0; b < W; ++b) {
          int l2 = i2 + b;
          l2 = l2 < 0 ? l2 + nf : (l2 >= nf ? l2 - nf : l2);
          const float* row = g + ((int64_t)l1 * nf + l2) * nf;
          float rb = 0.f;
#pragma unroll
          for (int c = 0; c < W; ++c) {
            int l3 = i3 + c;
            l3 = l3 < 0 ? l3 + nf : (l3 >= nf ? l3 - nf : l3);
            rb += row[l3] * k3[c];
          }
          ra += rb * k2[b];
        }
        acc += ra * k1[a];
      }
    } else {
      const float* g = grid + (int64_t)t * nf * nf;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        int l1 = i1 + a;
        l1 = l1 < 0 ? l1 + nf : (l1 >= nf ? l1 - nf : l1);
        const float* row = g + (int64_t)l1 * nf;
        float ra = 0.f;
#pragma unroll
        for (int b = 0; b < W; ++b) {
          int l2 = i2 + b;
          l2 = l2 < 0 ? l2 + nf : (l2 >= nf ? l2 - nf : l2);
          ra += row[l2] * k2[b];
        }
        acc += ra * k1[a];
      }
    }
    out[(int64_t)t * nq + j] = acc;
  }
}

// ------------------------------------------------------------------ 2-D prediction from an LDS grid
// For d = 2 the oversampled grid of one coefficient set is small enough for LDS when its length is
// any even number near 2.2 (2m + 1) (not a power of two): the inverse transforms are then plain
// FP64 DFTs (a few hundred lines of at most 186 outputs), and every interpolation read is an LDS
// read instead of an L2 request.

constexpr int kNf2Max = 186;   // (nf + kMaxW)^2 FP32 values fit 160 KB of LDS

// Grid length of the LDS path for d = 2 (0 when the grid would not fit LDS).
static int predict_nf2(int m) {
  const int L = 2 * m + 1;
  const int nf = ((int)std::ceil(2.2 * L) + 7) & ~7;
  return nf <= kNf2Max ? nf : 0;
}

static size_t pad_stride(int nf, int W) { return ((size_t)(nf + W) * (nf + W) + 63) & ~size_t(63); }

// Inverse DFT along axis 0 of theta (one line per (set, q2)), pruned input frequencies q1 = -K..K,
// deconvolved:  tmp[t][l1][q2] = sum_q1 theta[t][q1][q2] (-1)^q1 / phihat[|q1|] e^{+2 pi i q1 l1 / nf}.
__global__ __launch_bounds__(256) void k_idft_cols(const double* __restrict__ theta, int K, int nf,
                                                   const double* __restrict__ phihat, double* __restrict__ tmp) {
  __shared__ double twr[kNf2Max], twi[kNf2Max];
  __shared__ double ar[129], ai[129];
  const int L = 2 * K + 1;
  const int line = blockIdx.x;   // t * L + q2
  const int t = line / L, q2 = line - t * L;
  for (int i = threadIdx.x; i < nf; i += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * i / nf, &sn, &cs);
    twr[i] = cs;
    twi[i] = sn;
  }
  const double* src = theta + 2 * ((size_t)t * L * L + q2);
  for (int q = threadIdx.x; q < L; q += blockDim.x) {
    const int aq = q - K < 0 ? K - q : q - K;
    double f = 1.0 / phihat[aq];
    if (aq & 1) f = -f;
    ar[q] = src[2 * (size_t)q * L] * f;
    ai[q] = src[2 * (size_t)q * L + 1] * f;
  }
  __syncthreads();
  double* dst = tmp + 2 * ((size_t)t * nf * L + q2);
  for (int l = threadIdx.x; l < nf; l += blockDim.x) {
    int r = (int)(((int64_t)(nf - K) * l) % nf);   // (-K) l mod nf
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < L; ++q) {
      sr += ar[q] * twr[r] - ai[q] * twi[r];
      si += ar[q] * twi[r] + ai[q] * twr[r];
      r += l;
      if (r >= nf) r -= nf;
    }
    dst[2 * (size_t)l * L] = sr;
    dst[2 * (size_t)l * L + 1] = si;
  }
}

// Inverse DFT along axis 1 (one line per (set, l1)), deconvolved, real part in FP32, written into
// the periodically padded grid g[t][p1][p2] (P = nf + W rows and columns, padded index p holding the
// grid point (p - W/2) mod nf), so that every window of W cells is contiguous without wrapping.
__global__ __launch_bounds__(256) void k_idft_rows_pad(const double* __restrict__ tmp, int K, int nf, int W,
                                                       const double* __restrict__ phihat, size_t pstride,
                                                       float* __restrict__ g) {
  __shared__ double twr[kNf2Max], twi[kNf2Max];
  __shared__ double ar[129], ai[129];
  const int L = 2 * K + 1, P = nf + W, H = W / 2;
  const int line = blockIdx.x;   // t * nf + l1
  const int t = line / nf, l1 = line - t * nf;
  for (int i = threadIdx.x; i < nf; i += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * i / nf, &sn, &cs);
    twr[i] = cs;
    twi[i] = sn;
  }
  const double* src = tmp + 2 * ((size_t)t * nf * L + (size_t)l1 * L);
  for (int q = threadIdx.x; q < L; q += blockDim.x) {
    const int aq = q - K < 0 ? K - q : q - K;
    double f = 1.0 / phihat[aq];
    if (aq & 1) f = -f;
    ar[q] = src[2 * q] * f;
    ai[q] = src[2 * q + 1] * f;
  }
  __syncthreads();
  float* gt = g + (size_t)t * pstride;
  for (int p2 = threadIdx.x; p2 < P; p2 += blockDim.x) {
    int l = p2 - H;
    l = l < 0 ? l + nf : (l >= nf ? l - nf : l);
    int r = (int)(((int64_t)(nf - K) * l) % nf);
    double sr = 0.0;
    for (int q = 0; q < L; ++q) {
      sr += ar[q] * twr[r] - ai[q] * twi[r];
      r += l;
      if (r >= nf) r -= nf;
    }
    const float v = (float)sr;
    // padded rows of grid row l1: l1 + H, and its periodic copies inside [0, P)
    for (int p1 = l1 + H - nf; p1 < P; p1 += nf)
      if (p1 >= 0) gt[(size_t)p1 * P + p2] = v;
  }
}

// f_t(x_j) for one coefficient set t and one chunk of points, from the padded grid in LDS.
// Blocks: the T sets of a chunk are consecutive among the blocks one XCD receives (blocks go to
// the 8 XCDs round robin), so the chunk's coordinates are read from HBM once per chunk and then
// from that XCD's L2.
template <int W>
__global__ __launch_bounds__(1024) void k_interp2_lds(const float* __restrict__ gpad, size_t pstride, int nf, int T,
                                                      const void* __restrict__ Xq, fk_dtype dt, int64_t nq,
                                                      int64_t per_chunk, int64_t nchunk, double scale, EsDev2 es,
                                                      float* __restrict__ out, int* flags) {
  extern __shared__ float gl[];
  constexpr int H = W / 2;
  const int P = nf + W;
  const int64_t b = blockIdx.x, xcd = b & 7, k = b >> 3;
  const int t = (int)(k % T);
  const int64_t chunk = (k / T) * 8 + xcd;
  if (chunk >= nchunk) return;
  const int64_t j0 = chunk * per_chunk;
  const int64_t j1 = min(nq, j0 + per_chunk);
  if (j0 >= j1) return;
  {
    const float4* src = reinterpret_cast<const float4*>(gpad + (size_t)t * pstride);
    float4* dst = reinterpret_cast<float4*>(gl);
    const int n4 = (int)(pstride / 4);
    for (int i = threadIdx.x; i < n4; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  auto ld = [&](int64_t idx) -> double {
    return dt == FK_F64 ? static_cast<const double*>(Xq)[idx] : (double)static_cast<const float*>(Xq)[idx];
  };
  // one point: f_t(x_j), or NaN and the range flag for a coordinate outside [-2 pi, 2 pi)
  auto one = [&](int64_t j) -> float {
    int i1, i2;
    float s1, s2;
    const bool ok1 = window_at(ld(j), scale, W, &i1, &s1);
    const bool ok2 = window_at(ld(nq + j), scale, W, &i2, &s2);
    if (!(ok1 && ok2)) {
      atomicOr(&flags[kFlagRange], 1);
      return __int_as_float(0x7fc00000);
    }
    float k1[W], k2[W];
#pragma unroll
    for (int a = 0; a < W; ++a) {
      k1[a] = es_eval2(s1 + (float)a, es);
      k2[a] = es_eval2(s2 + (float)a, es);
    }
    const float* gp = gl + (i1 + H) * P + (i2 + H);
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const float* row = gp + a * P;
      float ra = 0.f;
#pragma unroll
      for (int c = 0; c < W; ++c) ra += row[c] * k2[c];
      acc += ra * k1[a];
    }
    return acc;
  };
  // two points per thread and step (independent chains of LDS reads)
  const int64_t stride = blockDim.x;
  int64_t j = j0 + threadIdx.x;
  for (; j + stride < j1; j += 2 * stride) {
    const float a = one(j), b = one(j + stride);
    out[(int64_t)t * nq + j] = a;
    out[(int64_t)t * nq + j + stride] = b;
  }
  if (j < j1) out[(int64_t)t * nq + j] = one(j);
}

static int ilog2i(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

static size_t grid_cells(int d, int nf) {
  size_t g = 1;
  for (int a = 0; a < d; ++a) g *= (size_t)nf;
  return g;
}

static size_t predict_ws(int d, int m, int T) {
  int nf = 16;
  while (nf < 2 * (2 * m + 1)) nf <<= 1;
  const int L = 2 * m + 1;
  Carve cv(nullptr, 0);
  if (d == 2 && predict_nf2(m)) {
    const int nf2 = predict_nf2(m);
    cv.take<double>((size_t)T * nf2 * L * 2);
    cv.take<float>((size_t)T * pad_stride(nf2, kMaxW));
    return cv.off + 512;
  }
  if (d == 2) cv.take<double>((size_t)T * nf * L * 2);
  if (d == 3) {
    cv.take<double>((size_t)T * nf * L * L * 2);
    cv.take<double>((size_t)T * nf * nf * L * 2);
  }
  cv.take<double>((size_t)T * grid_cells(d, nf));
  cv.take<float>((size_t)T * grid_cells(d, nf));
  return cv.off + 512;
}

// d = 3 is limited to m <= 31 (grid 128^3) and 64 coefficient sets per call.
static bool predict_shape_ok(int d, int m, int T) {
  if (d < 1 || d > 3 || m < 1 || m > 64 || T < 1 || T > 4096) return false;
  return d < 3 || (m <= 31 && T <= 64);
}

}  // namespace fk

using namespace fk;

extern "C" fk_status fk_predict_workspace_size(fk_ctx* ctx, int d, int m, int ntheta, size_t* bytes) {
  if (!bytes || !predict_shape_ok(d, m, ntheta)) return FK_EINVAL;
  *bytes = predict_ws(d, m, ntheta);
  return FK_OK;
}

#define FK_W_SWITCH2(w, CALL)                        \
  switch (w) {                                       \
    case 4: { constexpr int WW = 4; CALL; } break;   \
    case 5: { constexpr int WW = 5; CALL; } break;   \
    case 6: { constexpr int WW = 6; CALL; } break;   \
    case 7: { constexpr int WW = 7; CALL; } break;   \
    case 8: { constexpr int WW = 8; CALL; } break;   \
    case 9: { constexpr int WW = 9; CALL; } break;   \
    case 10: { constexpr int WW = 10; CALL; } break; \
    case 11: { constexpr int WW = 11; CALL; } break; \
    case 12: { constexpr int WW = 12; CALL; } break; \
    case 13: { constexpr int WW = 13; CALL; } break; \
    case 14: { constexpr int WW = 14; CALL; } break; \
    case 15: { constexpr int WW = 15; CALL; } break; \
    case 16: { constexpr int WW = 16; CALL; } break; \
    default: return FK_EINVAL;                       \
  }

namespace fk {

// The type-2 stage on a caller-given workspace and deconvolution table (device, plan.K + 1 doubles).
static fk_status predict_impl(fk_ctx* ctx, const EsPlan& plan, const double* phihat, int d, int m, int T,
                              const double* theta, int64_t nq, fk_dtype dt, const void* Xq, float* out, void* ws,
                              size_t ws_bytes) {
  fk_status st = reset_flags(ctx);
  if (st != FK_OK) return st;
  const int nf = plan.nf, logn = ilog2i(nf), L = 2 * m + 1;
  Carve cv(ws, ws_bytes);
  if (d == 2 && predict_nf2(m) == nf) {
    // two pruned FP64 DFTs into padded FP32 grids, then one LDS-resident grid per workgroup
    const int W = plan.w;
    const size_t pst = pad_stride(nf, W);
    double* t2 = cv.take<double>((size_t)T * nf * L * 2);
    float* gp = cv.take<float>((size_t)T * pst);
    if (!cv.ok()) return FK_ENOMEM;
    hipLaunchKernelGGL(k_idft_cols, dim3(T * L), dim3(256), 0, ctx->stream, theta, m, nf, phihat, t2);
    hipLaunchKernelGGL(k_idft_rows_pad, dim3(T * nf), dim3(256), 0, ctx->stream, t2, m, nf, W, phihat, pst, gp);
    int64_t per_chunk = 32768;
    if ((nq + per_chunk - 1) / per_chunk * T < 2048)
      per_chunk = std::max<int64_t>(1024, (nq * T + 2047) / 2048);
    const int64_t nchunk = (nq + per_chunk - 1) / per_chunk;
    const int64_t nchunk8 = (nchunk + 7) & ~int64_t(7);
    const int64_t blocks = nchunk8 * T;
    if (blocks > 0x7fffffff) return FK_EINVAL;
    EsDev2 es{(float)(plan.beta * 1.44269504088896340736), 2.0f / (float)W};
    const size_t lds = sizeof(float) * pst;
    FK_W_SWITCH2(W, hipLaunchKernelGGL(k_interp2_lds<WW>, dim3((unsigned)blocks), dim3(1024), lds, ctx->stream, gp,
                                       pst, nf, T, Xq, dt, nq, per_chunk, nchunk, (double)nf / (2.0 * 3.14159265358979323846),
                                       es, out, ctx->flags));
    FK_HIP(hipGetLastError());
    return read_flags(ctx);
  }
  double* tmp = d == 2 ? cv.take<double>((size_t)T * nf * L * 2) : nullptr;
  double* ta = d == 3 ? cv.take<double>((size_t)T * nf * L * L * 2) : nullptr;
  double* tb = d == 3 ? cv.take<double>((size_t)T * nf * nf * L * 2) : nullptr;
  double* g64 = cv.take<double>((size_t)T * grid_cells(d, nf));
  float* g32 = cv.take<float>((size_t)T * grid_cells(d, nf));
  if (!cv.ok()) return FK_ENOMEM;
  if (d == 1) {
    // one line per target: theta[t][q + m] -> g64[t][l] (real part)
    hipLaunchKernelGGL(k_ifft_line, dim3(T), dim3(256), 0, ctx->stream, theta, (int64_t)1, (int64_t)L, (int64_t)0,
                       1, m, phihat, nf, logn, g64, 1, (int64_t)1, (int64_t)nf, (int64_t)0);
  } else if (d == 3) {
    // axis 0: for each (t, q2, q3) the line over q1 (stride L^2) -> ta[t][l1][q2][q3]
    hipLaunchKernelGGL(k_ifft_line, dim3(T * L * L), dim3(256), 0, ctx->stream, theta, (int64_t)L * L,
                       (int64_t)L * L * L, (int64_t)1, L * L, m, phihat, nf, logn, ta, 0, (int64_t)L * L,
                       (int64_t)nf * L * L, (int64_t)1);
    // axis 1: for each (t, l1, q3) the line over q2 (stride L) -> tb[t][l1][l2][q3]
    hipLaunchKernelGGL(k_ifft_line, dim3(T * nf * L), dim3(256), 0, ctx->stream, ta, (int64_t)L, (int64_t)L * L,
                       (int64_t)1, L, m, phihat, nf, logn, tb, 0, (int64_t)L, (int64_t)nf * L, (int64_t)1);
    // axis 2: for each (t, l1, l2) the contiguous line over q3 -> g64[t][l1][l2][l3] real part
    hipLaunchKernelGGL(k_ifft_line, dim3(T * nf * nf), dim3(256), 0, ctx->stream, tb, (int64_t)1, (int64_t)L,
                       (int64_t)0, 1, m, phihat, nf, logn, g64, 1, (int64_t)1, (int64_t)nf, (int64_t)0);
  } else {
    // pass A: for each (t, q2): line over q1 (stride L) -> tmp[t][l1][q2] (complex, stride L)
    hipLaunchKernelGGL(k_ifft_line, dim3(T * L), dim3(256), 0, ctx->stream, theta, (int64_t)L, (int64_t)L * L,
                       (int64_t)1, L, m, phihat, nf, logn, tmp, 0, (int64_t)L, (int64_t)nf * L, (int64_t)1);
    // pass B: for each (t, l1): line over q2 (contiguous) -> g64[t][l1][l2] real part
    hipLaunchKernelGGL(k_ifft_line, dim3(T * nf), dim3(256), 0, ctx->stream, tmp, (int64_t)1, (int64_t)L,
                       (int64_t)0, 1, m, phihat, nf, logn, g64, 1, (int64_t)1, (int64_t)nf, (int64_t)0);
  }
  const int64_t gsz = (int64_t)T * (int64_t)grid_cells(d, nf);
  hipLaunchKernelGGL(k_d2f_grid, dim3((gsz + 255) / 256), dim3(256), 0, ctx->stream, g64, g32, gsz);
  EsDev2 es{(float)(plan.beta * 1.44269504088896340736), 2.0f / (float)plan.w};
  const int blocks = (int)((nq + 255) / 256);
  FK_W_SWITCH2(plan.w, hipLaunchKernelGGL(k_interp<WW>, dim3(blocks), dim3(256), 0, ctx->stream, g32, d, nf, T, Xq,
                                          dt, nq, es, out, ctx->flags));
  FK_HIP(hipGetLastError());
  return read_flags(ctx);
}

static bool predict_args_ok(fk_ctx* ctx, int d, int m, int T, const double* theta, int64_t nq, fk_dtype dt,
                            const void* Xq, const float* out) {
  return ctx && theta && Xq && out && predict_shape_ok(d, m, T) && nq >= 1 && (dt == FK_F32 || dt == FK_F64);
}

// ------------------------------------------------------------------ allocation-free prediction
// A file-scope device array holds the intermediates of fk_predict_noalloc: the deconvolution table
// at its start, then the workspace that fk_predict would take from the caller.  Each device has its
// own copy; host code uses only the address hipGetSymbolAddress returns for the device (the array's
// name on the host is a stand-in, not a device address).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchTable = 1024;   // phihat, at most 65 doubles
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};

// Resolves this device's copy of the array; called with the device current (from fk_create, and
// again by the entry point if that failed).  Returns FK_EHIP if the address cannot be taken.
fk_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return FK_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return FK_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FK_EHIP;
  g_scratch[device] = ptr;
  return FK_OK;
}

struct Table65 {
  double v[65];
};

__global__ void k_put_table(Table65 t, int count, double* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = t.v[i];
}

}  // namespace fk

extern "C" fk_status fk_predict(fk_ctx* ctx, int d, int m, int T, const double* theta, int64_t nq, fk_dtype dt,
                                const void* Xq, float* out, void* ws, size_t ws_bytes) {
  if (!predict_args_ok(ctx, d, m, T, theta, nq, dt, Xq, out)) return FK_EINVAL;
  if (!ws || ws_bytes < predict_ws(d, m, T)) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  kept_invalidate(ws, ws_bytes);
  EsPlan plan;
  const double* phihat;
  fk_status st = get_es_plan(ctx, m, &plan, &phihat, d == 2 ? predict_nf2(m) : 0);
  if (st != FK_OK) return st;
  return predict_impl(ctx, plan, phihat, d, m, T, theta, nq, dt, Xq, out, ws, ws_bytes);
}

extern "C" size_t fk_predict_noalloc_max_bytes(void) { return kScratchBytes - kScratchTable; }

extern "C" fk_status fk_predict_noalloc(fk_ctx* ctx, int d, int m, int T, const double* theta, int64_t nq,
                                        fk_dtype dt, const void* Xq, float* out) {
  if (!predict_args_ok(ctx, d, m, T, theta, nq, dt, Xq, out)) return FK_EINVAL;
  if (predict_ws(d, m, T) > kScratchBytes - kScratchTable) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  fk_status st = scratch_init(ctx->device);
  if (st != FK_OK) return st;
  unsigned char* base = static_cast<unsigned char*>(g_scratch[ctx->device]);
  EsPlan plan;
  st = get_es_plan_host(ctx, m, &plan, d == 2 ? predict_nf2(m) : 0);
  if (st != FK_OK) return st;
  if (plan.phihat.size() != (size_t)m + 1 || m + 1 > 65) return FK_EINVAL;
  // the deconvolution table goes in by value (a kernel argument), so no host buffer must outlive the call
  Table65 tab{};
  for (int i = 0; i <= m; ++i) tab.v[i] = plan.phihat[i];
  double* phihat = reinterpret_cast<double*>(base);
  hipLaunchKernelGGL(k_put_table, dim3(1), dim3(128), 0, ctx->stream, tab, m + 1, phihat);
  FK_HIP(hipGetLastError());
  return predict_impl(ctx, plan, phihat, d, m, T, theta, nq, dt, Xq, out, base + kScratchTable,
                      kScratchBytes - kScratchTable);
}

// ------------------------------------------------------------------ Philox4x32-10 generator
// Salmon et al., SC'11: ten rounds of (hi, lo) = M * c with the Weyl key schedule.

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

struct Box16 {
  double lo[16], hi[16];
};

__global__ void k_gen_uniform(uint64_t seed, int d, int64_t n, int64_t start, Box16 box, float* __restrict__ X) {
  const double* lo = box.lo;
  const double* hi = box.hi;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t j = (uint64_t)(i + start);
  for (int g = 0; g < (d + 3) / 4; ++g) {
    uint32_t c[4] = {(uint32_t)j, (uint32_t)(j >> 32), (uint32_t)(g == 0 ? 0 : 16 + g), 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int r = 0; r < 4; ++r) {
      int a = 4 * g + r;
      if (a >= d) break;
      double u = (double)(c[r] >> 8) * 5.9604644775390625e-08;  // 2^-24
      double span = __dadd_rn(hi[a], -lo[a]);
      X[(int64_t)a * n + i] = (float)__dadd_rn(lo[a], __dmul_rn(span, u));
    }
  }
}

__global__ void k_gen_targets(uint64_t seed, int ntgt, int64_t n, int64_t start, const float* __restrict__ X,
                              double sigma, float* __restrict__ Y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t j = (uint64_t)(i + start);
  const double x1 = X[i], x2 = X[n + i];
  const double c2 = cos(x2);
  for (int t = 1; t <= ntgt; ++t) {
    uint32_t c[4] = {(uint32_t)j, (uint32_t)(j >> 32), (uint32_t)t, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    double u1 = ((double)c[0] + 1.0) * 2.3283064365386963e-10;  // (0, 1]
    double u2 = (double)c[1] * 2.3283064365386963e-10;          // [0, 1)
    double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    double v = sin((double)t * x1) * c2 + sigma * z;
    Y[(int64_t)(t - 1) * n + i] = (float)v;
  }
}

extern "C" fk_status fk_generate_uniform(fk_ctx* ctx, uint64_t seed, int d, int64_t n, int64_t start,
                                         const double* lo, const double* hi, float* X) {
  if (!ctx || !lo || !hi || !X || d < 1 || d > 16 || n < 1 || start < 0) return FK_EINVAL;
  FK_HIP(hipSetDevice(ctx->device));
  Box16 box;
  for (int a = 0; a < 16; ++a) {
    box.lo[a] = a < d ? lo[a] : 0.0;
    box.hi[a] = a < d ? hi[a] : 0.0;
  }
  hipLaunchKernelGGL(k_gen_uniform, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, seed, d, n, start,
                     box, X);
  FK_HIP(hipGetLastError());
  FK_HIP(hipStreamSynchronize(ctx->stream));
  return FK_OK;
}

extern "C" fk_status fk_generate_targets(fk_ctx* ctx, uint64_t seed, int ntgt, int64_t n, int64_t start,
                                         const float* X, double sigma, float* Y) {
  if (!ctx || !X || !Y || ntgt < 1 || ntgt > 1024 || n < 1 || start < 0) return FK_EINVAL;
  FK_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(k_gen_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, seed, ntgt, n,
                     start, X, sigma, Y);
  FK_HIP(hipGetLastError());
  FK_HIP(hipStreamSynchronize(ctx->stream));
  return FK_OK;
}
