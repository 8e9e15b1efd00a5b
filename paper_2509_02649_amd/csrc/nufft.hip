// Type-1 non-uniform FFT on gfx950: exponential-of-semicircle spreading onto an
// oversampled grid, FP64 FFT, deconvolution.
//
// What is computed (Sec. 2.3 of the paper, "Covariance vector" / "Covariance
// matrix"): for C real weight channels w_c and points x_j on the torus,
//     c_c[q] = sum_j w_cj exp(-i q.x_j),   |q_a| <= K.
// Method (Barnett, Magland, af Klinteberg, SIAM J. Sci. Comput. 41(5), 2019):
// with grid spacing h = 2 pi / nf and grid point l <-> x = -pi + l h, spread
//     g_c[l] = sum_j w_cj phi(l - u_j),  u_j = (x_j + pi) / h,
// phi(t) = psi(2 t / w), psi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1, then
//     c_c[q] ~= (-1)^q DFT(g_c)[q mod nf] / prod_a Phihat(q_a h),
// Phihat(omega) = int phi(t) exp(-i omega t) dt (Poisson summation; the
// aliased terms are the error, bounded here by the plan's error estimate).
//
// Design for MI355X:
// * 1-D grids (<= 1024 points per channel) live whole in LDS: each workgroup
//   streams a contiguous chunk of points (coalesced), accumulates partials
//   with LDS atomics and flushes them once into an FP64 global grid.
// * 2-D grids (up to 512 x 512) do not fit in 160 KB of LDS, so points are
//   counting-sorted by bin (a T x T tile of the grid): per-workgroup LDS
//   histograms, a scan, and a scatter into bin-contiguous records
//   (two 32-bit fixed-point grid coordinates + FP32 weights).  One workgroup
//   per (bin, slice of the bin's points) then spreads into an LDS subgrid of
//   (T + 2 ceil(w/2))^2 cells x C channels and flushes it with FP64 atomics.
// * LDS partials are FP64: on gfx950 ds_add_f64 sustains ~7 lane-ops/clk/CU
//   while ds_add_f32 sustains ~0.33 (measured), so the wider type is also the
//   fast one, and the per-bin partials carry no FP32 rounding.
// * Grid coordinates are computed in FP64 and carried as fixed point (error
//   <= 2^-(33 - log2 nf) grid units), so the phase error stays below 1e-7
//   even at the highest frequency.
// * The FFT and deconvolution run in FP64 (the grids are tiny).
#include "fk_internal.h"
#include "fk_device.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace fk {

// ------------------------------------------------------------------ plan (host)

static double es_psi(double z, double beta) {
  double r = 1.0 - z * z;
  return r < 0 ? 0.0 : std::exp(beta * (std::sqrt(r) - 1.0));
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on the Legendre recurrence).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Phihat(omega) = (w/2) int_{-1}^{1} psi(z) cos(omega w z / 2) dz.
static double es_phihat(double omega, int w, double beta, const std::vector<double>& gx,
                        const std::vector<double>& gw) {
  double s = 0.0;
  for (size_t i = 0; i < gx.size(); ++i) s += gw[i] * es_psi(gx[i], beta) * std::cos(omega * w * gx[i] * 0.5);
  return 0.5 * w * s;
}

// Worst case over sub-grid shifts of |sum_l phi(l - u) e^{-i omega (l-u)} - Phihat(omega)| / Phihat(omega)
// for omega = q h, 0 <= q <= K.
static double es_error(int nf, int K, int w, double beta, const std::vector<double>& gx,
                       const std::vector<double>& gw) {
  const double h = 2.0 * kPi / nf;
  std::vector<double> ph(K + 1);
  for (int q = 0; q <= K; ++q) ph[q] = es_phihat(q * h, w, beta, gx, gw);
  double worst = 0.0;
  const int nu = 24;
  for (int iu = 0; iu <= nu; ++iu) {
    double u = double(iu) / nu;
    for (int q = 0; q <= K; q += std::max(1, K / 48)) {
      double re = 0.0, im = 0.0;
      for (int l = -w; l <= w + 1; ++l) {
        double t = l - u;
        double z = 2.0 * t / w;
        if (std::fabs(z) > 1.0) continue;
        double v = es_psi(z, beta);
        re += v * std::cos(q * h * t);
        im -= v * std::sin(q * h * t);
      }
      double e = std::hypot(re - ph[q], im) / std::fabs(ph[q]);
      worst = std::max(worst, e);
    }
  }
  return worst;
}

EsPlan make_es_plan(int K, double eps, int nf_fixed) {
  // Fine grid: nf_fixed when given, else the smallest power of two with oversampling
  // nf / (2K+1) >= 2.
  EsPlan p;
  p.K = K;
  int nf = 16;
  while (nf < 2 * (2 * K + 1)) nf <<= 1;
  if (nf_fixed > 0) nf = nf_fixed;
  p.nf = nf;
  std::vector<double> gx, gw;
  gauss_legendre(160, gx, gw);
  const double sigma = double(nf) / (2 * K + 1);
  int best_w = kMaxW;
  double best_beta = 2.3 * kMaxW, best_err = 1.0;
  for (int w = 4; w <= kMaxW; ++w) {
    // shape parameter: scan around the published heuristic beta ~ pi w (1 - 1/(2 sigma)) * 0.97
    double b0 = 0.97 * kPi * w * (1.0 - 0.5 / sigma);
    double bb = b0, be = 1.0;
    for (int i = -6; i <= 6; ++i) {
      double beta = b0 * (1.0 + 0.02 * i);
      double e = es_error(nf, K, w, beta, gx, gw);
      if (e < be) { be = e; bb = beta; }
    }
    if (be <= eps || w == kMaxW) {
      best_w = w;
      best_beta = bb;
      best_err = be;
      break;
    }
  }
  p.w = best_w;
  p.beta = best_beta;
  p.err = best_err;
  p.phihat.resize(K + 1);
  const double h = 2.0 * kPi / nf;
  for (int q = 0; q <= K; ++q) p.phihat[q] = es_phihat(q * h, p.w, p.beta, gx, gw);
  return p;
}

fk_status get_es_plan(fk_ctx* ctx, int K, EsPlan* plan, const double** d_phihat, int nf_fixed) {
  double eps = ctx->opt.eps > 0 ? ctx->opt.eps : 2e-7;
  uint64_t bits;
  std::memcpy(&bits, &eps, 8);
  auto key = std::make_pair(K + (nf_fixed << 16), bits);
  auto it = ctx->es_cache.find(key);
  if (it == ctx->es_cache.end()) {
    EsPlan p = make_es_plan(K, eps, nf_fixed);
    double* d = nullptr;
    FK_HIP(hipMalloc(&d, sizeof(double) * (K + 1)));
    FK_HIP(hipMemcpy(d, p.phihat.data(), sizeof(double) * (K + 1), hipMemcpyHostToDevice));
    it = ctx->es_cache.emplace(key, std::make_pair(p, d)).first;
  }
  *plan = it->second.first;
  *d_phihat = it->second.second;
  return FK_OK;
}

fk_status get_es_plan_host(fk_ctx* ctx, int K, EsPlan* plan, int nf_fixed) {
  double eps = ctx->opt.eps > 0 ? ctx->opt.eps : 2e-7;
  uint64_t bits;
  std::memcpy(&bits, &eps, 8);
  auto key = std::make_pair(K + (nf_fixed << 16), bits);
  auto dev = ctx->es_cache.find(key);
  if (dev != ctx->es_cache.end()) {
    *plan = dev->second.first;
    return FK_OK;
  }
  auto it = ctx->es_host_cache.find(key);
  if (it == ctx->es_host_cache.end()) it = ctx->es_host_cache.emplace(key, make_es_plan(K, eps, nf_fixed)).first;
  *plan = it->second;
  return FK_OK;
}

// ------------------------------------------------------------------ device helpers

// beta is pre-multiplied by log2(e): the exponent lies in [-beta log2 e, 0], so the hardware exp2
// needs no range handling, and the hardware square root no denormal scaling.
struct EsDev {
  float beta_log2e;
  float two_over_w;
};

__device__ __forceinline__ float es_eval(float s, EsDev es) {
  // s: distance in grid units; |s| <= w/2 inside the support.
  const float z = s * es.two_over_w;
  const float r = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
  return __builtin_amdgcn_exp2f(fmaf(es.beta_log2e, __builtin_amdgcn_sqrtf(r), -es.beta_log2e));
}

// Window start i0 = ceil(u - w/2) and first offset s0 = i0 - u (grid units) from
// a fixed-point coordinate with fb fraction bits.
__device__ __forceinline__ void window_start(uint32_t U, int fb, int w, int* i0, float* s0) {
  int64_t V = (int64_t)U - ((int64_t)w << (fb - 1));
  int64_t one = (int64_t)1 << fb;
  int64_t c = (V >= 0) ? ((V + one - 1) >> fb) : -((-V) >> fb);
  *i0 = (int)c;
  *s0 = (float)((double)((c << fb) - (int64_t)U) * (1.0 / (double)one));
}

// ------------------------------------------------------------------ 1-D spread (whole grid in LDS)
// grid: gridDim.x workgroups over contiguous chunks of points.  LDS: C * nf floats.
// Channel 0 carries weight 1 when ones != 0; channels ones..C-1 read Y rows.
template <int W>
__global__ __launch_bounds__(256) void k_spread_1d(const void* __restrict__ X, fk_dtype dt, int64_t n,
                                                   const void* __restrict__ Y, int nw, int ones,
                                                   int nf, int fb, double scale, EsDev es,
                                                   double* __restrict__ grid, int* flags,
                                                   int64_t chunk) {
  extern __shared__ double lds[];
  const int C = nw + ones;
  for (int i = threadIdx.x; i < C * nf; i += blockDim.x) lds[i] = 0.0;
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(n, beg + chunk);
  const uint32_t nf_fix = (uint32_t)nf << fb;
  for (int64_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
    uint32_t U;
    if (!to_fixed(load_coord(X, dt, j), scale, nf_fix, &U, flags)) continue;
    int i0;
    float s0;
    window_start(U, fb, W, &i0, &s0);
    float k[W];
#pragma unroll
    for (int a = 0; a < W; ++a) k[a] = es_eval(s0 + (float)a, es);
    int base = i0 < 0 ? i0 + nf : i0;
    if (ones) {
#pragma unroll
      for (int a = 0; a < W; ++a) {
        int l = base + a;
        l = l >= nf ? l - nf : l;
        atomicAdd(&lds[l], (double)k[a]);
      }
    }
    for (int c = 0; c < nw; ++c) {
      float wc = load_weight(Y, dt, (int64_t)c * n + j);
      if (!(wc == wc) || isinf(wc)) { atomicOr(&flags[kFlagNaN], 1); continue; }
      double* g = lds + (c + ones) * nf;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        int l = base + a;
        l = l >= nf ? l - nf : l;
        atomicAdd(&g[l], (double)(wc * k[a]));
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < C * nf; i += blockDim.x) {
    double v = lds[i];
    if (v != 0.0) atomicAdd(&grid[i], v);
  }
}

// ------------------------------------------------------------------ 3-D spread (FP64 global atomics)
// One thread per point: the w^3 window of every channel (channel 0 with weight 1) is added into
// the FP64 grid [C][nf][nf][nf] by hardware FP64 atomics.  Kernel values in FP32, as in 1-D.
template <int W>
__global__ __launch_bounds__(256) void k_spread_3d(const void* __restrict__ X, fk_dtype dt, int64_t n,
                                                   int64_t xstride, const void* __restrict__ Y, int nw, int nf,
                                                   int fb, double scale, EsDev es, double* __restrict__ grid,
                                                   int* flags) {
  const uint32_t nf_fix = (uint32_t)nf << fb;
  const int64_t cube = (int64_t)nf * nf * nf;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    uint32_t U[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) ok = to_fixed(load_coord(X, dt, a * xstride + j), scale, nf_fix, &U[a], flags) && ok;
    if (!ok) continue;
    float k[3][W];
    int base[3];
    for (int a = 0; a < 3; ++a) {
      int i0;
      float s0;
      window_start(U[a], fb, W, &i0, &s0);
#pragma unroll
      for (int t = 0; t < W; ++t) k[a][t] = es_eval(s0 + (float)t, es);
      base[a] = i0 < 0 ? i0 + nf : i0;
    }
    for (int c = 0; c <= nw; ++c) {
      float wc = 1.0f;
      if (c > 0) {
        wc = load_weight(Y, dt, (int64_t)(c - 1) * n + j);
        if (!(wc == wc) || isinf(wc)) {
          atomicOr(&flags[kFlagNaN], 1);
          continue;
        }
      }
      double* g = grid + (int64_t)c * cube;
      for (int a1 = 0; a1 < W; ++a1) {
        int l1 = base[0] + a1;
        l1 = l1 >= nf ? l1 - nf : l1;
        const float v1 = wc * k[0][a1];
        for (int a2 = 0; a2 < W; ++a2) {
          int l2 = base[1] + a2;
          l2 = l2 >= nf ? l2 - nf : l2;
          const float v12 = v1 * k[1][a2];
          double* row = g + ((int64_t)l1 * nf + l2) * nf;
#pragma unroll
          for (int a3 = 0; a3 < W; ++a3) {
            int l3 = base[2] + a3;
            l3 = l3 >= nf ? l3 - nf : l3;
            atomicAdd(&row[l3], (double)(v12 * k[2][a3]));
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ 3-D binned spread
// Bins are T^3 blocks of window-start cells (nbx = nf / T per axis).  A point's window start
// i0 = ceil(u - w/2) per axis places it in bin (i0 mod nf) >> tshift, and its whole window then
// lies in the bin's subgrid of S = T + w - 1 cells per axis starting at the bin origin.

__device__ __forceinline__ bool fixed3(const void* X, fk_dtype dt, int64_t xstride, int64_t j, double scale,
                                       uint32_t nf_fix, uint32_t U[3], int* flags) {
  bool ok = true;
  for (int a = 0; a < 3; ++a) ok = to_fixed(load_coord(X, dt, a * xstride + j), scale, nf_fix, &U[a], flags) && ok;
  return ok;
}

__device__ __forceinline__ int bin3_of(const uint32_t U[3], int fb, int w, int nf, int tshift, int nbx) {
  int b = 0;
  for (int a = 0; a < 3; ++a) {
    int i0;
    float s0;
    window_start(U[a], fb, w, &i0, &s0);
    b = b * nbx + ((i0 & (nf - 1)) >> tshift);
  }
  return b;
}

__global__ __launch_bounds__(256) void k_bin3_count(const void* __restrict__ X, fk_dtype dt, int64_t n,
                                                    int64_t xstride, int nf, int fb, double scale, int w,
                                                    int tshift, int nbx, uint32_t* __restrict__ cnt, int* flags) {
  const uint32_t nf_fix = (uint32_t)nf << fb;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    uint32_t U[3];
    if (!fixed3(X, dt, xstride, j, scale, nf_fix, U, flags)) continue;
    atomicAdd(&cnt[bin3_of(U, fb, w, nf, tshift, nbx)], 1u);
  }
}

// start[b] = sum of cnt[< b] (start[nb] = valid points), cursor[b] = start[b].  One workgroup.
__global__ __launch_bounds__(1024) void k_bin3_scan(const uint32_t* __restrict__ cnt, int nb,
                                                    uint64_t* __restrict__ start, uint64_t* __restrict__ cursor) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
  uint64_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += cnt[b];
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    uint64_t run = 0;
    for (int k = 0; k < 1024; ++k) {
      const uint64_t v = part[k];
      part[k] = run;
      run += v;
    }
    start[nb] = run;
  }
  __syncthreads();
  uint64_t run = part[t];
  for (int b = b0; b < b1; ++b) {
    start[b] = run;
    cursor[b] = run;
    run += cnt[b];
  }
}

// Records of 3 + nw words: the fixed-point coordinates, then the weights (a NaN or Inf weight
// raises the flag and is stored as 0).
__global__ __launch_bounds__(256) void k_bin3_scatter(const void* __restrict__ X, fk_dtype dt, int64_t n,
                                                      int64_t xstride, const void* __restrict__ Y, int nw, int nf,
                                                      int fb, double scale, int w, int tshift, int nbx,
                                                      unsigned long long* __restrict__ cursor,
                                                      uint32_t* __restrict__ rec, int* flags) {
  const uint32_t nf_fix = (uint32_t)nf << fb;
  const int R = 3 + nw;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    uint32_t U[3];
    if (!fixed3(X, dt, xstride, j, scale, nf_fix, U, flags)) continue;
    const unsigned long long pos = atomicAdd(&cursor[bin3_of(U, fb, w, nf, tshift, nbx)], 1ull);
    uint32_t* r = rec + pos * R;
    r[0] = U[0];
    r[1] = U[1];
    r[2] = U[2];
    for (int c = 0; c < nw; ++c) {
      float wc = load_weight(Y, dt, (int64_t)c * n + j);
      if (!(wc == wc) || isinf(wc)) {
        atomicOr(&flags[kFlagNaN], 1);
        wc = 0.f;
      }
      r[3 + c] = __float_as_uint(wc);
    }
  }
}

// One workgroup per (bin, slice): the slice's points add their windows into the bin's LDS
// subgrid [C][S][S][S] by FP64 LDS atomics; the subgrid is then added into the FP64 grid.
template <int W>
__global__ __launch_bounds__(256) void k_spread_3d_binned(const uint32_t* __restrict__ rec, int nw,
                                                          const uint64_t* __restrict__ start, int nbx, int T,
                                                          int nf, int fb, EsDev es, int slices,
                                                          double* __restrict__ grid) {
  extern __shared__ double sub[];
  const int S = T + W - 1, S3 = S * S * S, C = nw + 1, R = 3 + nw;
  const int bin = blockIdx.x / slices, sl = blockIdx.x - bin * slices;
  for (int i = threadIdx.x; i < C * S3; i += blockDim.x) sub[i] = 0.0;
  __syncthreads();
  const uint64_t p0 = start[bin], len = start[bin + 1] - p0;
  const uint64_t q0 = p0 + len * sl / slices, q1 = p0 + len * (sl + 1) / slices;
  const int bz = bin % nbx, by = (bin / nbx) % nbx, bx = bin / (nbx * nbx);
  const int o[3] = {bx * T, by * T, bz * T};
  for (uint64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    const uint32_t* r = rec + q * R;
    float k[3][W];
    int rel[3];
    for (int a = 0; a < 3; ++a) {
      int i0;
      float s0;
      window_start(r[a], fb, W, &i0, &s0);
      rel[a] = (i0 & (nf - 1)) - o[a];
#pragma unroll
      for (int t = 0; t < W; ++t) k[a][t] = es_eval(s0 + (float)t, es);
    }
    for (int c = 0; c < C; ++c) {
      const float wc = c == 0 ? 1.0f : __uint_as_float(r[2 + c]);
      double* g = sub + c * S3;
      for (int a1 = 0; a1 < W; ++a1) {
        const float v1 = wc * k[0][a1];
        for (int a2 = 0; a2 < W; ++a2) {
          const float v12 = v1 * k[1][a2];
          double* row = g + ((rel[0] + a1) * S + (rel[1] + a2)) * S + rel[2];
#pragma unroll
          for (int a3 = 0; a3 < W; ++a3) atomicAdd(&row[a3], (double)(v12 * k[2][a3]));
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < C * S3; i += blockDim.x) {
    const double v = sub[i];
    if (v == 0.0) continue;
    const int c = i / S3, cell = i - c * S3;
    const int x = cell / (S * S), y = (cell / S) % S, z = cell % S;
    int gx = o[0] + x, gy = o[1] + y, gz = o[2] + z;
    gx -= gx >= nf ? nf : 0;
    gy -= gy >= nf ? nf : 0;
    gz -= gz >= nf ? nf : 0;
    atomicAdd(&grid[(((int64_t)c * nf + gx) * nf + gy) * nf + gz], v);
  }
}

// ------------------------------------------------------------------ 2-D binned spread
// Bins are T x T tiles of the nf x nf grid: nbx = nf / T bins per axis.

__global__ __launch_bounds__(256) void k_bin_count(const void* __restrict__ X, fk_dtype dt, int64_t n,
                                                   int64_t xstride, int nf, int fb, double scale,
                                                   int tshift, int nbx, uint32_t* __restrict__ cnt,
                                                   int nblk, int64_t chunk, int* flags) {
  extern __shared__ uint32_t hist[];
  const int nb = nbx * nbx;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(n, beg + chunk);
  const uint32_t nf_fix = (uint32_t)nf << fb;
  for (int64_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
    uint32_t U1, U2;
    bool ok = to_fixed(load_coord(X, dt, j), scale, nf_fix, &U1, flags);
    ok = to_fixed(load_coord(X, dt, xstride + j), scale, nf_fix, &U2, flags) && ok;
    if (!ok) continue;
    int b = ((U1 >> fb) >> tshift) * nbx + ((U2 >> fb) >> tshift);
    atomicAdd(&hist[b], 1u);
  }
  __syncthreads();
  // count table is [workgroup][bin]: one contiguous row per workgroup
  uint32_t* row = cnt + (int64_t)blockIdx.x * nb;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) row[i] = hist[i];
  (void)nblk;
}

// Exclusive scan over workgroups of cnt[.][bin] in place, one thread per bin
// (consecutive threads read consecutive bins of a row); bin totals out.
__global__ __launch_bounds__(256) void k_scan_cols(uint32_t* __restrict__ cnt, int nb, int nblk,
                                                   uint32_t* __restrict__ totals) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  uint32_t run = 0;
  for (int k = 0; k < nblk; ++k) {
    uint32_t* p = cnt + (int64_t)k * nb + b;
    uint32_t c = *p;
    *p = run;
    run += c;
  }
  totals[b] = run;
}

// Exclusive scan of the bin totals (nb <= 65536) by one workgroup; start[nb] = total.
__global__ __launch_bounds__(1024) void k_scan_totals(const uint32_t* __restrict__ totals, int nb,
                                                      uint64_t* __restrict__ start) {
  __shared__ uint64_t part[1024];
  const int per = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  uint64_t s = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) s += totals[b0 + i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint64_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint64_t run = part[threadIdx.x] - s;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) {
      start[b0 + i] = run;
      run += totals[b0 + i];
    }
  if (threadIdx.x == 1023) start[nb] = part[1023];
}

// Scatter points into bin-contiguous records [U1, U2, w_0 .. w_{nw-1}] (32-bit words).
// Each workgroup keeps the next write position of every bin in LDS (64-bit,
// seeded from the scans) and claims a slot with one LDS atomic per point.
__global__ __launch_bounds__(1024) void k_bin_scatter(const void* __restrict__ X, fk_dtype dt, int64_t n,
                                                      int64_t xstride, const void* __restrict__ Y,
                                                      int nw, int nf, int fb, double scale, int tshift,
                                                      int nbx, const uint32_t* __restrict__ cnt,
                                                      const uint64_t* __restrict__ start, int64_t chunk,
                                                      uint32_t* __restrict__ rec, int* flags) {
  extern __shared__ unsigned long long nextpos[];
  const int nb = nbx * nbx;
  const uint32_t* row = cnt + (int64_t)blockIdx.x * nb;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) nextpos[i] = start[i] + row[i];
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(n, beg + chunk);
  const uint32_t nf_fix = (uint32_t)nf << fb;
  const int R = 2 + nw;
  for (int64_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
    uint32_t U1, U2;
    bool ok = to_fixed(load_coord(X, dt, j), scale, nf_fix, &U1, flags);
    ok = to_fixed(load_coord(X, dt, xstride + j), scale, nf_fix, &U2, flags) && ok;
    if (!ok) continue;
    int b = ((U1 >> fb) >> tshift) * nbx + ((U2 >> fb) >> tshift);
    uint64_t pos = atomicAdd(&nextpos[b], 1ull);
    uint32_t* o = rec + pos * R;
    o[0] = U1;
    o[1] = U2;
    for (int c = 0; c < nw; ++c) {
      float wc = load_weight(Y, dt, (int64_t)c * n + j);
      if (!(wc == wc) || isinf(wc)) {
        atomicOr(&flags[kFlagNaN], 1);
        wc = 0.f;
      }
      o[2 + c] = __float_as_uint(wc);
    }
  }
}

// One workgroup per (bin, slice).  LDS subgrid S x S cells x C channels,
// cell-major ([cell][channel]) so the channels of one cell are adjacent.
template <int W>
__global__ __launch_bounds__(256) void k_spread_2d_binned(const uint32_t* __restrict__ rec, int nw,
                                                          int ones, const uint64_t* __restrict__ start,
                                                          int nbx, int T, int nf, int fb, EsDev es,
                                                          int slices, double* __restrict__ grid) {
  extern __shared__ double sub[];
  constexpr int H = (W + 1) / 2;     // halo each side
  const int S = T + 2 * H;
  const int C = nw + ones;
  const int b = blockIdx.x / slices;
  const int sl = blockIdx.x - b * slices;
  const uint64_t p0 = start[b], p1 = start[b + 1];
  const uint64_t len = p1 - p0;
  const uint64_t q0 = p0 + len * sl / slices;
  const uint64_t q1 = p0 + len * (sl + 1) / slices;
  if (q0 == q1) return;
  for (int i = threadIdx.x; i < S * S * C; i += blockDim.x) sub[i] = 0.0;
  __syncthreads();
  const int bx = b / nbx, by = b - bx * nbx;
  const int o1 = bx * T - H, o2 = by * T - H;   // subgrid origin (may be negative: periodic)
  const int R = 2 + nw;
  for (uint64_t j = q0 + threadIdx.x; j < q1; j += blockDim.x) {
    const uint32_t* r = rec + j * R;
    int i1, i2;
    float s1, s2;
    window_start(r[0], fb, W, &i1, &s1);
    window_start(r[1], fb, W, &i2, &s2);
    float k1[W], k2[W];
#pragma unroll
    for (int a = 0; a < W; ++a) {
      k1[a] = es_eval(s1 + (float)a, es);
      k2[a] = es_eval(s2 + (float)a, es);
    }
    const int l1 = i1 - o1, l2 = i2 - o2;      // in [0, S - W]
    if (ones) {
#pragma unroll
      for (int a = 0; a < W; ++a) {
        double* row = sub + ((l1 + a) * S + l2) * C;
#pragma unroll
        for (int c2 = 0; c2 < W; ++c2) atomicAdd(&row[c2 * C], (double)(k1[a] * k2[c2]));
      }
    }
    for (int cg = 0; cg < nw; cg += 4) {
      float wv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) wv[u] = (cg + u < nw) ? __uint_as_float(r[2 + cg + u]) : 0.f;
      const int cn = min(4, nw - cg);
#pragma unroll
      for (int a = 0; a < W; ++a) {
        double* row = sub + ((l1 + a) * S + l2) * C + ones + cg;
#pragma unroll
        for (int c2 = 0; c2 < W; ++c2) {
          float kk = k1[a] * k2[c2];
          double* cell = row + c2 * C;
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (u < cn) atomicAdd(&cell[u], (double)(wv[u] * kk));
        }
      }
    }
  }
  __syncthreads();
  // flush: periodic wrap into the FP64 global grid [C][nf][nf]
  for (int i = threadIdx.x; i < S * S * C; i += blockDim.x) {
    double v = sub[i];
    if (v == 0.0) continue;
    int c = i % C;
    int cell = i / C;
    int a = cell / S, bb = cell - a * S;
    int g1 = o1 + a, g2 = o2 + bb;
    g1 = g1 < 0 ? g1 + nf : (g1 >= nf ? g1 - nf : g1);
    g2 = g2 < 0 ? g2 + nf : (g2 >= nf ? g2 - nf : g2);
    atomicAdd(&grid[((int64_t)c * nf + g1) * nf + g2], v);
  }
}

// ------------------------------------------------------------------ FFT (FP64, radix-2, in LDS)
// One workgroup transforms one line of length nf (power of two <= 1024) and
// writes the pruned, deconvolved frequencies q = -K..K:
//   out[line][q + K] = scale * (-1)^q / phihat[|q|] * sum_l in[l] e^{-2 pi i q l / nf}.
// Input line `line` starts at in + line_off(line) with element stride `istride`
// (complex elements when icomplex, else real doubles).
__global__ __launch_bounds__(256) void k_fft_line(const double* __restrict__ in, int icomplex,
                                                  int64_t istride, int64_t in_line_stride_outer,
                                                  int64_t in_line_stride_inner, int lines_inner,
                                                  int nf, int logn, const double* __restrict__ phihat,
                                                  int K, double scale, double* __restrict__ out,
                                                  int64_t ostride, int64_t out_line_stride_outer,
                                                  int64_t out_line_stride_inner) {
  __shared__ double re[1024], im[1024];
  const int line = blockIdx.x;
  const int lo = line / lines_inner, li = line - lo * lines_inner;
  const double* src = in + (lo * in_line_stride_outer + li * in_line_stride_inner) * (icomplex ? 2 : 1);
  for (int i = threadIdx.x; i < nf; i += blockDim.x) {
    int r = __brev((unsigned)i) >> (32 - logn);
    if (icomplex) {
      re[r] = src[2 * i * istride];
      im[r] = src[2 * i * istride + 1];
    } else {
      re[r] = src[i * istride];
      im[r] = 0.0;
    }
  }
  __syncthreads();
  for (int len = 2; len <= nf; len <<= 1) {
    const int half = len >> 1;
    for (int t = threadIdx.x; t < nf / 2; t += blockDim.x) {
      int grp = t / half, pos = t - grp * half;
      int i = grp * len + pos, j = i + half;
      double sn, cs;
      sincospi(-2.0 * pos / len, &sn, &cs);
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
  double* dst = out + (lo * out_line_stride_outer + li * out_line_stride_inner) * 2;
  for (int q = -K + (int)threadIdx.x; q <= K; q += blockDim.x) {
    int l = q < 0 ? q + nf : q;
    int aq = q < 0 ? -q : q;
    double f = scale / phihat[aq];
    if (aq & 1) f = -f;
    dst[2 * (q + K) * ostride] = re[l] * f;
    dst[2 * (q + K) * ostride + 1] = im[l] * f;
  }
}

// ------------------------------------------------------------------ host driver

static int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

struct BinGeom {
  int T, tshift, nbx, nb, nblk;
  int64_t chunk;
};

// Spread used by the 2-D type-1 stage.  kRows: 8..16 weighted channels as the rows
// of matrix-core products (spread_mfma.hip); kOuter: 0..7 weighted channels as
// per-channel outer products (spread_op.hip); both after the two-pass bin sort.
// kAtomic: one counting pass and FP64 LDS atomics (other channel counts or widths).
enum class Spread2 { kAtomic, kRows, kOuter };

static Spread2 spread2_kind(int nw, int nf, int W, int64_t n) {
  if (nw >= 8 && nw <= 16 && spread_mfma_ok(nw, W) && sort2_ok(nf / spread_mfma_bin(nf, n))) return Spread2::kRows;
  if (spread_op_ok(nw, W) && nf % spread_op_bin() == 0 && sort2_ok(nf / spread_op_bin())) return Spread2::kOuter;
  return Spread2::kAtomic;
}

// Bin edge of the channel-row spread: the shape's choice when the sort can take it, else the
// density rule.
static int rows_bin(int nf, int64_t n, int mb) {
  if ((mb == 2 || mb == 4) && sort2_ok(nf / mb)) return mb;
  return spread_mfma_bin(nf, n);
}

static BinGeom bin_geom(int nf, int C, int64_t n, Spread2 kind, int mb = 0) {
  BinGeom g;
  g.T = kind == Spread2::kRows ? rows_bin(nf, n, mb)
        : kind == Spread2::kOuter ? spread_op_bin() : ((C > 8) ? 16 : 32);
  if (g.T > nf) g.T = nf;
  g.tshift = ilog2(g.T);
  g.nbx = nf / g.T;
  g.nb = g.nbx * g.nbx;
  const int64_t cap = std::max<int64_t>(1, (int64_t)(1 << 23) / g.nb);   // count table <= 8M entries
  g.nblk = (int)std::min<int64_t>(std::min<int64_t>(2048, cap), std::max<int64_t>(1, (n + 8191) / 8192));
  g.chunk = (n + g.nblk - 1) / g.nblk;
  return g;
}

// Workspace of type1(): the largest layout any kernel width can select (the width
// follows from K and the context's tolerance, not known here).
size_t type1_workspace(int d, int64_t n, int nw, int K, double eps) {
  (void)eps;
  int nf = 16;
  while (nf < 2 * (2 * K + 1)) nf <<= 1;
  const int C = nw + 1;
  const int L = 2 * K + 1;
  auto layout = [&](Spread2 kind) {
    Carve cv(nullptr, 0);
    if (d == 1) {
      cv.take<double>((size_t)C * nf);
      return cv.off;
    }
    if (d == 3) {
      cv.take<double>((size_t)C * nf * nf * nf);      // FP64 grid
      cv.take<double>((size_t)C * nf * nf * L * 2);   // after the axis-2 transform
      cv.take<double>((size_t)C * nf * L * L * 2);    // after the axis-1 transform
      const size_t nb = (size_t)(nf / 2) * (nf / 2) * (nf / 2);   // the smallest bins (T = 2)
      cv.take<uint32_t>(nb);                          // counts
      cv.take<uint64_t>(nb + 1);                      // starts
      cv.take<uint64_t>(nb);                          // cursors
      cv.take<uint32_t>((size_t)n * (3 + nw));        // records
      return cv.off;
    }
    cv.take<double>((size_t)C * nf * nf);          // FP64 grid
    cv.take<double>((size_t)C * nf * L * 2);        // row-FFT output
    BinGeom g = bin_geom(nf, C, n, kind);
    if (kind == Spread2::kRows) {                   // bin starts for the finest bins any shape takes
      const BinGeom g2 = bin_geom(nf, C, n, kind, 2);
      if (g2.nb > g.nb) g = g2;
    }
    cv.take<uint32_t>((size_t)g.nb * g.nblk);
    cv.take<uint32_t>((size_t)g.nb);
    cv.take<uint64_t>((size_t)g.nb + 1);
    if (kind != Spread2::kAtomic) {
      const int wv = sort2_words(nw);
      cv.take<uint32_t>((size_t)n * 2);
      cv.take<uint32_t>((size_t)n * (kind == Spread2::kRows ? 1 : wv));
      Sort2Bufs sb;
      sort2_carve(cv, n, g.nbx, wv, &sb);
    } else {
      cv.take<uint32_t>((size_t)n * (2 + nw));
    }
    return cv.off;
  };
  size_t sz = layout(Spread2::kAtomic);
  for (int w = 4; w <= 8; ++w) sz = std::max(sz, layout(spread2_kind(nw, nf, w, n)));
  return sz + 256;
}

template <int W>
static void launch_spread_1d(fk_ctx* ctx, int blocks, size_t lds, const void* X, fk_dtype dt, int64_t n,
                             const void* Y, int nw, int ones, int nf, int fb, double scale, EsDev es, double* grid,
                             int64_t chunk) {
  hipLaunchKernelGGL(k_spread_1d<W>, dim3(blocks), dim3(256), lds, ctx->stream, X, dt, n, Y, nw, ones, nf,
                     fb, scale, es, grid, ctx->flags, chunk);
}

template <int W>
static void launch_spread_3d_binned(fk_ctx* ctx, int blocks, size_t lds, const uint32_t* rec, int nw,
                                    const uint64_t* start, int nbx, int T, int nf, int fb, EsDev es, int slices,
                                    double* grid) {
  hipLaunchKernelGGL(k_spread_3d_binned<W>, dim3(blocks), dim3(256), lds, ctx->stream, rec, nw, start, nbx, T, nf,
                     fb, es, slices, grid);
}

template <int W>
static void launch_spread_3d(fk_ctx* ctx, const void* X, fk_dtype dt, int64_t n, int64_t xstride, const void* Y,
                             int nw, int nf, int fb, double scale, EsDev es, double* grid) {
  const int blocks = (int)std::min<int64_t>(65536, std::max<int64_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_spread_3d<W>, dim3(blocks), dim3(256), 0, ctx->stream, X, dt, n, xstride, Y, nw, nf, fb,
                     scale, es, grid, ctx->flags);
}

template <int W>
static void launch_spread_2d(fk_ctx* ctx, int blocks, size_t lds, const uint32_t* rec, int nw,
                             const uint64_t* start, int nbx, int T, int nf, int fb, EsDev es, int slices,
                             double* grid) {
  hipLaunchKernelGGL(k_spread_2d_binned<W>, dim3(blocks), dim3(256), lds, ctx->stream, rec, nw, 1, start,
                     nbx, T, nf, fb, es, slices, grid);
}

#define FK_W_SWITCH(w, CALL)                         \
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

// Launch shape of the sorted 2-D type-1 stage: the table's entry for this shape, or (when the
// problem is large enough for shapes to matter and the mode allows) coordinate descent over the
// candidates, each run on the call's own data and timed between ev[0] and ev[2].
template <class Run>
static fk_status tune_t1(fk_ctx* ctx, int d, int nf, int W, int nw, int64_t n, bool rows, Run& run, T1Shape* out) {
  T1Shape sh;
  const int mode = tune_mode(ctx);
  if (mode == kTuneOff) {
    *out = sh;
    return FK_OK;
  }
  char key[160];
  std::snprintf(key, sizeof(key), "%s t1 d=%d nf=%d w=%d nw=%d n=2^%d", tune_arch(ctx->device).c_str(), d, nf, W, nw,
                ilog2((int)std::min<int64_t>(n >> 10, 1 << 30)) + 10);
  std::map<std::string, double> v;
  if (mode != kTuneForce && tune_lookup(key, &v)) {
    if (v.count("mb")) sh.mb = (int)v["mb"];
    if (v.count("spread_pts") && v["spread_pts"] >= 256) sh.spread_pts = (int)v["spread_pts"];
    if (v.count("sort_blk") && v["sort_blk"] >= 1 && v["sort_blk"] <= kSortBlkMax) sh.sort_blk = (int)v["sort_blk"];
    if (v.count("sort_slice") && v["sort_slice"] >= kSortSliceMin) sh.sort_slice = (int)v["sort_slice"];
    *out = sh;
    return FK_OK;
  }
  if (n < ((int64_t)1 << 22)) {   // small problems: launch and latency bound, the defaults
    *out = sh;
    return FK_OK;
  }
  // a candidate's time is the better of two runs: the candidates of a knob differ by about as much
  // as one run varies (1-2 % of the stage), and the first run of the stage also pays first touches
  auto time_of = [&](const T1Shape& s, float* ms) -> fk_status {
    *ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      fk_status st = run(s);
      if (st != FK_OK) return st;
      FK_HIP(hipEventSynchronize(ctx->ev[2]));
      float t = 0.f;
      FK_HIP(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[2]));
      *ms = rep == 0 ? t : std::min(*ms, t);
    }
    return FK_OK;
  };
  float best;
  fk_status st = time_of(sh, &best);
  if (st != FK_OK) return st;
  auto knob = [&](int T1Shape::*field, std::initializer_list<int> cands) -> fk_status {
    for (int c : cands) {
      if (sh.*field == c) continue;
      T1Shape t = sh;
      t.*field = c;
      float ms;
      fk_status s = time_of(t, &ms);
      if (s != FK_OK) return s;
      if (ms < best) {
        best = ms;
        sh = t;
      }
    }
    return FK_OK;
  };
  if (rows) {
    sh.mb = spread_mfma_bin(nf, n);
    st = knob(&T1Shape::mb, {2, 4});
    if (st != FK_OK) return st;
  }
  if ((st = knob(&T1Shape::spread_pts, {4096, 8192, 16384, 32768})) != FK_OK) return st;
  if ((st = knob(&T1Shape::sort_blk, {256, 512, 1024})) != FK_OK) return st;
  if ((st = knob(&T1Shape::sort_slice, {32768, 65536, 131072})) != FK_OK) return st;
  std::map<std::string, double> rec{{"spread_pts", sh.spread_pts}, {"sort_blk", sh.sort_blk},
                                    {"sort_slice", sh.sort_slice}};
  if (rows) rec["mb"] = sh.mb;
  tune_store(key, rec, best);
  *out = sh;
  return FK_OK;
}

// out: complex128 [C][(2K+1)^d], C = nw + 1, channel 0 = weight 1.
// out_c[q] = sign_scale * sum_j w_cj exp(-i q.x_j).
fk_status type1(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int64_t xstride, int nw,
                const void* Y, int K, double sign_scale, double* out, Carve& cv, fk_fit_info* info) {
  EsPlan plan;
  const double* phihat;
  fk_status st = get_es_plan(ctx, K, &plan, &phihat);
  if (st != FK_OK) return st;
  const int nf = plan.nf, W = plan.w, logn = ilog2(nf);
  const int fb = 32 - ilog2(nf) - 1;        // fixed-point fraction bits (u < nf <= 2^(31-fb))
  const double scale = (double)nf / (2.0 * kPi) * (double)(1u << fb);
  EsDev es{(float)(plan.beta * 1.44269504088896340736), 2.0f / (float)W};
  const int C = nw + 1;
  const int L = 2 * K + 1;
  if (info) {
    info->w = W;
    info->nf = nf;
    info->beta = plan.beta;
  }
  hipEvent_t* ev = ctx->ev;
  if (d == 1) {
    double* grid = cv.take<double>((size_t)C * nf);
    if (!cv.ok()) return FK_ENOMEM;
    FK_HIP(hipEventRecord(ev[0], ctx->stream));
    FK_HIP(hipMemsetAsync(grid, 0, sizeof(double) * C * nf, ctx->stream));
    int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 4095) / 4096));
    int64_t chunk = (n + blocks - 1) / blocks;
    // channels per launch: as many whole FP64 grids as 160 KB of LDS holds (the ones channel
    // goes with the first launch); the grid is [C][nf], so a launch writes channels ones + c0 ..
    const int per = (int)((160 * 1024) / (sizeof(double) * nf));
    if (per < 2) return FK_EINVAL;
    const size_t esz = dt == FK_F64 ? sizeof(double) : sizeof(float);
    FK_HIP(hipEventRecord(ev[1], ctx->stream));
    for (int c0 = 0, first = 1; first || c0 < nw; first = 0) {
      const int cnt = std::min(per - first, nw - c0);
      const void* Yc = Y ? static_cast<const void*>(static_cast<const char*>(Y) + esz * (size_t)c0 * n) : nullptr;
      double* gc = grid + (size_t)(first ? 0 : 1 + c0) * nf;
      const size_t lds = sizeof(double) * (size_t)(cnt + first) * nf;
      FK_W_SWITCH(W, launch_spread_1d<WW>(ctx, blocks, lds, X, dt, n, Yc, cnt, first, nf, fb, scale, es, gc,
                                          chunk));
      c0 += cnt;
    }
    FK_HIP(hipGetLastError());
    FK_HIP(hipEventRecord(ev[2], ctx->stream));
    hipLaunchKernelGGL(k_fft_line, dim3(C), dim3(256), 0, ctx->stream, grid, 0, (int64_t)1, (int64_t)nf,
                       (int64_t)0, 1, nf, logn, phihat, K, sign_scale, out, (int64_t)1, (int64_t)L, (int64_t)0);
    FK_HIP(hipGetLastError());
    FK_HIP(hipEventRecord(ev[3], ctx->stream));
    if (info) info->bin = 0;
    return FK_OK;
  }
  if (d == 3) {
    // spread, then transforms along axis 2 (C nf^2 lines), axis 1 (C nf L lines) and axis 0
    // (C L^2 lines), each pruned to |q| <= K and deconvolved along its own axis
    const int64_t nf3 = (int64_t)nf * nf * nf;
    double* grid = cv.take<double>((size_t)C * nf3);
    double* ta = cv.take<double>((size_t)C * nf * nf * L * 2);
    double* tb = cv.take<double>((size_t)C * nf * L * L * 2);
    // bins of T^3 window-start cells, T the largest of 8, 4, 2 whose subgrid fits 96 KB of LDS
    int T3 = 0;
    for (int t = 8; t >= 2; t >>= 1) {
      const size_t Sx = (size_t)(t + W - 1);
      if (nf % t == 0 && (size_t)C * Sx * Sx * Sx * sizeof(double) <= 96 * 1024) {
        T3 = t;
        break;
      }
    }
    const int nbx3 = T3 ? nf / T3 : 1;
    const int64_t nb3 = (int64_t)nbx3 * nbx3 * nbx3;
    uint32_t* cnt3 = nullptr;
    uint64_t *start3 = nullptr, *cursor3 = nullptr;
    uint32_t* rec3 = nullptr;
    if (T3) {
      cnt3 = cv.take<uint32_t>((size_t)nb3);
      start3 = cv.take<uint64_t>((size_t)nb3 + 1);
      cursor3 = cv.take<uint64_t>((size_t)nb3);
      rec3 = cv.take<uint32_t>((size_t)n * (3 + nw));
    }
    if (!cv.ok()) return FK_ENOMEM;
    if (info) info->bin = T3;
    FK_HIP(hipEventRecord(ev[0], ctx->stream));
    FK_HIP(hipMemsetAsync(grid, 0, sizeof(double) * C * nf3, ctx->stream));
    const int pblocks = (int)std::min<int64_t>(65536, std::max<int64_t>(1, (n + 255) / 256));
    if (T3) {
      const int tshift = ilog2(T3);
      FK_HIP(hipMemsetAsync(cnt3, 0, sizeof(uint32_t) * nb3, ctx->stream));
      hipLaunchKernelGGL(k_bin3_count, dim3(pblocks), dim3(256), 0, ctx->stream, X, dt, n, xstride, nf, fb, scale, W,
                         tshift, nbx3, cnt3, ctx->flags);
      hipLaunchKernelGGL(k_bin3_scan, dim3(1), dim3(1024), 0, ctx->stream, cnt3, (int)nb3, start3, cursor3);
      hipLaunchKernelGGL(k_bin3_scatter, dim3(pblocks), dim3(256), 0, ctx->stream, X, dt, n, xstride, Y, nw, nf, fb,
                         scale, W, tshift, nbx3, reinterpret_cast<unsigned long long*>(cursor3), rec3, ctx->flags);
      FK_HIP(hipGetLastError());
    }
    FK_HIP(hipEventRecord(ev[1], ctx->stream));
    if (T3) {
      const int64_t per_bin = (n + nb3 - 1) / nb3;
      const int slices = (int)std::max<int64_t>(1, std::min<int64_t>(256, (per_bin + 2047) / 2048));
      const int S = T3 + W - 1;
      const size_t lds = sizeof(double) * C * S * S * S;
      const int64_t blocks = nb3 * slices;
      if (blocks > 0x7fffffff) return FK_EINVAL;
      FK_W_SWITCH(W, launch_spread_3d_binned<WW>(ctx, (int)blocks, lds, rec3, nw, start3, nbx3, T3, nf, fb, es, slices,
                                                 grid));
    } else {
      FK_W_SWITCH(W, launch_spread_3d<WW>(ctx, X, dt, n, xstride, Y, nw, nf, fb, scale, es, grid));
    }
    FK_HIP(hipGetLastError());
    FK_HIP(hipEventRecord(ev[2], ctx->stream));
    hipLaunchKernelGGL(k_fft_line, dim3(C * nf * nf), dim3(256), 0, ctx->stream, grid, 0, (int64_t)1, (int64_t)nf,
                       (int64_t)0, 1, nf, logn, phihat, K, 1.0, ta, (int64_t)1, (int64_t)L, (int64_t)0);
    hipLaunchKernelGGL(k_fft_line, dim3(C * nf * L), dim3(256), 0, ctx->stream, ta, 1, (int64_t)L,
                       (int64_t)nf * L, (int64_t)1, L, nf, logn, phihat, K, 1.0, tb, (int64_t)L, (int64_t)L * L,
                       (int64_t)1);
    hipLaunchKernelGGL(k_fft_line, dim3(C * L * L), dim3(256), 0, ctx->stream, tb, 1, (int64_t)L * L,
                       (int64_t)nf * L * L, (int64_t)1, L * L, nf, logn, phihat, K, sign_scale, out,
                       (int64_t)L * L, (int64_t)L * L * L, (int64_t)1);
    FK_HIP(hipGetLastError());
    FK_HIP(hipEventRecord(ev[3], ctx->stream));
    return FK_OK;
  }
  if (d != 2) return FK_EINVAL;
  double* grid = cv.take<double>((size_t)C * nf * nf);
  double* rowfft = cv.take<double>((size_t)C * nf * L * 2);
  const Spread2 kind = spread2_kind(nw, nf, W, n);
  const bool split = kind != Spread2::kAtomic;   // two-pass sort, then an MFMA spread
  const int wv = sort2_words(nw);
  BinGeom gmax = bin_geom(nf, C, n, kind);
  if (kind == Spread2::kRows) {
    const BinGeom g2 = bin_geom(nf, C, n, kind, 2);
    if (g2.nb > gmax.nb) gmax = g2;
  }
  uint32_t* cnt = cv.take<uint32_t>((size_t)gmax.nb * gmax.nblk);
  uint32_t* totals = cv.take<uint32_t>((size_t)gmax.nb);
  uint64_t* start = cv.take<uint64_t>((size_t)gmax.nb + 1);
  uint32_t* rec = cv.take<uint32_t>((size_t)n * (split ? 2 : 2 + nw));
  // second sorted array: weight words (outer-product spread) or, for the channel-row
  // spread, each point's position in the row-grouped weight blocks sb.wts1
  uint32_t* wts = split ? cv.take<uint32_t>((size_t)n * (kind == Spread2::kRows ? 1 : wv)) : nullptr;
  Sort2Bufs sb;
  if (split) sort2_carve(cv, n, gmax.nbx, wv, &sb);
  if (!cv.ok()) return FK_ENOMEM;
  // The binning and the spread for one launch shape, between events ev[0] .. ev[2].
  auto run = [&](const T1Shape& sh) -> fk_status {
    const BinGeom g = bin_geom(nf, C, n, kind, sh.mb);
    if (info) info->bin = g.T;
    FK_HIP(hipEventRecord(ev[0], ctx->stream));
    FK_HIP(hipMemsetAsync(grid, 0, sizeof(double) * C * nf * nf, ctx->stream));
    if (split) {
      // records for the MFMA spreads: two-pass sort, coordinates and weight words
      fk_status s2 = sort2(ctx->stream, X, dt, n, xstride, Y, nw, nf, fb, W, scale, g.tshift, g.nbx, sh, sb, rec, wts,
                           start, ctx->flags);
      if (s2 != FK_OK) return s2;
    } else {
      hipLaunchKernelGGL(k_bin_count, dim3(g.nblk), dim3(256), sizeof(uint32_t) * g.nb, ctx->stream, X, dt, n,
                         xstride, nf, fb, scale, g.tshift, g.nbx, cnt, g.nblk, g.chunk, ctx->flags);
      FK_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_scan_cols, dim3((g.nb + 255) / 256), dim3(256), 0, ctx->stream, cnt, g.nb, g.nblk,
                         totals);
      hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, ctx->stream, totals, g.nb, start);
      hipLaunchKernelGGL(k_bin_scatter, dim3(g.nblk), dim3(1024), sizeof(unsigned long long) * g.nb, ctx->stream, X,
                         dt, n, xstride, Y, nw, nf, fb, scale, g.tshift, g.nbx, cnt, start, g.chunk, rec,
                         ctx->flags);
    }
    FK_HIP(hipGetLastError());
    FK_HIP(hipEventRecord(ev[1], ctx->stream));
    int64_t per_bin = (n + g.nb - 1) / g.nb;
    if (kind == Spread2::kRows) {
      fk_status s2 = launch_spread_mfma(ctx->stream, W, g.T, rec, wts, sb.wts1, nw, start, g.nbx, g.nb, nf, fb,
                                        plan.beta, n, sh.spread_pts, grid);
      if (s2 != FK_OK) return s2;
      if (info) info->bin = -g.T;   // negative: MFMA spread over T x T bins
    } else if (kind == Spread2::kOuter) {
      fk_status s2 = launch_spread_op(ctx->stream, W, rec, wts, nw, start, g.nbx, g.nb, nf, fb, plan.beta, n,
                                      sh.spread_pts, grid);
      if (s2 != FK_OK) return s2;
      if (info) info->bin = -g.T;
    } else {
      const int H = (W + 1) / 2;
      const int S = g.T + 2 * H;
      size_t lds = sizeof(double) * S * S * C;
      if (lds > 160 * 1024) return FK_EINVAL;
      int slices = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (per_bin + 8191) / 8192));
      int blocks = g.nb * slices;
      FK_W_SWITCH(W, launch_spread_2d<WW>(ctx, blocks, lds, rec, nw, start, g.nbx, g.T, nf, fb, es, slices, grid));
    }
    FK_HIP(hipGetLastError());
    FK_HIP(hipEventRecord(ev[2], ctx->stream));
    return FK_OK;
  };
  T1Shape shape;
  if (split) {
    fk_status s2 = tune_t1(ctx, d, nf, W, nw, n, kind == Spread2::kRows, run, &shape);
    if (s2 != FK_OK) return s2;
  }
  st = run(shape);
  if (st != FK_OK) return st;
  // rows: lines along dim 2 (contiguous), C*nf lines -> rowfft[c][i1][q2]
  hipLaunchKernelGGL(k_fft_line, dim3(C * nf), dim3(256), 0, ctx->stream, grid, 0, (int64_t)1, (int64_t)nf,
                     (int64_t)0, 1, nf, logn, phihat, K, 1.0, rowfft, (int64_t)1, (int64_t)L, (int64_t)0);
  // columns: for each (c, q2) the line along i1 with stride L (complex)
  hipLaunchKernelGGL(k_fft_line, dim3(C * L), dim3(256), 0, ctx->stream, rowfft, 1, (int64_t)L,
                     (int64_t)nf * L, (int64_t)1, L, nf, logn, phihat, K, sign_scale, out, (int64_t)L,
                     (int64_t)L * L, (int64_t)1);
  FK_HIP(hipGetLastError());
  FK_HIP(hipEventRecord(ev[3], ctx->stream));
  return FK_OK;
}

}  // namespace fk
