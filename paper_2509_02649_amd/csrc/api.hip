// C ABI entry points of libfastkernel (declared in include/fk.h).
#include "fk_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

namespace fk {
// dense.hip kernels (same library, separate translation unit)
struct ToeplitzQ;
}

using namespace fk;

// ------------------------------------------------------------------ context

extern "C" fk_status fk_create(fk_ctx** ctx, int device, void* hip_stream) {
  if (!ctx) return FK_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FK_EINVAL;
  FK_HIP(hipSetDevice(device));
  fk_ctx* c = new fk_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->opt.eps = 2e-7;
  c->opt.max_refine = 8;
  c->opt.refine_tol = 1e-10;
  if (hipMalloc(&c->flags, sizeof(int) * kFlagCount) != hipSuccess ||
      hipHostMalloc(&c->flags_host, sizeof(int) * 2 * kFlagCount, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return FK_EHIP;
  }
  for (auto& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) return FK_EHIP;
  // the allocation-free prediction's device array, resolved once per device
  fk_status st = scratch_init(device);
  if (st != FK_OK) {
    fk_destroy(c);
    return st;
  }
  *ctx = c;
  return FK_OK;
}

extern "C" fk_status fk_destroy(fk_ctx* ctx) {
  if (!ctx) return FK_EINVAL;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->es_cache) hipFree(kv.second.second);
  if (ctx->aux_stream) {
    hipStreamSynchronize(ctx->aux_stream);
    hipStreamDestroy(ctx->aux_stream);
    for (auto& e : ctx->aux_ev) hipEventDestroy(e);
  }
  hipFree(ctx->flags);
  hipHostFree(ctx->flags_host);
  if (ctx->stage) hipHostFree(ctx->stage);
  for (auto& e : ctx->ev) hipEventDestroy(e);
  delete ctx;
  return FK_OK;
}

extern "C" fk_status fk_set_stream(fk_ctx* ctx, void* s) {
  if (!ctx) return FK_EINVAL;
  ctx->stream = static_cast<hipStream_t>(s);
  return FK_OK;
}

extern "C" fk_status fk_set_options(fk_ctx* ctx, const fk_options* o) {
  if (!ctx || !o) return FK_EINVAL;
  fk_options v = *o;
  if (v.eps <= 0) v.eps = 2e-7;
  if (v.eps < 1e-14 || v.eps > 1e-2) return FK_EINVAL;
  if (v.max_refine < 0 || v.max_refine > 100) return FK_EINVAL;
  if (v.refine_tol <= 0) v.refine_tol = 1e-10;
  ctx->opt = v;
  return FK_OK;
}

extern "C" const char* fk_status_string(fk_status s) {
  switch (s) {
    case FK_OK: return "ok";
    case FK_EINVAL: return "invalid argument";
    case FK_ERANGE: return "coordinate outside [-2pi, 2pi)";
    case FK_ENAN: return "NaN or Inf in the input";
    case FK_ENOTPD: return "system matrix not positive definite in FP32";
    case FK_ENOCONV: return "iterative refinement did not converge";
    case FK_ENOMEM: return "workspace too small";
    case FK_EHIP: return "HIP runtime error";
  }
  return "unknown status";
}

namespace fk {

fk_status reset_flags(fk_ctx* ctx) {
  int init[kFlagCount] = {0, 0, 0, 0x7fffffff, 0, 0x7fffffff, 0, 0};
  std::memcpy(ctx->flags_host, init, sizeof(init));
  FK_HIP(hipMemcpyAsync(ctx->flags, ctx->flags_host, sizeof(init), hipMemcpyHostToDevice, ctx->stream));
  return FK_OK;
}

void* stage_take(fk_ctx* ctx, size_t bytes) {
  bytes = (bytes + 15) & ~size_t(15);
  if (ctx->stage_off + bytes > ctx->stage_cap) {
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return nullptr;
    ctx->stage_off = 0;
    if (bytes > ctx->stage_cap) {
      const size_t cap = std::max(bytes, (size_t)4 << 20);
      if (ctx->stage) hipHostFree(ctx->stage);
      ctx->stage = nullptr;
      ctx->stage_cap = 0;
      void* p = nullptr;
      if (hipHostMalloc(&p, cap, hipHostMallocDefault) != hipSuccess) return nullptr;
      ctx->stage = static_cast<char*>(p);
      ctx->stage_cap = cap;
    }
  }
  void* p = ctx->stage + ctx->stage_off;
  ctx->stage_off += bytes;
  return p;
}

fk_status stage_upload(fk_ctx* ctx, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return FK_OK;
  void* h = stage_take(ctx, bytes);
  if (!h) return FK_EHIP;
  std::memcpy(h, src, bytes);
  FK_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, ctx->stream));
  return FK_OK;
}

fk_status read_flags(fk_ctx* ctx) {
  FK_HIP(hipMemcpyAsync(ctx->flags_host, ctx->flags, sizeof(int) * kFlagCount, hipMemcpyDeviceToHost,
                        ctx->stream));
  FK_HIP(hipStreamSynchronize(ctx->stream));
  return flag_status(ctx);
}

fk_status flag_status(const fk_ctx* ctx) {
  if (ctx->flags_host[kFlagNaN]) return FK_ENAN;
  if (ctx->flags_host[kFlagRange]) return FK_ERANGE;
  if (ctx->flags_host[kFlagNotPD]) return FK_ENOTPD;
  return FK_OK;
}

static float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.f;
  return ms;
}

// extraction of M and b from the type-1 output (complex [C][(2K+1)^d], K = 2m)
__global__ void k_extract_gram(const double* __restrict__ c, int d, int m, int ntgt, double* __restrict__ M,
                               double* __restrict__ b) {
  const int K = 2 * m, LK = 2 * K + 1, L = 2 * m + 1;
  const int totK = d == 1 ? LK : (d == 2 ? LK * LK : LK * LK * LK);
  const int totN = d == 1 ? L : (d == 2 ? L * L : L * L * L);
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.y == 0) {
    if (i >= totK) return;
    // M[q] = c_0[-q]: reversal of the flattened index
    int j = totK - 1 - i;
    M[2 * i] = c[2 * j];
    M[2 * i + 1] = c[2 * j + 1];
    return;
  }
  const int t = blockIdx.y - 1;
  if (i >= totN) return;
  int src;
  if (d == 1) {
    src = i + m;
  } else if (d == 2) {
    int k1 = i / L, k2 = i - k1 * L;
    src = (k1 + m) * LK + (k2 + m);
  } else {
    int k1 = i / (L * L), r = i - k1 * L * L, k2 = r / L, k3 = r - k2 * L;
    src = ((k1 + m) * LK + (k2 + m)) * LK + (k3 + m);
  }
  const double* ct = c + 2 * (size_t)(t + 1) * totK;
  b[2 * ((size_t)t * totN + i)] = ct[2 * src];
  b[2 * ((size_t)t * totN + i) + 1] = ct[2 * src + 1];
}

// Centred sub-block of `count` row-major d-dimensional arrays: out[c][i] = in[c][i + off] per
// coordinate, off = (Lin - Lout) / 2 (the frequencies |q| <= (Lout - 1) / 2 of a larger set).
__global__ void k_restrict(const double2* __restrict__ in, int d, int Lin, int Lout, int64_t tot_out, int count,
                           double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tot_out * count) return;
  const int64_t c = e / tot_out;
  int64_t rem = e - c * tot_out, src = 0, mul = 1, tot_in = 1;
  const int off = (Lin - Lout) / 2;
  for (int a = 0; a < d; ++a) {
    const int64_t j = rem % Lout;
    rem /= Lout;
    src += (j + off) * mul;
    mul *= Lin;
  }
  for (int a = 0; a < d; ++a) tot_in *= Lin;
  out[e] = in[c * tot_in + src];
}

}  // namespace fk

// ------------------------------------------------------------------ kept factors
// A workspace holding the factors and solutions of a solve stays registered until any library
// call writes a workspace that overlaps it; fk_heldout_mse / fk_fit_backward look it up.
namespace fk {
namespace {
struct KeptEntry {
  uintptr_t base;
  size_t bytes;
  int device, kind, d, m, N, nlam, ntgt, stage;
};
std::mutex g_kept_mu;
std::vector<KeptEntry> g_kept;
}  // namespace

void kept_invalidate(const void* ws, size_t bytes) {
  if (!ws) return;
  const uintptr_t a = reinterpret_cast<uintptr_t>(ws), b = a + bytes;
  std::lock_guard<std::mutex> lk(g_kept_mu);
  g_kept.erase(std::remove_if(g_kept.begin(), g_kept.end(),
                              [&](const KeptEntry& e) { return e.base < b && a < e.base + e.bytes; }),
               g_kept.end());
}

void kept_register(const void* ws, size_t bytes, int device, int kind, int d, int m, int N, int nlam, int ntgt,
                   int stage) {
  kept_invalidate(ws, bytes);
  std::lock_guard<std::mutex> lk(g_kept_mu);
  g_kept.push_back({reinterpret_cast<uintptr_t>(ws), bytes, device, kind, d, m, N, nlam, ntgt, stage});
}

bool kept_find(const void* ws, int device, int kind, int d, int m, int N, int nlam, int ntgt, int min_stage) {
  std::lock_guard<std::mutex> lk(g_kept_mu);
  for (const KeptEntry& e : g_kept)
    if (e.base == reinterpret_cast<uintptr_t>(ws) && e.device == device && e.kind == kind && e.d == d && e.m == m &&
        e.N == N && e.nlam == nlam && e.ntgt == ntgt && e.stage >= min_stage)
      return true;
  return false;
}
}  // namespace fk

// ------------------------------------------------------------------ fk_gram

static int64_t ipow(int64_t a, int d) {
  int64_t r = 1;
  while (d-- > 0) r *= a;
  return r;
}

static size_t gram_ws(int d, int64_t n, int ntgt, int m) {
  const int K = 2 * m;
  const int LK = 2 * K + 1;
  const int64_t tot = ipow(LK, d);
  Carve cv(nullptr, 0);
  cv.take<double>((size_t)2 * (ntgt + 1) * tot);
  return cv.off + type1_workspace(d, n, ntgt, K, 0) + 512;
}

static fk_status check_gram_args(int d, int64_t n, int ntgt, int m, const void* X, const void* Y) {
  if (d < 1 || d > 3) return FK_EINVAL;
  if (n < 1 || m < 1 || m > 64 || ntgt < 0 || ntgt > 32) return FK_EINVAL;
  if (d == 3 && (m > 31 || ntgt > 8)) return FK_EINVAL;   // FP64 grid 256^3 per channel
  if (!X || (ntgt > 0 && !Y)) return FK_EINVAL;
  if (d == 2 && n > (int64_t)1 << 34) return FK_EINVAL;
  return FK_OK;
}

extern "C" fk_status fk_gram_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m, size_t* bytes) {
  if (!bytes) return FK_EINVAL;
  if (check_gram_args(d, n, ntgt, m, (void*)1, (void*)1) != FK_OK) return FK_EINVAL;
  *bytes = gram_ws(d, n, ntgt, m);
  return FK_OK;
}

namespace fk {
fk_status gram_impl(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int ntgt, const void* Y, int m,
                    double* M_out, double* b_out, Carve& cv, fk_fit_info* info) {
  const int K = 2 * m;
  const int LK = 2 * K + 1;
  const int64_t tot = ipow(LK, d);
  double* c = cv.take<double>((size_t)2 * (ntgt + 1) * tot);
  if (!cv.ok()) return FK_ENOMEM;
  fk_status st = type1(ctx, d, n, dt, X, n, ntgt, Y, K, 1.0 / (double)n, c, cv, info);
  if (st != FK_OK) return st;
  const int64_t totN = ipow(2 * m + 1, d);
  int mx = (int)std::max<int64_t>(tot, totN);
  hipLaunchKernelGGL(k_extract_gram, dim3((mx + 255) / 256, ntgt + 1), dim3(256), 0, ctx->stream, c, d, m, ntgt,
                     M_out, b_out);
  FK_HIP(hipGetLastError());
  FK_HIP(hipEventRecord(ctx->ev[4], ctx->stream));
  return FK_OK;
}
}  // namespace fk

extern "C" fk_status fk_gram(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int ntgt, const void* Y,
                             int m, double* M_out, double* b_out, void* ws, size_t ws_bytes, fk_fit_info* info) {
  if (!ctx) return FK_EINVAL;
  if (check_gram_args(d, n, ntgt, m, X, Y) != FK_OK || !M_out || (ntgt > 0 && !b_out)) return FK_EINVAL;
  if (dt != FK_F32 && dt != FK_F64) return FK_EINVAL;
  if (ws_bytes < gram_ws(d, n, ntgt, m) || !ws) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  kept_invalidate(ws, ws_bytes);
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->bad_index = -1;
  }
  Carve cv(ws, ws_bytes);
  fk_status st = reset_flags(ctx);
  if (st == FK_OK) st = gram_impl(ctx, d, n, dt, X, ntgt, Y, m, M_out, b_out, cv, info);
  if (st != FK_OK) return st;
  st = read_flags(ctx);
  if (info) {
    info->status = st;
    info->t_sort_ms = elapsed(ctx->ev[0], ctx->ev[1]);
    info->t_spread_ms = elapsed(ctx->ev[1], ctx->ev[2]);
    info->spread_kernel_ms = info->t_spread_ms;
    info->t_fft_ms = elapsed(ctx->ev[2], ctx->ev[4]);
    info->t_total_ms = elapsed(ctx->ev[0], ctx->ev[4]);
  }
  return st;
}

// ------------------------------------------------------------------ fk_solve / fk_fit


static fk_status penalty_weights(const fk_penalty* pen, int d, int m, std::vector<double>& p) {
  const int L = 2 * m + 1;
  const int64_t N = ipow(L, d);
  p.assign(N, 1.0);
  const int kind = pen ? pen->kind : FK_PEN_SOBOLEV;
  const double s = pen ? pen->s : 1.0;
  for (int64_t i = 0; i < N; ++i) {
    int64_t ii = i;
    double r2 = 0.0;
    for (int a = 0; a < d; ++a) {
      int k = (int)(ii % L) - m;
      ii /= L;
      r2 += (double)k * k;
    }
    switch (kind) {
      case FK_PEN_SOBOLEV: p[i] = 1.0 + std::pow(r2, s); break;
      case FK_PEN_SOBOLEV_BESSEL: p[i] = std::pow(1.0 + r2, s); break;
      case FK_PEN_IDENTITY: p[i] = 1.0; break;
      case FK_PEN_DIAG:
        if (!pen->p) return FK_EINVAL;
        p[i] = pen->p[i];
        break;
      case FK_PEN_HEAT_BOX: p[i] = 1.0 + r2; break;
      case FK_PEN_PDE_BOX: p[i] = 1.0 + std::pow(r2, s); break;
      default: return FK_EINVAL;
    }
    if (!(p[i] > 0.0) || std::isinf(p[i])) return FK_EINVAL;
  }
  if (kind == FK_PEN_DIAG)
    for (int64_t i = 0; i < N; ++i)
      if (p[i] != p[N - 1 - i]) return FK_EINVAL;   // p_{-k} = p_k required for the real form
  if (kind == FK_PEN_SOBOLEV || kind == FK_PEN_SOBOLEV_BESSEL || kind == FK_PEN_PDE_BOX)
    if (!(s >= 0.0) || s > 64) return FK_EINVAL;
  return FK_OK;
}

// Operator symbol D_k = sum_t coef[t] prod_a (i k_a)^alpha[t][a] (Sec. 4: the derivative of exp(i k.x)
// along axis a is i k_a exp(i k.x)), complex interleaved over the N modes.  The heat box is the
// operator d_t - d_xx.
static fk_status pde_symbol(const fk_penalty* pen, int d, int m, std::vector<double>& D) {
  static const int heat_alpha[4] = {1, 0, 0, 2};
  static const double heat_coef[2] = {1.0, -1.0};
  const bool heat = pen->kind == FK_PEN_HEAT_BOX;
  const int nt = heat ? 2 : pen->nterms;
  const int* alpha = heat ? heat_alpha : pen->alpha;
  const double* coef = heat ? heat_coef : pen->coef;
  if (nt < 1 || nt > 16 || !alpha || !coef) return FK_EINVAL;
  for (int t = 0; t < nt; ++t) {
    if (!std::isfinite(coef[t])) return FK_EINVAL;
    for (int a = 0; a < d; ++a)
      if (alpha[t * d + a] < 0 || alpha[t * d + a] > 8) return FK_EINVAL;
  }
  const int L = 2 * m + 1;
  const int64_t N = ipow(L, d);
  D.assign(2 * N, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    int k[2] = {0, 0};
    int64_t ii = i;
    for (int a = d - 1; a >= 0; --a) {
      k[a] = (int)(ii % L) - m;
      ii /= L;
    }
    double re = 0.0, im = 0.0;
    for (int t = 0; t < nt; ++t) {
      double tr = coef[t], ti = 0.0;   // coef * prod_a (i k_a)^alpha
      for (int a = 0; a < d; ++a)
        for (int e = 0; e < alpha[t * d + a]; ++e) {   // multiply by i k_a
          const double nr = -ti * k[a], ni = tr * k[a];
          tr = nr;
          ti = ni;
        }
      re += tr;
      im += ti;
    }
    D[2 * i] = re;
    D[2 * i + 1] = im;
  }
  return FK_OK;
}

static fk_status build_problem(int d, int m, const double* M, const double* b, const double* lambdas, int nlam,
                               const fk_penalty* pen, SolveProblem& P) {
  if ((d != 1 && d != 2) || m < 1 || m > 64 || nlam < 1 || nlam > 1024 || !lambdas) return FK_EINVAL;
  P.kind = SolveProblem::kToeplitz;
  if (pen && (pen->kind == FK_PEN_HEAT_BOX || pen->kind == FK_PEN_PDE_BOX)) {
    if ((pen->kind == FK_PEN_HEAT_BOX && d != 2) || !(pen->mu >= 0.0) || std::isinf(pen->mu)) return FK_EINVAL;
    P.kind = SolveProblem::kToeplitzPde;
    P.mu = pen->mu;
    for (int a = 0; a < d; ++a) {
      P.lo[a] = pen->box_lo[a];
      P.hi[a] = pen->box_hi[a];
      if (!(P.hi[a] > P.lo[a]) || std::isinf(P.hi[a]) || std::isinf(P.lo[a])) return FK_EINVAL;
    }
    fk_status st = pde_symbol(pen, d, m, P.dsym);
    if (st != FK_OK) return st;
  }
  P.M = M;
  P.b = b;
  P.m = m;
  P.d = d;
  P.L = (int)ipow(2 * m + 1, d);
  fk_status st = penalty_weights(pen, d, m, P.p);
  if (st != FK_OK) return st;
  P.lams.assign(lambdas, lambdas + nlam);
  for (double l : P.lams)
    if (!(l > 0.0) || std::isinf(l)) return FK_EINVAL;
  return FK_OK;
}

extern "C" fk_status fk_solve_workspace_size(fk_ctx* ctx, int d, int m, int ntgt, int nlam, size_t* bytes) {
  if (!bytes || (d != 1 && d != 2) || m < 1 || m > 64 || ntgt < 1 || ntgt > 32 || nlam < 1 || nlam > 1024)
    return FK_EINVAL;
  *bytes = solve_layout((int)ipow(2 * m + 1, d), nlam, ntgt, nullptr, 0).bytes;
  return FK_OK;
}

extern "C" fk_status fk_solve(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                              const double* lambdas, int nlam, const fk_penalty* pen, double* theta_out, void* ws,
                              size_t ws_bytes, fk_fit_info* info) {
  if (!ctx || !M || !b || !theta_out || ntgt < 1 || ntgt > 32) return FK_EINVAL;
  SolveProblem P;
  fk_status st = build_problem(d, m, M, b, lambdas, nlam, pen, P);
  if (st != FK_OK) return st;
  SolveLayout s = solve_layout(P.L, nlam, ntgt, ws, ws_bytes);
  if (!ws || s.bytes > ws_bytes) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  kept_invalidate(ws, ws_bytes);
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->bad_index = -1;
  }
  st = reset_flags(ctx);
  if (st == FK_OK) st = solve_impl(ctx, P, s, theta_out, info);
  if (st == FK_OK || st == FK_ENOCONV)
    kept_register(ws, s.bytes, ctx->device, kKeptToeplitz, d, m, P.L, nlam, ntgt, 1);
  if (info) info->status = st;
  return st;
}

// ---------------------------------------------------------------- restriction to a smaller m

extern "C" fk_status fk_restrict(fk_ctx* ctx, int d, int m_from, int m_to, int ntgt, const double* M_in,
                                 const double* b_in, double* M_out, double* b_out) {
  if (!ctx || d < 1 || d > 3 || m_to < 1 || m_to > m_from || m_from > 255 || ntgt < 0 || ntgt > 65536)
    return FK_EINVAL;
  if (!M_in || !M_out || (ntgt > 0 && (!b_in || !b_out))) return FK_EINVAL;
  FK_HIP(hipSetDevice(ctx->device));
  const int64_t totM = ipow(4 * m_to + 1, d), totB = ipow(2 * m_to + 1, d);
  hipLaunchKernelGGL(k_restrict, dim3((unsigned)((totM + 255) / 256)), dim3(256), 0, ctx->stream,
                     reinterpret_cast<const double2*>(M_in), d, 4 * m_from + 1, 4 * m_to + 1, totM, 1,
                     reinterpret_cast<double2*>(M_out));
  if (ntgt > 0)
    hipLaunchKernelGGL(k_restrict, dim3((unsigned)((totB * ntgt + 255) / 256)), dim3(256), 0, ctx->stream,
                       reinterpret_cast<const double2*>(b_in), d, 2 * m_from + 1, 2 * m_to + 1, totB, ntgt,
                       reinterpret_cast<double2*>(b_out));
  FK_HIP(hipGetLastError());
  FK_HIP(hipStreamSynchronize(ctx->stream));
  return FK_OK;
}

// ---------------------------------------------------------------- iterative solve

extern "C" fk_status fk_toeplitz_apply_workspace_size(fk_ctx* ctx, int d, int m, int nvec, size_t* bytes) {
  if (!bytes || !toeplitz_fft_ok(d, m) || nvec < 1) return FK_EINVAL;
  *bytes = toeplitz_apply_workspace(d, m, nvec);
  return FK_OK;
}

extern "C" fk_status fk_toeplitz_apply(fk_ctx* ctx, int d, int m, const double* M, int nvec, const double* x,
                                       double* y, void* ws, size_t ws_bytes) {
  if (!ctx || !M || !x || !y || !toeplitz_fft_ok(d, m) || nvec < 1) return FK_EINVAL;
  if (!ws || ws_bytes < toeplitz_apply_workspace(d, m, nvec)) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  kept_invalidate(ws, ws_bytes);
  Carve cv(ws, ws_bytes);
  return toeplitz_apply_impl(ctx, d, m, M, nvec, x, y, cv);
}

static bool cg_shape_ok(int d, int m, int ntgt, int nlam) {
  return toeplitz_fft_ok(d, m) && ntgt >= 1 && nlam >= 1 && nlam <= 1024 && (int64_t)ntgt * nlam <= 65536;
}

extern "C" fk_status fk_solve_cg_workspace_size(fk_ctx* ctx, int d, int m, int ntgt, int nlam, size_t* bytes) {
  if (!bytes || !cg_shape_ok(d, m, ntgt, nlam)) return FK_EINVAL;
  *bytes = cg_workspace(d, m, ntgt * nlam, nlam, false);
  return FK_OK;
}

extern "C" fk_status fk_solve_cg_collocation_workspace_size(fk_ctx* ctx, int d, int m, int ntgt, int nlam,
                                                            size_t* bytes) {
  if (!bytes || !cg_shape_ok(d, m, ntgt, nlam)) return FK_EINVAL;
  *bytes = cg_workspace(d, m, ntgt * nlam, nlam, true);
  return FK_OK;
}

static fk_status cg_common(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                           const double* lambdas, int nlam, const fk_penalty* pen, double mu, const double* Mr,
                           const double* Dsym, double tol, int maxit, double* theta_out, int* iters,
                           double* relres, void* ws, size_t ws_bytes) {
  if (!ctx || !M || !b || !theta_out || !lambdas || !cg_shape_ok(d, m, ntgt, nlam)) return FK_EINVAL;
  if (!(tol > 0.0) || !(tol < 1.0) || maxit < 1 || maxit > 1000000) return FK_EINVAL;
  if (pen && (pen->kind == FK_PEN_HEAT_BOX || pen->kind == FK_PEN_PDE_BOX)) return FK_EINVAL;   // dense: fk_solve
  std::vector<double> pw;
  fk_status st = penalty_weights(pen, d, m, pw);
  if (st != FK_OK) return st;
  std::vector<double> lams(lambdas, lambdas + nlam);
  for (double l : lams)
    if (!(l > 0.0) || std::isinf(l)) return FK_EINVAL;
  if (!ws || ws_bytes < cg_workspace(d, m, ntgt * nlam, nlam, Mr != nullptr)) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  kept_invalidate(ws, ws_bytes);
  st = reset_flags(ctx);
  if (st != FK_OK) return st;
  Carve cv(ws, ws_bytes);
  return cg_solve_impl(ctx, d, m, M, ntgt, b, lams, pw, mu, Mr, Dsym, tol, maxit, theta_out, iters, relres, cv);
}

extern "C" fk_status fk_solve_cg(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                                 const double* lambdas, int nlam, const fk_penalty* pen, double tol, int maxit,
                                 double* theta_out, int* iters, double* relres, void* ws, size_t ws_bytes) {
  return cg_common(ctx, d, m, M, ntgt, b, lambdas, nlam, pen, 0.0, nullptr, nullptr, tol, maxit, theta_out, iters,
                   relres, ws, ws_bytes);
}

extern "C" fk_status fk_solve_cg_collocation(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                                             const double* lambdas, int nlam, const fk_penalty* pen, double mu,
                                             const double* Mr, const double* Dsym, double tol, int maxit,
                                             double* theta_out, int* iters, double* relres, void* ws,
                                             size_t ws_bytes) {
  if (!Mr || !Dsym || !(mu >= 0.0) || std::isinf(mu)) return FK_EINVAL;
  return cg_common(ctx, d, m, M, ntgt, b, lambdas, nlam, pen, mu, Mr, Dsym, tol, maxit, theta_out, iters, relres, ws,
                   ws_bytes);
}

static size_t fit_scratch(int d, int64_t n, int ntgt, int m);
static size_t fit_ws(int d, int64_t n, int ntgt, int m, int nlam) {
  const int64_t N = ipow(2 * m + 1, d);
  return solve_layout((int)N, nlam, ntgt, nullptr, 0).bytes + fit_scratch(d, n, ntgt, m);
}

extern "C" fk_status fk_fit_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m, int nlam,
                                           size_t* bytes) {
  if (!bytes) return FK_EINVAL;
  if (check_gram_args(d, n, ntgt, m, (void*)1, (void*)1) != FK_OK || ntgt < 1 || nlam < 1 || nlam > 1024 || d > 2)
    return FK_EINVAL;
  *bytes = fit_ws(d, n, ntgt, m, nlam);
  return FK_OK;
}

// The type-1 stage's part of a fit: M, b and the stage's scratch.
static size_t fit_scratch(int d, int64_t n, int ntgt, int m) {
  const int64_t N = ipow(2 * m + 1, d);
  Carve cv(nullptr, 0);
  cv.take<double>((size_t)2 * ipow(4 * m + 1, d));
  cv.take<double>((size_t)2 * ntgt * N);
  return cv.off + gram_ws(d, n, ntgt, m) + 1024;
}

// fk_fit with the solve's layout (factors, FP64 Gram, solutions: what the gradients read) in wss and
// the type-1 stage (M, b and its scratch) in wst.
static fk_status fit_impl(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int ntgt, const void* Y, int m,
                          const double* lambdas, int nlam, const fk_penalty* pen, double* theta_out, void* wss,
                          size_t wss_bytes, void* wst, size_t wst_bytes, fk_fit_info* info) {
  if (!ctx || !theta_out) return FK_EINVAL;
  if (check_gram_args(d, n, ntgt, m, X, Y) != FK_OK || ntgt < 1) return FK_EINVAL;
  if (dt != FK_F32 && dt != FK_F64) return FK_EINVAL;
  SolveProblem P;
  fk_status st = build_problem(d, m, nullptr, nullptr, lambdas, nlam, pen, P);
  if (st != FK_OK) return st;
  if (!wss || !wst) return FK_ENOMEM;
  SolveLayout s = solve_layout(P.L, nlam, ntgt, wss, wss_bytes);
  if (s.bytes > wss_bytes || wst_bytes < fit_scratch(d, n, ntgt, m)) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  kept_invalidate(wss, wss_bytes);
  kept_invalidate(wst, wst_bytes);
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->bad_index = -1;
  }
  Carve cv(wst, wst_bytes);
  double* M = cv.take<double>((size_t)2 * ipow(4 * m + 1, d));
  double* b = cv.take<double>((size_t)2 * ntgt * P.L);
  P.M = M;
  P.b = b;
  st = reset_flags(ctx);
  if (st == FK_OK) st = gram_impl(ctx, d, n, dt, X, ntgt, Y, m, M, b, cv, info);
  if (st != FK_OK) return st;
  // No synchronization here: the solve is queued behind the type-1 stage, and the flags the stage
  // raises (NaN, range) come back with the solve's first residual norms, ahead of its own status.
  st = solve_impl(ctx, P, s, theta_out, info);
  if (st == FK_OK || st == FK_ENOCONV)
    kept_register(wss, s.bytes, ctx->device, kKeptToeplitz, d, m, P.L, nlam, ntgt, 1);
  if (info) {
    info->status = st;
    info->t_sort_ms = elapsed(ctx->ev[0], ctx->ev[1]);
    info->t_spread_ms = elapsed(ctx->ev[1], ctx->ev[2]);
    info->spread_kernel_ms = info->t_spread_ms;
    info->t_fft_ms = elapsed(ctx->ev[2], ctx->ev[4]);
    info->t_total_ms = elapsed(ctx->ev[0], ctx->ev[8]);
  }
  return st;
}

extern "C" fk_status fk_fit(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int ntgt, const void* Y,
                            int m, const double* lambdas, int nlam, const fk_penalty* pen, double* theta_out,
                            void* ws, size_t ws_bytes, fk_fit_info* info) {
  if (!ctx || !theta_out) return FK_EINVAL;
  if (check_gram_args(d, n, ntgt, m, X, Y) != FK_OK || ntgt < 1 || nlam < 1) return FK_EINVAL;
  if (!ws || ws_bytes < fit_ws(d, n, ntgt, m, nlam)) return FK_ENOMEM;
  const size_t sb = solve_layout((int)ipow(2 * m + 1, d), nlam, ntgt, nullptr, 0).bytes;
  return fit_impl(ctx, d, n, dt, X, ntgt, Y, m, lambdas, nlam, pen, theta_out, ws, sb,
                  static_cast<char*>(ws) + sb, ws_bytes - sb, info);
}

extern "C" fk_status fk_fit_kept_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m, int nlam,
                                                size_t* solve_bytes, size_t* scratch_bytes) {
  if (!solve_bytes || !scratch_bytes) return FK_EINVAL;
  if (check_gram_args(d, n, ntgt, m, (void*)1, (void*)1) != FK_OK || ntgt < 1 || nlam < 1 || nlam > 1024 || d > 2)
    return FK_EINVAL;
  *solve_bytes = solve_layout((int)ipow(2 * m + 1, d), nlam, ntgt, nullptr, 0).bytes;
  *scratch_bytes = fit_scratch(d, n, ntgt, m);
  return FK_OK;
}

extern "C" fk_status fk_fit_kept(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int ntgt,
                                 const void* Y, int m, const double* lambdas, int nlam, const fk_penalty* pen,
                                 double* theta_out, void* ws_solve, size_t ws_solve_bytes, void* ws_scratch,
                                 size_t ws_scratch_bytes, fk_fit_info* info) {
  if (ws_solve && ws_scratch) {
    const char* a = static_cast<const char*>(ws_solve);
    const char* b = static_cast<const char*>(ws_scratch);
    if (a < b + ws_scratch_bytes && b < a + ws_solve_bytes) return FK_EINVAL;   // overlapping workspaces
  }
  return fit_impl(ctx, d, n, dt, X, ntgt, Y, m, lambdas, nlam, pen, theta_out, ws_solve, ws_solve_bytes, ws_scratch,
                  ws_scratch_bytes, info);
}

// ------------------------------------------------------------------ held-out loss / backward

extern "C" fk_status fk_heldout_mse(fk_ctx* ctx, int d, int m, int ntgt, int nlam, const double* Mv,
                                    const double* bv, const double* yv2, double* mse_out, void* ws,
                                    size_t ws_bytes) {
  if (!ctx || !Mv || !bv || !yv2 || !mse_out || (d != 1 && d != 2) || m < 1 || m > 64 || ntgt < 1 || ntgt > 32 ||
      nlam < 1 || nlam > 1024)
    return FK_EINVAL;
  SolveLayout s = solve_layout((int)ipow(2 * m + 1, d), nlam, ntgt, ws, ws_bytes);
  if (!ws || s.bytes > ws_bytes) return FK_ENOMEM;
  if (!kept_find(ws, ctx->device, kKeptToeplitz, d, m, s.N, nlam, ntgt, 1)) return FK_EINVAL;
  FK_HIP(hipSetDevice(ctx->device));
  fk_status st = heldout_mse_impl(ctx, s, d, m, Mv, bv, yv2, mse_out);
  if (st != FK_OK) return st;
  FK_HIP(hipStreamSynchronize(ctx->stream));
  kept_register(ws, s.bytes, ctx->device, kKeptToeplitz, d, m, s.N, nlam, ntgt, 2);
  return FK_OK;
}

namespace fk {
// out[t] += sum_j Y[t][j]^2 over this workgroup's part of row t (FP64; grid.y = t).
template <typename TY>
__global__ __launch_bounds__(256) void k_sum_squares(const TY* __restrict__ Y, int64_t n, double* __restrict__ out) {
  __shared__ double part[4];
  const TY* y = Y + (int64_t)blockIdx.y * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // four loads in flight per thread, four partial sums
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (; j + 3 * stride < n; j += 4 * stride) {
    const double v0 = (double)y[j], v1 = (double)y[j + stride], v2 = (double)y[j + 2 * stride],
                 v3 = (double)y[j + 3 * stride];
    s0 = fma(v0, v0, s0);
    s1 = fma(v1, v1, s1);
    s2 = fma(v2, v2, s2);
    s3 = fma(v3, v3, s3);
  }
  for (; j < n; j += stride) {
    const double v = (double)y[j];
    s0 = fma(v, v, s0);
  }
  double s = (s0 + s1) + (s2 + s3);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&out[blockIdx.y], part[0] + part[1] + part[2] + part[3]);
}
__global__ void k_fill_zero(double* __restrict__ p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}
__global__ void k_scale(double* __restrict__ p, int count, double a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] *= a;
}
}  // namespace fk

extern "C" fk_status fk_mean_square(fk_ctx* ctx, int ntgt, int64_t n, fk_dtype dtype, const void* Y, double* out) {
  if (!ctx || !Y || !out || ntgt < 1 || ntgt > 65535 || n < 1 || (dtype != FK_F32 && dtype != FK_F64))
    return FK_EINVAL;
  FK_HIP(hipSetDevice(ctx->device));
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_fill_zero, dim3((ntgt + 255) / 256), dim3(256), 0, ctx->stream, out, ntgt);
  if (dtype == FK_F32)
    hipLaunchKernelGGL(k_sum_squares<float>, dim3(blocks, ntgt), dim3(256), 0, ctx->stream,
                       static_cast<const float*>(Y), n, out);
  else
    hipLaunchKernelGGL(k_sum_squares<double>, dim3(blocks, ntgt), dim3(256), 0, ctx->stream,
                       static_cast<const double*>(Y), n, out);
  hipLaunchKernelGGL(k_scale, dim3((ntgt + 255) / 256), dim3(256), 0, ctx->stream, out, ntgt, 1.0 / (double)n);
  FK_HIP(hipGetLastError());
  return FK_OK;
}

extern "C" fk_status fk_fit_backward(fk_ctx* ctx, int d, int m, int ntgt, int nlam, const double* grad_mse,
                                     const double* grad_theta_in, double* grad_loglam, double* grad_p,
                                     double* grad_theta, void* ws, size_t ws_bytes) {
  if (!ctx || !grad_mse || !grad_loglam || (d != 1 && d != 2) || m < 1 || m > 64 || ntgt < 1 || ntgt > 32 ||
      nlam < 1 || nlam > 1024)
    return FK_EINVAL;
  SolveLayout s = solve_layout((int)ipow(2 * m + 1, d), nlam, ntgt, ws, ws_bytes);
  if (!ws || s.bytes > ws_bytes) return FK_ENOMEM;
  if (!kept_find(ws, ctx->device, kKeptToeplitz, d, m, s.N, nlam, ntgt, 2)) return FK_EINVAL;
  FK_HIP(hipSetDevice(ctx->device));
  fk_status st = backward_impl(ctx, s, d, grad_mse, grad_theta_in, grad_loglam, grad_p, grad_theta);
  if (st != FK_OK) return st;
  FK_HIP(hipStreamSynchronize(ctx->stream));
  return FK_OK;
}

// ------------------------------------------------------------------ additive model (Sec. 5)
namespace fk {

// Assemble the complex block Gram B [Nc][Nc] (Nc = d L, L = 2m+1) and stacked RHS from
//   c1[a]: 1-D type-1 outputs [T+1][4m+1] (K = 2m, already scaled by 1/n),
//   c2[p]: 2-D type-1 outputs [(2m+1)^2] (K = m) of the pair p = (a < b), scaled by 1/n.
// B[a,a][k,l] = M_a[l-k] = c1_a,0[k-l]; B[a,b][k,l] = c2_ab[k, -l]; B[b,a] = B[a,b]^*.
__global__ void k_additive_assemble(const double* __restrict__ c1, const double* __restrict__ c2, int d, int m,
                                    int T, double* __restrict__ B, double* __restrict__ b) {
  const int L = 2 * m + 1, K1 = 4 * m + 1, Nc = d * L;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < Nc * Nc) {
    int r = idx / Nc, s = idx - r * Nc;
    int a = r / L, k = r % L - m, bb = s / L, l = s % L - m;
    double re, im;
    if (a == bb) {
      const double* c = c1 + 2 * (size_t)a * (T + 1) * K1;
      int q = k - l + 2 * m;
      re = c[2 * q];
      im = c[2 * q + 1];
    } else {
      int lo = a < bb ? a : bb, hi = a < bb ? bb : a;
      int p = lo * d - lo * (lo + 1) / 2 + (hi - lo - 1);   // pair index
      const double* c = c2 + 2 * (size_t)p * L * L;
      if (a < bb) {
        int o = (k + m) * L + (-l + m);
        re = c[2 * o];
        im = c[2 * o + 1];
      } else {  // B[a,b][k,l] = conj(B[b,a][l,k]) with b < a
        int o = (l + m) * L + (-k + m);
        re = c[2 * o];
        im = -c[2 * o + 1];
      }
    }
    B[2 * (size_t)idx] = re;
    B[2 * (size_t)idx + 1] = im;
  }
  if (idx < T * Nc) {
    int t = idx / Nc, r = idx - t * Nc;
    int a = r / L, k = r % L - m;
    const double* c = c1 + 2 * ((size_t)a * (T + 1) + (t + 1)) * K1;
    int q = k + 2 * m;
    b[2 * (size_t)idx] = c[2 * q];
    b[2 * (size_t)idx + 1] = c[2 * q + 1];
  }
}

// Workspace of one type-1 transform of the additive model (the larger of the 1-D and pairwise ones).
static size_t additive_region(int64_t n, int T, int m) {
  const size_t t1 = type1_workspace(1, n, T, 2 * m, 0);
  const size_t t2 = type1_workspace(2, n, 0, m, 0);
  return (std::max(t1, t2) + 1023) & ~size_t(255);
}

static size_t additive_gram_ws(int d, int64_t n, int T, int m) {
  const int L = 2 * m + 1, K1 = 4 * m + 1;
  const int npair = d * (d - 1) / 2;
  Carve cv(nullptr, 0);
  cv.take<double>((size_t)2 * d * (T + 1) * K1);
  cv.take<double>((size_t)2 * npair * L * L);
  cv.take<char>(additive_region(n, T, m));   // two transforms in flight, one region each
  cv.take<char>(additive_region(n, T, m));
  return cv.off + 1024;
}

// The second stream of the additive model's transforms (created on first use, default priority).
static fk_status aux_stream(fk_ctx* ctx) {
  if (ctx->aux_stream) return FK_OK;
  FK_HIP(hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking));
  for (auto& e : ctx->aux_ev) FK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return FK_OK;
}

fk_status additive_gram_impl(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int T, const void* Y,
                             int m, double* B, double* b, Carve& cv, fk_fit_info* info) {
  const int L = 2 * m + 1, K1 = 4 * m + 1;
  const int npair = d * (d - 1) / 2;
  double* c1 = cv.take<double>((size_t)2 * d * (T + 1) * K1);
  double* c2 = cv.take<double>((size_t)2 * npair * L * L);
  const size_t region = additive_region(n, T, m);
  char* reg[2] = {cv.take<char>(region), cv.take<char>(region)};
  if (!cv.ok()) return FK_ENOMEM;
  fk_status st = aux_stream(ctx);
  if (st != FK_OK) return st;
  const size_t esz = dt == FK_F64 ? 8 : 4;
  const char* Xc = static_cast<const char*>(X);
  // The d(d-1)/2 pairwise and d one-dimensional transforms, two in flight: task k runs on the
  // caller's stream (even k) or the aux stream (odd k), each side in a workspace region of its own.
  // Both kinds are HBM-bound (sorting passes, record gathers), so the gain is the filling of each
  // other's launch tails and gaps.  Task 0, the first pair, runs alone first: the pairwise launch
  // shape, tuned at its first use (the one-dimensional transforms have none), is then measured without
  // the other stream, and the later pairs find it in the table.
  std::vector<std::pair<int, int>> tasks;
  for (int a = 0; a < d; ++a)
    for (int bb = a + 1; bb < d; ++bb) tasks.push_back({a, bb});
  for (int a = 0; a < d; ++a) tasks.push_back({a, -1});
  hipStream_t S = ctx->stream, Bs = ctx->aux_stream;
  int p = 0;
  for (size_t k = 0; k < tasks.size() && st == FK_OK; ++k) {
    if (k == 1) {
      FK_HIP(hipEventRecord(ctx->aux_ev[0], S));
      FK_HIP(hipStreamWaitEvent(Bs, ctx->aux_ev[0], 0));
    }
    const int side = (int)(k & 1);
    ctx->stream = side ? Bs : S;
    Carve sub(reg[side], region);
    const int a = tasks[k].first, bb = tasks[k].second;
    if (bb < 0) {
      st = type1(ctx, 1, n, dt, Xc + esz * (size_t)a * n, n, T, Y, 2 * m, 1.0 / (double)n,
                 c1 + 2 * (size_t)a * (T + 1) * K1, sub, info);
    } else {
      st = type1(ctx, 2, n, dt, Xc + esz * (size_t)a * n, (int64_t)(bb - a) * n, 0, nullptr, m, 1.0 / (double)n,
                 c2 + 2 * (size_t)p * L * L, sub, info);
      ++p;
    }
    ctx->stream = S;
  }
  // join: the caller's stream waits for the aux stream's work (also on an error, before returning)
  FK_HIP(hipEventRecord(ctx->aux_ev[1], Bs));
  FK_HIP(hipStreamWaitEvent(S, ctx->aux_ev[1], 0));
  if (st != FK_OK) return st;
  const int Nc = d * L;
  const int tot = std::max(Nc * Nc, T * Nc);
  hipLaunchKernelGGL(k_additive_assemble, dim3((tot + 255) / 256), dim3(256), 0, ctx->stream, c1, c2, d, m, T, B, b);
  FK_HIP(hipGetLastError());
  return FK_OK;
}

}  // namespace fk

static fk_status check_additive(int d, int64_t n, int T, int m, const void* X, const void* Y) {
  if (d < 2 || d > 16 || n < 1 || m < 1 || m > 64 || T < 1 || T > 32 || !X || !Y) return FK_EINVAL;
  return FK_OK;
}

extern "C" fk_status fk_additive_gram_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m,
                                                     size_t* bytes) {
  (void)ctx;
  if (!bytes || check_additive(d, n, ntgt, m, (void*)1, (void*)1) != FK_OK) return FK_EINVAL;
  *bytes = additive_gram_ws(d, n, ntgt, m);
  return FK_OK;
}

extern "C" fk_status fk_additive_gram(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int ntgt,
                                      const void* Y, int m, double* B_out, double* b_out, void* ws, size_t ws_bytes,
                                      fk_fit_info* info) {
  if (!ctx || check_additive(d, n, ntgt, m, X, Y) != FK_OK || !B_out || !b_out) return FK_EINVAL;
  if (dt != FK_F32 && dt != FK_F64) return FK_EINVAL;
  if (!ws || ws_bytes < additive_gram_ws(d, n, ntgt, m)) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  kept_invalidate(ws, ws_bytes);
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->bad_index = -1;
  }
  Carve cv(ws, ws_bytes);
  fk_status st = reset_flags(ctx);
  FK_HIP(hipEventRecord(ctx->ev[9], ctx->stream));
  if (st == FK_OK) st = additive_gram_impl(ctx, d, n, dt, X, ntgt, Y, m, B_out, b_out, cv, info);
  if (st != FK_OK) return st;
  FK_HIP(hipEventRecord(ctx->ev[10], ctx->stream));
  st = read_flags(ctx);
  if (info) {
    info->status = st;
    info->t_total_ms = elapsed(ctx->ev[9], ctx->ev[10]);
  }
  return st;
}

static size_t additive_fit_ws(int d, int64_t n, int T, int m, int nlam) {
  const int Nc = d * (2 * m + 1);
  size_t a = solve_layout(Nc, nlam, T, nullptr, 0).bytes;
  Carve cv(nullptr, 0);
  cv.take<double>((size_t)2 * Nc * Nc);
  cv.take<double>((size_t)2 * T * Nc);
  return a + cv.off + additive_gram_ws(d, n, T, m) + 1024;
}

extern "C" fk_status fk_additive_fit_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m, int nlam,
                                                    size_t* bytes) {
  (void)ctx;
  if (!bytes || check_additive(d, n, ntgt, m, (void*)1, (void*)1) != FK_OK || nlam < 1 || nlam > 1024)
    return FK_EINVAL;
  *bytes = additive_fit_ws(d, n, ntgt, m, nlam);
  return FK_OK;
}

extern "C" fk_status fk_additive_fit(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int ntgt,
                                     const void* Y, int m, const double* lambdas, int nlam, double s,
                                     double* theta_out, void* ws, size_t ws_bytes, fk_fit_info* info) {
  if (!ctx || check_additive(d, n, ntgt, m, X, Y) != FK_OK || !theta_out || !lambdas || nlam < 1 || nlam > 1024)
    return FK_EINVAL;
  if (dt != FK_F32 && dt != FK_F64) return FK_EINVAL;
  if (!(s >= 0.0) || s > 64) return FK_EINVAL;
  if (!ws || ws_bytes < additive_fit_ws(d, n, ntgt, m, nlam)) return FK_ENOMEM;
  FK_HIP(hipSetDevice(ctx->device));
  kept_invalidate(ws, ws_bytes);
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->bad_index = -1;
  }
  const int L = 2 * m + 1, Nc = d * L;
  SolveProblem P;
  P.kind = SolveProblem::kDense;
  P.m = m;
  P.d = 1;
  P.L = L;
  P.p.resize(Nc);
  for (int a = 0; a < d; ++a)
    for (int k = -m; k <= m; ++k) P.p[a * L + k + m] = 1.0 + (s == 0.0 ? 0.0 : std::pow((double)k * k, s));
  if (s == 0.0)
    for (auto& v : P.p) v = 1.0;
  P.lams.assign(lambdas, lambdas + nlam);
  for (double l : P.lams)
    if (!(l > 0.0) || std::isinf(l)) return FK_EINVAL;
  SolveLayout sl = solve_layout(Nc, nlam, ntgt, ws, ws_bytes);
  Carve cv(static_cast<char*>(ws) + sl.bytes, ws_bytes - sl.bytes);
  double* B = cv.take<double>((size_t)2 * Nc * Nc);
  double* b = cv.take<double>((size_t)2 * ntgt * Nc);
  P.B = B;
  P.b = b;
  fk_status st = reset_flags(ctx);
  FK_HIP(hipEventRecord(ctx->ev[9], ctx->stream));
  if (st == FK_OK) st = additive_gram_impl(ctx, d, n, dt, X, ntgt, Y, m, B, b, cv, info);
  if (st != FK_OK) return st;
  FK_HIP(hipEventRecord(ctx->ev[10], ctx->stream));
  // (the transforms' flags come back with the solve's first residual norms)
  st = solve_impl(ctx, P, sl, theta_out, info);
  if (info) {
    info->status = st;
    info->t_spread_ms = elapsed(ctx->ev[9], ctx->ev[10]);
    info->t_total_ms = elapsed(ctx->ev[9], ctx->ev[8]);
  }
  return st;
}
