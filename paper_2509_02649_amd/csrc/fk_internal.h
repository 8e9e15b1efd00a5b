// Internal declarations shared by the HIP translation units of libfastkernel.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fk.h"

#define FK_HIP(call)                                                         \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) return FK_EHIP;                                    \
  } while (0)

namespace fk {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxW = 16;

// Device error flags (one int array per context, reset at the start of a call).
enum Flag { kFlagRange = 0, kFlagNaN = 1, kFlagNotPD = 2, kFlagCount = 8 };

// Exponential-of-semicircle spreading plan for one dimension: grid size nf,
// width w, shape beta, and the FP64 Fourier transform of the kernel at the
// integer frequencies 0..K (deconvolution factors, host copy).
struct EsPlan {
  int nf = 0;
  int w = 0;
  int K = 0;          // largest |frequency| needed
  double beta = 0.0;
  double err = 0.0;   // estimated worst-case relative aliasing error
  std::vector<double> phihat;  // size K+1
};

// nf_fixed > 0 fixes the grid size (any even length), else the smallest power of two >= 2(2K+1).
EsPlan make_es_plan(int K, double eps, int nf_fixed = 0);

// Workspace carving: bump allocator over the caller's buffer.
// Every array starts on a 256-byte boundary of the device address space: a base that is not
// aligned is first moved up to the next boundary (the workspace sizes carry that much slack).
// The 64-byte weight blocks of the sort and the spread's gathers rely on it: one block per half
// cache line, not one straddling two lines.
struct Carve {
  char* base;
  size_t off = 0;
  size_t cap;
  Carve(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {
    const size_t mis = reinterpret_cast<uintptr_t>(base) & 255u;
    if (base && mis) {
      const size_t skip = 256 - mis;
      base += skip;
      cap = cap > skip ? cap - skip : 0;
    }
  }
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
  bool ok() const { return off <= cap; }
};

// Workspace layout of the dense stage (fixed from N, nlam, ntgt, at the start
// of the caller's workspace so that later calls on the same workspace find it).
struct SolveLayout {
  int N = 0, Np = 0, nlam = 0, ntgt = 0;
  double* H64 = nullptr;   // Np x Np real-form Gram (+ dense penalty), FP64
  float* A32 = nullptr;    // nlam x Np x Np FP32 matrices / factors
  float* Linv = nullptr;   // nlam x (Np/64) x 64 x 64 inverses of diagonal blocks
  double* preal = nullptr; // Np real-form diagonal weights
  double* lams = nullptr;  // nlam
  double* Bre = nullptr;   // ntgt x Np real right-hand sides
  double* X64 = nullptr;   // nlam x ntgt x Np solutions (real form)
  double* R64 = nullptr;   // residuals
  double* U64 = nullptr;   // adjoint solutions
  double* G64 = nullptr;   // held-out gradient directions
  double* Gadj = nullptr;  // adjoint right-hand sides
  float* R32 = nullptr;
  float* Y32 = nullptr;
  float* D32 = nullptr;
  double* norms = nullptr;
  double* Hv = nullptr;    // held-out real-form Gram
  double* Bv = nullptr;    // held-out real right-hand sides
  double* pcx = nullptr;   // N complex-mode weights
  double* scl = nullptr;   // nlam x Np diagonal equilibration of the FP32 factor
  double* dsym = nullptr;  // N complex: operator symbol of a physics-informed penalty
  float* upart = nullptr;  // part_tiles x 64 x 128: parts of the split paired updates
  int part_tiles = 0;
  size_t bytes = 0;
};
SolveLayout solve_layout(int N, int nlam, int ntgt, void* base, size_t cap);

struct SolveProblem {
  enum Kind { kToeplitz = 0, kToeplitzPde = 1, kDense = 2 } kind = kToeplitz;
  const double* M = nullptr;  // generator (Toeplitz kinds)
  const double* B = nullptr;  // dense complex matrix (kDense)
  const double* b = nullptr;  // complex right-hand sides ntgt x N
  int m = 0, d = 0, L = 0;    // L: complex modes per real-form block
  std::vector<double> p;      // complex-mode diagonal weights (N)
  std::vector<double> lams;   // nlam
  // kToeplitzPde: mu D^* C D with the operator symbol D (N complex, interleaved) and the box
  // [lo, hi] of the Fourier matrix C (d <= 2)
  std::vector<double> dsym;
  double mu = 0, lo[2] = {0, 0}, hi[2] = {0, 0};
};
fk_status solve_impl(fk_ctx* ctx, const SolveProblem& P, const SolveLayout& s, double* theta_out,
                     fk_fit_info* info);
fk_status heldout_mse_impl(fk_ctx* ctx, const SolveLayout& s, int d, int m, const double* Mv, const double* bv,
                           const double* yv2, double* mse);
// gin: device complex [nlam][ntgt][N] dLoss/dconj(theta) from other uses of theta, or null.
fk_status backward_impl(fk_ctx* ctx, const SolveLayout& s, int d, const double* gm, const double* gin,
                        double* grad_loglam, double* grad_p, double* grad_theta);

// Registry of workspaces that hold kept factors (process-wide, all contexts and devices).
// stage 1: factors and solutions of a solve; stage 2: held-out gradient directions as well.
enum KeptKind { kKeptToeplitz = 0, kKeptDense = 1 };
void kept_invalidate(const void* ws, size_t bytes);
void kept_register(const void* ws, size_t bytes, int device, int kind, int d, int m, int N, int nlam, int ntgt,
                   int stage);
bool kept_find(const void* ws, int device, int kind, int d, int m, int N, int nlam, int ntgt, int min_stage);
fk_status reset_flags(fk_ctx* ctx);

// MFMA spread for 8..16 weight channels over MB x MB-cell bins (spread_mfma.hip):
// sorted coordinates, per point its position in the row-grouped weight blocks wrow.
int spread_mfma_bin(int nf, int64_t n);
bool spread_mfma_ok(int nw, int W);
fk_status launch_spread_mfma(hipStream_t st, int W, int MB, const uint32_t* crd, const uint32_t* pos,
                             const uint32_t* wrow, int nw, const uint64_t* start, int nbx, int nb, int nf, int fb,
                             double beta, int64_t n, int spread_pts, double* grid);

// MFMA spread for 0..7 weight channels as per-channel outer products over 8 x 8-cell
// bins (spread_op.hip).
int spread_op_bin();
bool spread_op_ok(int nw, int W);
fk_status launch_spread_op(hipStream_t st, int W, const uint32_t* crd, const uint32_t* wts, int nw,
                           const uint64_t* start, int nbx, int nb, int nf, int fb, double beta, int64_t n,
                           int spread_pts, double* grid);

// Autotuner (tune.hip): process-wide table of measured launch shapes.
enum TuneMode { kTuneEnv = 0, kTuneOff = 1, kTuneForce = 2, kTuneAuto = 3 };
int tune_mode(const fk_ctx* ctx);
std::string tune_arch(int device);
bool tune_lookup(const std::string& key, std::map<std::string, double>* values);
void tune_store(const std::string& key, const std::map<std::string, double>& values, double ms);

// Launch shape of the sorted 2-D type-1 stage.
struct T1Shape {
  int mb = 0;                 // bin edge of the channel-row spread (2 or 4 cells); 0: by density
  int spread_pts = 16384;     // points per spreading workgroup (a slice of one bin)
  int sort_blk = 512;         // workgroups of the first sort pass (at most; fewer for small n)
  int sort_slice = 65536;     // points per workgroup of the second sort pass
};
constexpr int kSortBlkMax = 1024;
constexpr int kSortSliceMin = 32768;

// Launch shape of the dense solve.
struct DenseShape {
  int trsm_wg = 768;          // workgroups per triangular-solve launch (over all lambdas; 3 per CU)
  int pair = 1;               // factor block columns in pairs (row panels read once for two)
  int diag64 = 0;             // diagonal blocks factored in FP64 (1) or FP32 (0)
};

// Two-pass bin sort for the MFMA spreads (sort2.hip): scratch buffers carved from
// the caller's workspace, and the sort itself (bin starts in start[0..nbx^2]).
// Records: coordinates (2 words) and sort2_words(nw) weight words per point
// (16 for 8..16 channels, else the next power of two >= nw, at least 1).  With 16
// words the second pass writes, instead of the weights, each point's position in
// the row-grouped records of the first pass (b.wts1), one word per point.
struct Sort2Bufs {
  uint32_t* cnt1 = nullptr;
  uint32_t* off1 = nullptr;
  uint64_t* start1 = nullptr;
  uint32_t* cnt2 = nullptr;
  uint32_t* off2 = nullptr;
  uint32_t* crd1 = nullptr;
  uint32_t* wts1 = nullptr;
};
bool sort2_ok(int nbx);
int sort2_words(int nw);
// Buffers for any shape with at most kSortBlkMax first-pass workgroups and slices of at least
// kSortSliceMin points.
void sort2_carve(Carve& cv, int64_t n, int nbx, int wv, Sort2Bufs* b);
fk_status sort2(hipStream_t st, const void* X, fk_dtype dt, int64_t n, int64_t xstride, const void* Y, int nw,
                int nf, int fb, int W, double scale, int tshift, int nbx, const T1Shape& shape, const Sort2Bufs& b,
                uint32_t* crd, uint32_t* wts, uint64_t* start, int* flags);

}  // namespace fk

struct fk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  fk_options opt{};
  int* flags = nullptr;           // device, fk::kFlagCount ints
  int* flags_host = nullptr;      // pinned host mirror (kFlagCount ints), then kFlagCount words for counters
  hipEvent_t ev[16] = {};
  // cached deconvolution tables keyed by (K, eps bits)
  std::map<std::pair<int, uint64_t>, std::pair<fk::EsPlan, double*>> es_cache;
  // the same plans without device tables (for the allocation-free entry point)
  std::map<std::pair<int, uint64_t>, fk::EsPlan> es_host_cache;
  // second stream (default priority) and events of the additive model's overlapped transforms
  hipStream_t aux_stream = nullptr;
  hipEvent_t aux_ev[2] = {};
  // pinned host staging area for small uploads and read-backs on the context's stream
  char* stage = nullptr;
  size_t stage_cap = 0, stage_off = 0;
};

namespace fk {
// Returns the ES plan and a device copy of its phihat table (owned by ctx).
fk_status get_es_plan(fk_ctx* ctx, int K, EsPlan* plan, const double** d_phihat, int nf_fixed = 0);
// The same plan, host tables only (no device memory is allocated).
fk_status get_es_plan_host(fk_ctx* ctx, int K, EsPlan* plan, int nf_fixed = 0);
// Resolves this device's copy of the allocation-free prediction's device array (device current).
fk_status scratch_init(int device);
fk_status finish(fk_ctx* ctx, fk_status st, fk_fit_info* info);
fk_status read_flags(fk_ctx* ctx);
// `bytes` of the context's pinned staging area (16-byte aligned), for an asynchronous copy on the
// context's stream; nullptr on failure.  Space is handed out in order; when the area is full the
// stream is synchronized (every copy through it has then completed) and it restarts, grown if needed.
void* stage_take(fk_ctx* ctx, size_t bytes);
// Upload of a small host array through the staging area (asynchronous on the context's stream).
fk_status stage_upload(fk_ctx* ctx, void* dst, const void* src, size_t bytes);
// the status the host mirror of the flags holds (after a read-back that the caller synchronized)
fk_status flag_status(const fk_ctx* ctx);

// Type-1 stage.  Computes c_c[q] = sum_j w_cj exp(-i q.x_j) for |q_a| <= K on C
// channels (channel 0 has weight 1 when `ones_channel`), written as complex128
// [C][(2K+1)^d]. Used by fk_gram and the additive path.
size_t type1_workspace(int d, int64_t n, int nw, int K, double eps);
fk_status type1(fk_ctx* ctx, int d, int64_t n, fk_dtype dt, const void* X, int64_t xstride,
                int nw, const void* Y, int K, double sign_scale, double* out,
                Carve& cv, fk_fit_info* info);

// Multilevel-Toeplitz product by FFT and the conjugate-gradient solve (cg.hip).
// pw: complex-mode diagonal penalty weights (N, host); theta_out: nlam x ntgt x N complex.
bool toeplitz_fft_ok(int d, int m);
size_t toeplitz_apply_workspace(int d, int m, int nvec);
fk_status toeplitz_apply_impl(fk_ctx* ctx, int d, int m, const double* M, int nvec, const double* x, double* y,
                              Carve& cv);
// Mr, Dsym (device, nullable together): generator of the collocation points and the operator
// symbol of the physics term mu D^* Sigma_r D.
size_t cg_workspace(int d, int m, int nsys, int nlam, bool colloc);
fk_status cg_solve_impl(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                        const std::vector<double>& lams, const std::vector<double>& pw, double mu, const double* Mr,
                        const double* Dsym, double tol, int maxit, double* theta_out, int* iters_out,
                        double* relres_out, Carve& cv);
}  // namespace fk
