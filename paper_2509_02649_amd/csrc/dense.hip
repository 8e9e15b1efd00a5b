// Dense stage: assembly of the normal equations in real cosine/sine form, a
// batched blocked Cholesky of FP32 matrices on MFMA (finished panels kept as FP16
// pairs, products on the FP16 matrix cores), FP32 triangular solves, and FP64
// iterative refinement (eq. kenrel_reg; the paper's additive model solves the
// same kind of system directly, Sec. 5 "Complexity").
//
// Real form.  For real data the complex system A theta = b with
// A[-k,-l] = conj A[k,l] and b[-k] = conj b[k] has a Hermitian-symmetric
// solution, and theta = U c with the unitary change of basis
//   c_0 <-> exp(0),  c_{k,cos} <-> sqrt2 cos(k.x),  c_{k,sin} <-> sqrt2 sin(k.x)
// (k in a half space) turns it into the real symmetric system
// (U^* A U) c = U^* b of the same size N and condition number, which costs
// a quarter of the complex factorization.  Real index r of a block of L modes:
// r = 0 constant, r = 2h-1 cosine and r = 2h sine of mode h = 1..(L-1)/2 (the
// modes are counted from the centre of the block in row-major order).
//
// Layout in HBM: every real matrix is Np x Np row-major, Np = N rounded up to a
// multiple of 64, padded with the identity (factor) or zeros (FP64 Gram), so the
// blocked kernels never see a ragged edge.  One FP64 Gram H64 (with any dense,
// lambda-independent penalty folded in) serves all lambdas; each lambda has its
// own FP32 matrix, overwritten by its Cholesky factor (FP32 diagonal blocks, the
// blocks below them as FP16 pairs in the same 32-bit slots), and the inverses of
// its 64 x 64 diagonal blocks.
#include "fk_internal.h"

#include <cmath>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

namespace fk {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int NB = 64;     // block size of the factorization
constexpr int LDT = NB + 4; // LDS row stride (floats) of a 64 x 64 tile

// ------------------------------------------------------------------ factor panels as FP16 pairs
// A finished panel of the factor keeps each entry as two FP16 halves in its 32-bit slot:
// a = hi + 2^-11 lo with hi = fp16(a) and lo = fp16(2^11 (a - hi)), both rounded to nearest (the
// splitting of Ootomo and Yokota, 2022, for FP32-accurate products on FP16 matrix units).  The
// left-looking updates multiply such panels as hi*hi + 2^-11 (hi*lo + lo*hi) with FP32 accumulation,
// the lo*lo term (2^-22 relative) dropped: about 22 significant bits per operand at the FP16 matrix
// rate (one v_mfma_f32_16x16x32_f16, 16 cycles, per 16 x 16 x 32 term against eight FP32 16x16x4
// steps, 256 cycles).  The equilibrated factor's entries are at most 1 in magnitude, far inside the
// FP16 range, and the scaled lo keeps entries below the FP16 normal range to 2^-35 absolute.
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
constexpr float kSplitScale = 2048.f;

__device__ __forceinline__ uint32_t split_pack(float a) {
  const _Float16 hi = (_Float16)a;
  const _Float16 lo = (_Float16)((a - (float)hi) * kSplitScale);
  return (uint32_t)__builtin_bit_cast(uint16_t, hi) | ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
}

__device__ __forceinline__ float split_unpack(uint32_t w) {
  const float hi = (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
  const float lo = (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
  return fmaf(lo, 1.f / kSplitScale, hi);
}

// A 64 x 64 split tile in LDS: the hi and the lo halves as two row-major FP16 tiles of 128-byte
// rows, unpadded (three tiles per workgroup, three workgroups per CU).  The 16-byte chunk j of row r
// is stored at chunk j ^ sw(r), sw(r) = (r mod 8) ^ (r / 8 mod 2): the 16 rows that one matrix-core
// operand read touches (16 lanes, 16 bytes each) then fall on distinct banks.
struct SplitTile {
  _Float16 hi[NB * NB];
  _Float16 lo[NB * NB];
};
__device__ __forceinline__ int split_off(int r, int c) {   // c: first of 4 (staging) or 8 (reads) columns
  return r * NB + ((((c >> 3) ^ (r & 7) ^ ((r >> 3) & 1))) << 3) + (c & 7);
}

// Four packed entries of one tile row (LDS offset off = split_off(row, first column)) into the hi
// and lo tiles.
__device__ __forceinline__ void split_stage(SplitTile& T, int off, uint4 v) {
  uint2 h, o;
  h.x = (v.x & 0xffffu) | (v.y << 16);
  h.y = (v.z & 0xffffu) | (v.w << 16);
  o.x = (v.x >> 16) | (v.y & 0xffff0000u);
  o.y = (v.z >> 16) | (v.w & 0xffff0000u);
  *reinterpret_cast<uint2*>(&T.hi[off]) = h;
  *reinterpret_cast<uint2*>(&T.lo[off]) = o;
}

// ------------------------------------------------------------------ real-form index maps

struct RealMap {
  int L;      // complex modes per block
  int nblk;   // number of blocks (1, or d for the additive model)
};

// complex index of the mode of real index r, its negation, and the entry type
// (0 const, 1 cos, 2 sin)
__device__ __forceinline__ void real_to_complex(int r, int L, int* type, int* kidx, int* nkidx) {
  int a = r / L, rho = r - a * L;
  int c0 = a * L + (L - 1) / 2;
  if (rho == 0) {
    *type = 0;
    *kidx = c0;
    *nkidx = c0;
  } else {
    int h = (rho + 1) >> 1;
    *type = (rho & 1) ? 1 : 2;
    *kidx = c0 + h;
    *nkidx = c0 - h;
  }
}

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }

// Real-form entry from four complex entries (see header comment).
template <class Q>
__device__ double real_entry(const Q& q, int r, int s, int L) {
  int tr, k, nk, ts, l, nl;
  real_to_complex(r, L, &tr, &k, &nk);
  real_to_complex(s, L, &ts, &l, &nl);
  const double rs2 = 0.70710678118654752440;
  if (tr == 0 && ts == 0) return q(k, l).re;
  if (tr == 0) {
    cplx a = q(k, l), b = q(k, nl);
    // (0, cos): (Q(0,l) + Q(0,-l))/sqrt2 ; (0, sin): Re[i (Q(0,-l) - Q(0,l))]/sqrt2
    return ts == 1 ? (a.re + b.re) * rs2 : -(b.im - a.im) * rs2;
  }
  if (ts == 0) {
    cplx a = q(k, l), b = q(nk, l);
    // (cos, 0): (Q(k,0) + Q(-k,0))/sqrt2 ; (sin, 0): Re[-i (Q(-k,0) - Q(k,0))]/sqrt2
    return tr == 1 ? (a.re + b.re) * rs2 : (b.im - a.im) * rs2;
  }
  cplx kl = q(k, l), knl = q(k, nl), nkl = q(nk, l), nknl = q(nk, nl);
  if (tr == 1 && ts == 1) return 0.5 * (kl.re + knl.re + nkl.re + nknl.re);
  if (tr == 2 && ts == 2) return 0.5 * (nknl.re - nkl.re - knl.re + kl.re);
  if (tr == 1) {  // (cos k, sin l) = Re[(i/2)(Q(k,-l) - Q(k,l) + Q(-k,-l) - Q(-k,l))]
    cplx z = csub(cadd(knl, nknl), cadd(kl, nkl));
    return -0.5 * z.im;
  }
  // (sin k, cos l) = Re[(-i/2)(Q(-k,l) + Q(-k,-l) - Q(k,l) - Q(k,-l))]
  cplx z = csub(cadd(nkl, nknl), cadd(kl, knl));
  return 0.5 * z.im;
}

// Complex entry providers ------------------------------------------------

// Toeplitz Gram Sigma[k, l] = M[l - k] from the generator over {-2m..2m}^d.
struct ToeplitzQ {
  const double* M;
  int m, d;
  __device__ cplx operator()(int i, int j) const {
    const int L = 2 * m + 1, G = 4 * m + 1;
    int idx = 0;
    int ii = i, jj = j;
    int mul = 1;
    for (int a = d - 1; a >= 0; --a) {
      int ki = ii % L - m, kj = jj % L - m;
      ii /= L;
      jj /= L;
      idx += (kj - ki + 2 * m) * mul;
      mul *= G;
    }
    return {M[2 * idx], M[2 * idx + 1]};
  }
  // Linear offset of mode i in the generator grid (sum over axes of k_a G^a): the entry (i, j) is at
  // off(j) - off(i) + centre, so four entries of one real-form element need four decodes, not eight.
  __device__ int off(int i) const {
    const int L = 2 * m + 1, G = 4 * m + 1;
    int o = 0, mul = 1;
    for (int a = d - 1; a >= 0; --a) {
      const int qd = i / L;
      o += (i - qd * L - m) * mul;
      i = qd;
      mul *= G;
    }
    return o;
  }
  __device__ int centre() const {
    const int G = 4 * m + 1;
    int c = 0, mul = 1;
    for (int a = 0; a < d; ++a) {
      c += 2 * m * mul;
      mul *= G;
    }
    return c;
  }
};

// The four complex entries that real_entry reads for one real-form element (modes k, -k of the
// row and l, -l of the column), through mode offsets: entry (i, j) at M[off(j) - off(i) + centre].
struct ToeplitzPairQ {
  const double* M;
  int c, k, l, ok, onk, ol, onl;
  __device__ cplx operator()(int i, int j) const {
    const int idx = (j == l ? ol : onl) - (i == k ? ok : onk) + c;
    return {M[2 * idx], M[2 * idx + 1]};
  }
};

// Physics-informed penalty of a box (Sec. 4, tractable domains): mu conj(D_k) C[k, l] D_l with the
// operator symbol D (device, N complex) and C[k, l] = (2 pi)^-d prod_a int_{lo_a}^{hi_a}
// exp(i (l_a - k_a) u) du, so that theta^* C theta = (2 pi)^-d int_box |f_theta|^2 for
// f_theta = sum_k theta_k exp(i k.x).  d = 1 or 2.
struct PdeQ {
  const double* dsym;
  int m, d;
  double mu, lo0, hi0, lo1, hi1;
  __device__ static cplx box(int q, double lo, double hi) {
    if (q == 0) return {hi - lo, 0.0};
    double s1, c1, s0, c0;
    sincos(q * hi, &s1, &c1);
    sincos(q * lo, &s0, &c0);
    // (e^{iqhi} - e^{iqlo}) / (iq) = ((s1 - s0) - i (c1 - c0)) / q
    return {(s1 - s0) / q, -(c1 - c0) / q};
  }
  __device__ cplx operator()(int i, int j) const {
    const int L = 2 * m + 1;
    cplx C;
    if (d == 1) {
      C = box((j - m) - (i - m), lo0, hi0);
      const double s = 1.0 / (2.0 * kPi);
      C = {C.re * s, C.im * s};
    } else {
      const int k0 = i / L - m, k1 = i % L - m, l0 = j / L - m, l1 = j % L - m;
      const cplx c0 = box(l0 - k0, lo0, hi0), c1 = box(l1 - k1, lo1, hi1);
      const double s = 1.0 / (4.0 * kPi * kPi);
      C = {(c0.re * c1.re - c0.im * c1.im) * s, (c0.re * c1.im + c0.im * c1.re) * s};
    }
    const cplx Dk = {dsym[2 * i], dsym[2 * i + 1]}, Dl = {dsym[2 * j], dsym[2 * j + 1]};
    // conj(Dk) * C * Dl
    const cplx t = {Dk.re * C.re + Dk.im * C.im, Dk.re * C.im - Dk.im * C.re};
    return {mu * (t.re * Dl.re - t.im * Dl.im), mu * (t.re * Dl.im + t.im * Dl.re)};
  }
};

// Dense complex matrix [Nc][Nc] (additive block Gram).
struct DenseQ {
  const double* B;
  int Nc;
  __device__ cplx operator()(int i, int j) const {
    size_t o = 2 * ((size_t)i * Nc + j);
    return {B[o], B[o + 1]};
  }
};

template <class Q1, class Q2>
struct SumQ {
  Q1 a;
  Q2 b;
  __device__ cplx operator()(int i, int j) const { return cadd(a(i, j), b(i, j)); }
};

// H64[r][s] = real form of Q (r, s < N); zero padding up to Np.
template <class Q>
__global__ __launch_bounds__(256) void k_assemble_real(Q q, int N, int L, int Np, double* __restrict__ H) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Np * Np) return;
  int r = (int)(idx / Np), s = (int)(idx - (int64_t)r * Np);
  double v = 0.0;
  if (r < N && s < N) {
    if constexpr (std::is_same<Q, ToeplitzQ>::value) {
      int tr, k, nk, ts, l, nl;
      real_to_complex(r, L, &tr, &k, &nk);
      real_to_complex(s, L, &ts, &l, &nl);
      const ToeplitzPairQ pq{q.M, q.centre(), k, l, q.off(k), q.off(nk), q.off(l), q.off(nl)};
      v = real_entry(pq, r, s, L);
    } else {
      v = real_entry(q, r, s, L);
    }
  }
  H[idx] = v;
}

// Symmetric diagonal equilibration of each lambda's matrix: scl[l][r] =
// 1/sqrt(H64[r][r] + lambda_l preal[r]) (1 on the padding).  The FP32 factor is
// taken of S A S, which keeps the PDE-penalty systems (diagonal spread over many
// decades) inside FP32's reach; refinement applies S on both sides.
__global__ void k_make_scale(const double* __restrict__ H, const double* __restrict__ preal,
                             const double* __restrict__ lams, int N, int Np, double* __restrict__ scl) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (r >= Np) return;
  double v = 1.0;
  if (r < N) {
    double dgl = H[(size_t)r * Np + r] + lams[l] * preal[r];
    v = dgl > 0.0 ? 1.0 / sqrt(dgl) : 1.0;
  }
  scl[(size_t)l * Np + r] = v;
}

// A32[l] = S_l (H64 + lambda_l diag(p_real)) S_l in FP32, identity padding; blocks
// above the block diagonal are not written (no kernel reads them).  One workgroup per 64 x 64
// tile of the lower block triangle (blockIdx.x enumerates them row by row); a thread takes four
// consecutive columns of four rows of H64, read once, and writes them for every lambda.
__global__ __launch_bounds__(256) void k_make_a32(const double* __restrict__ H, const double* __restrict__ preal,
                                                  const double* __restrict__ lams, const double* __restrict__ scl,
                                                  int N, int Np, int nlam, float* __restrict__ A) {
  // tile index x -> (rb, cb), cb <= rb, x = rb (rb + 1) / 2 + cb
  const int x = blockIdx.x;
  int rb = (int)((sqrt(8.0 * x + 1.0) - 1.0) * 0.5);
  while ((rb + 1) * (rb + 2) / 2 <= x) ++rb;
  while (rb * (rb + 1) / 2 > x) --rb;
  const int cb = x - rb * (rb + 1) / 2;
  const int cc = (threadIdx.x & 15) * 4, r0 = threadIdx.x >> 4;
  const int s = cb * NB + cc;
  double h[4][4], pr[4];
  int rows[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = rb * NB + r0 + 16 * u;
    rows[u] = r;
    pr[u] = (r < N) ? preal[r] : 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) h[u][e] = (r < N && s + e < N) ? H[(size_t)r * Np + s + e] : 0.0;
  }
  for (int l = 0; l < nlam; ++l) {
    const double* sl = scl + (size_t)l * Np;
    const double lam = lams[l];
    double ss[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) ss[e] = sl[s + e];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = rows[u];
      const double sr = sl[r];
      float o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = s + e;
        const bool in = r < N && c < N;
        const double pd = (in && r == c) ? pr[u] : 0.0;
        o[e] = in ? (float)(sr * (h[u][e] + lam * pd) * ss[e]) : (r == c ? 1.0f : 0.0f);
      }
      *reinterpret_cast<float4*>(A + (size_t)l * Np * Np + (size_t)r * Np + s) = make_float4(o[0], o[1], o[2], o[3]);
    }
  }
}

// Workgroups of k_make_a32: the 64 x 64 tiles of the lower block triangle.
static unsigned a32_tiles(int Np) {
  const unsigned nb = (unsigned)(Np / NB);
  return nb * (nb + 1) / 2;
}

// preal[r] = p[complex mode of r]
__global__ void k_real_weights(const double* __restrict__ p, int N, int L, double* __restrict__ preal) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int t, k, nk;
  real_to_complex(r, L, &t, &k, &nk);
  preal[r] = p[k];
}

// Real right-hand sides Bre[t][r] (Np rows, zero padded) from complex b[t][k].  The real form reads
// the mode k of each pair (k, -k) only (b_-k = conj b_k for real data); a NaN or Inf in either entry
// of the pair is carried into the row, so that the residual norms report it.
__global__ void k_rhs_real(const double* __restrict__ b, int N, int L, int Np, int ntgt,
                           double* __restrict__ Bre) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  int t = blockIdx.y;
  if (r >= Np) return;
  double v = 0.0;
  if (r < N) {
    int ty, k, nk;
    real_to_complex(r, L, &ty, &k, &nk);
    const double* bt = b + 2 * (size_t)t * N;
    const double s2 = 1.41421356237309504880;
    v = ty == 0 ? bt[2 * k] : (ty == 1 ? s2 * bt[2 * k] : -s2 * bt[2 * k + 1]);
    const double pair = bt[2 * k] + bt[2 * k + 1] + bt[2 * nk] + bt[2 * nk + 1];
    if (!isfinite(pair)) v = pair - pair;   // NaN
  }
  Bre[(size_t)t * Np + r] = v;
}

// theta[l][t][k] (complex) from real solutions X[l][t][r].
__global__ void k_theta_from_real(const double* __restrict__ X, int N, int L, int Np, int ntgt,
                                  double* __restrict__ theta) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  int lt = blockIdx.y;  // l * ntgt + t
  if (r >= N) return;
  const double* x = X + (size_t)lt * Np;
  double* th = theta + 2 * (size_t)lt * N;
  int ty, k, nk;
  real_to_complex(r, L, &ty, &k, &nk);
  const double rs2 = 0.70710678118654752440;
  if (ty == 0) {
    th[2 * k] = x[r];
    th[2 * k + 1] = 0.0;
  } else if (ty == 1) {
    double c = x[r], s = x[r + 1];
    th[2 * k] = c * rs2;
    th[2 * k + 1] = -s * rs2;
    th[2 * nk] = c * rs2;
    th[2 * nk + 1] = s * rs2;
  }
}

// ------------------------------------------------------------------ MFMA 64x64x64 tile
// acc += As * Bs^T, As and Bs are 64 x 64 FP32 tiles in LDS with row stride LDT
// (As[row][k], Bs[col][k]).  Wave w owns rows 32*(w>>1).. and cols 32*(w&1)..,
// as 2 x 2 blocks of v_mfma_f32_16x16x4f32.  For that instruction lane l holds
// A[l%16][l/16] and B[l/16][l%16]; the 16 x 16 result row 4*(l/16)+v, column
// l%16 sits in element v of the lane's accumulator.
__device__ __forceinline__ void mfma_tile64(const float* As, const float* Bs, floatx4 acc[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int k = 0; k < NB; k += 4) {
    float a0 = As[(r0 + li) * LDT + k + lk];
    float a1 = As[(r0 + 16 + li) * LDT + k + lk];
    float b0 = Bs[(c0 + li) * LDT + k + lk];
    float b1 = Bs[(c0 + 16 + li) * LDT + k + lk];
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// Load a 64 x 64 FP32 tile (row-major, leading dimension ld) into LDS (rows of LDT
// floats, 16-byte aligned).
// A 64 x 64 FP32 tile (row stride ld) in four float4 registers per lane of a 256-thread
// workgroup, and its store into an LDS tile of row stride LDT (named registers: an array would be
// kept in scratch memory by the compiler where it lives across other work).
#define FK_F32_LOAD4(src, ld, a0, a1, a2, a3)                                                \
  do {                                                                                       \
    _Pragma("unroll") for (int u_ = 0; u_ < 4; ++u_) {                                       \
      const int i_ = threadIdx.x + 256 * u_, r_ = i_ / (NB / 4), c_ = (i_ - r_ * (NB / 4)) * 4; \
      const float4 v_ = *reinterpret_cast<const float4*>((src) + r_ * (ld) + c_);          \
      if (u_ == 0) a0 = v_;                                                                  \
      if (u_ == 1) a1 = v_;                                                                  \
      if (u_ == 2) a2 = v_;                                                                  \
      if (u_ == 3) a3 = v_;                                                                  \
    }                                                                                        \
  } while (0)
#define FK_F32_STORE4(T, a0, a1, a2, a3)                                                     \
  do {                                                                                       \
    _Pragma("unroll") for (int u_ = 0; u_ < 4; ++u_) {                                       \
      const int i_ = threadIdx.x + 256 * u_, r_ = i_ / (NB / 4), c_ = (i_ - r_ * (NB / 4)) * 4; \
      *reinterpret_cast<float4*>((T) + r_ * LDT + c_) = u_ == 0 ? a0 : u_ == 1 ? a1 : u_ == 2 ? a2 : a3; \
    }                                                                                        \
  } while (0)

// Two tiles into LDS, all eight loads of a lane issued before any store (one memory latency).
__device__ __forceinline__ void load_tiles2(float* T0, const float* src0, int64_t ld0, float* T1, const float* src1,
                                            int64_t ld1) {
  float4 v0, v1, v2, v3, w0, w1, w2, w3;
  FK_F32_LOAD4(src0, ld0, v0, v1, v2, v3);
  FK_F32_LOAD4(src1, ld1, w0, w1, w2, w3);
  FK_F32_STORE4(T0, v0, v1, v2, v3);
  FK_F32_STORE4(T1, w0, w1, w2, w3);
}

// dst tile (+)= sign * acc
__device__ __forceinline__ void store_acc(float* dst, int64_t ld, const floatx4 acc[2][2], bool add, float sign) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = r0 + rb * 16 + 4 * (lane >> 4) + v;
        int c = c0 + cb * 16 + (lane & 15);
        float x = sign * acc[rb][cb][v];
        if (add) dst[r * ld + c] += x;
        else dst[r * ld + c] = x;
      }
}

// acc[t] += As Bt^T over the 64 k of split tiles (t = 0: B0, t = 1: B1), for the 2 x 2 blocks of
// 16 x 16 a wave owns (rows 32 (w >> 1).., columns 32 (w & 1)..): hi*hi into acc, hi*lo + lo*hi into
// accx.  For v_mfma_f32_16x16x32_f16 lane l supplies row l % 16 of A and column l % 16 of B at the
// 8 k of its lane group l / 16 (the same 8 for both operands); its result layout is the one of
// the FP32 instruction above.
template <int NBT>
__device__ __forceinline__ void mfma_split64(const SplitTile& As, const SplitTile& B0, const SplitTile& B1,
                                             floatx4 (&acc)[NBT][2][2], floatx4 (&accx)[NBT][2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  const int li = lane & 15, kq = 8 * (lane >> 4);
#pragma unroll
  for (int k = 0; k < NB; k += 32) {
    half8 ah[2], al[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int o = split_off(r0 + 16 * u + li, k + kq);
      ah[u] = *reinterpret_cast<const half8*>(&As.hi[o]);
      al[u] = *reinterpret_cast<const half8*>(&As.lo[o]);
    }
#pragma unroll
    for (int t = 0; t < NBT; ++t) {
      const SplitTile& Bt = t == 0 ? B0 : B1;
      half8 bh[2], bl[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int o = split_off(c0 + 16 * u + li, k + kq);
        bh[u] = *reinterpret_cast<const half8*>(&Bt.hi[o]);
        bl[u] = *reinterpret_cast<const half8*>(&Bt.lo[o]);
      }
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[t][rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[rb], bh[cb], acc[t][rb][cb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          accx[t][rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[rb], bl[cb], accx[t][rb][cb], 0, 0, 0);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          accx[t][rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[rb], bh[cb], accx[t][rb][cb], 0, 0, 0);
    }
  }
}

// dst tile -= acc + 2^-11 accx
__device__ __forceinline__ void store_split_update(float* dst, int64_t ld, const floatx4 (&acc)[2][2],
                                                   const floatx4 (&accx)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + rb * 16 + 4 * (lane >> 4) + v;
        const int c = c0 + cb * 16 + (lane & 15);
        dst[r * ld + c] -= fmaf(accx[rb][cb][v], 1.f / kSplitScale, acc[rb][cb][v]);
      }
}

// dst tile = acc as packed FP16 pairs (a finished panel tile of the factor)
__device__ __forceinline__ void store_acc_split(float* dst, int64_t ld, const floatx4 acc[2][2]) {
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + rb * 16 + 4 * (lane >> 4) + v;
        const int c = c0 + cb * 16 + (lane & 15);
        d[r * ld + c] = split_pack(acc[rb][cb][v]);
      }
}

// ------------------------------------------------------------------ Cholesky kernels

// XCD-aware placement of a (rows x nlam) grid launched as one dimension.  The hardware deals the
// workgroups round-robin over the 8 XCDs (XCD = id mod 8); this bijection gives XCD x the
// consecutive run of pairs (lambda, row) in the order (lambda mod 8, lambda / 8, row), so that the
// workgroups of one lambda share one L2, which then holds the column tiles they all read.  Any
// dealing order gives the same result; only the locality depends on it.
__device__ __forceinline__ void xcd_place(int rows, int nlam, int* lam, int* row) {
  const int G = rows * nlam, id = blockIdx.x;
  const int x = id & 7, slot = id >> 3;
  int off = 0;   // workgroups dealt to the XCDs before x
  for (int y = 0; y < x; ++y) off += (G - y + 7) >> 3;
  const int q = off + slot;
  int c = 0, base = 0;   // lambda class c = lambda mod 8 holds ceil((nlam - c) / 8) lambdas
  while (c < 7) {
    const int n = ((nlam - c + 7) >> 3) * rows;
    if (q < base + n) break;
    base += n;
    ++c;
  }
  const int r = q - base;
  *lam = c + 8 * (r / rows);
  *row = r % rows;
}

// 1/x for a positive normal x: hardware reciprocal and two Newton steps
// (r <- r + r (1 - x r)), a few ulp in FP64.
__device__ inline double recip64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double recip_t(double x) { return recip64(x); }
// 1/x for a positive normal FP32 x: hardware reciprocal and one Newton step (about 1 ulp).
__device__ inline float recip_t(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// The same update for the two block columns kb and kb + 1 at once, over the panels
// k < kb:  A[i][kb] -= sum L[i][k] L[kb][k]^T  and (i > kb) A[i][kb+1] -= sum
// L[i][k] L[kb+1][k]^T.  The row panel L[i][.], the bulk of the traffic, is read once
// for both columns.  The finished panels are FP16 pairs (split tiles in LDS, products on the
// FP16 matrix cores); one LDS buffer per operand, the next k's tiles loaded into registers
// while the current ones are multiplied.
template <bool PART>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_left_update2(float* __restrict__ A,
                                                                                             int Np, int kb,
                                                                                             int nlam, int nsplit,
                                                                                             float* __restrict__ part) {
  __shared__ __align__(16) SplitTile As;
  __shared__ __align__(16) SplitTile B0;
  __shared__ __align__(16) SplitTile B1;
  const int rows = Np / NB - kb;
  int l, i, k0 = 0, k1 = kb, sidx = 0;
  if constexpr (PART) {
    // workgroup (sidx, l, i): panels k0 <= k < k1 of the split sidx of the sum
    const int b = blockIdx.x;
    i = b % rows;
    l = (b / rows) % nlam;
    sidx = b / (rows * nlam);
    k0 = (int)((int64_t)kb * sidx / nsplit);
    k1 = (int)((int64_t)kb * (sidx + 1) / nsplit);
  } else {
    xcd_place(rows, nlam, &l, &i);
  }
  i += kb;
  float* Al = A + (size_t)l * Np * Np;
  const uint32_t* Ai = reinterpret_cast<const uint32_t*>(Al + (size_t)i * NB * Np);
  const uint32_t* A0 = reinterpret_cast<const uint32_t*>(Al + (size_t)kb * NB * Np);
  const uint32_t* A1 = reinterpret_cast<const uint32_t*>(Al + (size_t)(kb + 1) * NB * Np);
  int off_g[4], off_s[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = threadIdx.x + q * 256, r = idx / (NB / 4), c = (idx % (NB / 4)) * 4;
    off_g[q] = r * Np + c;
    off_s[q] = split_off(r, c);
  }
  uint4 ra[4], rb[4], rc[4];
  auto gload = [&](int k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = *reinterpret_cast<const uint4*>(Ai + k * NB + off_g[q]);
      rb[q] = *reinterpret_cast<const uint4*>(A0 + k * NB + off_g[q]);
      rc[q] = *reinterpret_cast<const uint4*>(A1 + k * NB + off_g[q]);
    }
  };
  floatx4 acc[2][2][2] = {}, accx[2][2][2] = {};
  if (k0 < k1) gload(k0);
  for (int k = k0; k < k1; ++k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      split_stage(As, off_s[q], ra[q]);
      split_stage(B0, off_s[q], rb[q]);
      split_stage(B1, off_s[q], rc[q]);
    }
    __syncthreads();
    if (k + 1 < k1) gload(k + 1);
    mfma_split64<2>(As, B0, B1, acc, accx);
    __syncthreads();
  }
  if constexpr (PART) {
    // this split's part of the 64 x 128 update, row-major, columns kb then kb + 1
    float* dst = part + ((size_t)(sidx * nlam + l) * rows + (i - kb)) * (NB * 2 * NB);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = r0 + rb2 * 16 + 4 * (lane >> 4) + v;
            const int c = c0 + cb * 16 + (lane & 15);
            dst[r * (2 * NB) + t * NB + c] = fmaf(accx[t][rb2][cb][v], 1.f / kSplitScale, acc[t][rb2][cb][v]);
          }
  } else {
    store_split_update(Al + (size_t)i * NB * Np + kb * NB, Np, acc[0], accx[0]);
    if (i > kb) store_split_update(Al + (size_t)i * NB * Np + (kb + 1) * NB, Np, acc[1], accx[1]);
  }
}

// The split update's parts added in a fixed order (the result does not depend on timing) and
// subtracted from block columns kb, kb + 1 (the tile above the diagonal left alone).  Workgroup
// (tile, eighth): 256 threads x 4 consecutive entries; all parts of an entry are loaded before the
// first addition, so a workgroup waits for memory once.
constexpr int kMaxSplit = 16;
__global__ __launch_bounds__(256) void k_left_update2_sum(float* __restrict__ A, int Np, int kb, int nlam,
                                                          int nsplit, const float* __restrict__ part) {
  const int rows = Np / NB - kb;
  const int tile_id = blockIdx.x >> 3, eighth = blockIdx.x & 7;
  const int ii = tile_id % rows, l = tile_id / rows, i = kb + ii;
  const size_t tile = (size_t)NB * 2 * NB, stride = (size_t)nlam * rows * tile;
  const int e = (eighth * 256 + threadIdx.x) * 4, r = e / (2 * NB), c = e - r * (2 * NB);
  if (c >= NB && i == kb) return;   // above the diagonal (all four entries: c is a multiple of 4)
  const float* src = part + ((size_t)l * rows + ii) * tile + e;
  float4 v[kMaxSplit];
#pragma unroll
  for (int sp = 0; sp < kMaxSplit; ++sp)
    if (sp < nsplit) v[sp] = *reinterpret_cast<const float4*>(src + sp * stride);
  float4 sum = v[0];
#pragma unroll
  for (int sp = 1; sp < kMaxSplit; ++sp)
    if (sp < nsplit) {
      sum.x += v[sp].x;
      sum.y += v[sp].y;
      sum.z += v[sp].z;
      sum.w += v[sp].w;
    }
  float4* dst = reinterpret_cast<float4*>(A + (size_t)l * Np * Np + (size_t)i * NB * Np + kb * NB + (size_t)r * Np + c);
  float4 d = *dst;
  d.x -= sum.x;
  d.y -= sum.y;
  d.z -= sum.z;
  d.w -= sum.w;
  *dst = d;
}

// Factor the diagonal block kb of every lambda (one workgroup per lambda) in Real (FP32, or FP64
// when the launch shape asks for it); write L_kk (lower) back and inv(L_kk) to Linv[l][kb].
// Within the 64 x 64 block the sweep is right-looking:
// Thread (r, q) = (tid / 8, tid % 8) keeps entries r, q + 8u (u = 0..7) of the block, and
// of T below, in registers.  Unscaled: at step j column j has received every
// update, its owners publish it to P[.][j] (never written again), one barrier, and each row
// below applies a[r][k] -= f P[k][j] with f = P[r][j] / P[j][j].  Then L[r][c] = P[r][c] /
// sqrt(P[c][c]).  The same row operations turn the identity into T = diag(sqrt P) inv(L):
// T[i][c] = delta_ic - sum_{k<i} (P[i][k] / P[k][k]) T[k][c], so row j of T is final at step j,
// is published with column j (two-slot LDS buffer), and rows r > j take t[r][.] -= f T[j][.]
// in the same step: one sweep of 64 barriers for the factor and its inverse.
constexpr int kPotrfThreads = 512;
template <typename Real>
__global__ __launch_bounds__(kPotrfThreads) void k_potrf_diag(float* __restrict__ A, int Np, int kb,
                                                    float* __restrict__ Linv, int* flags) {
  __shared__ Real P[NB][NB + 1];
  __shared__ Real trow[2][NB];
  __shared__ Real piv[NB], sq[NB], rsq[NB];
  __shared__ int bad;
  constexpr int TPR = kPotrfThreads / NB, EPT = NB / TPR;   // threads per row, entries per thread
  const int l = blockIdx.x;
  float* Ab = A + (size_t)l * Np * Np + (size_t)kb * NB * Np + kb * NB;
  const int r = threadIdx.x / TPR, q = threadIdx.x % TPR;
  Real a[EPT], t[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int k = TPR * u + q;
    a[u] = (k <= r) ? (Real)Ab[(size_t)r * Np + k] : Real(0);
    t[u] = (k == r) ? Real(1) : Real(0);
  }
  if (threadIdx.x == 0) bad = 0;
  // unrolled, so that the register holding column j is known at compile time
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (q == (j % TPR) && r >= j) {
      Real v = a[0];
#pragma unroll
      for (int u = 1; u < EPT; ++u)
        if (u == (j / TPR)) v = a[u];
      P[r][j] = v;
    }
    if (r == j) {
#pragma unroll
      for (int u = 0; u < EPT; ++u) trow[j & 1][TPR * u + q] = t[u];
    }
    __syncthreads();
    // all loads first and unconditionally (rows k < j of P[.][j] are not yet written:
    // their values are discarded by the select), so the reads share one wait
    const Real pj = P[j][j];
    const Real prj = P[r][j];
    Real pk[EPT], tv[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      pk[u] = P[TPR * u + q][j];
      tv[u] = trow[j & 1][TPR * u + q];
    }
    const bool badj = !(pj > Real(0));  // non-positive or NaN pivot
    const Real rp = recip_t(badj ? Real(1) : pj);
    const Real f = r > j ? prj * rp : Real(0);
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int k = TPR * u + q;
      const Real upd = fma(-f, pk[u], a[u]);
      a[u] = (k > j && k <= r) ? upd : a[u];
      t[u] = fma(-f, tv[u], t[u]);   // T[j][c] = 0 for c > j: no change there
    }
    if (threadIdx.x == 0) {
      piv[j] = badj ? Real(1) : pj;
      if (badj) bad = 1;
    }
  }
  // t[] holds T[r][q + TPR u]
#pragma unroll
  for (int u = 0; u < EPT; ++u) a[u] = t[u];
  __syncthreads();   // the last pivot (thread 0, after the last step's barrier)
  if (threadIdx.x < NB) {
    const Real d = sqrt(piv[threadIdx.x]);
    sq[threadIdx.x] = d;
    rsq[threadIdx.x] = Real(1) / d;
  }
  __syncthreads();
  float* Li = Linv + ((size_t)l * (Np / NB) + kb) * NB * NB;
  const Real rs = rsq[r];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int c = TPR * u + q;
    Li[r * NB + c] = (c <= r) ? (float)(a[u] * rs) : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < NB * NB / kPotrfThreads; ++u) {
    const int i = threadIdx.x + kPotrfThreads * u, rr = i / NB, c = i - rr * NB;
    float v = 0.0f;
    if (c == rr) v = (float)sq[c];
    else if (c < rr) v = (float)(P[rr][c] * rsq[c]);
    Ab[(size_t)rr * Np + c] = v;
  }
  if (threadIdx.x == 0 && bad) {
    atomicOr(&flags[kFlagNotPD], 1);
    atomicMin(&flags[kFlagNotPD + 1], l);
  }
}

// Panel: L[i][kb] = A[i][kb] * inv(L_kk)^T for block rows i > kb.
__global__ __launch_bounds__(256) void k_trsm_panel(float* __restrict__ A, int Np, int kb,
                                                    const float* __restrict__ Linv, int nlam) {
  __shared__ float As[NB * LDT], Bs[NB * LDT];
  int l, ib;
  xcd_place(Np / NB - kb - 1, nlam, &l, &ib);
  ib += kb + 1;
  float* Al = A + (size_t)l * Np * Np;
  float* src = Al + (size_t)ib * NB * Np + kb * NB;
  const float* Li = Linv + ((size_t)l * (Np / NB) + kb) * NB * NB;
  load_tiles2(As, src, Np, Bs, Li, NB);
  __syncthreads();
  floatx4 acc[2][2] = {};
  mfma_tile64(As, Bs, acc);
  store_acc_split(src, Np, acc);   // finished: FP16 pairs for the updates and the solves
}

// Left-looking update of block column kb for every lambda (grid.y):
//   A[i][kb] -= sum_{k0 <= k < k1} L[i][k] L[kb][k]^T,   i = kb + blockIdx.x,
// the K loop over the finished panels (FP16 pairs, split tiles in LDS) with the next pair of
// tiles loaded into registers while the current pair is on the matrix cores.
__global__ __launch_bounds__(256) void k_left_update(float* __restrict__ A, int Np, int kb, int k0, int k1,
                                                     int nlam) {
  __shared__ __align__(16) SplitTile As;
  __shared__ __align__(16) SplitTile Bs;
  int l, i;
  xcd_place(Np / NB - kb, nlam, &l, &i);
  i += kb;
  float* Al = A + (size_t)l * Np * Np;
  const uint32_t* Ai = reinterpret_cast<const uint32_t*>(Al + (size_t)i * NB * Np);
  const uint32_t* Ak = reinterpret_cast<const uint32_t*>(Al + (size_t)kb * NB * Np);
  int off_g[4], off_s[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = threadIdx.x + q * 256, r = idx / (NB / 4), c = (idx % (NB / 4)) * 4;
    off_g[q] = r * Np + c;
    off_s[q] = split_off(r, c);
  }
  uint4 ra[4], rb[4];
  auto gload = [&](int k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = *reinterpret_cast<const uint4*>(Ai + k * NB + off_g[q]);
      rb[q] = *reinterpret_cast<const uint4*>(Ak + k * NB + off_g[q]);
    }
  };
  floatx4 acc[1][2][2] = {}, accx[1][2][2] = {};
  gload(k0);
  for (int k = k0; k < k1; ++k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      split_stage(As, off_s[q], ra[q]);
      split_stage(Bs, off_s[q], rb[q]);
    }
    __syncthreads();
    if (k + 1 < k1) gload(k + 1);
    mfma_split64<1>(As, Bs, Bs, acc, accx);
    __syncthreads();
  }
  store_split_update(Al + (size_t)i * NB * Np + kb * NB, Np, acc[0], accx[0]);
}

// ------------------------------------------------------------------ triangular solves (FP32)
// R, Y: [lambda][ncol][Np] (column-major per lambda: column t contiguous).

// MFMA product of a 64 x 64 LDS tile (or its transpose) with a 64 x (16*NCT) LDS
// block: wave w computes rows 16w..16w+15.  Lane layout as in mfma_tile64.
constexpr int LDB = 33;   // row stride of the 64 x ncol blocks (ncol <= 32)
template <bool TRANS, int NCT, bool ACC = false>
__device__ __forceinline__ void mfma_64xK(const float* Ls, const float (*Bs)[LDB], floatx4 acc[NCT]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (!ACC) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll 4
  for (int k0 = 0; k0 < NB; k0 += 4) {
    const float a = TRANS ? Ls[(k0 + lk) * LDT + 16 * w + li] : Ls[(16 * w + li) * LDT + k0 + lk];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const float b = Bs[k0 + lk][ct * 16 + li];
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[ct], 0, 0, 0);
    }
  }
}

// One 64 x 64 tile of a finished panel (FP16 pairs) in four uint4 registers per thread
// (256 threads: thread t holds the four entries number t + 256 u of the row-major tile),
// for loading the next tile of a sweep while the current one is on the matrix cores; the
// staging into LDS unpacks it to FP32.
#define FK_TILE_FETCH_TO(src, ld, a0, a1, a2, a3)                                            \
  do {                                                                                       \
    _Pragma("unroll") for (int u_ = 0; u_ < 4; ++u_) {                                       \
      const int i_ = threadIdx.x + 256 * u_, r_ = i_ / (NB / 4), c_ = (i_ - r_ * (NB / 4)) * 4; \
      const uint4 v_ = *reinterpret_cast<const uint4*>((src) + r_ * (ld) + c_);            \
      if (u_ == 0) a0 = v_;                                                                  \
      if (u_ == 1) a1 = v_;                                                                  \
      if (u_ == 2) a2 = v_;                                                                  \
      if (u_ == 3) a3 = v_;                                                                  \
    }                                                                                        \
  } while (0)
#define FK_TILE_STAGE_FROM(T, a0, a1, a2, a3)                                                \
  do {                                                                                       \
    _Pragma("unroll") for (int u_ = 0; u_ < 4; ++u_) {                                       \
      const int i_ = threadIdx.x + 256 * u_, r_ = i_ / (NB / 4), c_ = (i_ - r_ * (NB / 4)) * 4; \
      const uint4 q_ = u_ == 0 ? a0 : u_ == 1 ? a1 : u_ == 2 ? a2 : a3;                     \
      *reinterpret_cast<float4*>((T) + r_ * LDT + c_) =                                      \
          make_float4(split_unpack(q_.x), split_unpack(q_.y), split_unpack(q_.z), split_unpack(q_.w)); \
    }                                                                                        \
  } while (0)
#define FK_TILE_FETCH(src, ld) FK_TILE_FETCH_TO(src, ld, nt0, nt1, nt2, nt3)
#define FK_TILE_STAGE(T) FK_TILE_STAGE_FROM(T, nt0, nt1, nt2, nt3)

// Forward step kb of L y = r for every lambda (grid.y): y_kb = inv(L_kk) r_kb, written
// by block 0; block x then updates rows ib = kb + 1 + x, kb + 1 + x + gridDim.x, ...:
// r_ib -= L[ib][kb] y_kb, with the next row's tile loaded while the current one is
// multiplied (two LDS buffers, one barrier per row).
template <int NCT>
__global__ __launch_bounds__(256) void k_fwd_mfma(const float* __restrict__ A, int Np, int kb,
                                                  const float* __restrict__ Linv, float* __restrict__ R,
                                                  float* __restrict__ Y, int ncol) {
  __shared__ float Ls[2][NB * LDT];
  __shared__ float Bs[NB][LDB];
  const int l = blockIdx.y;
  const int nb = Np / NB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float* Rl = R + (size_t)l * ncol * Np;
  const float* Al = A + (size_t)l * Np * Np;
  // every load of the prologue goes out before any is used
  int ib = kb + 1 + blockIdx.x;
  uint4 nt0, nt1, nt2, nt3;
  if (ib < nb) FK_TILE_FETCH(Al + (size_t)ib * NB * Np + kb * NB, Np);
  constexpr int NBS = NB * 16 * NCT / 256;   // right-hand-side entries per thread
  float bsv[NBS];
#pragma unroll
  for (int u = 0; u < NBS; ++u) {
    const int i = threadIdx.x + 256 * u, t = i / NB, k = i - t * NB;
    bsv[u] = t < ncol ? Rl[(size_t)t * Np + kb * NB + k] : 0.f;
  }
  float4 d0, d1, d2, d3;
  FK_F32_LOAD4(Linv + ((size_t)l * nb + kb) * NB * NB, NB, d0, d1, d2, d3);
#pragma unroll
  for (int u = 0; u < NBS; ++u) {
    const int i = threadIdx.x + 256 * u, t = i / NB, k = i - t * NB;
    Bs[k][t] = bsv[u];
  }
  FK_F32_STORE4(Ls[0], d0, d1, d2, d3);
  __syncthreads();
  floatx4 acc[NCT];
  mfma_64xK<false, NCT>(Ls[0], Bs, acc);
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[16 * w + 4 * lk + v][ct * 16 + li] = acc[ct][v];
  if (ib < nb) FK_TILE_STAGE(Ls[1]);
  __syncthreads();
  if (blockIdx.x == 0) {
    float* Yl = Y + (size_t)l * ncol * Np;
    for (int i = threadIdx.x; i < ncol * NB; i += blockDim.x) {
      const int t = i / NB, r = i - t * NB;
      Yl[(size_t)t * Np + kb * NB + r] = Bs[r][t];
    }
  }
  // this lane's part of the right-hand-side block of a row: 4 rows x NCT columns
  float rr[NCT][4];
#define FK_R_FETCH(RB)                                                                         \
  _Pragma("unroll") for (int ct = 0; ct < NCT; ++ct) {                                         \
    const int t_ = min(ct * 16 + li, ncol - 1);                                                \
    _Pragma("unroll") for (int v = 0; v < 4; ++v)                                              \
      rr[ct][v] = Rl[(size_t)t_ * Np + (RB) * NB + 16 * w + 4 * lk + v];                       \
  }
  if (ib < nb) FK_R_FETCH(ib)
  int cur = 1;
  for (; ib < nb; ib += gridDim.x) {
    const int nx = ib + gridDim.x;
    if (nx < nb) FK_TILE_FETCH(Al + (size_t)nx * NB * Np + kb * NB, Np);
    mfma_64xK<false, NCT>(Ls[cur], Bs, acc);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = ct * 16 + li;
        if (t < ncol) Rl[(size_t)t * Np + ib * NB + 16 * w + 4 * lk + v] = rr[ct][v] - acc[ct][v];
      }
    if (nx < nb) FK_R_FETCH(nx)
    if (nx < nb) FK_TILE_STAGE(Ls[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
  }
#undef FK_R_FETCH
}

// Backward step kb of L^T x = y: x_kb = inv(L_kk)^T y_kb (block 0 writes X); block x
// then updates rows jb = x, x + gridDim.x, ... < kb: y_jb -= L[kb][jb]^T x_kb, the
// next row's tile loaded while the current one is multiplied.
template <int NCT>
__global__ __launch_bounds__(256) void k_bwd_mfma(const float* __restrict__ A, int Np, int kb,
                                                  const float* __restrict__ Linv, float* __restrict__ Yv,
                                                  float* __restrict__ X, int ncol) {
  __shared__ float Ls[2][NB * LDT];
  __shared__ float Bs[NB][LDB];
  const int l = blockIdx.y;
  const int nb = Np / NB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float* Yl = Yv + (size_t)l * ncol * Np;
  const float* Ak = A + (size_t)l * Np * Np + (size_t)kb * NB * Np;
  // every load of the prologue goes out before any is used
  int jb = blockIdx.x;
  uint4 nt0, nt1, nt2, nt3;
  if (jb < kb) FK_TILE_FETCH(Ak + jb * NB, Np);
  constexpr int NBS = NB * 16 * NCT / 256;   // right-hand-side entries per thread
  float bsv[NBS];
#pragma unroll
  for (int u = 0; u < NBS; ++u) {
    const int i = threadIdx.x + 256 * u, t = i / NB, k = i - t * NB;
    bsv[u] = t < ncol ? Yl[(size_t)t * Np + kb * NB + k] : 0.f;
  }
  float4 d0, d1, d2, d3;
  FK_F32_LOAD4(Linv + ((size_t)l * nb + kb) * NB * NB, NB, d0, d1, d2, d3);
#pragma unroll
  for (int u = 0; u < NBS; ++u) {
    const int i = threadIdx.x + 256 * u, t = i / NB, k = i - t * NB;
    Bs[k][t] = bsv[u];
  }
  FK_F32_STORE4(Ls[0], d0, d1, d2, d3);
  __syncthreads();
  floatx4 acc[NCT];
  mfma_64xK<true, NCT>(Ls[0], Bs, acc);
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[16 * w + 4 * lk + v][ct * 16 + li] = acc[ct][v];
  if (jb < kb) FK_TILE_STAGE(Ls[1]);
  __syncthreads();
  if (blockIdx.x == 0) {
    float* Xl = X + (size_t)l * ncol * Np;
    for (int i = threadIdx.x; i < ncol * NB; i += blockDim.x) {
      const int t = i / NB, r = i - t * NB;
      Xl[(size_t)t * Np + kb * NB + r] = Bs[r][t];
    }
  }
  float rr[NCT][4];
#define FK_R_FETCH(RB)                                                                         \
  _Pragma("unroll") for (int ct = 0; ct < NCT; ++ct) {                                         \
    const int t_ = min(ct * 16 + li, ncol - 1);                                                \
    _Pragma("unroll") for (int v = 0; v < 4; ++v)                                              \
      rr[ct][v] = Yl[(size_t)t_ * Np + (RB) * NB + 16 * w + 4 * lk + v];                       \
  }
  if (jb < kb) FK_R_FETCH(jb)
  int cur = 1;
  for (; jb < kb; jb += gridDim.x) {
    const int nx = jb + gridDim.x;
    if (nx < kb) FK_TILE_FETCH(Ak + nx * NB, Np);
    mfma_64xK<true, NCT>(Ls[cur], Bs, acc);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = ct * 16 + li;
        if (t < ncol) Yl[(size_t)t * Np + jb * NB + 16 * w + 4 * lk + v] = rr[ct][v] - acc[ct][v];
      }
    if (nx < kb) FK_R_FETCH(nx)
    if (nx < kb) FK_TILE_STAGE(Ls[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
  }
#undef FK_R_FETCH
}


// Two forward steps kb, kb + 1 in one launch (kb + 1 < nb).  Every workgroup solves the 128-row
// diagonal part itself: y_kb = inv(L_kk) r_kb, then r_{kb+1} -= L[kb+1][kb] y_kb and y_{kb+1} =
// inv(L_{kb+1,kb+1}) r_{kb+1}; block 0 writes both blocks of Y.  Block x then updates rows ib = kb + 2
// + x, kb + 2 + x + gridDim.x, ...: r_ib -= L[ib][kb] y_kb + L[ib][kb+1] y_{kb+1}, the tiles streamed
// through the two LDS buffers in the order (ib, kb), (ib, kb + 1), (next ib, kb), ... (one barrier
// per tile).  Half the dependent launches of the one-step sweep.
template <int NCT>
__global__ __launch_bounds__(256) void k_fwd2_mfma(const float* __restrict__ A, int Np, int kb,
                                                   const float* __restrict__ Linv, float* __restrict__ R,
                                                   float* __restrict__ Y, int ncol) {
  __shared__ float Ls[2][NB * LDT];
  __shared__ float Bs[2 * NB][LDB];
  const int l = blockIdx.y;
  const int nb = Np / NB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float* Rl = R + (size_t)l * ncol * Np;
  const float* Al = A + (size_t)l * Np * Np;
  const int ib0 = kb + 2 + blockIdx.x;
  // Every global load of the two diagonal steps and of the first row goes out here, before any
  // is used: the prologue waits for memory once instead of three times.
  constexpr int NBS = 2 * NB * 16 * NCT / 256;   // right-hand-side entries per thread
  float bsv[NBS];
#pragma unroll
  for (int u = 0; u < NBS; ++u) {
    const int i = threadIdx.x + 256 * u, t = i / (2 * NB), k = i - t * (2 * NB);
    bsv[u] = t < ncol ? Rl[(size_t)t * Np + kb * NB + k] : 0.f;
  }
  float4 d00, d01, d02, d03, d10, d11, d12, d13;
  FK_F32_LOAD4(Linv + ((size_t)l * nb + kb) * NB * NB, NB, d00, d01, d02, d03);
  FK_F32_LOAD4(Linv + ((size_t)l * nb + kb + 1) * NB * NB, NB, d10, d11, d12, d13);
  uint4 nt0, nt1, nt2, nt3, ns0, ns1, ns2, ns3;
  FK_TILE_FETCH(Al + (size_t)(kb + 1) * NB * Np + kb * NB, Np);
  if (ib0 < nb) FK_TILE_FETCH_TO(Al + (size_t)ib0 * NB * Np + kb * NB, Np, ns0, ns1, ns2, ns3);
  // this lane's part of the right-hand-side block of a row: 4 rows x NCT columns
  float rr[NCT][4];
#define FK_R_FETCH(RB)                                                                         \
  _Pragma("unroll") for (int ct = 0; ct < NCT; ++ct) {                                         \
    const int t_ = min(ct * 16 + li, ncol - 1);                                                \
    _Pragma("unroll") for (int v = 0; v < 4; ++v)                                              \
      rr[ct][v] = Rl[(size_t)t_ * Np + (RB) * NB + 16 * w + 4 * lk + v];                       \
  }
  if (ib0 < nb) FK_R_FETCH(ib0)
#pragma unroll
  for (int u = 0; u < NBS; ++u) {
    const int i = threadIdx.x + 256 * u, t = i / (2 * NB), k = i - t * (2 * NB);
    Bs[k][t] = bsv[u];
  }
  FK_F32_STORE4(Ls[0], d00, d01, d02, d03);
  FK_TILE_STAGE(Ls[1]);
  __syncthreads();
  floatx4 acc[NCT];
  mfma_64xK<false, NCT>(Ls[0], Bs, acc);   // y_kb
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[16 * w + 4 * lk + v][ct * 16 + li] = acc[ct][v];
  __syncthreads();
  mfma_64xK<false, NCT>(Ls[1], Bs, acc);   // L[kb+1][kb] y_kb
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[NB + 16 * w + 4 * lk + v][ct * 16 + li] -= acc[ct][v];
  FK_F32_STORE4(Ls[0], d10, d11, d12, d13);
  __syncthreads();
  mfma_64xK<false, NCT>(Ls[0], Bs + NB, acc);   // y_{kb+1}
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[NB + 16 * w + 4 * lk + v][ct * 16 + li] = acc[ct][v];
  if (ib0 < nb) FK_TILE_STAGE_FROM(Ls[1], ns0, ns1, ns2, ns3);
  __syncthreads();
  if (blockIdx.x == 0) {
    float* Yl = Y + (size_t)l * ncol * Np;
    for (int i = threadIdx.x; i < ncol * 2 * NB; i += blockDim.x) {
      const int t = i / (2 * NB), r = i - t * (2 * NB);
      Yl[(size_t)t * Np + kb * NB + r] = Bs[r][t];
    }
  }
  int cur = 1;
  for (int ib = ib0; ib < nb; ib += gridDim.x) {
    // tile (ib, kb) is in Ls[cur]; (ib, kb + 1) comes next
    FK_TILE_FETCH(Al + (size_t)ib * NB * Np + (kb + 1) * NB, Np);
    mfma_64xK<false, NCT>(Ls[cur], Bs, acc);
    FK_TILE_STAGE(Ls[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
    const int nx = ib + gridDim.x;
    if (nx < nb) FK_TILE_FETCH(Al + (size_t)nx * NB * Np + kb * NB, Np);
    mfma_64xK<false, NCT, true>(Ls[cur], Bs + NB, acc);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = ct * 16 + li;
        if (t < ncol) Rl[(size_t)t * Np + ib * NB + 16 * w + 4 * lk + v] = rr[ct][v] - acc[ct][v];
      }
    if (nx < nb) FK_R_FETCH(nx)
    if (nx < nb) FK_TILE_STAGE(Ls[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
  }
#undef FK_R_FETCH
}

// Two backward steps kb, kb - 1 in one launch (kb >= 1): x_kb = inv(L_kk)^T y_kb, then y_{kb-1} -=
// L[kb][kb-1]^T x_kb and x_{kb-1} = inv(L_{kb-1,kb-1})^T y_{kb-1} in every workgroup (block 0 writes
// both blocks of X); block x then updates rows jb = x, x + gridDim.x, ... < kb - 1: y_jb -= L[kb][jb]^T
// x_kb + L[kb-1][jb]^T x_{kb-1}, the two tiles of a row streamed one after the other.
template <int NCT>
__global__ __launch_bounds__(256) void k_bwd2_mfma(const float* __restrict__ A, int Np, int kb,
                                                   const float* __restrict__ Linv, float* __restrict__ Yv,
                                                   float* __restrict__ X, int ncol) {
  __shared__ float Ls[2][NB * LDT];
  __shared__ float Bs[2 * NB][LDB];
  const int l = blockIdx.y;
  const int nb = Np / NB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float* Yl = Yv + (size_t)l * ncol * Np;
  const float* Ak = A + (size_t)l * Np * Np + (size_t)kb * NB * Np;         // block row kb
  const float* Ak1 = A + (size_t)l * Np * Np + (size_t)(kb - 1) * NB * Np;  // block row kb - 1
  const int jb0 = blockIdx.x;
  // every global load of the two diagonal steps and of the first row goes out here
  constexpr int NBS = 2 * NB * 16 * NCT / 256;   // right-hand-side entries per thread
  float bsv[NBS];
#pragma unroll
  for (int u = 0; u < NBS; ++u) {
    const int i = threadIdx.x + 256 * u, t = i / (2 * NB), k = i - t * (2 * NB);
    const int row = k < NB ? kb * NB + k : (kb - 1) * NB + (k - NB);
    bsv[u] = t < ncol ? Yl[(size_t)t * Np + row] : 0.f;
  }
  float4 d00, d01, d02, d03, d10, d11, d12, d13;
  FK_F32_LOAD4(Linv + ((size_t)l * nb + kb) * NB * NB, NB, d00, d01, d02, d03);
  FK_F32_LOAD4(Linv + ((size_t)l * nb + kb - 1) * NB * NB, NB, d10, d11, d12, d13);
  uint4 nt0, nt1, nt2, nt3, ns0, ns1, ns2, ns3;
  FK_TILE_FETCH(Ak + (kb - 1) * NB, Np);   // L[kb][kb-1]
  if (jb0 < kb - 1) FK_TILE_FETCH_TO(Ak + jb0 * NB, Np, ns0, ns1, ns2, ns3);
  float rr[NCT][4];
#define FK_R_FETCH(RB)                                                                         \
  _Pragma("unroll") for (int ct = 0; ct < NCT; ++ct) {                                         \
    const int t_ = min(ct * 16 + li, ncol - 1);                                                \
    _Pragma("unroll") for (int v = 0; v < 4; ++v)                                              \
      rr[ct][v] = Yl[(size_t)t_ * Np + (RB) * NB + 16 * w + 4 * lk + v];                       \
  }
  if (jb0 < kb - 1) FK_R_FETCH(jb0)
#pragma unroll
  for (int u = 0; u < NBS; ++u) {
    const int i = threadIdx.x + 256 * u, t = i / (2 * NB), k = i - t * (2 * NB);
    Bs[k][t] = bsv[u];
  }
  FK_F32_STORE4(Ls[0], d00, d01, d02, d03);
  FK_TILE_STAGE(Ls[1]);
  __syncthreads();
  floatx4 acc[NCT];
  mfma_64xK<true, NCT>(Ls[0], Bs, acc);   // x_kb
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[16 * w + 4 * lk + v][ct * 16 + li] = acc[ct][v];
  __syncthreads();
  mfma_64xK<true, NCT>(Ls[1], Bs, acc);   // L[kb][kb-1]^T x_kb
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[NB + 16 * w + 4 * lk + v][ct * 16 + li] -= acc[ct][v];
  FK_F32_STORE4(Ls[0], d10, d11, d12, d13);
  __syncthreads();
  mfma_64xK<true, NCT>(Ls[0], Bs + NB, acc);   // x_{kb-1}
  __syncthreads();
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[NB + 16 * w + 4 * lk + v][ct * 16 + li] = acc[ct][v];
  if (jb0 < kb - 1) FK_TILE_STAGE_FROM(Ls[1], ns0, ns1, ns2, ns3);
  __syncthreads();
  if (blockIdx.x == 0) {
    float* Xl = X + (size_t)l * ncol * Np;
    for (int i = threadIdx.x; i < ncol * 2 * NB; i += blockDim.x) {
      const int t = i / (2 * NB), k = i - t * (2 * NB);
      const int row = k < NB ? kb * NB + k : (kb - 1) * NB + (k - NB);
      Xl[(size_t)t * Np + row] = Bs[k][t];
    }
  }
  int cur = 1;
  for (int jb = jb0; jb < kb - 1; jb += gridDim.x) {
    // tile (kb, jb) is in Ls[cur]; (kb - 1, jb) comes next
    FK_TILE_FETCH(Ak1 + jb * NB, Np);
    mfma_64xK<true, NCT>(Ls[cur], Bs, acc);
    FK_TILE_STAGE(Ls[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
    const int nx = jb + gridDim.x;
    if (nx < kb - 1) FK_TILE_FETCH(Ak + nx * NB, Np);
    mfma_64xK<true, NCT, true>(Ls[cur], Bs + NB, acc);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = ct * 16 + li;
        if (t < ncol) Yl[(size_t)t * Np + jb * NB + 16 * w + 4 * lk + v] = rr[ct][v] - acc[ct][v];
      }
    if (nx < kb - 1) FK_R_FETCH(nx)
    if (nx < kb - 1) FK_TILE_STAGE(Ls[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
  }
#undef FK_R_FETCH
}


// ------------------------------------------------------------------ FP64 residual
// Rres[l][t] = Bre[t] - (H64 + lambda_l diag(preal)) X[l][t], for all (l, t) at once:
// one FP64 GEMM H64 (Np x Np) times X (Np x ncolsTotal), then the diagonal and the
// subtraction.  Column c of X/Rres is (l, t) with l = c / ntgt.
// On the FP64 matrix cores (v_mfma_f64_16x16x4f64): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; element v of lane l's accumulator is D[l / 16 + 4 v][l % 16]
// (the FP32 form holds D[4 (l / 16) + v][l % 16] instead).  A workgroup computes 64 rows
// x 32 WN columns, its four waves 32 rows x 16 WN columns each (2 x WN blocks of
// 16 x 16).  The k dimension streams in chunks of 16 through double-buffered LDS (the
// next chunk in registers meanwhile).  Every operand value read from LDS feeds 16
// multiply-adds (a 4 x 4 register block on the vector units gets 2), so the kernel is
// bound by the FP64 matrix rate.
template <int WN>
__global__ __launch_bounds__(256) void k_resid64_mfma(const double* __restrict__ H, int N, int Np,
                                                      const double* __restrict__ X, int ncols, int ntgt,
                                                      int rhs_per_col, const double* __restrict__ Bre,
                                                      const double* __restrict__ preal,
                                                      const double* __restrict__ lams, double* __restrict__ Rres) {
  constexpr int TM = 64, TN = 32 * WN, KC = 16;
  constexpr int PH = TM * KC / 256, PX = TN * KC / 256;
  __shared__ double Hs[2][KC][TM + 4];  // Hs[k][row]
  __shared__ double Xs[2][KC][TN + 4];  // Xs[k][col]
  const int row0 = blockIdx.x * TM, col0 = blockIdx.y * TN;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 16 * WN;
  const int li = lane & 15, lk = lane >> 4;
  // global element e = tid + 256 u of a chunk: (row or column e / 16, k e % 16)
  const int gk = threadIdx.x & (KC - 1), gr = threadIdx.x >> 4;
  const int cmax = ncols - 1;
  double ph[PH], px[PX];
#define FK_RLOAD(k0)                                                                              \
  do {                                                                                            \
    _Pragma("unroll") for (int u = 0; u < PH; ++u)                                                \
      ph[u] = H[(size_t)(row0 + gr + 16 * u) * Np + (k0) + gk];                                  \
    _Pragma("unroll") for (int u = 0; u < PX; ++u)                                                \
      px[u] = X[(size_t)min(col0 + gr + 16 * u, cmax) * Np + (k0) + gk];                         \
  } while (0)
#define FK_RSTORE(buf)                                                                            \
  do {                                                                                            \
    _Pragma("unroll") for (int u = 0; u < PH; ++u) Hs[buf][gk][gr + 16 * u] = ph[u];              \
    _Pragma("unroll") for (int u = 0; u < PX; ++u)                                                \
      Xs[buf][gk][gr + 16 * u] = (col0 + gr + 16 * u <= cmax) ? px[u] : 0.0;                      \
  } while (0)
  doublex4 acc[2][WN];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  FK_RLOAD(0);
  FK_RSTORE(0);
  __syncthreads();
  const int nk = Np / KC;
  for (int kc = 0; kc < nk; ++kc) {
    const int cur = kc & 1;
    if (kc + 1 < nk) FK_RLOAD((kc + 1) * KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      double a[2], b[WN];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = Hs[cur][ks + lk][wr + 16 * i + li];
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = Xs[cur][ks + lk][wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kc + 1 < nk) FK_RSTORE(cur ^ 1);
    __syncthreads();
  }
#undef FK_RLOAD
#undef FK_RSTORE
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int c = col0 + wc + 16 * j + li;
    if (c >= ncols) continue;
    const int l = c / ntgt, t = c - l * ntgt;
    const double lam = lams[l];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = row0 + wr + 16 * i + lk + 4 * v;
        const double xv = X[(size_t)c * Np + r];
        const double ax = acc[i][j][v] + (r < N ? lam * preal[r] * xv : 0.0);
        const double bv = (r < N) ? Bre[(size_t)(rhs_per_col ? c : t) * Np + r] : 0.0;
        Rres[(size_t)c * Np + r] = bv - ax;
      }
  }
}

// Same residual for a few columns (ncols <= 8): one wave per row streams the row of
// H64 once (coalesced) against all columns; the tiled kernel above would leave
// most of each column tile empty.
constexpr int NARROW = 8;
__global__ __launch_bounds__(256) void k_resid64_narrow(const double* __restrict__ H, int N, int Np,
                                                        const double* __restrict__ X, int ncols, int ntgt,
                                                        int rhs_per_col, const double* __restrict__ Bre,
                                                        const double* __restrict__ preal,
                                                        const double* __restrict__ lams, double* __restrict__ Rres) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= Np) return;
  double acc[NARROW];
#pragma unroll
  for (int c = 0; c < NARROW; ++c) acc[c] = 0.0;
  const double* h = H + (size_t)r * Np;
  for (int k = lane; k < Np; k += 64) {
    const double hv = h[k];
#pragma unroll
    for (int c = 0; c < NARROW; ++c)
      if (c < ncols) acc[c] = fma(hv, X[(size_t)c * Np + k], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < NARROW; ++c)
    for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
  if (lane < ncols) {
    const int c = lane;
    double a = 0.0;
#pragma unroll
    for (int cc = 0; cc < NARROW; ++cc)
      if (cc == c) a = acc[cc];
    const int l = c / ntgt, t = c - l * ntgt;
    const double xv = X[(size_t)c * Np + r];
    const double ax = a + (r < N ? lams[l] * preal[r] * xv : 0.0);
    const double bv = (r < N) ? Bre[(size_t)(rhs_per_col ? c : t) * Np + r] : 0.0;
    Rres[(size_t)c * Np + r] = bv - ax;
  }
}

static void launch_resid(hipStream_t st, const double* H, int N, int Np, const double* X, int ncols, int ntgt,
                         int rhs_per_col, const double* Bre, const double* preal, const double* lams, double* R) {
  if (ncols <= NARROW) {
    hipLaunchKernelGGL(k_resid64_narrow, dim3((Np + 3) / 4), dim3(256), 0, st, H, N, Np, X, ncols, ntgt,
                       rhs_per_col, Bre, preal, lams, R);
    return;
  }
  // Column tile of 32 WN: the one with the fewest tile columns per CU, counting every CU's last
  // round as full (ceil(tiles / 256 CUs) rounds x TN columns of work each); ties to the wider tile,
  // which reuses each loaded H value more.  For 1024 columns: WN = 3 (737 tiles, 3 rounds x 96)
  // against WN = 4 (536 tiles, 3 rounds x 128).
  int best_wn = 4;
  long best = -1;
  for (int wn = 4; wn >= 2; --wn) {
    const long tiles = (long)(Np / 64) * ((ncols + 32 * wn - 1) / (32 * wn));
    const long cost = (tiles + 255) / 256 * (32 * wn);
    if (best < 0 || cost < best) {
      best = cost;
      best_wn = wn;
    }
  }
  const int TN = 32 * best_wn;
  const dim3 grid(Np / 64, (ncols + TN - 1) / TN);
  if (best_wn == 4)
    hipLaunchKernelGGL(k_resid64_mfma<4>, grid, dim3(256), 0, st, H, N, Np, X, ncols, ntgt, rhs_per_col, Bre, preal,
                       lams, R);
  else if (best_wn == 3)
    hipLaunchKernelGGL(k_resid64_mfma<3>, grid, dim3(256), 0, st, H, N, Np, X, ncols, ntgt, rhs_per_col, Bre, preal,
                       lams, R);
  else
    hipLaunchKernelGGL(k_resid64_mfma<2>, grid, dim3(256), 0, st, H, N, Np, X, ncols, ntgt, rhs_per_col, Bre, preal,
                       lams, R);
}

// Column norms squared of Rres and of the right-hand sides (per column), FP64.
__global__ __launch_bounds__(256) void k_colnorm2(const double* __restrict__ V, int Np, double* __restrict__ out) {
  __shared__ double part[256];
  const double* v = V + (size_t)blockIdx.x * Np;
  double s = 0.0;
  for (int i = threadIdx.x; i < Np; i += blockDim.x) s += v[i] * v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// b = (float)(S a) and x += S d, with the per-lambda scaling; element i is
// (lambda, target, row) = (i / (ntgt Np), ., i % Np).
__global__ void k_scale_d2f(const double* __restrict__ a, const double* __restrict__ scl, int Np, int ntgt,
                            float* __restrict__ b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t l = i / ((int64_t)ntgt * Np);
  int r = (int)(i % Np);
  b[i] = (float)(a[i] * scl[l * Np + r]);
}
__global__ void k_scale_axpy_f2d(const float* __restrict__ a, const double* __restrict__ scl, int Np, int ntgt,
                                 double* __restrict__ b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t l = i / ((int64_t)ntgt * Np);
  int r = (int)(i % Np);
  b[i] += scl[l * Np + r] * (double)a[i];
}
__global__ void k_rep_rhs(const double* __restrict__ Bre, int Np, int ntgt, int nlam, double* __restrict__ R) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)nlam * ntgt * Np;
  if (i >= tot) return;
  int64_t c = i / Np;
  int t = (int)(c % ntgt);
  R[i] = Bre[(size_t)t * Np + (i - c * Np)];
}

}  // namespace fk

// ==================================================================== host drivers
namespace fk {

static int round64(int n) { return (n + NB - 1) / NB * NB; }

SolveLayout solve_layout(int N, int nlam, int ntgt, void* base, size_t cap) {
  SolveLayout s;
  s.N = N;
  s.Np = round64(N);
  s.nlam = nlam;
  s.ntgt = ntgt;
  const size_t Np = s.Np;
  const size_t nc = (size_t)nlam * ntgt;
  Carve cv(base, cap);
  s.H64 = cv.take<double>(Np * Np);
  s.A32 = cv.take<float>((size_t)nlam * Np * Np);
  s.Linv = cv.take<float>((size_t)nlam * Np * NB);
  s.preal = cv.take<double>(Np);
  s.lams = cv.take<double>(nlam);
  s.Bre = cv.take<double>((size_t)ntgt * Np);
  s.X64 = cv.take<double>(nc * Np);
  s.R64 = cv.take<double>(nc * Np);
  s.U64 = cv.take<double>(nc * Np);
  s.G64 = cv.take<double>(nc * Np);
  s.Gadj = cv.take<double>(nc * Np);
  s.R32 = cv.take<float>(nc * Np);
  s.Y32 = cv.take<float>(nc * Np);
  s.D32 = cv.take<float>(nc * Np);
  s.norms = cv.take<double>(2 * nc + nlam + 64);
  s.Hv = cv.take<double>(Np * Np);
  s.Bv = cv.take<double>((size_t)ntgt * Np);
  s.pcx = cv.take<double>((size_t)N);
  s.scl = cv.take<double>((size_t)nlam * Np);
  s.dsym = cv.take<double>((size_t)2 * N);
  // parts of the split paired updates: 768 tiles of 64 x 128 at most (fewer for small systems)
  const int nb = (int)(Np / NB);
  s.part_tiles = (int)std::min<int64_t>(768, (int64_t)nb * nb * nlam);
  s.upart = cv.take<float>((size_t)s.part_tiles * NB * 2 * NB);
  s.bytes = ((cv.off + 255) & ~size_t(255)) + 256;   // a multiple of 256: what follows stays aligned
  return s;
}

// Splits of the paired update's sum over panels when its grid is small (few lambdas, or the last
// block columns): about three workgroups per CU in all, at least two panels per split, within the
// workspace's part tiles.  1 = no split.
static int update_split(int wgs, int kb, int part_tiles) {
  if (wgs >= 512 || kb < 4) return 1;
  int ns = std::min(std::min(kb / 2, kMaxSplit), 768 / wgs);
  ns = std::min(ns, part_tiles / wgs);
  return std::max(ns, 1);
}

// Factor A32[l] = L L^T for every lambda: left-looking blocked Cholesky, per block column an
// update with the finished panels (one pass over the column), the factorization of the
// diagonal block, the solve of the panel below it.
static fk_status factor_all(fk_ctx* ctx, const SolveLayout& s, const DenseShape& sh) {
  const int nb = s.Np / NB;
  auto finish = [&](int kb) {   // diagonal block and the panel below it
    if (sh.diag64)
      hipLaunchKernelGGL(k_potrf_diag<double>, dim3(s.nlam), dim3(kPotrfThreads), 0, ctx->stream, s.A32, s.Np, kb, s.Linv,
                         ctx->flags);
    else
      hipLaunchKernelGGL(k_potrf_diag<float>, dim3(s.nlam), dim3(kPotrfThreads), 0, ctx->stream, s.A32, s.Np, kb, s.Linv,
                         ctx->flags);
    const int rem = nb - kb - 1;
    if (rem > 0)
      hipLaunchKernelGGL(k_trsm_panel, dim3(rem * s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv,
                         s.nlam);
  };
  // Block columns in pairs (kb, kb + 1): one pass over the panels k < kb updates both,
  // then column kb is finished, then column kb + 1 takes its remaining term k = kb.
  for (int kb = 0; kb < nb;) {
    if (sh.pair && kb > 0 && kb + 1 < nb) {
      const int wgs = (nb - kb) * s.nlam;
      const int nsplit = update_split(wgs, kb, s.part_tiles);
      if (nsplit > 1) {
        hipLaunchKernelGGL(k_left_update2<true>, dim3(wgs * nsplit), dim3(256), 0, ctx->stream, s.A32, s.Np, kb,
                           s.nlam, nsplit, s.upart);
        hipLaunchKernelGGL(k_left_update2_sum, dim3(wgs * 8), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.nlam,
                           nsplit, s.upart);
      } else {
        hipLaunchKernelGGL(k_left_update2<false>, dim3(wgs), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.nlam, 1,
                           nullptr);
      }
      finish(kb);
      hipLaunchKernelGGL(k_left_update, dim3((nb - kb - 1) * s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np,
                         kb + 1, kb, kb + 1, s.nlam);
      finish(kb + 1);
      kb += 2;
    } else {
      if (kb > 0)
        hipLaunchKernelGGL(k_left_update, dim3((nb - kb) * s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, 0,
                           kb, s.nlam);
      finish(kb);
      kb += 1;
    }
  }
  FK_HIP(hipGetLastError());
  return FK_OK;
}

// D32 = A^-1 R32 per lambda (ncol = ntgt columns each), through Y32.
static fk_status trsm_all(fk_ctx* ctx, const SolveLayout& s, const DenseShape& sh, float* R, float* Y, float* X) {
  const int nb = s.Np / NB;
  const bool two = s.ntgt > 16;
  // workgroups per lambda: about sh.trsm_wg in all, each sweeping several rows
  const int gmax = std::max(1, sh.trsm_wg / s.nlam);
  // two block columns per launch (the last one alone when nb is odd)
  for (int kb = 0; kb < nb;) {
    if (kb + 1 < nb) {
      const int g = std::max(1, std::min(gmax, nb - kb - 2));
      if (two)
        hipLaunchKernelGGL(k_fwd2_mfma<2>, dim3(g, s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv, R,
                           Y, s.ntgt);
      else
        hipLaunchKernelGGL(k_fwd2_mfma<1>, dim3(g, s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv, R,
                           Y, s.ntgt);
      kb += 2;
    } else {
      const int g = std::max(1, std::min(gmax, nb - kb - 1));
      if (two)
        hipLaunchKernelGGL(k_fwd_mfma<2>, dim3(g, s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv, R,
                           Y, s.ntgt);
      else
        hipLaunchKernelGGL(k_fwd_mfma<1>, dim3(g, s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv, R,
                           Y, s.ntgt);
      kb += 1;
    }
  }
  for (int kb = nb - 1; kb >= 0;) {
    if (kb >= 1) {
      const int g = std::max(1, std::min(gmax, kb - 1));
      if (two)
        hipLaunchKernelGGL(k_bwd2_mfma<2>, dim3(g, s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv, Y,
                           X, s.ntgt);
      else
        hipLaunchKernelGGL(k_bwd2_mfma<1>, dim3(g, s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv, Y,
                           X, s.ntgt);
      kb -= 2;
    } else {
      const int g = std::max(1, std::min(gmax, kb));
      if (two)
        hipLaunchKernelGGL(k_bwd_mfma<2>, dim3(g, s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv, Y,
                           X, s.ntgt);
      else
        hipLaunchKernelGGL(k_bwd_mfma<1>, dim3(g, s.nlam), dim3(256), 0, ctx->stream, s.A32, s.Np, kb, s.Linv, Y,
                           X, s.ntgt);
      kb -= 1;
    }
  }
  FK_HIP(hipGetLastError());
  return FK_OK;
}

// Solve (H64 + lambda diag(preal)) X = RHS for all (lambda, target) with FP32
// factors and FP64 refinement.  RHS given per target (Bre) or per column (rhs_cols).
// Returns the number of refinement steps and the worst relative residual.
// With check_flags, every step's norm read-back also brings the context's error flags (the stages
// queued before the solve raised them: input NaN, range, not positive definite), and those are
// reported first: the caller then needs no synchronization of its own before the solve.
static fk_status refine_solve(fk_ctx* ctx, const SolveLayout& s, const DenseShape& sh, const double* rhs_cols,
                              double* X, int* iters_out, double* resid_out, int* bad_out,
                              bool check_flags = false) {
  const int64_t tot = (int64_t)s.nlam * s.ntgt * s.Np;
  const int nc = s.nlam * s.ntgt;
  const int thr = 256;
  const int blocks = (int)((tot + thr - 1) / thr);
  // R64 = rhs
  if (rhs_cols) {
    FK_HIP(hipMemcpyAsync(s.R64, rhs_cols, sizeof(double) * tot, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    hipLaunchKernelGGL(k_rep_rhs, dim3(blocks), dim3(thr), 0, ctx->stream, s.Bre, s.Np, s.ntgt, s.nlam, s.R64);
  }
  FK_HIP(hipMemsetAsync(X, 0, sizeof(double) * tot, ctx->stream));
  // norms of the right-hand sides
  hipLaunchKernelGGL(k_colnorm2, dim3(nc), dim3(256), 0, ctx->stream, s.R64, s.Np, s.norms + nc);
  const int maxit = ctx->opt.max_refine;
  const double tol = ctx->opt.refine_tol;
  // the norms come back through the context's pinned staging area (an asynchronous copy)
  double* nh = static_cast<double*>(stage_take(ctx, sizeof(double) * 2 * nc));
  if (!nh) return FK_EHIP;
  int it = 0;
  double worst = 0.0;
  int bad = -1;
  for (;; ++it) {
    hipLaunchKernelGGL(k_scale_d2f, dim3(blocks), dim3(thr), 0, ctx->stream, s.R64, s.scl, s.Np, s.ntgt, s.R32,
                       tot);
    fk_status st = trsm_all(ctx, s, sh, s.R32, s.Y32, s.D32);
    if (st != FK_OK) return st;
    hipLaunchKernelGGL(k_scale_axpy_f2d, dim3(blocks), dim3(thr), 0, ctx->stream, s.D32, s.scl, s.Np, s.ntgt, X,
                       tot);
    // R64 = rhs - A X
    launch_resid(ctx->stream, s.H64, s.N, s.Np, X, nc, s.ntgt, rhs_cols ? 1 : 0, rhs_cols ? rhs_cols : s.Bre,
                 s.preal, s.lams, s.R64);
    FK_HIP(hipGetLastError());
    // Below 1e-8 the FP32-class first solve never meets the tolerance on its own: its check (a host
    // wait) is skipped and the first refinement step queued behind it; errors it would have found
    // (NaN, flags) are found by the next check with the same status.
    if (it == 0 && maxit > 0 && tol < 1e-8) continue;
    hipLaunchKernelGGL(k_colnorm2, dim3(nc), dim3(256), 0, ctx->stream, s.R64, s.Np, s.norms);
    FK_HIP(hipMemcpyAsync(nh, s.norms, sizeof(double) * 2 * nc, hipMemcpyDeviceToHost, ctx->stream));
    if (check_flags)
      FK_HIP(hipMemcpyAsync(ctx->flags_host, ctx->flags, sizeof(int) * kFlagCount, hipMemcpyDeviceToHost,
                            ctx->stream));
    FK_HIP(hipStreamSynchronize(ctx->stream));
    if (check_flags) {
      const fk_status fs = flag_status(ctx);
      if (fs != FK_OK) {
        *iters_out = it;
        *resid_out = 0.0;
        *bad_out = fs == FK_ENOTPD ? ctx->flags_host[kFlagNotPD + 1] : -1;
        return fs;
      }
    }
    worst = 0.0;
    bad = -1;
    for (int c = 0; c < nc; ++c) {
      // a NaN or Inf right-hand side (or one that the solve turned into one) is an input error,
      // not a refinement stall
      if (!std::isfinite(nh[c]) || !std::isfinite(nh[nc + c])) {
        *iters_out = it;
        *resid_out = nh[c];
        *bad_out = c / s.ntgt;
        return FK_ENAN;
      }
      double rel = nh[nc + c] > 0 ? std::sqrt(nh[c] / nh[nc + c]) : std::sqrt(nh[c]);
      if (!(rel <= worst)) {
        worst = rel;
        bad = c / s.ntgt;
      }
    }
    if (worst <= tol || it >= maxit) break;
  }
  *iters_out = it;
  *resid_out = worst;
  *bad_out = bad;
  return worst <= tol ? FK_OK : FK_ENOCONV;
}

static std::string dense_key(const fk_ctx* ctx, const SolveLayout& s) {
  char key[128];
  std::snprintf(key, sizeof(key), "%s dense Np=%d nlam=%d ntgt=%d", tune_arch(ctx->device).c_str(), s.Np, s.nlam,
                s.ntgt);
  return key;
}

static bool dense_tunable(const SolveLayout& s) { return (double)s.Np * s.Np * s.nlam >= (double)(1 << 28); }

// The table's launch shape of this dense shape (the defaults when there is none).
static DenseShape dense_shape(const fk_ctx* ctx, const SolveLayout& s) {
  DenseShape sh;
  std::map<std::string, double> v;
  if (tune_mode(ctx) == kTuneOff || !tune_lookup(dense_key(ctx, s), &v)) return sh;
  if (v.count("trsm_wg") && v["trsm_wg"] >= 64 && v["trsm_wg"] <= 4096) sh.trsm_wg = (int)v["trsm_wg"];
  if (v.count("pair")) sh.pair = v["pair"] != 0.0;
  if (v.count("diag64")) sh.diag64 = v["diag64"] != 0.0;
  return sh;
}

// Launch shape of the factorization and the triangular solves.  Tuning (large batched solves whose
// shape has no table entry): each pairing candidate rebuilds the FP32 matrices and factors them, and
// the chosen one's factors are left in place (*factored; rebuilt if another candidate ran last);
// each solve width is timed on zero right-hand sides.
static fk_status tune_dense(fk_ctx* ctx, const SolveLayout& s, DenseShape* out, bool* factored) {
  const int mode = tune_mode(ctx);
  *factored = false;
  *out = dense_shape(ctx, s);
  if (mode == kTuneOff || !dense_tunable(s)) return FK_OK;
  std::map<std::string, double> v;
  if (mode != kTuneForce && tune_lookup(dense_key(ctx, s), &v)) return FK_OK;
  // the trials synchronize anyway: no shape is measured on a system the earlier stages flagged
  fk_status fs = read_flags(ctx);
  if (fs != FK_OK) return fs;
  hipEvent_t e0 = ctx->ev[11], e1 = ctx->ev[12];
  DenseShape sh;
  float best_f = 0.f;
  for (int pair : {1, 0}) {
    DenseShape c = sh;
    c.pair = pair;
    hipLaunchKernelGGL(k_make_a32, dim3(a32_tiles(s.Np)), dim3(256), 0, ctx->stream, s.H64, s.preal, s.lams, s.scl, s.N, s.Np,
                       s.nlam, s.A32);
    FK_HIP(hipEventRecord(e0, ctx->stream));
    fk_status st = factor_all(ctx, s, c);
    if (st != FK_OK) return st;
    FK_HIP(hipEventRecord(e1, ctx->stream));
    FK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    FK_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (pair == 1 || ms < best_f) {
      best_f = ms;
      sh.pair = pair;
    }
  }
  // the factors the call goes on with are those of the chosen pairing, so that the first call of a
  // shape gives the same bits as the later ones
  if (sh.pair != 0) {
    hipLaunchKernelGGL(k_make_a32, dim3(a32_tiles(s.Np)), dim3(256), 0, ctx->stream, s.H64, s.preal, s.lams, s.scl,
                       s.N, s.Np, s.nlam, s.A32);
    fk_status st = factor_all(ctx, s, sh);
    if (st != FK_OK) return st;
  }
  *factored = true;
  const size_t nv = (size_t)s.nlam * s.ntgt * s.Np;
  FK_HIP(hipMemsetAsync(s.R32, 0, sizeof(float) * nv, ctx->stream));
  float best_t = 0.f;
  for (int wg : {512, 768, 256, 1024}) {
    DenseShape c = sh;
    c.trsm_wg = wg;
    FK_HIP(hipEventRecord(e0, ctx->stream));
    fk_status st = trsm_all(ctx, s, c, s.R32, s.Y32, s.D32);
    if (st != FK_OK) return st;
    FK_HIP(hipEventRecord(e1, ctx->stream));
    FK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    FK_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (wg == 512 || ms < best_t) {
      best_t = ms;
      sh.trsm_wg = wg;
    }
  }
  tune_store(dense_key(ctx, s), {{"pair", sh.pair}, {"trsm_wg", sh.trsm_wg}}, best_f + best_t);
  *out = sh;
  return FK_OK;
}

fk_status solve_impl(fk_ctx* ctx, const SolveProblem& P, const SolveLayout& s, double* theta_out,
                     fk_fit_info* info) {
  const int N = s.N, Np = s.Np;
  const int L = P.L;
  hipEvent_t* ev = ctx->ev;
  FK_HIP(hipEventRecord(ev[5], ctx->stream));
  // penalty weights (complex modes) -> device, real-form weights
  fk_status up = stage_upload(ctx, s.pcx, P.p.data(), sizeof(double) * N);
  if (up == FK_OK) up = stage_upload(ctx, s.lams, P.lams.data(), sizeof(double) * s.nlam);
  if (up != FK_OK) return up;
  FK_HIP(hipMemsetAsync(s.preal, 0, sizeof(double) * Np, ctx->stream));
  hipLaunchKernelGGL(k_real_weights, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, s.pcx, N, L, s.preal);
  // FP64 real-form Gram (+ dense lambda-independent penalty)
  const int64_t tot2 = (int64_t)Np * Np;
  const int gb = (int)((tot2 + 255) / 256);
  if (P.kind == SolveProblem::kToeplitz) {
    ToeplitzQ q{P.M, P.m, P.d};
    hipLaunchKernelGGL(k_assemble_real<ToeplitzQ>, dim3(gb), dim3(256), 0, ctx->stream, q, N, L, Np, s.H64);
  } else if (P.kind == SolveProblem::kToeplitzPde) {
    up = stage_upload(ctx, s.dsym, P.dsym.data(), sizeof(double) * 2 * N);
    if (up != FK_OK) return up;
    using PQ = SumQ<ToeplitzQ, PdeQ>;
    PQ q{ToeplitzQ{P.M, P.m, P.d}, PdeQ{s.dsym, P.m, P.d, P.mu, P.lo[0], P.hi[0], P.lo[1], P.hi[1]}};
    hipLaunchKernelGGL(k_assemble_real<PQ>, dim3(gb), dim3(256), 0, ctx->stream, q, N, L, Np, s.H64);
  } else {
    DenseQ q{P.B, N};
    hipLaunchKernelGGL(k_assemble_real<DenseQ>, dim3(gb), dim3(256), 0, ctx->stream, q, N, L, Np, s.H64);
  }
  hipLaunchKernelGGL(k_make_scale, dim3((Np + 255) / 256, s.nlam), dim3(256), 0, ctx->stream, s.H64, s.preal,
                     s.lams, N, Np, s.scl);
  hipLaunchKernelGGL(k_make_a32, dim3(a32_tiles(Np)), dim3(256), 0, ctx->stream, s.H64, s.preal, s.lams, s.scl, N, Np,
                     s.nlam, s.A32);
  hipLaunchKernelGGL(k_rhs_real, dim3((Np + 255) / 256, s.ntgt), dim3(256), 0, ctx->stream, P.b, N, L, Np,
                     s.ntgt, s.Bre);
  FK_HIP(hipGetLastError());
  DenseShape sh;
  bool factored = false;
  fk_status st = tune_dense(ctx, s, &sh, &factored);
  if (st != FK_OK) return st;
  FK_HIP(hipEventRecord(ev[6], ctx->stream));
  if (!factored) {
    st = factor_all(ctx, s, sh);
    if (st != FK_OK) return st;
  }
  FK_HIP(hipEventRecord(ev[7], ctx->stream));
  // the flags of the earlier stages and of the factorization come back with the first residual norms
  int iters = 0, bad = -1;
  double resid = 0.0;
  st = refine_solve(ctx, s, sh, nullptr, s.X64, &iters, &resid, &bad, true);
  hipLaunchKernelGGL(k_theta_from_real, dim3((N + 255) / 256, s.nlam * s.ntgt), dim3(256), 0, ctx->stream, s.X64,
                     N, L, Np, s.ntgt, theta_out);
  FK_HIP(hipGetLastError());
  FK_HIP(hipEventRecord(ev[8], ctx->stream));
  FK_HIP(hipEventSynchronize(ev[8]));
  if (info) {
    info->refine_iters = iters;
    info->resid_rel = resid;
    if (st != FK_OK) info->bad_index = bad;
    float a = 0, f = 0, so = 0;
    hipEventElapsedTime(&a, ev[5], ev[6]);
    hipEventElapsedTime(&f, ev[6], ev[7]);
    hipEventElapsedTime(&so, ev[7], ev[8]);
    info->t_assemble_ms = a;
    info->t_factor_ms = f;
    info->t_solve_ms = so;
  }
  return st;
}

// ------------------------------------------------------------------ held-out loss and backward

// out[c] = x_c . v_c  (dot products of matching columns)
__global__ __launch_bounds__(256) void k_coldot(const double* __restrict__ A, const double* __restrict__ B,
                                                int Np, int bstride_cols, int ntgt, double* __restrict__ out) {
  __shared__ double part[256];
  const int c = blockIdx.x;
  const double* a = A + (size_t)c * Np;
  const double* b = B + (size_t)(bstride_cols ? c : (c % ntgt)) * Np;
  double s = 0.0;
  for (int i = threadIdx.x; i < Np; i += blockDim.x) s += a[i] * b[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = part[0];
}

__global__ void k_mse_combine(const double* __restrict__ xg, const double* __restrict__ bx,
                              const double* __restrict__ yv2, int nc, int ntgt, double* __restrict__ mse) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  mse[c] = xg[c] - bx[c] + yv2[c % ntgt];   // x.(Hv x - bv) - x.bv + mean(Yv^2)
}

// G64[c] = Hv X[c] - Bv[t]   (gradient direction g in real form)
// (the residual kernels with lambda = 0:  Rres = Bv - Hv X  -> negate)
__global__ void k_negate(double* __restrict__ v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = -v[i];
}

fk_status heldout_mse_impl(fk_ctx* ctx, const SolveLayout& s, int d, int m, const double* Mv, const double* bv,
                           const double* yv2, double* mse) {
  const int N = s.N, Np = s.Np, L = N;   // one real-form block of all N modes
  const int64_t tot2 = (int64_t)Np * Np;
  const int gb = (int)((tot2 + 255) / 256);
  ToeplitzQ q{Mv, m, d};
  hipLaunchKernelGGL(k_assemble_real<ToeplitzQ>, dim3(gb), dim3(256), 0, ctx->stream, q, N, L, Np, s.Hv);
  hipLaunchKernelGGL(k_rhs_real, dim3((Np + 255) / 256, s.ntgt), dim3(256), 0, ctx->stream, bv, N, L, Np, s.ntgt,
                     s.Bv);
  const int nc = s.nlam * s.ntgt;
  // zero "lambda" for the validation product: reuse norms scratch as a zero lambda array
  FK_HIP(hipMemsetAsync(s.norms, 0, sizeof(double) * (2 * nc + s.nlam + 64), ctx->stream));
  // R = Bv - Hv X   (lambda = 0 via a zero lambda array of length nlam in norms[2nc..])
  launch_resid(ctx->stream, s.Hv, N, Np, s.X64, nc, s.ntgt, 0, s.Bv, s.preal, s.norms + 2 * nc, s.G64);
  const int64_t tot = (int64_t)nc * Np;
  hipLaunchKernelGGL(k_negate, dim3((tot + 255) / 256), dim3(256), 0, ctx->stream, s.G64, tot);
  // xGx = x.(Hv x) = x.(g + bv) ; bx = bv.x
  hipLaunchKernelGGL(k_coldot, dim3(nc), dim3(256), 0, ctx->stream, s.X64, s.G64, Np, 1, s.ntgt, s.norms);
  hipLaunchKernelGGL(k_coldot, dim3(nc), dim3(256), 0, ctx->stream, s.X64, s.Bv, Np, 0, s.ntgt, s.norms + nc);
  // mse = x.g + x.bv - 2 x.bv + yv2 = x.g - x.bv + yv2
  hipLaunchKernelGGL(k_mse_combine, dim3((nc + 255) / 256), dim3(256), 0, ctx->stream, s.norms, s.norms + nc, yv2,
                     nc, s.ntgt, mse);
  FK_HIP(hipGetLastError());
  (void)L;
  return FK_OK;
}

// Adjoint right-hand sides in real form: Gadj[c] = gm[c] G64[c] + (1/2) d(Loss)/dc of the incoming
// Wirtinger gradient gin[c] = dLoss/dconj(theta_c) (complex, N modes).  With theta = U c (real c),
// dLoss/dc_r = 2 Re(gin^* dtheta/dc_r), so the real-form entry is Re gin_0 (constant),
// (Re gin_k + Re gin_-k)/sqrt2 (cosine of k) and (Im gin_-k - Im gin_k)/sqrt2 (sine of k): the
// projection onto Hermitian-symmetric theta, where every fitted theta lies.
__global__ void k_adjoint_rhs(const double* __restrict__ G64, const double* __restrict__ gm,
                              const double* __restrict__ gin, int N, int L, int Np, double* __restrict__ Gadj) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= Np) return;
  double v = gm[c] * G64[(size_t)c * Np + r];
  if (gin && r < N) {
    int ty, k, nk;
    real_to_complex(r, L, &ty, &k, &nk);
    const double* g = gin + 2 * (size_t)c * N;
    const double rs2 = 0.70710678118654752440;
    v += ty == 0 ? g[2 * k] : (ty == 1 ? rs2 * (g[2 * k] + g[2 * nk]) : rs2 * (g[2 * nk + 1] - g[2 * k + 1]));
  }
  Gadj[(size_t)c * Np + r] = v;
}

// grad_loglam[l] = sum_t (-2 lambda_l) u.(preal o x), u the adjoint solution of the combined
// right-hand side;  grad_p (complex modes) likewise.
// One workgroup of 1024 threads per lambda (the sum runs over ntgt x Np terms).
__global__ __launch_bounds__(1024) void k_grad_loglam(const double* __restrict__ U, const double* __restrict__ X,
                                                      const double* __restrict__ preal, const double* __restrict__ lams,
                                                      int Np, int ntgt, double* __restrict__ out) {
  __shared__ double part[1024];
  const int l = blockIdx.x;
  double s = 0.0;
  for (int t = 0; t < ntgt; ++t) {
    const double* u = U + ((size_t)l * ntgt + t) * Np;
    const double* x = X + ((size_t)l * ntgt + t) * Np;
    double a = 0.0;
    for (int i = threadIdx.x; i < Np; i += blockDim.x) a += u[i] * preal[i] * x[i];
    s += a;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[l] = -2.0 * lams[l] * part[0];
}

// grad_p over the (lambda, target) systems: blockIdx.y takes one slice of them, its four waves
// a quarter of the slice each, lane = real-form row; the slices' sums are added into gp, which
// k_zero_d cleared.
constexpr int kGradPSlices = 16;
__global__ void k_zero_d(double* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_grad_p(const double* __restrict__ U, const double* __restrict__ X,
                                                const double* __restrict__ lams, int N, int L, int Np, int nlam,
                                                int ntgt, double* __restrict__ gp) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + lane;
  const int nc = nlam * ntgt;
  const int c0 = (int)((int64_t)nc * blockIdx.y / gridDim.y), c1 = (int)((int64_t)nc * (blockIdx.y + 1) / gridDim.y);
  int ty = 2, k = 0, nk = 0;
  if (r < N) real_to_complex(r, L, &ty, &k, &nk);
  double s = 0.0;
  if (ty != 2)
    for (int c = c0 + wv; c < c1; c += 4) {
      const int l = c / ntgt;
      const size_t o = (size_t)c * Np;
      const double v = ty == 0 ? U[o + r] * X[o + r] : 0.5 * (U[o + r] * X[o + r] + U[o + r + 1] * X[o + r + 1]);
      s += (-2.0 * lams[l]) * v;
    }
  part[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && ty != 2) {
    const double t = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
    atomicAdd(&gp[k], t);
    if (ty == 1) atomicAdd(&gp[nk], t);
  }
}

__global__ void k_scale_cols_cplx(double* __restrict__ th, const double* __restrict__ gm, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  if (i >= 2 * N) return;
  th[(size_t)c * 2 * N + i] *= gm[c];
}

fk_status backward_impl(fk_ctx* ctx, const SolveLayout& s, int d, const double* gm, const double* gin,
                        double* grad_loglam, double* grad_p, double* grad_theta) {
  const int N = s.N, Np = s.Np, L = N;   // one real-form block of all N modes
  const int nc = s.nlam * s.ntgt;
  int iters = 0, bad = -1;
  double resid = 0.0;
  // u = A^-1 (gm g + gin) for every (lambda, target)
  hipLaunchKernelGGL(k_adjoint_rhs, dim3((Np + 255) / 256, nc), dim3(256), 0, ctx->stream, s.G64, gm, gin, N, L, Np,
                     s.Gadj);
  fk_status st = refine_solve(ctx, s, dense_shape(ctx, s), s.Gadj, s.U64, &iters, &resid, &bad);
  if (st != FK_OK && st != FK_ENOCONV) return st;
  hipLaunchKernelGGL(k_grad_loglam, dim3(s.nlam), dim3(1024), 0, ctx->stream, s.U64, s.X64, s.preal, s.lams, Np,
                     s.ntgt, grad_loglam);
  if (grad_p) {
    hipLaunchKernelGGL(k_zero_d, dim3((N + 255) / 256), dim3(256), 0, ctx->stream, grad_p, N);
    hipLaunchKernelGGL(k_grad_p, dim3((N + 63) / 64, kGradPSlices), dim3(256), 0, ctx->stream, s.U64, s.X64, s.lams,
                       N, L, Np, s.nlam, s.ntgt, grad_p);
  }
  if (grad_theta) {
    hipLaunchKernelGGL(k_theta_from_real, dim3((N + 255) / 256, nc), dim3(256), 0, ctx->stream, s.G64, N, L, Np,
                       s.ntgt, grad_theta);
    hipLaunchKernelGGL(k_scale_cols_cplx, dim3((2 * N + 255) / 256, nc), dim3(256), 0, ctx->stream, grad_theta, gm,
                       N);
  }
  FK_HIP(hipGetLastError());
  return st;
}

}  // namespace fk
