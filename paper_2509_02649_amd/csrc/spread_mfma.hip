// 2-D binned spread on MFMA, for 8..16 weight channels (the batched targets).
//
// The type-1 sums of Sec. 2.3 for T targets share the kernel weights of each
// point: every point adds W[c] psi1[a] psi2[b] to the w x w grid cells of its
// window, for the ones channel (the Gram, c = 0) and the T target channels.
// With LDS atomics that is w^2 (T+1) atomic adds per point; here it is a dense
// matrix product on the matrix cores.
//
// * Bins are MB x MB grid cells, sorted beforehand (sort2.hip) so a bin's points
//   are contiguous: fixed-point coordinates [U1, U2] (8 B) and the point's
//   position in the row-grouped output of the sort's first pass, where its 64-byte
//   block of 16 FP32 weights (zero padded) stays.  A point belongs to the bin
//   holding the first cell of its window (not its own cell), so the windows of a
//   bin's points start in MB consecutive cells per axis.  MB = 2 when the bins are
//   well filled (fewer subgrid cells per point: (1 + w)^2 against (3 + w)^2), else 4.
// * A workgroup of SWAVE waves takes a slice of one bin; each wave takes the
//   slice's points 4 at a time (one "chunk"), in stored order and on its own
//   (no workgroup barrier in the loop).  All windows of a bin's points lie in
//   its S x S subgrid, S = MB + w - 1, so with the kernel value zero outside a
//   point's own window,
//     D[c][cell] += sum_k W[c][k] * psi1_k[cell / S] * psi2_k[cell % S]
//   over the S^2 cells is NT = ceil(S^2 / 16) v_mfma_f32_16x16x4f32 per chunk:
//   rows = the 16 target channels, columns = 16 subgrid cells, K = the 4 points.
//   The ones channel is the column sum of the same kernel products (vector ALUs).
// * Per batch of 64 points, one lane per point writes the point's w kernel values
//   per axis (at their subgrid offsets, zeros elsewhere) into an LDS table row; the
//   B operand of cell (a, b) is the product of two table entries.
// * The weights are gathered by position (64-byte blocks, one batch ahead: into
//   alternating register sets for MB = 2); coordinates and positions stream one
//   batch ahead.
// * FP32 accumulators are added into the workgroup's FP64 LDS subgrid (ds_add_f64)
//   every SFLUSH batches and at the end; the subgrid is then added into the FP64
//   fine grid with global FP64 atomics.
//
// Lane layout of v_mfma_f32_16x16x4f32 (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; element v of the result holds row 4*(l/16)+v, column l%16.
#include "fk_internal.h"

#include <algorithm>

namespace fk {

namespace {

typedef float floatx4_t __attribute__((ext_vector_type(4)));

// Exponential of semicircle psi(s) = exp(beta (sqrt(1 - (2s/w)^2) - 1)), with beta
// pre-multiplied by log2(e): the exponent lies in [-beta log2 e, 0], far from the
// denormal range, so the hardware exp2 needs no range handling, and the hardware square
// root needs no denormal scaling (1 - z^2 below 2^-126 gives psi ~ e^-beta either way).
__device__ __forceinline__ float psi_es2(float s, float beta_log2e, float two_over_w) {
  const float z = s * two_over_w;
  const float r = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
  return __builtin_amdgcn_exp2f(fmaf(beta_log2e, __builtin_amdgcn_sqrtf(r), -beta_log2e));
}

// i0 = ceil(u - w/2), s0 = i0 - u from a fixed-point coordinate U = u 2^fb < 2^31,
// in 32-bit integer arithmetic: the bias of 8 cells keeps the dividend positive, and
// i0 2^fb - U is small, so its 32-bit wrap-around difference is exact, as is its
// conversion to float (|.| < 2^24) and the scaling by a power of two.
__device__ __forceinline__ void win_start(uint32_t U, int fb, int w, int* i0, float* s0) {
  const uint32_t one = 1u << fb;
  const uint32_t t = U + (one - 1u) + 8u * one - ((uint32_t)w << (fb - 1));
  const int c = (int)(t >> fb) - 8;
  *i0 = c;
  *s0 = (float)(int)(((uint32_t)c << fb) - U) * __uint_as_float((uint32_t)(127 - fb) << 23);
}

constexpr int SWAVE = 4;     // waves per workgroup, each independent
constexpr int SFLUSH = 16;   // batches of 64 points between FP32 -> FP64 flushes
// Kernel-value table row of one point: S + 1 slots per axis (offsets 0..S-1 of the subgrid, and
// slot S kept zero for the padding cells of the last column tile), rounded up to whole 16-byte units.
__host__ __device__ constexpr int tab_sp(int S) { return S + 1; }
__host__ __device__ constexpr int tab_ps(int S) { return (2 * tab_sp(S) + 3) / 4 * 4; }

template <int W, int MB>
__device__ __forceinline__ void spread_mfma_body(const uint2* __restrict__ crd, const uint32_t* __restrict__ pos,
                                                 const float* __restrict__ wrow, int nw,
                                                 const uint64_t* __restrict__ start, int nbx, int nf, int fb,
                                                 float beta, int slices, double* __restrict__ grid) {
  constexpr int S = MB + W - 1;
  constexpr int NT = (S * S + 15) / 16;
  constexpr int SP = tab_sp(S), PS = tab_ps(S);
  static_assert(S <= 15, "subgrid offsets 0..S-1");
  extern __shared__ double smem_d[];
  const int C = nw + 1;
  const float two_over_w = 2.0f / (float)W;
  const float bl2 = beta * 1.44269504088896340736f;
  const int subn = (S * S * C + 1) & ~1;   // keep the tables 16-byte aligned
  double* sub = smem_d;                    // S*S*C doubles

  const int b = blockIdx.x / slices;
  const int sl = blockIdx.x - b * slices;
  const uint64_t p0 = start[b], p1 = start[b + 1];
  const uint64_t len = p1 - p0;
  const uint64_t q0 = p0 + len * sl / slices;
  const uint64_t q1 = p0 + len * (sl + 1) / slices;
  if (q0 == q1) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  float* tab = reinterpret_cast<float*>(sub + subn) + wv * 64 * PS;   // this wave's 64 rows
  const int bx = b / nbx, by = b - bx * nbx;
  const int o1 = bx * MB, o2 = by * MB;   // first subgrid cell (window starts o .. o + MB - 1)
  for (int i = tid; i < S * S * C; i += 64 * SWAVE) sub[i] = 0.0;
  __syncthreads();

  const int k = lane >> 4, j = lane & 15;
  // Table offsets of psi1[a] and psi2[b] for the cell (a, b) of column tile t.
  // Padding cells (>= S*S) read slot S of each half, which stays zero.
  int offa[NT], offb[NT];
  bool cin[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int cell = t * 16 + j;
    cin[t] = cell < S * S;
    offa[t] = cin[t] ? cell / S : S;
    offb[t] = SP + (cin[t] ? cell - (cell / S) * S : S);
  }
  floatx4_t acc[NT];
  float ones[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    acc[t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    ones[t] = 0.f;
  }

  auto flush = [&]() {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      float o = ones[t];
      o += __shfl_xor(o, 16, 64);
      o += __shfl_xor(o, 32, 64);
      if (cin[t]) {
        double* cp = sub + (t * 16 + j) * C;
        if (k == 0 && o != 0.f) atomicAdd(cp, (double)o);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 4 * k + v;
          const float x = acc[t][v];
          if (row < nw && x != 0.f) atomicAdd(cp + 1 + row, (double)x);
        }
      }
      acc[t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
      ones[t] = 0.f;
    }
  };

  // Slice-relative 32-bit indices (a slice holds < 2^31 points).  A wave takes
  // batches of 64 points (16 chunks of 4): batch bb covers points 64 bb ..
  const uint32_t npts = (uint32_t)(q1 - q0);
  const uint32_t nbatch = (npts + 63) / 64;
  const uint2* __restrict__ cs = crd + q0;
  const uint32_t* __restrict__ ps = pos + q0;
  // Loads are unconditional (index clamped to the slice) so that no branch makes the
  // compiler wait for them early.  Coordinates and positions are read one lane per
  // point; the weights of chunk q of a batch are gathered for lane (k, j) as
  // W[4q + k][j] from the 64-byte block at the point's position, which lane 4q + k
  // holds.  A batch's gathers are issued one batch ahead, into the other of two
  // register sets.
  auto cload = [&](uint32_t batch) { return cs[min(batch * 64 + lane, npts - 1)]; };
  auto pload = [&](uint32_t batch) { return ps[min(batch * 64 + lane, npts - 1)]; };
#define FK_GATHER(DST, P)                                                                    \
  _Pragma("unroll") for (int q = 0; q < 16; ++q)                                             \
    DST[q] = wrow[(size_t)(uint32_t)__shfl((int)(P), 4 * q + k, 64) * 16 + j];
  uint2 Un = cload(wv);
  uint32_t Pn = pload(wv);
  float Wa[16], Wb[16];
  FK_GATHER(Wa, Pn)
  Pn = pload(wv + SWAVE);
  float* row = tab + lane * PS;
  int since = 0;
  // One batch: phase 1 builds the kernel-value table of the batch's points (one lane
  // per point: window starts and the w kernel values per axis, zeros elsewhere),
  // the next batch's gathers go out, phase 2 runs 16 chunks of 4 points on the
  // matrix cores with the weights in WC.
#define FK_BATCH(BB, WC, WN)                                                                 \
  {                                                                                          \
    const uint2 U = Un;                                                                      \
    Un = cload((BB) + SWAVE);                                                                \
    {                                                                                        \
      const bool valid = (BB) * 64 + lane < npts;                                            \
      int i1, i2;                                                                            \
      float s1, s2;                                                                          \
      win_start(U.x, fb, W, &i1, &s1);                                                       \
      win_start(U.y, fb, W, &i2, &s2);                                                       \
      float4* r4 = reinterpret_cast<float4*>(row);                                           \
      _Pragma("unroll") for (int q = 0; q < PS / 4; ++q) r4[q] = make_float4(0.f, 0.f, 0.f, 0.f); \
      const int rel1 = (i1 - o1) & (nf - 1), rel2 = SP + ((i2 - o2) & (nf - 1));            \
      if (valid && rel1 < MB && rel2 < SP + MB) {                                            \
        _Pragma("unroll") for (int r = 0; r < W; ++r) {                                     \
          row[rel1 + r] = psi_es2(s1 + (float)r, bl2, two_over_w);                           \
          row[rel2 + r] = psi_es2(s2 + (float)r, bl2, two_over_w);                           \
        }                                                                                    \
      }                                                                                      \
    }                                                                                        \
    FK_GATHER(WN, Pn)                                                                        \
    Pn = pload((BB) + 2 * SWAVE);                                                            \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");                                   \
    __builtin_amdgcn_wave_barrier();                                                         \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");                                   \
    _Pragma("unroll") for (int q = 0; q < 16; ++q) {                                         \
      const float aop = WC[q];                                                               \
      const float* rk = tab + (4 * q + k) * PS;                                              \
      _Pragma("unroll") for (int t = 0; t < NT; ++t) {                                       \
        const float bv = rk[offa[t]] * rk[offb[t]];                                          \
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bv, acc[t], 0, 0, 0);             \
        ones[t] += bv;                                                                       \
      }                                                                                      \
    }                                                                                        \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");                                   \
    __builtin_amdgcn_wave_barrier();                                                         \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");                                   \
    if (++since == SFLUSH) {                                                                 \
      flush();                                                                               \
      since = 0;                                                                             \
    }                                                                                        \
  }
  if constexpr (MB == 2) {
    for (uint32_t bb = wv; bb < nbatch; bb += 2 * SWAVE) {
      FK_BATCH(bb, Wa, Wb)
      if (bb + SWAVE < nbatch) FK_BATCH(bb + SWAVE, Wb, Wa)
    }
  } else {
    // (more tiles per chunk: one register set copied forward keeps the kernel at
    // three waves per SIMD, where the unrolled pair would not)
    for (uint32_t bb = wv; bb < nbatch; bb += SWAVE) {
      FK_BATCH(bb, Wa, Wb)
#pragma unroll
      for (int q = 0; q < 16; ++q) Wa[q] = Wb[q];
    }
  }
#undef FK_BATCH
#undef FK_GATHER
  flush();
  __syncthreads();
  for (int i = tid; i < S * S * C; i += 64 * SWAVE) {
    double v = sub[i];
    if (v == 0.0) continue;
    int ch = i % C;
    int cell = i / C;
    int a = cell / S, bb = cell - a * S;
    int g1 = o1 + a, g2 = o2 + bb;
    g1 = g1 < 0 ? g1 + nf : (g1 >= nf ? g1 - nf : g1);
    g2 = g2 < 0 ? g2 + nf : (g2 >= nf ? g2 - nf : g2);
    atomicAdd(&grid[((int64_t)ch * nf + g1) * nf + g2], v);
  }
}

// Four waves per SIMD (at most 128 registers): the kernel is issue-bound (matrix cores and
// vector ALUs together), and the fourth wave hides more of the gathers' latency than the
// registers it takes from the unrolled chunk loop cost (29.7 against 30.4 ms at 1e9 points).
template <int W, int MB>
__global__ __launch_bounds__(64 * SWAVE) __attribute__((amdgpu_waves_per_eu(4))) void k_spread_mfma(
    const uint2* __restrict__ crd, const uint32_t* __restrict__ pos, const float* __restrict__ wrow, int nw,
    const uint64_t* __restrict__ start, int nbx, int nf, int fb, float beta, int slices, double* __restrict__ grid) {
  spread_mfma_body<W, MB>(crd, pos, wrow, nw, start, nbx, nf, fb, beta, slices, grid);
}
// 4 x 4-cell bins with w <= 7: the compiler is held to the registers of three waves
// per SIMD (LDS allows three workgroups per CU); left alone it takes more.
template <int W, int MB>
__global__ __launch_bounds__(64 * SWAVE) __attribute__((amdgpu_waves_per_eu(3))) void k_spread_mfma_w3(
    const uint2* __restrict__ crd, const uint32_t* __restrict__ pos, const float* __restrict__ wrow, int nw,
    const uint64_t* __restrict__ start, int nbx, int nf, int fb, float beta, int slices, double* __restrict__ grid) {
  spread_mfma_body<W, MB>(crd, pos, wrow, nw, start, nbx, nf, fb, beta, slices, grid);
}

}  // namespace

int spread_mfma_bin(int nf, int64_t n) {
  const int64_t nb2 = (int64_t)(nf / 2) * (nf / 2);
  return (sort2_ok(nf / 2) && n >= 4096 * nb2) ? 2 : 4;
}

bool spread_mfma_ok(int nw, int W) { return nw >= 8 && nw <= 16 && W >= 4 && W <= 8; }

template <int W, int MB>
static void launch_w(hipStream_t st, int blocks, size_t lds, const uint2* c2, const uint32_t* pos, const float* wf,
                     int nw, const uint64_t* start, int nbx, int nf, int fb, float bt, int slices, double* grid) {
  if constexpr (MB == 4 && W <= 7)
    hipLaunchKernelGGL((k_spread_mfma_w3<W, MB>), dim3(blocks), dim3(64 * SWAVE), lds, st, c2, pos, wf, nw, start,
                       nbx, nf, fb, bt, slices, grid);
  else
    hipLaunchKernelGGL((k_spread_mfma<W, MB>), dim3(blocks), dim3(64 * SWAVE), lds, st, c2, pos, wf, nw, start, nbx,
                       nf, fb, bt, slices, grid);
}

fk_status launch_spread_mfma(hipStream_t st, int W, int MB, const uint32_t* crd, const uint32_t* pos,
                             const uint32_t* wrow, int nw, const uint64_t* start, int nbx, int nb, int nf, int fb,
                             double beta, int64_t n, int spread_pts, double* grid) {
  if (!spread_mfma_ok(nw, W) || (MB != 2 && MB != 4) || spread_pts < 256) return FK_EINVAL;
  const int64_t per_bin = (n + nb - 1) / nb;
  const int slices = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (per_bin + spread_pts - 1) / spread_pts));
  const int blocks = nb * slices;
  const size_t lds = sizeof(double) * (((MB + W - 1) * (MB + W - 1) * (nw + 1) + 1) & ~1) +
                     sizeof(float) * SWAVE * 64 * tab_ps(MB + W - 1);
  const float bt = (float)beta;
  const uint2* c2 = reinterpret_cast<const uint2*>(crd);
  const float* wf = reinterpret_cast<const float*>(wrow);
#define FK_SPREAD_W(WW)                                                                                   \
  case WW:                                                                                                \
    if (MB == 2) launch_w<WW, 2>(st, blocks, lds, c2, pos, wf, nw, start, nbx, nf, fb, bt, slices, grid); \
    else launch_w<WW, 4>(st, blocks, lds, c2, pos, wf, nw, start, nbx, nf, fb, bt, slices, grid);         \
    break;
  switch (W) {
    FK_SPREAD_W(4)
    FK_SPREAD_W(5)
    FK_SPREAD_W(6)
    FK_SPREAD_W(7)
    FK_SPREAD_W(8)
    default: return FK_EINVAL;
  }
#undef FK_SPREAD_W
  return hipGetLastError() == hipSuccess ? FK_OK : FK_EHIP;
}

}  // namespace fk
