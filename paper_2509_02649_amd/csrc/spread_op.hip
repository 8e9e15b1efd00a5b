// 2-D binned spread on MFMA for 0..7 weight channels (one target, a few targets, or
// the Gram channel alone).
//
// The kernel is a tensor product, so the contribution of point k with channel
// weight W_c[k] (W_0 = 1: the Gram) to subgrid cell (x, y) is W_c[k] psi1_k[x] psi2_k[y].
// Four points at a time, the subgrid of channel c takes
//   D_c[x][y] += sum_k (W_c[k] psi1_k[x]) psi2_k[y],
// one v_mfma_f32_16x16x4f32 on a 16 x 16 subgrid: A[x][k] = W_c[k] psi1_k[x] and
// B[k][y] = psi2_k[y].  Lane l = j + 16 k supplies A[j][k] and B[k][j], the kernel
// values of point k at subgrid offset j; element v of its result is D[4 k + v][j].
// Per point that is CH / 4 MFMAs (CH = WV + 1 channels), against ceil(S^2 / 16) / 4
// for the channel-row form of spread_mfma.hip, which pays off only with many
// channels.
//
// * Bins are OMB x OMB cells (OMB = 8), sorted beforehand (sort2.hip, records of WV
//   = 0, 1, 2, 4 or 8 weight words, WV = 0 for the Gram channel alone); a point
//   belongs to the bin holding the first cell of its window,
//   so all windows of a bin lie in its S x S subgrid, S = OMB + w - 1 <= 16.
// * A workgroup of OWAVE waves takes a slice of one bin, each wave its batches of 64
//   points in turn.  Per batch, one lane per point writes the point's w kernel values
//   per axis (at their subgrid offsets, zeros elsewhere) and its weights into an LDS
//   table row; then 16 chunks of 4 points read their operands from the table.  The
//   next batch's coordinates and weights are loaded meanwhile.
// * FP32 accumulators go into the workgroup's FP64 LDS subgrid every OFLUSH batches
//   (1024 points per wave) and at the end; the subgrid is added into the FP64 fine
//   grid with global FP64 atomics.
#include "fk_internal.h"

#include <algorithm>

namespace fk {

namespace {

typedef float floatx4_o __attribute__((ext_vector_type(4)));

constexpr int OMB = 8;       // bin width in cells
constexpr int OWAVE = 4;     // waves per workgroup
constexpr int OFLUSH = 16;   // batches of 64 points per wave between FP32 -> FP64 flushes

// Exponential of semicircle psi(s) = exp(beta (sqrt(1 - (2s/w)^2) - 1)) with beta
// pre-multiplied by log2(e) (exponent in [-beta log2 e, 0]: the hardware exp2 needs no range
// handling, and the hardware square root no denormal scaling).
__device__ __forceinline__ float psi_es(float s, float beta_log2e, float two_over_w) {
  const float z = s * two_over_w;
  const float r = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
  return __builtin_amdgcn_exp2f(fmaf(beta_log2e, __builtin_amdgcn_sqrtf(r), -beta_log2e));
}

// i0 = ceil(u - w/2) and s0 = i0 - u for the fixed-point coordinate U = u 2^fb, in
// 32-bit integer arithmetic (8 cells of bias keep the sum positive; i0 2^fb - U is
// small, so its wrap-around difference and its conversion to float are exact).
__device__ __forceinline__ void window(uint32_t U, int fb, int w, int* i0, float* s0) {
  const uint32_t one = 1u << fb;
  const uint32_t t = U + (one - 1u) + 8u * one - ((uint32_t)w << (fb - 1));
  const int c = (int)(t >> fb) - 8;
  *i0 = c;
  *s0 = (float)(int)(((uint32_t)c << fb) - U) * __uint_as_float((uint32_t)(127 - fb) << 23);
}

template <int WV>
struct WBlk {
  float v[WV > 0 ? WV : 1];
};

template <int WV>
__device__ __forceinline__ WBlk<WV> load_w(const uint32_t* __restrict__ p) {
  WBlk<WV> r;
  if constexpr (WV == 0) {
    r.v[0] = 0.f;
  } else if constexpr (WV == 1) {
    r.v[0] = __uint_as_float(p[0]);
  } else if constexpr (WV == 2) {
    const uint2 a = *reinterpret_cast<const uint2*>(p);
    r.v[0] = __uint_as_float(a.x);
    r.v[1] = __uint_as_float(a.y);
  } else {
#pragma unroll
    for (int q = 0; q < WV / 4; ++q) {
      const uint4 a = reinterpret_cast<const uint4*>(p)[q];
      r.v[4 * q + 0] = __uint_as_float(a.x);
      r.v[4 * q + 1] = __uint_as_float(a.y);
      r.v[4 * q + 2] = __uint_as_float(a.z);
      r.v[4 * q + 3] = __uint_as_float(a.w);
    }
  }
  return r;
}

// Table row: psi1[16], psi2[16], weights, padded to a multiple of 4 floats that is an
// odd number of 16-byte words, so that the float4 row writes of 8 consecutive lanes fall
// into distinct LDS banks (36 floats, or 44 with 8 weight words).
template <int WV>
constexpr int op_row() {
  const int r = (32 + WV + 3) & ~3;
  return ((r / 4) % 2 == 0) ? r + 4 : r;
}

template <int W, int WV>
__global__ __launch_bounds__(64 * OWAVE) void k_spread_op(const uint2* __restrict__ crd,
                                                          const uint32_t* __restrict__ wts, int C,
                                                          const uint64_t* __restrict__ start, int nbx, int nf,
                                                          int fb, float beta, int slices,
                                                          double* __restrict__ grid) {
  constexpr int S = OMB + W - 1;
  constexpr int CH = WV + 1;
  constexpr int PR = op_row<WV>();
  static_assert(S <= 16, "the subgrid must fit one 16 x 16 MFMA tile");
  __shared__ double sub[CH * 256];                      // sub[c][x][y], 16 x 16 per channel
  __shared__ __align__(16) float tabs[OWAVE * 64 * PR];  // per wave: 64 rows
  const int b = blockIdx.x / slices;
  const int sl = blockIdx.x - b * slices;
  const uint64_t p0 = start[b], len = start[b + 1] - p0;
  const uint64_t q0 = p0 + len * sl / slices;
  const uint64_t q1 = p0 + len * (sl + 1) / slices;
  if (q0 == q1) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int k = lane >> 4, j = lane & 15;
  const int bx = b / nbx, by = b - bx * nbx;
  const int o1 = bx * OMB, o2 = by * OMB;   // first subgrid cell on each axis
  for (int i = tid; i < CH * 256; i += 64 * OWAVE) sub[i] = 0.0;
  __syncthreads();

  const float two_over_w = 2.0f / (float)W;
  const float bl2 = beta * 1.44269504088896340736f;
  const uint32_t npts = (uint32_t)(q1 - q0);   // a slice holds < 2^31 points
  const uint32_t nbatch = (npts + 63) / 64;
  const uint2* __restrict__ cs = crd + q0;
  const uint32_t* __restrict__ ws = wts + q0 * WV;
  float* tab = tabs + wv * 64 * PR;
  float* row = tab + lane * PR;
  // phase-1 inputs of the wave's next batch in flight (one point per lane; index
  // clamped to the slice)
  uint2 Un = cs[min(wv * 64u + lane, npts - 1)];
  WBlk<WV> Wn = load_w<WV>(ws + (size_t)min(wv * 64u + lane, npts - 1) * WV);
  floatx4_o acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = floatx4_o{0.f, 0.f, 0.f, 0.f};

  auto flush = [&]() {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float x = acc[c][v];
        if (x != 0.f) atomicAdd(&sub[c * 256 + (4 * k + v) * 16 + j], (double)x);
      }
      acc[c] = floatx4_o{0.f, 0.f, 0.f, 0.f};
    }
  };

  int since = 0;
  for (uint32_t bb = wv; bb < nbatch; bb += OWAVE) {
    // Phase 1, one lane per point: its window starts, the w kernel values per axis at
    // their subgrid offsets (zeros elsewhere) and its weights, in its table row.
    const uint2 U = Un;
    const WBlk<WV> Wk = Wn;
    {
      const uint32_t p = min((bb + OWAVE) * 64u + lane, npts - 1);
      Un = cs[p];
      Wn = load_w<WV>(ws + (size_t)p * WV);
    }
    {
      const bool valid = bb * 64u + lane < npts;
      int i1, i2;
      float s1, s2;
      window(U.x, fb, W, &i1, &s1);
      window(U.y, fb, W, &i2, &s2);
      float4* r4 = reinterpret_cast<float4*>(row);
#pragma unroll
      for (int q = 0; q < 8; ++q) r4[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      // the sort keeps the window start within the bin's first OMB cells, so
      // rel + W - 1 <= S - 1 <= 15; the test keeps the row in bounds regardless
      const int rel1 = (i1 - o1) & (nf - 1), rel2 = (i2 - o2) & (nf - 1);
      if (valid && rel1 < OMB && rel2 < OMB) {
#pragma unroll
        for (int r = 0; r < W; ++r) {
          row[rel1 + r] = psi_es(s1 + (float)r, bl2, two_over_w);
          row[16 + rel2 + r] = psi_es(s2 + (float)r, bl2, two_over_w);
        }
      }
#pragma unroll
      for (int c = 0; c < WV; ++c) row[32 + c] = Wk.v[c];
    }
    // the rows written by other lanes of this wave are read below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Phase 2: 16 chunks of 4 points on the matrix cores.
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const float* rk = tab + (4 * q + k) * PR;
      const float a = rk[j];
      const float bv = rk[16 + j];
      acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[0], 0, 0, 0);
#pragma unroll
      for (int c = 1; c < CH; ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a * rk[32 + c - 1], bv, acc[c], 0, 0, 0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (++since == OFLUSH) {
      flush();
      since = 0;
    }
  }
  flush();
  __syncthreads();
  for (int i = tid; i < C * 256; i += 64 * OWAVE) {
    const double v = sub[i];
    if (v == 0.0) continue;
    const int c = i >> 8, x = (i >> 4) & 15, y = i & 15;
    if (x >= S || y >= S) continue;
    int g1 = o1 + x, g2 = o2 + y;
    g1 = g1 >= nf ? g1 - nf : g1;
    g2 = g2 >= nf ? g2 - nf : g2;
    atomicAdd(&grid[((int64_t)c * nf + g1) * nf + g2], v);
  }
}

template <int W, int WV>
void launch_op(hipStream_t st, int blocks, const uint2* c2, const uint32_t* w, int C, const uint64_t* start, int nbx,
               int nf, int fb, float bt, int slices, double* grid) {
  hipLaunchKernelGGL((k_spread_op<W, WV>), dim3(blocks), dim3(64 * OWAVE), 0, st, c2, w, C, start, nbx, nf, fb, bt,
                     slices, grid);
}

template <int W>
fk_status launch_op_w(hipStream_t st, int wv, int blocks, const uint2* c2, const uint32_t* w, int C,
                      const uint64_t* start, int nbx, int nf, int fb, float bt, int slices, double* grid) {
  switch (wv) {
    case 0: launch_op<W, 0>(st, blocks, c2, w, C, start, nbx, nf, fb, bt, slices, grid); break;
    case 1: launch_op<W, 1>(st, blocks, c2, w, C, start, nbx, nf, fb, bt, slices, grid); break;
    case 2: launch_op<W, 2>(st, blocks, c2, w, C, start, nbx, nf, fb, bt, slices, grid); break;
    case 4: launch_op<W, 4>(st, blocks, c2, w, C, start, nbx, nf, fb, bt, slices, grid); break;
    case 8: launch_op<W, 8>(st, blocks, c2, w, C, start, nbx, nf, fb, bt, slices, grid); break;
    default: return FK_EINVAL;
  }
  return FK_OK;
}

}  // namespace

int spread_op_bin() { return OMB; }

bool spread_op_ok(int nw, int W) { return nw >= 0 && nw <= 7 && W >= 4 && W <= 8; }

fk_status launch_spread_op(hipStream_t st, int W, const uint32_t* crd, const uint32_t* wts, int nw,
                           const uint64_t* start, int nbx, int nb, int nf, int fb, double beta, int64_t n,
                           int spread_pts, double* grid) {
  if (!spread_op_ok(nw, W) || nbx * OMB != nf || spread_pts < 256) return FK_EINVAL;
  const int wv = sort2_words(nw);
  const int64_t per_bin = (n + nb - 1) / nb;
  const int slices = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (per_bin + spread_pts - 1) / spread_pts));
  const int blocks = nb * slices;
  const uint2* c2 = reinterpret_cast<const uint2*>(crd);
  const float bt = (float)beta;
  fk_status s = FK_EINVAL;
  switch (W) {
    case 4: s = launch_op_w<4>(st, wv, blocks, c2, wts, nw + 1, start, nbx, nf, fb, bt, slices, grid); break;
    case 5: s = launch_op_w<5>(st, wv, blocks, c2, wts, nw + 1, start, nbx, nf, fb, bt, slices, grid); break;
    case 6: s = launch_op_w<6>(st, wv, blocks, c2, wts, nw + 1, start, nbx, nf, fb, bt, slices, grid); break;
    case 7: s = launch_op_w<7>(st, wv, blocks, c2, wts, nw + 1, start, nbx, nf, fb, bt, slices, grid); break;
    case 8: s = launch_op_w<8>(st, wv, blocks, c2, wts, nw + 1, start, nbx, nf, fb, bt, slices, grid); break;
    default: return FK_EINVAL;
  }
  if (s != FK_OK) return s;
  return hipGetLastError() == hipSuccess ? FK_OK : FK_EHIP;
}

}  // namespace fk
