// 2-D binned spread on MFMA, for 8..16 weight channels (the batched targets).
//
// The type-1 sums of Sec. 2.3 for T targets share the kernel weights of each
// point: every point adds W[c] psi1[a] psi2[b] to the w x w grid cells of its
// window, for the ones channel (the Gram, c = 0) and the T target channels.
// With LDS atomics that is w^2 (T+1) atomic adds per point; here it becomes a
// dense matrix product on the matrix cores:
//
// * bins are MB x MB grid cells (MB = 4), counting-sorted beforehand so a bin's
//   points are contiguous: fixed-point coordinates [U1, U2] (8 B) and a
//   64-byte block of 16 FP32 weights (zero padded) per point;
// * a workgroup takes a slice of one bin and stages batches of MP points in
//   LDS (the next batch is loaded into registers while the current one is
//   processed); each point's window start (l1, l2) relative to the bin takes
//   (MB+1)^2 = 25 values, and the batch is counting-sorted by it;
// * the exponential-of-semicircle values psi1[0..w), psi2[0..w) of every point
//   are evaluated once per point into LDS;
// * for one window-start group, 4 points at a time,
//     D[c][cell] += sum_k W[c][k] * (psi1_k[cell / w] psi2_k[cell % w])
//   is v_mfma_f32_16x16x4f32 with rows = 16 target channels, columns = 16 of
//   the w^2 <= 64 window cells (4 column tiles), K = the 4 points; the ones
//   channel is the column sum of the same kernel products (vector ALUs);
// * each wave owns fixed groups, so its FP32 accumulators stay in registers
//   across batches; every MFLUSH batches they are added into an FP64 LDS
//   subgrid (LDS ds_add_f64), which is added into the FP64 grid at the end.
//
// Lane layout of v_mfma_f32_16x16x4f32 (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; element v of the result holds row 4*(l/16)+v, column l%16.
#include "fk_internal.h"

namespace fk {

namespace {

constexpr int MB = 4;                       // bin edge in grid cells
constexpr int MG = (MB + 1) * (MB + 1);     // window-start groups per bin
constexpr int NWAVE = 8;
constexpr int NTHR = 64 * NWAVE;
constexpr int MGW = (MG + NWAVE - 1) / NWAVE;   // groups per wave
constexpr int MP = 512;                     // points per LDS batch
constexpr int MFLUSH = 8;                   // batches between FP32 -> FP64 flushes
constexpr int WQ = MP * 4 / NTHR;           // 16-byte weight quads per thread per batch

typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float psi_es(float s, float beta, float two_over_w) {
  float z = s * two_over_w;
  float r = fmaxf(1.0f - z * z, 0.0f);
  return __expf(beta * (__fsqrt_rn(r) - 1.0f));
}

// i0 = ceil(u - w/2), s0 = i0 - u from a fixed-point coordinate with fb fraction bits.
__device__ __forceinline__ void win_start(uint32_t U, int fb, int w, int* i0, float* s0) {
  int64_t V = (int64_t)U - ((int64_t)w << (fb - 1));
  int64_t one = (int64_t)1 << fb;
  int64_t c = (V >= 0) ? ((V + one - 1) >> fb) : -((-V) >> fb);
  *i0 = (int)c;
  *s0 = (float)((double)((c << fb) - (int64_t)U) * (1.0 / (double)one));
}

struct Prefetch {
  uint2 c;
  uint4 w[WQ];
};

// Load the batch [base, base + np) of coordinates and weight blocks into registers.
__device__ __forceinline__ void prefetch(Prefetch& pf, const uint2* __restrict__ crd, const uint4* __restrict__ wts,
                                         uint64_t base, int np, int tid) {
  if (tid < np) pf.c = crd[base + tid];
#pragma unroll
  for (int q = 0; q < WQ; ++q) {
    const int i = tid + q * NTHR;
    if (i < np * 4) pf.w[q] = wts[base * 4 + i];
  }
}

template <int W>
__global__ __launch_bounds__(NTHR) void k_spread_mfma(const uint2* __restrict__ crd, const uint4* __restrict__ wts,
                                                      int nw, const uint64_t* __restrict__ start, int nbx, int nf,
                                                      int fb, float beta, int slices, double* __restrict__ grid) {
  static_assert(W <= 8, "the window must fit 4 column tiles and 16 lanes");
  static_assert(MP <= NTHR, "one coordinate per thread per batch");
  constexpr int S = MB + W;
  extern __shared__ double smem_d[];
  const int C = nw + 1;
  const float two_over_w = 2.0f / (float)W;
  const int subn = (S * S * C + 1) & ~1;                          // keep 16-byte alignment below
  double* sub = smem_d;                                            // S*S*C doubles
  float* psi = reinterpret_cast<float*>(sub + subn);               // MP*16 floats
  uint4* sw = reinterpret_cast<uint4*>(psi + MP * 16);             // MP*4 quads (16 weights per point)
  uint2* sc = reinterpret_cast<uint2*>(sw + MP * 4);               // MP coordinates
  uint16_t* perm = reinterpret_cast<uint16_t*>(sc + MP);           // MP
  uint16_t* rank = perm + MP;                                      // MP
  uint8_t* keyv = reinterpret_cast<uint8_t*>(rank + MP);           // MP
  int* gcount = reinterpret_cast<int*>(keyv + MP);                 // 32
  int* gstart = gcount + 32;                                       // 32
  const float* swf = reinterpret_cast<const float*>(sw);

  const int b = blockIdx.x / slices;
  const int sl = blockIdx.x - b * slices;
  const uint64_t p0 = start[b], p1 = start[b + 1];
  const uint64_t len = p1 - p0;
  const uint64_t q0 = p0 + len * sl / slices;
  const uint64_t q1 = p0 + len * (sl + 1) / slices;
  if (q0 == q1) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int bx = b / nbx, by = b - bx * nbx;
  const int o1 = bx * MB - W / 2, o2 = by * MB - W / 2;   // window starts lie in [o, o + MB]
  for (int i = tid; i < S * S * C; i += NTHR) sub[i] = 0.0;

  floatx4_t acc[MGW][4];
  float ones[MGW][4];
#pragma unroll
  for (int s = 0; s < MGW; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[s][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
      ones[s][t] = 0.f;
    }

  const int kslot = lane >> 4, jj = lane & 15;
  int ca[4], cb[4];
  bool cin[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int cell = t * 16 + jj;
    cin[t] = cell < W * W;
    ca[t] = cin[t] ? cell / W : 0;
    cb[t] = cin[t] ? cell - (cell / W) * W : 0;
  }

  Prefetch pf;
  prefetch(pf, crd, wts, q0, (int)min<uint64_t>(MP, q1 - q0), tid);
  int batch = 0;
  for (uint64_t base = q0; base < q1; base += MP, ++batch) {
    const int np = (int)min<uint64_t>(MP, q1 - base);
    __syncthreads();   // the previous batch is fully consumed
    if (tid < np) sc[tid] = pf.c;
#pragma unroll
    for (int q = 0; q < WQ; ++q) {
      const int i = tid + q * NTHR;
      if (i < np * 4) sw[i] = pf.w[q];
    }
    if (tid < 32) gcount[tid] = 0;
    if (base + MP < q1) prefetch(pf, crd, wts, base + MP, (int)min<uint64_t>(MP, q1 - base - MP), tid);
    __syncthreads();
    if (tid < np) {
      const int p = tid;
      int i1, i2;
      float s1, s2;
      const uint2 U = sc[p];
      win_start(U.x, fb, W, &i1, &s1);
      win_start(U.y, fb, W, &i2, &s2);
      const int k = (i1 - o1) * (MB + 1) + (i2 - o2);
      keyv[p] = (uint8_t)k;
      rank[p] = (uint16_t)atomicAdd(&gcount[k], 1);
      float* ps = psi + p * 16;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        ps[a] = psi_es(s1 + (float)a, beta, two_over_w);
        ps[W + a] = psi_es(s2 + (float)a, beta, two_over_w);
      }
    }
    __syncthreads();
    if (wv == 0) {   // exclusive scan of the 25 group counts in one wave
      int v = lane < MG ? gcount[lane] : 0;
      int x = v;
#pragma unroll
      for (int o = 1; o < 32; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (lane < MG) gstart[lane] = x - v;
    }
    __syncthreads();
    if (tid < np) perm[gstart[keyv[tid]] + rank[tid]] = (uint16_t)tid;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < MGW; ++s) {
      const int g = wv + NWAVE * s;
      if (g >= MG) continue;
      const int cnt = gcount[g], gs = gstart[g];
      for (int c0 = 0; c0 < cnt; c0 += 4) {
        const int idx = c0 + kslot;
        const bool valid = idx < cnt;
        const int p = valid ? perm[gs + idx] : 0;
        const float aop = (valid && jj < nw) ? swf[p * 16 + jj] : 0.f;
        const float* ps = psi + p * 16;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float bv = (valid && cin[t]) ? ps[ca[t]] * ps[W + cb[t]] : 0.f;
          acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bv, acc[s][t], 0, 0, 0);
          ones[s][t] += bv;
        }
      }
    }
    const bool last = base + MP >= q1;
    if (last || (batch % MFLUSH) == MFLUSH - 1) {
#pragma unroll
      for (int s = 0; s < MGW; ++s) {
        const int g = wv + NWAVE * s;
        if (g >= MG) continue;
        const int l1 = g / (MB + 1), l2 = g - (g / (MB + 1)) * (MB + 1);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          float o = ones[s][t];
          o += __shfl_xor(o, 16, 64);
          o += __shfl_xor(o, 32, 64);
          if (cin[t]) {
            double* cp = sub + ((l1 + ca[t]) * S + (l2 + cb[t])) * C;
            if (kslot == 0 && o != 0.f) atomicAdd(cp, (double)o);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = 4 * kslot + v;
              const float x = acc[s][t][v];
              if (row < nw && x != 0.f) atomicAdd(cp + 1 + row, (double)x);
            }
          }
          acc[s][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
          ones[s][t] = 0.f;
        }
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < S * S * C; i += NTHR) {
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

size_t lds_bytes(int W, int nw) {
  const int S = MB + W, C = nw + 1;
  size_t b = sizeof(double) * ((S * S * C + 1) & ~1) + sizeof(float) * MP * 16 + 16 * MP * 4 + 8 * MP +
             2 * sizeof(uint16_t) * MP + MP;
  b = (b + 3) & ~size_t(3);
  return b + 64 * sizeof(int);
}

}  // namespace

int spread_mfma_bin() { return MB; }

bool spread_mfma_ok(int nw, int W) { return nw >= 8 && nw <= 16 && W >= 4 && W <= 8; }

fk_status launch_spread_mfma(hipStream_t st, int W, const uint32_t* crd, const uint32_t* wts, int nw,
                             const uint64_t* start, int nbx, int nb, int nf, int fb, double beta, int64_t n,
                             double* grid) {
  const int64_t per_bin = (n + nb - 1) / nb;
  const int slices = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (per_bin + 16383) / 16384));
  const int blocks = nb * slices;
  const size_t lds = lds_bytes(W, nw);
  if (lds > 160 * 1024) return FK_EINVAL;
  const float bt = (float)beta;
  const uint2* c2 = reinterpret_cast<const uint2*>(crd);
  const uint4* w4 = reinterpret_cast<const uint4*>(wts);
  switch (W) {
    case 4: hipLaunchKernelGGL(k_spread_mfma<4>, dim3(blocks), dim3(NTHR), lds, st, c2, w4, nw, start, nbx, nf, fb,
                               bt, slices, grid); break;
    case 5: hipLaunchKernelGGL(k_spread_mfma<5>, dim3(blocks), dim3(NTHR), lds, st, c2, w4, nw, start, nbx, nf, fb,
                               bt, slices, grid); break;
    case 6: hipLaunchKernelGGL(k_spread_mfma<6>, dim3(blocks), dim3(NTHR), lds, st, c2, w4, nw, start, nbx, nf, fb,
                               bt, slices, grid); break;
    case 7: hipLaunchKernelGGL(k_spread_mfma<7>, dim3(blocks), dim3(NTHR), lds, st, c2, w4, nw, start, nbx, nf, fb,
                               bt, slices, grid); break;
    case 8: hipLaunchKernelGGL(k_spread_mfma<8>, dim3(blocks), dim3(NTHR), lds, st, c2, w4, nw, start, nbx, nf, fb,
                               bt, slices, grid); break;
    default: return FK_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? FK_OK : FK_EHIP;
}

}  // namespace fk
