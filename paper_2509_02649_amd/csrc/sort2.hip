// Two-pass bin sort of the point stream for the MFMA spreads.
//
// The matrix-core spreads take the points of one bin four at a time, so the type-1
// stage first orders the stream by bin.  A one-pass counting sort into the nbx^2
// bins sends consecutive points to unrelated addresses, and on HBM3E such
// scattered 8- and 64-byte writes run far below the streaming rate.  Here the order
// is reached in two counting passes over nbx buckets each (the bin row bx, then the
// bin column by inside a row).  A point's bin on an axis is set by the first cell of
// its kernel window, not by the cell it lies in, so that a bin's windows cover
// MB + w - 1 cells per axis.  A workgroup ranks a batch of points by bucket in LDS,
// stages the batch in bucket order, and writes each bucket's part as one contiguous
// run, so both passes write in runs and read in streams.
//
// 8..16 weight channels (records of 16 weight words, zero padded):
//   pass 1: X, Y (structure of arrays)          -> crd1 / wts1, grouped by bx
//   pass 2: one workgroup per (bx, slice) of it -> crd and, per point, its position
//           in crd1 / wts1, grouped by bin; the 64-byte weight blocks are not moved
//           again (the spread gathers them from wts1).
// 0..7 weight channels (records of 1, 2, 4 or 8 weight words):
//   pass 1 as above; pass 2 -> crd / wts, grouped by bin.
//
// The order of points inside a bin is not specified (LDS atomics rank them).
#include "fk_internal.h"
#include "fk_device.h"

#include <algorithm>

namespace fk {

namespace {

constexpr int BT = 1024;       // points per staged batch, one per thread
constexpr int KMAX = 256;      // largest bucket count (nf / MB for nf <= 1024)

struct Stage {
  unsigned long long cur[KMAX];   // next output position of every bucket
  uint32_t hist[KMAX];            // bucket counts of the current batch
  uint32_t lofs[KMAX];            // their exclusive prefix sums
  uint32_t total;
  uint16_t sbin[BT];              // bucket of every staged slot
  uint2 scrd[BT];
  uint4 swts[BT * 4];
};

// Rank of every point of the batch inside its bucket (LDS atomics), and the
// exclusive prefix sums of the batch's bucket counts (sm.lofs, sm.total).
template <class St>
__device__ __forceinline__ uint32_t rank_scan(St& sm, int nk, bool ok, int key) {
  const int tid = threadIdx.x;
  const uint32_t rank = ok ? atomicAdd(&sm.hist[key], 1u) : 0u;
  __syncthreads();
  if (tid < 64) {   // exclusive scan of the nk <= 256 counts in one wave
    const int per = (nk + 63) / 64;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i) {
      const int b = tid * per + i;
      if (b < nk) s += sm.hist[b];
    }
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (tid >= o) x += y;
    }
    uint32_t run = x - s;
    for (int i = 0; i < per; ++i) {
      const int b = tid * per + i;
      if (b < nk) {
        sm.lofs[b] = run;
        run += sm.hist[b];
      }
    }
    if (tid == 63) sm.total = x;
  }
  __syncthreads();
  return rank;
}

// Write the staged coordinates as runs, one per bucket (after the staging barrier).
template <class St>
__device__ __forceinline__ void write_coords(St& sm, uint2* __restrict__ crd_out) {
  const int tid = threadIdx.x;
  if ((uint32_t)tid < sm.total) {
    const int b = sm.sbin[tid];
    crd_out[sm.cur[b] + (tid - sm.lofs[b])] = sm.scrd[tid];
  }
}

// After the staged batch is written: advance the bucket cursors, clear the counts.
template <class St>
__device__ __forceinline__ void advance_cursors(St& sm, int nk) {
  __syncthreads();
  for (int b = threadIdx.x; b < nk; b += BT) {
    sm.cur[b] += sm.hist[b];
    sm.hist[b] = 0;
  }
  __syncthreads();
}

// Rank the batch by bucket, stage it in bucket order and write the runs.
// Every thread of the workgroup calls this once per batch with point t (key, U) and
// its weights v0..v3 (the four 16-byte quarters of its 64-byte block).
__device__ __forceinline__ void stage_batch(Stage& sm, int nk, bool ok, int key, uint2 U, uint4 v0, uint4 v1,
                                            uint4 v2, uint4 v3, uint2* __restrict__ crd_out,
                                            uint4* __restrict__ wts_out) {
  const int tid = threadIdx.x;
  const uint32_t rank = rank_scan(sm, nk, ok, key);
  if (ok) {
    const uint32_t s = sm.lofs[key] + rank;
    sm.sbin[s] = (uint16_t)key;
    sm.scrd[s] = U;
    sm.swts[s * 4 + 0] = v0;
    sm.swts[s * 4 + 1] = v1;
    sm.swts[s * 4 + 2] = v2;
    sm.swts[s * 4 + 3] = v3;
  }
  __syncthreads();
  const uint32_t total = sm.total;
  write_coords(sm, crd_out);
  for (uint32_t q = tid; q < total * 4; q += BT) {
    const uint32_t s = q >> 2;
    const int b = sm.sbin[s];
    wts_out[(sm.cur[b] + (s - sm.lofs[b])) * 4 + (q & 3)] = sm.swts[q];
  }
  advance_cursors(sm, nk);
}

// Pass 1 counts: bucket = bin row of every valid point, one row of nbx counts per
// workgroup (contiguous chunks of the input).  Each thread takes CU1 points per
// step, their loads issued together.
constexpr int CU1 = 4;
template <typename TX>
__global__ __launch_bounds__(BT) void k_s2_count1(const TX* __restrict__ X, int64_t n, int64_t xstride,
                                                  double scale, uint32_t nf_fix, int fb, uint32_t wbias,
                                                  int tshift, int nbx, int64_t chunk, uint32_t* __restrict__ cnt,
                                                  int* flags) {
  __shared__ uint32_t hist[KMAX];
  for (int i = threadIdx.x; i < nbx; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(n, beg + chunk);
  for (int64_t j0 = beg + threadIdx.x; j0 < end; j0 += (int64_t)CU1 * BT) {
    double x1[CU1], x2[CU1];
#pragma unroll
    for (int u = 0; u < CU1; ++u) {
      const int64_t jc = min(j0 + (int64_t)u * BT, end - 1);
      x1[u] = (double)X[jc];
      x2[u] = (double)X[xstride + jc];
    }
#pragma unroll
    for (int u = 0; u < CU1; ++u) {
      if (j0 + (int64_t)u * BT >= end) break;
      uint32_t U1, U2;
      bool ok = to_fixed(x1[u], scale, nf_fix, &U1, flags);
      ok = to_fixed(x2[u], scale, nf_fix, &U2, flags) && ok;
      if (ok) atomicAdd(&hist[window_bin(U1, fb, wbias, (int)(nf_fix >> fb), tshift)], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbx; i += blockDim.x) cnt[(int64_t)blockIdx.x * nbx + i] = hist[i];
}

// Pass 1 scatter.  off holds, per workgroup and bucket, the count of the bucket's
// points in earlier workgroups; start1 the bucket starts.  The inputs of the next
// batch are loaded (unconditionally, index clamped to the chunk) while the current
// batch is ranked, staged and written.
template <typename TX>
__global__ __launch_bounds__(BT) void k_s2_scatter1(const TX* __restrict__ X, int64_t n,
                                                    int64_t xstride, const TX* __restrict__ Y, int nw,
                                                    double scale, uint32_t nf_fix, int fb, uint32_t wbias,
                                                    int tshift, int nbx, int64_t chunk,
                                                    const uint32_t* __restrict__ off,
                                                    const uint64_t* __restrict__ start1,
                                                    uint2* __restrict__ crd1, uint4* __restrict__ wts1,
                                                    int* flags) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Stage& sm = *reinterpret_cast<Stage*>(smem_raw);
  const int tid = threadIdx.x;
  for (int b = tid; b < nbx; b += BT) {
    sm.cur[b] = start1[b] + off[(int64_t)blockIdx.x * nbx + b];
    sm.hist[b] = 0;
  }
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(n, beg + chunk);
  if (beg >= end) return;
  double nx1, nx2;
  float nw_[16];
  auto fetch = [&](int64_t j) {
    const int64_t jc = min(j, end - 1);
    nx1 = (double)X[jc];
    nx2 = (double)X[xstride + jc];
#pragma unroll
    for (int c = 0; c < 16; ++c) nw_[c] = (float)Y[(int64_t)min(c, nw - 1) * n + jc];
  };
  fetch(beg + tid);
  for (int64_t base = beg; base < end; base += BT) {
    const int64_t j = base + tid;
    const double x1 = nx1, x2 = nx2;
    float w[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) w[c] = nw_[c];
    fetch(base + BT + tid);
    bool ok = false;
    uint2 U = make_uint2(0u, 0u);
    if (j < end) {
      ok = to_fixed(x1, scale, nf_fix, &U.x, flags);
      ok = to_fixed(x2, scale, nf_fix, &U.y, flags) && ok;
    }
    uint32_t wb[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float wc = (ok && c < nw) ? w[c] : 0.f;
      if (!(wc == wc) || isinf(wc)) {
        atomicOr(&flags[kFlagNaN], 1);
        wc = 0.f;
      }
      wb[c] = __float_as_uint(wc);
    }
    const int key = ok ? window_bin(U.x, fb, wbias, (int)(nf_fix >> fb), tshift) : 0;
    stage_batch(sm, nbx, ok, key, U, make_uint4(wb[0], wb[1], wb[2], wb[3]), make_uint4(wb[4], wb[5], wb[6], wb[7]),
                make_uint4(wb[8], wb[9], wb[10], wb[11]), make_uint4(wb[12], wb[13], wb[14], wb[15]), crd1, wts1);
  }
}

// Pass 2 counts: workgroup (bx, slice) counts the bin columns of its slice of row bx,
// CU1 loads in flight per thread.
__global__ __launch_bounds__(BT) void k_s2_count2(const uint2* __restrict__ crd1,
                                                  const uint64_t* __restrict__ start1, int slices, int fb,
                                                  uint32_t wbias, int nf, int tshift, int nbx,
                                                  uint32_t* __restrict__ cnt2) {
  __shared__ uint32_t hist[KMAX];
  for (int i = threadIdx.x; i < nbx; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int bx = blockIdx.x / slices, sl = blockIdx.x - bx * slices;
  const uint64_t p0 = start1[bx], len = start1[bx + 1] - p0;
  const uint64_t q0 = p0 + len * sl / slices, q1 = p0 + len * (sl + 1) / slices;
  for (uint64_t p = q0 + threadIdx.x; p < q1; p += (uint64_t)CU1 * BT) {
    uint32_t y[CU1];
#pragma unroll
    for (int u = 0; u < CU1; ++u) y[u] = crd1[min(p + (uint64_t)u * BT, q1 - 1)].y;
#pragma unroll
    for (int u = 0; u < CU1; ++u)
      if (p + (uint64_t)u * BT < q1) atomicAdd(&hist[window_bin(y[u], fb, wbias, nf, tshift)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbx; i += blockDim.x) cnt2[(int64_t)blockIdx.x * nbx + i] = hist[i];
}

// Pass 2 offsets, one workgroup per row bx: off2[(bx, slice, by)] = count of bin
// (bx, by) in earlier slices of the row, and start[bx * nbx + by] = the bin start.
__global__ __launch_bounds__(KMAX) void k_s2_scan2(const uint32_t* __restrict__ cnt2,
                                                  const uint64_t* __restrict__ start1, int slices, int nbx,
                                                  uint32_t* __restrict__ off2, uint64_t* __restrict__ start) {
  __shared__ uint64_t tot[KMAX];
  const int bx = blockIdx.x, by = threadIdx.x;
  uint64_t run = 0;
  if (by < nbx) {
    for (int s = 0; s < slices; ++s) {
      const int64_t i = ((int64_t)bx * slices + s) * nbx + by;
      off2[i] = (uint32_t)run;
      run += cnt2[i];
    }
    tot[by] = run;
  }
  __syncthreads();
  if (by == 0) {
    uint64_t acc = start1[bx];
    for (int i = 0; i < nbx; ++i) {
      const uint64_t t = tot[i];
      tot[i] = acc;
      acc += t;
    }
  }
  __syncthreads();
  if (by < nbx) start[(int64_t)bx * nbx + by] = tot[by];
  if (bx == nbx - 1 && by == 0) start[(int64_t)nbx * nbx] = start1[nbx];
}


// ---------------------------------------------------------------- narrow records
// The same two passes for 0..7 weight channels (the outer-product spread): records of
// WV = 0, 1, 2, 4 or 8 weight words per point (zero padded), staged word by word.  A
// record is small, so each thread takes NPT points per batch (BT NPT points between
// barriers, longer runs per bucket).
template <int WV>
constexpr int narrow_ppt() { return WV <= 2 ? 4 : (WV == 4 ? 2 : 1); }
constexpr int kPosPpt = 8;   // points per thread of the position pass (116 KB of LDS)

template <int WV, int P = narrow_ppt<WV>()>
struct StageN {
  static constexpr int NPT = P;
  unsigned long long cur[KMAX];
  uint32_t hist[KMAX];
  uint32_t lofs[KMAX];
  uint32_t total;
  uint16_t sbin[BT * NPT];
  uint2 scrd[BT * NPT];
  uint32_t swts[BT * NPT * (WV > 0 ? WV : 1)];
};

// Exclusive prefix sums of the batch's bucket counts (after the rank atomics).
template <class St>
__device__ __forceinline__ void scan_counts(St& sm, int nk) {
  const int tid = threadIdx.x;
  __syncthreads();
  if (tid < 64) {
    const int per = (nk + 63) / 64;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i) {
      const int b = tid * per + i;
      if (b < nk) s += sm.hist[b];
    }
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (tid >= o) x += y;
    }
    uint32_t run = x - s;
    for (int i = 0; i < per; ++i) {
      const int b = tid * per + i;
      if (b < nk) {
        sm.lofs[b] = run;
        run += sm.hist[b];
      }
    }
    if (tid == 63) sm.total = x;
  }
  __syncthreads();
}

template <int WV, int P>
__device__ __forceinline__ void write_batch_n(StageN<WV, P>& sm, uint2* __restrict__ crd_out,
                                              uint32_t* __restrict__ wts_out) {
  const uint32_t total = sm.total;
  for (uint32_t q = threadIdx.x; q < total; q += BT) {
    const int b = sm.sbin[q];
    crd_out[sm.cur[b] + (q - sm.lofs[b])] = sm.scrd[q];
  }
  if constexpr (WV > 0) {
    for (uint32_t q = threadIdx.x; q < total * WV; q += BT) {
      const uint32_t s = q / WV;
      const int b = sm.sbin[s];
      wts_out[(sm.cur[b] + (s - sm.lofs[b])) * WV + q % WV] = sm.swts[q];
    }
  }
}

template <typename TX, int WV>
__global__ __launch_bounds__(BT) void k_s2n_scatter1(const TX* __restrict__ X, int64_t n, int64_t xstride,
                                                     const TX* __restrict__ Y, int nw, double scale,
                                                     uint32_t nf_fix, int fb, uint32_t wbias, int tshift, int nbx,
                                                     int64_t chunk, const uint32_t* __restrict__ off,
                                                     const uint64_t* __restrict__ start1,
                                                     uint2* __restrict__ crd1, uint32_t* __restrict__ wts1,
                                                     int* flags) {
  constexpr int NPT = narrow_ppt<WV>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  StageN<WV>& sm = *reinterpret_cast<StageN<WV>*>(smem_raw);
  const int tid = threadIdx.x;
  for (int b = tid; b < nbx; b += BT) {
    sm.cur[b] = start1[b] + off[(int64_t)blockIdx.x * nbx + b];
    sm.hist[b] = 0;
  }
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(n, beg + chunk);
  if (beg >= end) return;
  const int nf = (int)(nf_fix >> fb);
  // next batch in flight: point base + u BT + tid of slot u (index clamped to the
  // chunk; no target row is read when nw = 0)
  double nx1[NPT], nx2[NPT];
  float ny[NPT][WV > 0 ? WV : 1];
#define FK_FETCH1N(bb)                                                                     \
  _Pragma("unroll") for (int u = 0; u < NPT; ++u) {                                        \
    const int64_t jc = min((int64_t)(bb) + u * BT + tid, end - 1);                         \
    nx1[u] = (double)X[jc];                                                                \
    nx2[u] = (double)X[xstride + jc];                                                      \
    _Pragma("unroll") for (int c = 0; c < WV; ++c)                                         \
      ny[u][c] = nw > 0 ? (float)Y[(int64_t)min(c, nw - 1) * n + jc] : 0.f;               \
  }
  FK_FETCH1N(beg);
  for (int64_t base = beg; base < end; base += (int64_t)BT * NPT) {
    double x1[NPT], x2[NPT];
    float w[NPT][WV > 0 ? WV : 1];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      x1[u] = nx1[u];
      x2[u] = nx2[u];
#pragma unroll
      for (int c = 0; c < WV; ++c) w[u][c] = ny[u][c];
    }
    FK_FETCH1N(base + (int64_t)BT * NPT);
    bool ok[NPT];
    uint2 U[NPT];
    int key[NPT];
    uint32_t rank[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      ok[u] = false;
      U[u] = make_uint2(0u, 0u);
      if (base + u * BT + tid < end) {
        ok[u] = to_fixed(x1[u], scale, nf_fix, &U[u].x, flags);
        ok[u] = to_fixed(x2[u], scale, nf_fix, &U[u].y, flags) && ok[u];
      }
      key[u] = ok[u] ? window_bin(U[u].x, fb, wbias, nf, tshift) : 0;
      rank[u] = ok[u] ? atomicAdd(&sm.hist[key[u]], 1u) : 0u;
    }
    scan_counts(sm, nbx);
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      if (!ok[u]) continue;
      const uint32_t s = sm.lofs[key[u]] + rank[u];
      sm.sbin[s] = (uint16_t)key[u];
      sm.scrd[s] = U[u];
#pragma unroll
      for (int c = 0; c < WV; ++c) {
        float wc = c < nw ? w[u][c] : 0.f;
        if (!(wc == wc) || isinf(wc)) {
          atomicOr(&flags[kFlagNaN], 1);
          wc = 0.f;
        }
        sm.swts[s * WV + c] = __float_as_uint(wc);
      }
    }
    __syncthreads();
    write_batch_n(sm, crd1, wts1);
    advance_cursors(sm, nbx);
  }
#undef FK_FETCH1N
}

// Pass 2 for narrow records.  Slot u of the batch holds points base + u BT + tid; the
// wave's 64 weight records of a slot are read as 64 WV contiguous words (word
// lane + 64 v of the wave's block), and each word is staged at the slot of its
// point, taken from the owning lane by a wave shuffle.  With kPosition (WV = 1) the
// record word is not read but is the point's position in the pass-1 output: the
// sorted stream then refers back to the weight blocks grouped by bin row.
template <int WV, bool kPosition, int NPT = narrow_ppt<WV>()>
__global__ __launch_bounds__(BT) void k_s2n_scatter2(const uint2* __restrict__ crd1,
                                                     const uint32_t* __restrict__ wts1,
                                                     const uint64_t* __restrict__ start1,
                                                     const uint32_t* __restrict__ off2,
                                                     const uint64_t* __restrict__ start, int slices, int fb,
                                                     uint32_t wbias, int nf, int tshift, int nbx,
                                                     uint2* __restrict__ crd, uint32_t* __restrict__ wts) {
  constexpr int WD = WV > 0 ? WV : 1;   // divisor for the word index (no words when WV = 0)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  StageN<WV, NPT>& sm = *reinterpret_cast<StageN<WV, NPT>*>(smem_raw);
  const int tid = threadIdx.x;
  const int bx = blockIdx.x / slices, sl = blockIdx.x - bx * slices;
  for (int b = tid; b < nbx; b += BT) {
    sm.cur[b] = start[(int64_t)bx * nbx + b] + off2[(int64_t)blockIdx.x * nbx + b];
    sm.hist[b] = 0;
  }
  __syncthreads();
  const uint64_t p0 = start1[bx], len = start1[bx + 1] - p0;
  const uint64_t q0 = p0 + len * sl / slices, q1 = p0 + len * (sl + 1) / slices;
  if (q0 >= q1) return;
  const int lane = tid & 63;
  const uint64_t wb = (uint64_t)(tid & ~63);
  uint2 nU[NPT];
  uint32_t nv[NPT][WV > 0 ? WV : 1];
#define FK_FETCH2N(bb)                                                                      \
  _Pragma("unroll") for (int u = 0; u < NPT; ++u) {                                         \
    const uint64_t g0 = (uint64_t)(bb) + (uint64_t)u * BT;                                  \
    nU[u] = crd1[min(g0 + tid, q1 - 1)];                                                    \
    _Pragma("unroll") for (int v = 0; v < WV; ++v) {                                        \
      const uint32_t m = (uint32_t)lane + 64u * v;                                          \
      nv[u][v] = kPosition ? (uint32_t)(g0 + wb + m / WD)                                   \
                           : wts1[min(g0 + wb + m / WD, q1 - 1) * WV + m % WD];             \
    }                                                                                       \
  }
  FK_FETCH2N(q0);
  for (uint64_t base = q0; base < q1; base += (uint64_t)BT * NPT) {
    uint2 U[NPT];
    uint32_t v[NPT][WV > 0 ? WV : 1];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      U[u] = nU[u];
#pragma unroll
      for (int c = 0; c < WV; ++c) v[u][c] = nv[u][c];
    }
    FK_FETCH2N(base + (uint64_t)BT * NPT);
    bool ok[NPT];
    int key[NPT];
    uint32_t rank[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      ok[u] = base + (uint64_t)u * BT + tid < q1;
      key[u] = ok[u] ? window_bin(U[u].y, fb, wbias, nf, tshift) : 0;
      rank[u] = ok[u] ? atomicAdd(&sm.hist[key[u]], 1u) : 0u;
    }
    scan_counts(sm, nbx);
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const uint32_t s = ok[u] ? sm.lofs[key[u]] + rank[u] : 0xffffffffu;
      if (ok[u]) {
        sm.sbin[s] = (uint16_t)key[u];
        sm.scrd[s] = U[u];
      }
#pragma unroll
      for (int c = 0; c < WV; ++c) {
        const uint32_t m = (uint32_t)lane + 64u * c;
        const uint32_t su = __shfl(s, (int)(m / WD), 64);
        if (su != 0xffffffffu) sm.swts[su * WV + m % WD] = v[u][c];
      }
    }
    __syncthreads();
    write_batch_n(sm, crd, wts);
    advance_cursors(sm, nbx);
  }
#undef FK_FETCH2N
}

// Offsets of pass 1: off[k][b] = number of points of bucket b in workgroups < k,
// and start1[b] (start1[nk] = number of valid points).  One workgroup of 1024
// threads: thread (grp, b) sums a range of workgroups, the group sums are
// scanned, then each range is rewritten as running offsets.
constexpr int SG = 1024 / KMAX;   // workgroup ranges per bucket
__global__ __launch_bounds__(1024) void k_s2_scan1(const uint32_t* __restrict__ cnt, int nk, int nblk,
                                                  uint32_t* __restrict__ off, uint64_t* __restrict__ start1) {
  __shared__ uint64_t part[SG][KMAX];
  __shared__ uint64_t tot[KMAX];
  const int b = threadIdx.x % KMAX, grp = threadIdx.x / KMAX;
  const int per = (nblk + SG - 1) / SG;
  const int k0 = grp * per, k1 = min(nblk, k0 + per);
  uint64_t s = 0;
  if (b < nk)
    for (int k = k0; k < k1; ++k) s += cnt[(int64_t)k * nk + b];
  part[grp][b] = s;
  __syncthreads();
  if (grp == 0 && b < nk) {
    uint64_t run = 0;
    for (int g = 0; g < SG; ++g) {
      const uint64_t t = part[g][b];
      part[g][b] = run;
      run += t;
    }
    tot[b] = run;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t acc = 0;
    for (int i = 0; i < nk; ++i) {
      start1[i] = acc;
      acc += tot[i];
    }
    start1[nk] = acc;
  }
  if (b < nk) {
    uint64_t run = part[grp][b];
    for (int k = k0; k < k1; ++k) {
      off[(int64_t)k * nk + b] = (uint32_t)run;
      run += cnt[(int64_t)k * nk + b];
    }
  }
}

struct Sort2Geom {
  int nblk1, slices;
  int64_t chunk1;
};

// First pass: up to blk workgroups of at least 65536 points each; second pass: slices of about
// slice_pts points per bin row (at most 256).
Sort2Geom sort2_geom(int64_t n, int nbx, int blk, int64_t slice_pts) {
  Sort2Geom g;
  g.nblk1 = (int)std::min<int64_t>(blk, std::max<int64_t>(1, (n + 65535) / 65536));
  g.chunk1 = (n + g.nblk1 - 1) / g.nblk1;
  g.slices = (int)std::min<int64_t>(256, std::max<int64_t>(1, (n / nbx + slice_pts - 1) / slice_pts));
  return g;
}

// Counts (shared with the wide records), scans, and the narrow-record scatters.
template <int WV>
fk_status sort2_narrow(hipStream_t st, const void* X, fk_dtype dt, int64_t n, int64_t xstride, const void* Y, int nw,
                       uint32_t nf_fix, int fb, uint32_t wbias, double scale, int tshift, int nbx,
                       const Sort2Geom& g, const Sort2Bufs& b, uint32_t* crd, uint32_t* wts, uint64_t* start,
                       int* flags) {
  const size_t lds = sizeof(StageN<WV>);
  const int nf = (int)(nf_fix >> fb);
  if (dt == FK_F64) {
    const double* Xd = static_cast<const double*>(X);
    hipLaunchKernelGGL(k_s2_count1<double>, dim3(g.nblk1), dim3(BT), 0, st, Xd, n, xstride, scale, nf_fix, fb,
                       wbias, tshift, nbx, g.chunk1, b.cnt1, flags);
    hipLaunchKernelGGL(k_s2_scan1, dim3(1), dim3(1024), 0, st, b.cnt1, nbx, g.nblk1, b.off1, b.start1);
    hipLaunchKernelGGL((k_s2n_scatter1<double, WV>), dim3(g.nblk1), dim3(BT), lds, st, Xd, n, xstride,
                       static_cast<const double*>(Y), nw, scale, nf_fix, fb, wbias, tshift, nbx, g.chunk1, b.off1,
                       b.start1, reinterpret_cast<uint2*>(b.crd1), b.wts1, flags);
  } else {
    const float* Xf = static_cast<const float*>(X);
    hipLaunchKernelGGL(k_s2_count1<float>, dim3(g.nblk1), dim3(BT), 0, st, Xf, n, xstride, scale, nf_fix, fb,
                       wbias, tshift, nbx, g.chunk1, b.cnt1, flags);
    hipLaunchKernelGGL(k_s2_scan1, dim3(1), dim3(1024), 0, st, b.cnt1, nbx, g.nblk1, b.off1, b.start1);
    hipLaunchKernelGGL((k_s2n_scatter1<float, WV>), dim3(g.nblk1), dim3(BT), lds, st, Xf, n, xstride,
                       static_cast<const float*>(Y), nw, scale, nf_fix, fb, wbias, tshift, nbx, g.chunk1, b.off1,
                       b.start1, reinterpret_cast<uint2*>(b.crd1), b.wts1, flags);
  }
  hipLaunchKernelGGL(k_s2_count2, dim3(nbx * g.slices), dim3(BT), 0, st, reinterpret_cast<const uint2*>(b.crd1),
                     b.start1, g.slices, fb, wbias, nf, tshift, nbx, b.cnt2);
  hipLaunchKernelGGL(k_s2_scan2, dim3(nbx), dim3(KMAX), 0, st, b.cnt2, b.start1, g.slices, nbx, b.off2, start);
  hipLaunchKernelGGL((k_s2n_scatter2<WV, false>), dim3(nbx * g.slices), dim3(BT), lds, st,
                     reinterpret_cast<const uint2*>(b.crd1), b.wts1, b.start1, b.off2, start, g.slices, fb, wbias,
                     nf, tshift, nbx, reinterpret_cast<uint2*>(crd), wts);
  return hipGetLastError() == hipSuccess ? FK_OK : FK_EHIP;
}

}  // namespace

bool sort2_ok(int nbx) { return nbx >= 1 && nbx <= KMAX; }

int sort2_words(int nw) {
  if (nw >= 8) return 16;
  if (nw == 0) return 0;
  int wv = 1;
  while (wv < nw) wv <<= 1;
  return wv;
}

void sort2_carve(Carve& cv, int64_t n, int nbx, int wv, Sort2Bufs* b) {
  Sort2Geom g = sort2_geom(n, nbx, kSortBlkMax, kSortSliceMin);
  b->cnt1 = cv.take<uint32_t>((size_t)g.nblk1 * nbx);
  b->off1 = cv.take<uint32_t>((size_t)g.nblk1 * nbx);
  b->start1 = cv.take<uint64_t>((size_t)nbx + 1);
  b->cnt2 = cv.take<uint32_t>((size_t)nbx * g.slices * nbx);
  b->off2 = cv.take<uint32_t>((size_t)nbx * g.slices * nbx);
  b->crd1 = cv.take<uint32_t>((size_t)n * 2);
  b->wts1 = cv.take<uint32_t>((size_t)n * wv);
}

fk_status sort2(hipStream_t st, const void* X, fk_dtype dt, int64_t n, int64_t xstride, const void* Y, int nw,
                int nf, int fb, int W, double scale, int tshift, int nbx, const T1Shape& shape, const Sort2Bufs& b,
                uint32_t* crd, uint32_t* wts, uint64_t* start, int* flags) {
  if (!sort2_ok(nbx) || nw > 16 || (nf & (nf - 1)) != 0 || (nbx << tshift) != nf) return FK_EINVAL;
  if (n > (int64_t)0xffffffff) return FK_EINVAL;   // positions are 32-bit
  if (shape.sort_blk < 1 || shape.sort_blk > kSortBlkMax || shape.sort_slice < kSortSliceMin) return FK_EINVAL;
  const Sort2Geom g = sort2_geom(n, nbx, shape.sort_blk, shape.sort_slice);
  const uint32_t nf_fix = (uint32_t)nf << fb;
  const uint32_t one = 1u << fb;
  const uint32_t wbias = (one - 1u) + 8u * one - ((uint32_t)W << (fb - 1));
  const int wv = sort2_words(nw);
  if (wv < 16) {
    switch (wv) {
      case 0: return sort2_narrow<0>(st, X, dt, n, xstride, Y, nw, nf_fix, fb, wbias, scale, tshift, nbx, g, b, crd,
                                     wts, start, flags);
      case 1: return sort2_narrow<1>(st, X, dt, n, xstride, Y, nw, nf_fix, fb, wbias, scale, tshift, nbx, g, b, crd,
                                     wts, start, flags);
      case 2: return sort2_narrow<2>(st, X, dt, n, xstride, Y, nw, nf_fix, fb, wbias, scale, tshift, nbx, g, b, crd,
                                     wts, start, flags);
      case 4: return sort2_narrow<4>(st, X, dt, n, xstride, Y, nw, nf_fix, fb, wbias, scale, tshift, nbx, g, b, crd,
                                     wts, start, flags);
      default: return sort2_narrow<8>(st, X, dt, n, xstride, Y, nw, nf_fix, fb, wbias, scale, tshift, nbx, g, b, crd,
                                      wts, start, flags);
    }
  }
  const size_t lds = sizeof(Stage);
  if (dt == FK_F64) {
    const double* Xd = static_cast<const double*>(X);
    hipLaunchKernelGGL(k_s2_count1<double>, dim3(g.nblk1), dim3(BT), 0, st, Xd, n, xstride, scale, nf_fix, fb,
                       wbias, tshift, nbx, g.chunk1, b.cnt1, flags);
    hipLaunchKernelGGL(k_s2_scan1, dim3(1), dim3(1024), 0, st, b.cnt1, nbx, g.nblk1, b.off1, b.start1);
    hipLaunchKernelGGL(k_s2_scatter1<double>, dim3(g.nblk1), dim3(BT), lds, st, Xd, n, xstride,
                       static_cast<const double*>(Y), nw, scale, nf_fix, fb, wbias, tshift, nbx, g.chunk1, b.off1,
                       b.start1, reinterpret_cast<uint2*>(b.crd1), reinterpret_cast<uint4*>(b.wts1), flags);
  } else {
    const float* Xf = static_cast<const float*>(X);
    hipLaunchKernelGGL(k_s2_count1<float>, dim3(g.nblk1), dim3(BT), 0, st, Xf, n, xstride, scale, nf_fix, fb,
                       wbias, tshift, nbx, g.chunk1, b.cnt1, flags);
    hipLaunchKernelGGL(k_s2_scan1, dim3(1), dim3(1024), 0, st, b.cnt1, nbx, g.nblk1, b.off1, b.start1);
    hipLaunchKernelGGL(k_s2_scatter1<float>, dim3(g.nblk1), dim3(BT), lds, st, Xf, n, xstride,
                       static_cast<const float*>(Y), nw, scale, nf_fix, fb, wbias, tshift, nbx, g.chunk1, b.off1,
                       b.start1, reinterpret_cast<uint2*>(b.crd1), reinterpret_cast<uint4*>(b.wts1), flags);
  }
  hipLaunchKernelGGL(k_s2_count2, dim3(nbx * g.slices), dim3(BT), 0, st, reinterpret_cast<const uint2*>(b.crd1),
                     b.start1, g.slices, fb, wbias, nf, tshift, nbx, b.cnt2);
  hipLaunchKernelGGL(k_s2_scan2, dim3(nbx), dim3(KMAX), 0, st, b.cnt2, b.start1, g.slices, nbx, b.off2, start);
  // pass 2 moves the coordinates and each point's position in the pass-1 output
  // (into wts, one word per point); the weight blocks stay grouped by bin row in b.wts1.
  // Its records are 12 B, so a batch takes kPosPpt points per thread.
  hipLaunchKernelGGL((k_s2n_scatter2<1, true, kPosPpt>), dim3(nbx * g.slices), dim3(BT), sizeof(StageN<1, kPosPpt>), st,
                     reinterpret_cast<const uint2*>(b.crd1), static_cast<const uint32_t*>(nullptr), b.start1, b.off2,
                     start, g.slices, fb, wbias, nf, tshift, nbx, reinterpret_cast<uint2*>(crd), wts);
  return hipGetLastError() == hipSuccess ? FK_OK : FK_EHIP;
}

}  // namespace fk
