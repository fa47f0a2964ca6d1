// partition.hip -- sketch partitioning (Section 5.1): the two-dimensional
// sketch of a table that takes part in two joins, and the three-table chain
// estimate that combines it with the neighbours' one-dimensional sketches.
//
//  scan2d_*        fused selection scan (the same compaction as the
//                  one-dimensional build); per qualifying row and sketch
//                  row i, both keys are hashed with row i's functions of
//                  their join and xi1 * xi2 is added to entry
//                  [h1][h2] of row i's w1 x w2 matrix.  The matrices are far
//                  larger than LDS (8192 x 8192 per row for the 6a shape):
//                  the binned build below sorts the updates by LDS-sized
//                  tile; scan2d_kernel (one device-scope integer atomic per
//                  update) serves the widths no tiling fits.  Integer
//                  addition makes either exact and order-independent.
//  chain3_kernel   X_i = sum over (j1, j2) of A[j1] P[j1][j2] B[j2]: block
//                  (i, slab of j1 rows) streams its rows of P once with
//                  coalesced loads; each lane holds its columns of B in
//                  registers, sums P * B over them (int64 when n_P n_B <
//                  2^62, else 128-bit) and adds A[j1] times that sum to a
//                  128-bit total.
//  chain3_finish   row totals, median, round-to-nearest-even, certificate.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "build_params.hpp"
#include "device_math.hpp"
#include "scan_common.hpp"
#include "partition_params.hpp"

namespace compass {

struct Job2d {
  const BuildParams &P;
  __device__ int n_preds() const { return P.n_preds; }
  __device__ const PredDev &pred(int q) const { return P.preds[q]; }
};

template <typename C>
__device__ __forceinline__ void add_counter(C *p, int32_t v);
template <>
__device__ __forceinline__ void add_counter<int32_t>(int32_t *p, int32_t v) {
  atomicAdd(p, v);
}
template <>
__device__ __forceinline__ void add_counter<int64_t>(int64_t *p, int32_t v) {
  atomicAdd(reinterpret_cast<unsigned long long *>(p),
            (unsigned long long)(int64_t)v);
}

// hash of one key with a row's functions (the key's width class decides
// the Horner step)
__device__ __forceinline__ void hash_key(uint64_t x, const RowSeeds &s,
                                         const BucketMod &bm, int32_t &g,
                                         uint32_t &b) {
  if ((x >> 32) == 0)
    hash_xi_h<true>(x, s, bm, g, b);
  else
    hash_xi_h<false>(x, s, bm, g, b);
}

// The third and fourth joins of a row set: their buckets are appended to
// the flattened second index b2, their signs multiplied into g2.
template <int R>
__device__ __forceinline__ void hash_more(const BuildParams &P, const KdDims &kx,
                                          int i, const uint64_t *x3,
                                          const uint64_t *x4, int32_t *g2,
                                          uint32_t *b2) {
  if (kx.kd < 3) return;
  const int d = P.d;
  const RowSeeds s3 = P.seeds[2 * d + i];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    int32_t g;
    uint32_t b;
    hash_key(x3[k], s3, kx.bm3, g, b);
    b2[k] = b2[k] * (uint32_t)kx.w3 + b;
    g2[k] *= g;
  }
  if (kx.kd < 4) return;
  const RowSeeds s4 = P.seeds[3 * d + i];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    int32_t g;
    uint32_t b;
    hash_key(x4[k], s4, kx.bm4, g, b);
    b2[k] = b2[k] * (uint32_t)kx.w4 + b;
    g2[k] *= g;
  }
}

template <typename C>
__global__ __launch_bounds__(kBuildThreads) void scan2d_kernel(
    const BuildParams P, const KdDims kx) {
  __shared__ int32_t queue[kBuildTile];
  __shared__ int32_t s_qn;
  const Job2d job{P};
  const int d = P.d;
  const int64_t w1 = P.bm1.w, w2 = (int64_t)P.bm.w * kx.w3 * kx.w4;
  C *cnt = reinterpret_cast<C *>(P.counters[0]);
  uint64_t sel = 0;
  for (int64_t base = (int64_t)blockIdx.x * kBuildTile; base < P.n_rows;
       base += (int64_t)gridDim.x * kBuildTile) {
    const int nt = (int)min((int64_t)kBuildTile, P.n_rows - base);
    const int qn = compact_tile<Job2d, kBuildRowsPerThread>(
        job, base, nt, P.n_preds, queue, &s_qn);
    sel += (uint64_t)qn;
    int ridx[kBuildRowsPerThread];
    bool valid[kBuildRowsPerThread];
#pragma unroll
    for (int k = 0; k < kBuildRowsPerThread; ++k) {
      const int q = threadIdx.x + k * kBuildThreads;
      valid[k] = q < qn;
      ridx[k] = valid[k] ? (P.n_preds ? queue[q] : q) : 0;
    }
    uint64_t x1[kBuildRowsPerThread], x2[kBuildRowsPerThread];
    uint64_t x3[kBuildRowsPerThread], x4[kBuildRowsPerThread];
    load_fields<kBuildRowsPerThread>(P.keys[0], base, ridx, x1);
    load_fields<kBuildRowsPerThread>(P.keys[1], base, ridx, x2);
    if (kx.kd > 2) load_fields<kBuildRowsPerThread>(P.keys[2], base, ridx, x3);
    if (kx.kd > 3) load_fields<kBuildRowsPerThread>(P.keys[3], base, ridx, x4);
    for (int i = 0; i < d; ++i) {
      const RowSeeds s1 = P.seeds[i], s2 = P.seeds[d + i];
      int32_t g1[kBuildRowsPerThread], g2[kBuildRowsPerThread];
      uint32_t b1[kBuildRowsPerThread], b2[kBuildRowsPerThread];
#pragma unroll
      for (int k = 0; k < kBuildRowsPerThread; ++k) {
        hash_key(x1[k], s1, P.bm1, g1[k], b1[k]);
        hash_key(x2[k], s2, P.bm, g2[k], b2[k]);
      }
      hash_more<kBuildRowsPerThread>(P, kx, i, x3, x4, g2, b2);
#pragma unroll
      for (int k = 0; k < kBuildRowsPerThread; ++k) {
        if (!valid[k]) continue;
        add_counter<C>(cnt + ((int64_t)i * w1 + b1[k]) * w2 + b2[k],
                       g1[k] * g2[k]);
      }
    }
    __syncthreads();  // queue and s_qn are reused by the next tile
  }
  if (P.count_selected && threadIdx.x == 0 && sel)
    atomicAdd(reinterpret_cast<unsigned long long *>(P.n_selected),
              (unsigned long long)sel);
}

hipError_t launch_scan2d(const BuildParams &P, const KdDims &kx, int n_blocks,
                         hipStream_t st) {
  if (P.counter_bits == 32)
    hipLaunchKernelGGL(scan2d_kernel<int32_t>, dim3(n_blocks),
                       dim3(kBuildThreads), 0, st, P, kx);
  else
    hipLaunchKernelGGL(scan2d_kernel<int64_t>, dim3(n_blocks),
                       dim3(kBuildThreads), 0, st, P, kx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// Binned two-dimensional build.  The matrices are far larger than LDS, but
// a tile of R = 2^r_shift consecutive j1 rows of one sketch row's matrix
// (R * w2 int32 counters) is not.  Each update becomes a 32-bit record
//     tile << 16 | (offset in the tile) << 1 | [xi1 * xi2 = -1]
// (tiles < 2^15, offsets < 2^15); the records are counting-sorted by tile
// and one workgroup per tile adds its records in LDS and writes the tile
// once, so there is no zero fill and no device-scope atomic per update.
//   scan2d_bin_kernel      the fused predicate scan of a block's rows:
//                          records into the block's region, per-tile counts
//                          in an LDS histogram, written out per block
//   bin2d_offsets_kernel   per tile: exclusive sums over the blocks
//   bin2d_scan_kernel      exclusive sums over the tiles (tile starts)
//   bin2d_scatter_kernel   each block's records to their tile's range (the
//                          order inside a tile is free: integer sums)
//   bin2d_tile_kernel      per tile: LDS sums, one coalesced write
// ---------------------------------------------------------------------
__global__ __launch_bounds__(kBuildThreads) void scan2d_bin_kernel(
    const BuildParams P, const Bin2dArgs a, const KdDims kx) {
  extern __shared__ int32_t lds2[];
  int32_t *hist = lds2;                       // a.n_bins counts
  int32_t *queue = lds2 + ((a.n_bins + 3) & ~3);  // kBuildTile row offsets
  __shared__ int32_t s_qn;
  const Job2d job{P};
  const int d = a.d;
  const int w2 = a.w2;
  const uint32_t rmask = (1u << a.r_shift) - 1;
  const bool pow2 = P.bm1.pow2 && P.bm.pow2;
  for (int j = threadIdx.x; j < a.n_bins; j += kBuildThreads) hist[j] = 0;
  __syncthreads();
  const int b = blockIdx.x;
  const int64_t r0 = a.row0 + (int64_t)b * a.rows_per_block;
  const int64_t r1 = min(a.row1, r0 + a.rows_per_block);
  uint32_t *out = a.rec + (int64_t)b * a.rows_per_block * d;
  int64_t nrec = 0;  // block-uniform
  uint64_t sel = 0;
  for (int64_t base = r0; base < r1; base += kBuildTile) {
    const int nt = (int)min((int64_t)kBuildTile, r1 - base);
    const int qn = compact_tile<Job2d, kBuildRowsPerThread>(
        job, base, nt, P.n_preds, queue, &s_qn);
    sel += (uint64_t)qn;
    int ridx[kBuildRowsPerThread];
    bool valid[kBuildRowsPerThread];
#pragma unroll
    for (int k = 0; k < kBuildRowsPerThread; ++k) {
      const int q = threadIdx.x + k * kBuildThreads;
      valid[k] = q < qn;
      ridx[k] = valid[k] ? (P.n_preds ? queue[q] : q) : 0;
    }
    uint64_t x1[kBuildRowsPerThread], x2[kBuildRowsPerThread];
    uint64_t x3[kBuildRowsPerThread], x4[kBuildRowsPerThread];
    load_fields<kBuildRowsPerThread>(P.keys[0], base, ridx, x1);
    load_fields<kBuildRowsPerThread>(P.keys[1], base, ridx, x2);
    if (kx.kd > 2) load_fields<kBuildRowsPerThread>(P.keys[2], base, ridx, x3);
    if (kx.kd > 3) load_fields<kBuildRowsPerThread>(P.keys[3], base, ridx, x4);
    bool wide_key = false;
#pragma unroll
    for (int k = 0; k < kBuildRowsPerThread; ++k)
      wide_key = wide_key || ((x1[k] | x2[k]) >> 32) != 0;
    // power-of-two widths and 32-bit keys in the whole wave: the keys'
    // hash chains interleave (lanes without a row hash 0 and skip)
    const bool fast = pow2 && !__any(wide_key);
    for (int i = 0; i < d; ++i) {
      const RowSeeds s1 = P.seeds[i], s2 = P.seeds[d + i];
      uint32_t *dst = out + nrec + (int64_t)i * qn;
      int32_t g1[kBuildRowsPerThread], g2[kBuildRowsPerThread];
      uint32_t b1[kBuildRowsPerThread], b2[kBuildRowsPerThread];
      if (fast) {
        hash_many_pow2_auto<kBuildRowsPerThread>(x1, s1, P.bm1.mask, g1, b1);
        hash_many_pow2_auto<kBuildRowsPerThread>(x2, s2, P.bm.mask, g2, b2);
      } else {
#pragma unroll
        for (int k = 0; k < kBuildRowsPerThread; ++k) {
          if ((x1[k] >> 32) == 0)
            hash_xi_h<true>(x1[k], s1, P.bm1, g1[k], b1[k]);
          else
            hash_xi_h<false>(x1[k], s1, P.bm1, g1[k], b1[k]);
          if ((x2[k] >> 32) == 0)
            hash_xi_h<true>(x2[k], s2, P.bm, g2[k], b2[k]);
          else
            hash_xi_h<false>(x2[k], s2, P.bm, g2[k], b2[k]);
        }
      }
      hash_more<kBuildRowsPerThread>(P, kx, i, x3, x4, g2, b2);
#pragma unroll
      for (int k = 0; k < kBuildRowsPerThread; ++k) {
        if (!valid[k]) continue;
        const uint32_t tile = (uint32_t)(i * a.nbr) + (b1[k] >> a.r_shift);
        const uint32_t off = (b1[k] & rmask) * (uint32_t)w2 + b2[k];
        dst[threadIdx.x + k * kBuildThreads] =
            tile << 16 | off << 1 | (uint32_t)(g1[k] != g2[k]);
        atomicAdd(&hist[tile], 1);
      }
    }
    nrec += (int64_t)d * qn;
    __syncthreads();  // queue and s_qn are reused by the next tile
  }
  int32_t *h = a.hist + (int64_t)b * a.n_bins;
  for (int j = threadIdx.x; j < a.n_bins; j += kBuildThreads) h[j] = hist[j];
  if (threadIdx.x == 0) {
    a.rec_count[b] = (int32_t)nrec;
    if (P.count_selected && sel)
      atomicAdd(reinterpret_cast<unsigned long long *>(P.n_selected),
                (unsigned long long)sel);
  }
}

// one lane per tile: the counts of the blocks become their offsets inside
// the tile's range, the total is the tile's size
__global__ void bin2d_offsets_kernel(const Bin2dArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_bins) return;
  // sixteen blocks' counts loaded before any offset is written
  constexpr int kU = 16;
  int32_t run = 0;
  for (int b0 = 0; b0 < a.n_blocks; b0 += kU) {
    int32_t c[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      c[u] = b0 + u < a.n_blocks ? a.hist[(int64_t)(b0 + u) * a.n_bins + j] : 0;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (b0 + u < a.n_blocks) a.hist[(int64_t)(b0 + u) * a.n_bins + j] = run;
      run += c[u];
    }
  }
  a.bin_total[j] = run;
}

// one workgroup of kBinScanThreads lanes: bin_start = exclusive sums of
// bin_total, bin_start[n_bins] = the total (< 2^31: one batch's records)
constexpr int kBinScanThreads = 1024;
static_assert(kBinMaxBins % kBinScanThreads == 0, "whole tiles per lane");
__global__ __launch_bounds__(kBinScanThreads) void bin2d_scan_kernel(
    const Bin2dArgs a) {
  __shared__ int32_t part[kBinScanThreads];
  constexpr int kPer = kBinMaxBins / kBinScanThreads;  // tiles per lane at most
  const int n = a.n_bins;
  const int per = (n + kBinScanThreads - 1) / kBinScanThreads;
  const int j0 = threadIdx.x * per, j1 = min(n, j0 + per);
  int32_t t[kPer];  // all of the lane's loads in flight together
#pragma unroll
  for (int u = 0; u < kPer; ++u) t[u] = j0 + u < j1 ? a.bin_total[j0 + u] : 0;
  int32_t s = 0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) s += t[u];
  part[threadIdx.x] = s;
  __syncthreads();
  // inclusive scan of the lane sums (Hillis-Steele)
  for (int o = 1; o < kBinScanThreads; o <<= 1) {
    const int32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t run = part[threadIdx.x] - s;  // exclusive
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    if (j0 + u < j1) a.bin_start[j0 + u] = run;
    run += t[u];
  }
  if (threadIdx.x == kBinScanThreads - 1) a.bin_start[n] = part[threadIdx.x];
}

// block b moves its records to their tiles' ranges (16-bit records: the
// tile is known from the range)
__global__ __launch_bounds__(kBuildThreads) void bin2d_scatter_kernel(
    const Bin2dArgs a) {
  extern __shared__ int32_t lds2[];
  int32_t *pos = lds2;  // a.n_bins next free positions
  const int b = blockIdx.x;
  const int32_t *h = a.hist + (int64_t)b * a.n_bins;
  for (int j = threadIdx.x; j < a.n_bins; j += kBuildThreads)
    pos[j] = a.bin_start[j] + h[j];
  __syncthreads();
  const uint32_t *src = a.rec + (int64_t)b * a.rows_per_block * a.d;
  const int n = a.rec_count[b];
  for (int e0 = threadIdx.x; e0 < n; e0 += 4 * kBuildThreads) {
    uint32_t r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * kBuildThreads;
      r[u] = e < n ? src[e] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (e0 + u * kBuildThreads >= n) break;
      const int p = atomicAdd(&pos[r[u] >> 16], 1);
      a.sorted[p] = (uint16_t)(r[u] & 0xFFFFu);
    }
  }
}

// one workgroup per tile: LDS sums of the tile's records, then the tile's
// rows (contiguous in the d x w1 x w2 layout) written or added once
template <typename C>
__global__ __launch_bounds__(kBuildThreads) void bin2d_tile_kernel(
    const Bin2dArgs a, C *counters, int32_t accumulate) {
  extern __shared__ int32_t lds2[];
  int32_t *tile = lds2;
  const int t = blockIdx.x;
  const int i = t / a.nbr;
  const int j1a = (t % a.nbr) << a.r_shift;
  const int rows = min(1 << a.r_shift, a.w1 - j1a);
  const int words = rows * a.w2;
  // (w2 a multiple of 4: every tile starts on a 16-byte boundary)
  const bool quads = (a.w2 & 3) == 0;
  if (quads) {
    for (int j = threadIdx.x; j < words / 4; j += kBuildThreads)
      reinterpret_cast<int4 *>(tile)[j] = make_int4(0, 0, 0, 0);
  } else {
    for (int j = threadIdx.x; j < words; j += kBuildThreads) tile[j] = 0;
  }
  __syncthreads();
  const int e1 = a.bin_start[t + 1];
  for (int e0 = a.bin_start[t] + threadIdx.x; e0 < e1; e0 += 4 * kBuildThreads) {
    uint32_t r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * kBuildThreads;
      r[u] = e < e1 ? a.sorted[e] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e0 + u * kBuildThreads < e1)
        atomicAdd(&tile[r[u] >> 1], (r[u] & 1u) ? -1 : 1);
  }
  __syncthreads();
  C *dst = counters + ((int64_t)i * a.w1 + j1a) * a.w2;
  const bool aligned = (reinterpret_cast<uintptr_t>(counters) & 15) == 0;
  if (sizeof(C) == 4 && quads && aligned && !accumulate) {
    // written once and not read by this kernel: streaming stores
    for (int j = threadIdx.x; j < words / 4; j += kBuildThreads) {
      const int4 q = reinterpret_cast<const int4 *>(tile)[j];
      int *o = reinterpret_cast<int *>(dst) + 4 * j;
      __builtin_nontemporal_store(q.x, o);
      __builtin_nontemporal_store(q.y, o + 1);
      __builtin_nontemporal_store(q.z, o + 2);
      __builtin_nontemporal_store(q.w, o + 3);
    }
  } else if (accumulate) {
    for (int j = threadIdx.x; j < words; j += kBuildThreads)
      dst[j] += (C)tile[j];
  } else {
    for (int j = threadIdx.x; j < words; j += kBuildThreads)
      dst[j] = (C)tile[j];
  }
}

hipError_t launch_scan2d_binned(const BuildParams &P, const Bin2dArgs &a,
                                const KdDims &kx, int accumulate,
                                hipStream_t st) {
  const size_t hist_lds = (size_t)((a.n_bins + 3) & ~3) * 4;
  hipLaunchKernelGGL(scan2d_bin_kernel, dim3(a.n_blocks), dim3(kBuildThreads),
                     hist_lds + (size_t)kBuildTile * 4, st, P, a, kx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bin2d_offsets_kernel, dim3((a.n_bins + 255) / 256),
                     dim3(256), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bin2d_scan_kernel, dim3(1), dim3(kBinScanThreads), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bin2d_scatter_kernel, dim3(a.n_blocks), dim3(kBuildThreads),
                     hist_lds, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t tile_lds = (size_t)(a.w2 << a.r_shift) * 4;
  if (P.counter_bits == 32)
    hipLaunchKernelGGL(bin2d_tile_kernel<int32_t>, dim3(a.n_bins),
                       dim3(kBuildThreads), tile_lds, st, a,
                       reinterpret_cast<int32_t *>(P.counters[0]), accumulate);
  else
    hipLaunchKernelGGL(bin2d_tile_kernel<int64_t>, dim3(a.n_bins),
                       dim3(kBuildThreads), tile_lds, st, a,
                       reinterpret_cast<int64_t *>(P.counters[0]), accumulate);
  return hipGetLastError();
}

constexpr int kChainThreads = 512;
constexpr int kChainMaxW2 = 16384;
constexpr int kChainPerLane = kChainMaxW2 / kChainThreads;  // B values per lane

template <typename C>
__device__ __forceinline__ int64_t ld(const void *p, int64_t i) {
  return (int64_t)reinterpret_cast<const C *>(p)[i];
}

// Block (i, slab of kChainRows rows of P): lane l owns columns
// l, l + 512, ... of B (in registers, loaded once) and of every P row.
template <typename C>
__global__ __launch_bounds__(kChainThreads) void chain3_kernel(ChainArgs a) {
  __shared__ u128 red[kChainThreads];
  const int i = blockIdx.x;
  const int w1 = a.w1, w2 = a.w2;
  C bv[kChainPerLane];
#pragma unroll
  for (int k = 0; k < kChainPerLane; ++k) {
    const int j = threadIdx.x + k * kChainThreads;
    bv[k] = j < w2 ? reinterpret_cast<const C *>(a.B)[(int64_t)i * w2 + j] : (C)0;
  }
  // 64-bit inner sums are exact when n_P * n_B < 2^62: every partial sum
  // of |P| |B| over one row of P is at most n_P max|B| <= n_P n_B
  const uint64_t np = *a.n_p < 0 ? 0 : (uint64_t)*a.n_p;
  const uint64_t nb = *a.n_b < 0 ? 0 : (uint64_t)*a.n_b;
  const bool narrow = (u128)np * nb < ((u128)1 << 62);
  u128 G = 0;
  const int j1a = blockIdx.y * kChainRows, j1b = min(w1, j1a + kChainRows);
  for (int j1 = j1a; j1 < j1b; ++j1) {
    const C *prow = reinterpret_cast<const C *>(a.P) + ((int64_t)i * w1 + j1) * w2;
    const int64_t aj = ld<C>(a.A, (int64_t)i * w1 + j1);
    if (narrow) {
      int64_t t = 0;
#pragma unroll 8
      for (int k = 0; k < kChainPerLane; ++k) {
        const int j = threadIdx.x + k * kChainThreads;
        if (j < w2) t += (int64_t)prow[j] * (int64_t)bv[k];
      }
      G += mul_s64_s64(aj, t);
    } else {
      u128 t = 0;
#pragma unroll 4
      for (int k = 0; k < kChainPerLane; ++k) {
        const int j = threadIdx.x + k * kChainThreads;
        if (j < w2) t += mul_s64_s64((int64_t)prow[j], (int64_t)bv[k]);
      }
      G += mul_u128_s64(t, aj);
    }
  }
  red[threadIdx.x] = G;
  __syncthreads();
  for (int off = kChainThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[(size_t)i * gridDim.y + blockIdx.y] = red[0];
}

// int32 counters with w2 a multiple of 4 (16-byte aligned rows): the same
// sums with 16-byte loads.  Lane l owns the column quads l, l + 512, ...,
// Q of them (Q * 2048 >= w2), of B and of every P row; a row's loads are
// all issued before its products (branch-free: a lane past the row's end
// reloads the row's last quad and uses zeros).
template <int Q>
__global__ __launch_bounds__(kChainThreads) void chain3_vec_kernel(ChainArgs a) {
  __shared__ u128 red[kChainThreads];
  const int i = blockIdx.x;
  const int w1 = a.w1, nq = a.w2 / 4;  // quads per row
  const int4 *brow = reinterpret_cast<const int4 *>(a.B) + (int64_t)i * nq;
  int4 bv[Q];
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const int v = threadIdx.x + m * kChainThreads;
    const int4 t = brow[min(v, nq - 1)];
    bv[m] = v < nq ? t : make_int4(0, 0, 0, 0);
  }
  const uint64_t np = *a.n_p < 0 ? 0 : (uint64_t)*a.n_p;
  const uint64_t nb = *a.n_b < 0 ? 0 : (uint64_t)*a.n_b;
  const bool narrow = (u128)np * nb < ((u128)1 << 62);
  const int j1a = blockIdx.y * kChainRows, j1b = min(w1, j1a + kChainRows);
  const int4 *P4 = reinterpret_cast<const int4 *>(a.P) + (int64_t)i * w1 * nq;
  const int32_t *Ai = reinterpret_cast<const int32_t *>(a.A) + (int64_t)i * w1;
  u128 G = 0;
  for (int j1 = j1a; j1 < j1b; ++j1) {
    const int4 *prow = P4 + (int64_t)j1 * nq;
    const int64_t aj = Ai[j1];
    int4 cur[Q];
    // the matrix is read once: streaming loads
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      typedef int v4i __attribute__((ext_vector_type(4)));
      const v4i q = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(
          prow + min((int)threadIdx.x + m * kChainThreads, nq - 1)));
      cur[m] = make_int4(q.x, q.y, q.z, q.w);
    }
    // opaque, after every load is issued: B and the row stay in 32-bit
    // registers (no 64-bit copies, for B none hoisted out of the loop);
    // the multiply-adds widen them
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      __asm__("" : "+v"(bv[m].x), "+v"(bv[m].y), "+v"(bv[m].z), "+v"(bv[m].w));
      __asm__("" : "+v"(cur[m].x), "+v"(cur[m].y), "+v"(cur[m].z), "+v"(cur[m].w));
    }
    // (B is zero past the row's end, so the reloaded quads add nothing)
    if (narrow) {
      int64_t t = 0;
#pragma unroll
      for (int m = 0; m < Q; ++m) {
        t += (int64_t)cur[m].x * bv[m].x;
        t += (int64_t)cur[m].y * bv[m].y;
        t += (int64_t)cur[m].z * bv[m].z;
        t += (int64_t)cur[m].w * bv[m].w;
      }
      G += mul_s64_s64(aj, t);
    } else {
      // (an int32 x int32 product is exact in int64)
      u128 t = 0;
#pragma unroll
      for (int m = 0; m < Q; ++m) {
        t += s64_to_u128((int64_t)cur[m].x * bv[m].x);
        t += s64_to_u128((int64_t)cur[m].y * bv[m].y);
        t += s64_to_u128((int64_t)cur[m].z * bv[m].z);
        t += s64_to_u128((int64_t)cur[m].w * bv[m].w);
      }
      G += mul_u128_s64(t, aj);
    }
  }
  red[threadIdx.x] = G;
  __syncthreads();
  for (int off = kChainThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[(size_t)i * gridDim.y + blockIdx.y] = red[0];
}

__device__ __forceinline__ bool i128_less(u128 x, u128 y) {
  return (__int128)x < (__int128)y;
}

constexpr int kFinishThreads = 256;
__global__ __launch_bounds__(kFinishThreads) void chain3_finish_kernel(
    ChainArgs a, int32_t nblk, uint64_t *row_est, double *est,
    int32_t *flags) {
  __shared__ u128 xs[64];
  __shared__ u128 red[kFinishThreads];
  const int d = a.d;
  // row sums of the block partials: all lanes per row, then a tree in LDS
  for (int i = 0; i < d; ++i) {
    u128 x = 0;
    for (int k = threadIdx.x; k < nblk; k += kFinishThreads)
      x += a.partial[(size_t)i * nblk + k];
    red[threadIdx.x] = x;
    __syncthreads();
    for (int off = kFinishThreads / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      x = red[0];
      xs[i] = x;
      if (row_est) {
        row_est[2 * i] = (uint64_t)x;
        row_est[2 * i + 1] = (uint64_t)(x >> 64);
      }
    }
    __syncthreads();  // red is reused by the next row
  }
  if (threadIdx.x != 0) return;
  for (int p = 1; p < d; ++p) {  // insertion sort of d <= 32 values
    const u128 v = xs[p];
    int q = p - 1;
    while (q >= 0 && i128_less(v, xs[q])) {
      xs[q + 1] = xs[q];
      --q;
    }
    xs[q + 1] = v;
  }
  double m;
  if (d & 1) {
    m = i128_to_double(xs[d / 2]);
  } else {
    m = i128_to_double(xs[d / 2 - 1] + xs[d / 2]) * 0.5;
  }
  *est = m;
  // |X_i| <= n_A * n_P * n_B: certified below 2^127
  const u128 lim = (u128)1 << 127;
  u128 b = 1;
  bool ok = true;
  const int64_t ns[3] = {*a.n_a, *a.n_p, *a.n_b};
  for (int k = 0; k < 3 && ok; ++k) {
    const u128 f = (u128)(ns[k] < 0 ? 0 : ns[k]);
    if (f == 0) {
      b = 0;
      break;
    }
    u128 prod;  // b * f > 2^127 stops the product (no 128-bit division)
    if (__builtin_mul_overflow(b, f, &prod) || prod > lim) ok = false;
    else b = prod;
  }
  *flags = ok && b < lim ? 1 : 0;
}

hipError_t launch_chain3(const ChainArgs &a, uint64_t *row_est, double *est,
                         int32_t *flags, hipStream_t st) {
  const int nblk = (a.w1 + kChainRows - 1) / kChainRows;
  const bool aligned =
      ((reinterpret_cast<uintptr_t>(a.P) | reinterpret_cast<uintptr_t>(a.B)) & 15) == 0;
  const int quads = (a.w2 / 4 + kChainThreads - 1) / kChainThreads;  // <= 8
  if (a.counter_bits == 32 && a.w2 % 4 == 0 && aligned) {
    if (quads <= 1)
      hipLaunchKernelGGL(chain3_vec_kernel<1>, dim3(a.d, nblk),
                         dim3(kChainThreads), 0, st, a);
    else if (quads <= 2)
      hipLaunchKernelGGL(chain3_vec_kernel<2>, dim3(a.d, nblk),
                         dim3(kChainThreads), 0, st, a);
    else if (quads <= 4)
      hipLaunchKernelGGL(chain3_vec_kernel<4>, dim3(a.d, nblk),
                         dim3(kChainThreads), 0, st, a);
    else
      hipLaunchKernelGGL(chain3_vec_kernel<8>, dim3(a.d, nblk),
                         dim3(kChainThreads), 0, st, a);
  } else if (a.counter_bits == 32)
    hipLaunchKernelGGL(chain3_kernel<int32_t>, dim3(a.d, nblk),
                       dim3(kChainThreads), 0, st, a);
  else
    hipLaunchKernelGGL(chain3_kernel<int64_t>, dim3(a.d, nblk),
                       dim3(kChainThreads), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chain3_finish_kernel, dim3(1), dim3(kFinishThreads), 0, st,
                     a, nblk, row_est, est, flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------
// tree of partitioned sketches: grid (d x (parent width or root chunks),
// tasks of one tree level), kTensorThreads lanes
// ---------------------------------------------------------------------
template <typename C>
__device__ __forceinline__ u128 tensor_entry(const TensorTask &T, int row,
                                             int64_t off) {
  return s64_to_u128(
      (int64_t)reinterpret_cast<const C *>(T.tensor)[(int64_t)row * T.size + off]);
}

// the value of dimension k's message at bucket j (a leaf child's counter,
// or a computed message)
__device__ __forceinline__ u128 dim_msg(const TensorArgs &A, const TensorTask &T,
                                        int k, int row, int j) {
  const int s = T.child_msg[k];
  if (s >= 0) return A.msg[((size_t)s * A.d + row) * A.w_max + j];
  const int64_t idx = (int64_t)row * T.width[k] + j;
  if (A.counter_bits == 32)
    return s64_to_u128(reinterpret_cast<const int32_t *>(T.leaf[k])[idx]);
  return s64_to_u128(reinterpret_cast<const int64_t *>(T.leaf[k])[idx]);
}

__global__ __launch_bounds__(kTensorThreads) void tensor_node_kernel(
    TensorArgs A) {
  __shared__ u128 red[kTensorThreads];
  const TensorTask &T = A.tasks[blockIdx.y];
  const int root = T.parent_dim < 0;
  const int per_row = root ? T.n_chunks : T.width[T.parent_dim];
  const int row = blockIdx.x / per_row;
  const int jb = blockIdx.x % per_row;  // parent bucket, or root chunk
  if (row >= A.d) return;
  // entries of the block: root: a chunk of the flattened tensor; else the
  // slice at parent bucket jb, enumerated over the other dimensions
  int64_t n_ent, f0 = 0;
  if (root) {
    f0 = (int64_t)jb * kTensorChunk;
    n_ent = min((int64_t)kTensorChunk, T.size - f0);
  } else {
    n_ent = T.size / T.width[T.parent_dim];
  }
  u128 acc = 0;
  for (int64_t e = threadIdx.x; e < n_ent; e += kTensorThreads) {
    int64_t off;
    int idx[kTensorMaxDims];
    if (root) {
      off = f0 + e;
      int64_t r = off;
      for (int k = T.n_dims - 1; k >= 0; --k) {
        idx[k] = (int)(r % T.width[k]);
        r /= T.width[k];
      }
    } else {
      int64_t r = e;
      off = (int64_t)jb * T.stride[T.parent_dim];
      for (int k = T.n_dims - 1; k >= 0; --k) {
        if (k == T.parent_dim) {
          idx[k] = jb;
          continue;
        }
        idx[k] = (int)(r % T.width[k]);
        r /= T.width[k];
        off += (int64_t)idx[k] * T.stride[k];
      }
    }
    u128 v = A.counter_bits == 32 ? tensor_entry<int32_t>(T, row, off)
                                  : tensor_entry<int64_t>(T, row, off);
    for (int k = 0; k < T.n_dims; ++k)
      if (k != T.parent_dim) v *= dim_msg(A, T, k, row, idx[k]);
    acc += v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kTensorThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (root)
    A.partial[(size_t)row * T.n_chunks + jb] = red[0];
  else
    A.msg[((size_t)T.out_slot * A.d + row) * A.w_max + jb] = red[0];
}

hipError_t launch_tensor_level(const TensorArgs &A, int n_tasks, int max_blocks,
                               hipStream_t st) {
  hipLaunchKernelGGL(tensor_node_kernel, dim3(max_blocks, n_tasks),
                     dim3(kTensorThreads), 0, st, A);
  return hipGetLastError();
}

// row sums of the root's chunk partials, median, certificate (|X_i| <= the
// product of the tables' selected rows)
__global__ __launch_bounds__(kFinishThreads) void tensor_finish_kernel(
    const u128 *partial, int32_t n_chunks, int32_t d, const int64_t *n_sel,
    int32_t n_tables, uint64_t *row_est, double *est, int32_t *flags) {
  __shared__ u128 xs[64];
  __shared__ u128 red[kFinishThreads];
  for (int i = 0; i < d; ++i) {
    u128 x = 0;
    for (int k = threadIdx.x; k < n_chunks; k += kFinishThreads)
      x += partial[(size_t)i * n_chunks + k];
    red[threadIdx.x] = x;
    __syncthreads();
    for (int off = kFinishThreads / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      xs[i] = red[0];
      if (row_est) {
        row_est[2 * i] = (uint64_t)red[0];
        row_est[2 * i + 1] = (uint64_t)(red[0] >> 64);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  for (int p = 1; p < d; ++p) {
    const u128 v = xs[p];
    int q = p - 1;
    while (q >= 0 && i128_less(v, xs[q])) {
      xs[q + 1] = xs[q];
      --q;
    }
    xs[q + 1] = v;
  }
  *est = (d & 1) ? i128_to_double(xs[d / 2])
                 : i128_to_double(xs[d / 2 - 1] + xs[d / 2]) * 0.5;
  const u128 lim = (u128)1 << 127;
  u128 b = 1;
  bool ok = true;
  for (int t = 0; t < n_tables && ok; ++t) {
    const u128 f = (u128)(n_sel[t] < 0 ? 0 : n_sel[t]);
    if (f == 0) {
      b = 0;
      break;
    }
    u128 prod;
    if (__builtin_mul_overflow(b, f, &prod) || prod > lim) ok = false;
    else b = prod;
  }
  *flags = ok && b < lim ? 1 : 0;
}

hipError_t launch_tensor_finish(const u128 *partial, int n_chunks, int d,
                                const int64_t *n_sel, int n_tables,
                                uint64_t *row_est, double *est, int32_t *flags,
                                hipStream_t st) {
  hipLaunchKernelGGL(tensor_finish_kernel, dim3(1), dim3(kFinishThreads), 0, st,
                     partial, n_chunks, d, n_sel, n_tables, row_est, est, flags);
  return hipGetLastError();
}

}  // namespace compass
