// build_kernels.hip -- fused selection scan + Fast-AGMS sketch update (gfx950).
//
// What is computed (Section 3 "Workflow"/"Partitioned query execution",
// Section 4.2 counter definition): for every row that satisfies the
// conjunction of the pushed-down predicates, and for every attribute sketch
// s of the table and every sketch row i,
//     C_s[i][h_i(key_s)] += xi_i(key_s),
// plus the exact number of qualifying rows.
//
// How it maps to CDNA4:
//  * A "slice" is one (sketch, row) pair: w counters.  A workgroup owns a
//    group of slices whose int32 partial counters fit in LDS (privatised
//    sketch, as the paper's per-warp replicas, but one per workgroup) and
//    a contiguous chunk of table rows.
//  * Rows are read in coalesced 4-byte columns, 8192 rows per tile
//    (1024 lanes x 8) in the fused scan.  Where a scan has predicates they
//    are evaluated per row and survivors are compacted with a wave ballot +
//    mbcnt prefix into an LDS queue of row offsets, so hashing runs on
//    dense waves even at 0.1% selectivity.
//  * Each survivor's key is turned into its field element once per sketch;
//    the d row hashes then use wave-uniform seeds (scalar registers) and a
//    fire-and-forget ds_add into LDS.
//  * Each workgroup writes its LDS partials to its own slab row (plain
//    stores); one reduction kernel sums the chunks per counter.  Integer
//    addition is order-independent, so the result is bit-exact whatever
//    the schedule (Section 2: sketches of partitions add up to the sketch
//    of the whole).
//  * Block -> (chunk, group) pairs are numbered XCD by XCD (the hardware
//    deals workgroup b to XCD b mod 8), so the slice groups that re-read one
//    chunk's key columns run on one XCD and share them through its L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "build_params.hpp"
#include "device_math.hpp"
#include "scan_common.hpp"

namespace compass {

// Job view over the kernel-argument parameter block of one table.
struct ParamJob {
  const BuildParams &P;
  __device__ int n_preds() const { return P.n_preds; }
  __device__ const PredDev &pred(int q) const { return P.preds[q]; }
  __device__ KeyDev key(int s) const { return P.keys[s]; }
  __device__ int slice_sketch(int sl) const { return (P.slice_base + sl) / P.d; }
  __device__ int slice_row(int sl) const { return (P.slice_base + sl) % P.d; }
  __device__ RowSeeds seeds(int sl) const { return P.seeds[sl]; }
  __device__ BucketMod bm() const { return P.bm; }
  __device__ int counter_bits() const { return P.counter_bits; }
  __device__ void *counters(int s) const { return P.counters[s]; }
};

__global__ __launch_bounds__(kBuildThreads) void scan_sketch_kernel(
    const BuildParams P) {
  extern __shared__ int32_t lds[];
  __shared__ int32_t s_qn;

  const ParamJob job{P};
  const int ngroups = P.n_groups;
  // Workgroups are dealt to the XCDs round-robin (workgroup b to XCD
  // b mod kXcds).  Number the (chunk, group) pairs XCD by XCD, so that the
  // groups of one chunk run on the same XCD, one after another, and read
  // the chunk's key columns through that XCD's L2.
  const int per_xcd = (int)gridDim.x / kXcds;
  const int64_t lin = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (lin >= (int64_t)P.n_blocks) return;  // padding of the last XCD's share
  const int gi = (int)(lin % ngroups);
  const int64_t chunk = lin / ngroups;
  const int sb = P.group_begin[gi];
  const int se = P.group_begin[gi + 1];
  const int ns = se - sb;
  const int w = (int)P.bm.w;
  int32_t *cnt = lds;                       // ns * w partial counters
  int32_t *queue = lds + (size_t)ns * w;    // kScanTile row offsets (with
                                            // predicates only)

  for (int i = threadIdx.x; i < ns * w; i += kBuildThreads) cnt[i] = 0;
  __syncthreads();
  const int64_t row0 = chunk * P.rows_per_chunk;
  const int64_t row1 = min(row0 + P.rows_per_chunk, P.n_rows);
  RowSink sink = P.sink;
  if (gi != 0) sink.out = nullptr;  // one slice group writes the rows
  const uint64_t sel =
      scan_rows<ParamJob, kScanRowsPerThread>(job, row0, row1, sb, se, cnt,
                                              queue, &s_qn, sink);
  // partial counters of this chunk -> its slab rows (plain coalesced
  // stores; the reduction kernel sums the chunks in a fixed order)
  const size_t S = (size_t)P.n_slices_total;
  for (int l = 0; l < ns; ++l) {
    const int sl = sb + l;
    const size_t gs = (size_t)(P.slice_base + sl);
    int32_t *dst = P.slab + ((size_t)chunk * S + gs) * w;
    const int32_t *c = cnt + (size_t)l * w;
    for (int j = threadIdx.x; j < w; j += kBuildThreads) dst[j] = c[j];
  }
  if (P.count_selected && gi == 0 && threadIdx.x == 0 && sel)
    atomicAdd(reinterpret_cast<unsigned long long *>(P.n_selected),
              (unsigned long long)sel);
}

// Sketch rows too wide for LDS-private partials (w * 4 > the LDS budget,
// e.g. w = 65536): two phases per batch of rows, no global atomic per
// update (device-scope atomics run two orders of magnitude below LDS ones).
struct DirectJob {
  const BuildParams &P;
  __device__ int n_preds() const { return P.n_preds; }
  __device__ const PredDev &pred(int q) const { return P.preds[q]; }
};

// Wide sketches, phase A: the fused scan compacts the qualifying rows of
// [row_begin, row_end) and appends their key field elements, per sketch, to
// surv[s * cap + ...].  Each block strides over tiles, buffers the offsets
// of its survivors in LDS across tiles, and only when the buffer is nearly
// full (or its tiles are done) reserves space with one global atomic and
// gathers the keys of every (sketch, survivor) pair, four loads in flight
// per thread.
constexpr int kWideQueue = 16384;
// longer tiles than the fused scan's default: more predicate loads in
// flight per tile for this streaming pass
constexpr int kWideRows = 8;
constexpr int kWideTile = kBuildThreads * kWideRows;
static_assert(kWideQueue >= 2 * kWideTile, "a tile fits after a partial queue");

__global__ __launch_bounds__(kBuildThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void wide_compact_kernel(
    const BuildParams P, uint64_t *__restrict__ surv, int64_t cap,
    unsigned long long *__restrict__ count, int64_t row_begin,
    int64_t row_end) {
  __shared__ int32_t queue[kWideQueue];
  __shared__ int32_t s_qn;
  __shared__ unsigned long long s_off;
  const DirectJob job{P};
  uint64_t sel = 0;
  int qtot = 0;  // block-uniform
  const int64_t stride = (int64_t)gridDim.x * kWideTile;
  for (int64_t base = row_begin + (int64_t)blockIdx.x * kWideTile;
       base < row_end; base += stride) {
    const int nt = (int)min((int64_t)kWideTile, row_end - base);
    const int bias = (int)(base - row_begin);
    if (P.n_preds == 0) {
      for (int r = threadIdx.x; r < nt; r += kBuildThreads)
        queue[qtot + r] = bias + r;
      qtot += nt;
    } else {
      qtot = compact_tile<DirectJob, kWideRows>(
          job, base, nt, P.n_preds, queue, &s_qn, qtot, bias);
    }
    const bool last = base + stride >= row_end;
    if (qtot > kWideQueue - kWideTile || (last && qtot > 0)) {
      __syncthreads();  // queue complete
      if (threadIdx.x == 0) s_off = atomicAdd(count, (unsigned long long)qtot);
      __syncthreads();
      const int64_t off = (int64_t)s_off;
      for (int s = 0; s < P.n_groups; ++s) {  // n_groups = sketches here
        const KeyDev kd = P.keys[s];
        uint64_t *dst = surv + (int64_t)s * cap + off;
        for (int q0 = threadIdx.x; q0 < qtot; q0 += 4 * kBuildThreads) {
          uint64_t v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * kBuildThreads;
            v[u] = q < qtot ? load_field(kd, row_begin + queue[q]) : 0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * kBuildThreads;
            if (q < qtot) dst[q] = v[u];
          }
        }
      }
      if (P.sink.out) {  // selection output
        __syncthreads();  // every lane has read s_off
        if (threadIdx.x == 0)
          s_off = atomicAdd(P.sink.count, (unsigned long long)qtot);
        __syncthreads();
        const int64_t roff = (int64_t)s_off;
        for (int q = threadIdx.x; q < qtot; q += kBuildThreads)
          if (roff + q < P.sink.cap)
            P.sink.out[roff + q] = P.sink.row_base + row_begin + queue[q];
      }
      sel += (uint64_t)qtot;
      qtot = 0;
    }
    __syncthreads();  // queue, s_qn and s_off are reused
  }
  if (P.count_selected && threadIdx.x == 0 && sel)
    atomicAdd(reinterpret_cast<unsigned long long *>(P.n_selected),
              (unsigned long long)sel);
}

// Wide sketches, phase B: block (slice, bucket range, chunk) hashes its
// chunk of the compacted survivors of the slice's sketch into LDS counters
// for a range of up to 65536 buckets, two 16-bit counters per 32-bit word
// (bucket j of the range adds +-1 to the low half or +-65536 to the word,
// i.e. +-1 to the high half: the word holds lo + 65536 hi mod 2^32, which
// gives back lo and hi exactly while both stay within [-32767, 32767]).  The
// survivors are taken 32767 at a time, so no half can leave that range;
// after each piece every lane moves its 2 x kWidePairsPerLane counters into
// int32 registers and clears them.  One hash per update even at w = 65536.
constexpr int kWidePiece = 32767;
constexpr int kWidePairsPerLane = 32;   // 32768 words / 1024 lanes
constexpr int64_t kWideMinChunk = 16384;  // survivors per hashing chunk
constexpr int kWideRange = 2 * kWidePairsPerLane * kBuildThreads;  // 65536
constexpr int kWideKeys = 4;  // survivors per lane in flight (fast path)

// Chunks of the survivors that carry work: at least kWideMinChunk
// survivors each (a chunk's fixed cost is clearing, folding and writing w
// counters), at most `chunks`.  The slab reduction reads the same number.
__device__ __forceinline__ int64_t active_chunks(int64_t n, int64_t chunks) {
  const int64_t need = (n + kWideMinChunk - 1) / kWideMinChunk;
  return need < 1 ? 1 : (need < chunks ? need : chunks);
}

// A flush (hashing of the survivors buffered so far, then the slab
// reduction) runs when it is forced (last batch of a build) or when the
// next batch's rows might not fit the buffer: count + need > cap.  Every
// workgroup of both kernels reads the same count, so the decision is
// uniform over the launch.
__device__ __forceinline__ bool flush_due(const FlushCtl &f, int64_t n) {
  return f.force || n + f.need > f.cap;
}

__global__ __launch_bounds__(kBuildThreads) void wide_hash_kernel(
    const uint64_t *__restrict__ surv, FlushCtl fc,
    const RowSeeds *__restrict__ seeds, BucketMod bm, int32_t d,
    int32_t n_slices, int32_t ranges, int32_t chunks,
    int32_t *__restrict__ slab) {
  extern __shared__ uint32_t pairs[];
  const int64_t n = (int64_t)*fc.count;
  if (!flush_due(fc, n)) return;  // the buffer takes the next batch
  const int64_t cap = fc.cap;
  const int64_t act = active_chunks(n, chunks);
  // The act * n_slices * ranges items that carry work are numbered with
  // the slice fastest and split into kXcds contiguous runs, one per XCD
  // (workgroup b runs on XCD b mod kXcds): the d slices of one sketch read
  // the same survivors through one L2, and the XCDs share the work evenly
  // whatever the number of active chunks.
  const int64_t items = act * n_slices * ranges;
  const int xcd = (int)(blockIdx.x % kXcds);
  const int64_t t0 = items * xcd / kXcds, t1 = items * (xcd + 1) / kXcds;
  // a grid of about one workgroup per CU walks its XCD's items (a flush
  // that is not due costs one small launch)
  const int64_t per_xcd = gridDim.x / kXcds;
  for (int64_t t = t0 + blockIdx.x / kXcds; t < t1; t += per_xcd) {
    __syncthreads();  // the previous item's LDS words are read
    const int sl = (int)(t % n_slices);
    const int r = (int)((t / n_slices) % ranges);
    const int k = (int)(t / ((int64_t)n_slices * ranges));
    const int w = (int)bm.w;
    const int wr = (w + ranges - 1) / ranges;  // <= kWideRange
    const int lo = r * wr, hi = min(w, lo + wr);
    const int nwords = (hi - lo + 1) / 2;
    for (int j = threadIdx.x; j < nwords; j += kBuildThreads) pairs[j] = 0;
    int32_t acc[2 * kWidePairsPerLane];
#pragma unroll
    for (int i = 0; i < 2 * kWidePairsPerLane; ++i) acc[i] = 0;
    const int64_t a = n * k / act, b = n * (k + 1) / act;
    const int s = sl / d;
    const RowSeeds sd = seeds[sl];
    const uint64_t *x = surv + (int64_t)s * cap;
    const bool fast = bm.pow2 && ranges == 1;  // uniform
    for (int64_t p0 = a; p0 < b; p0 += kWidePiece) {
      const int64_t p1 = min(b, p0 + kWidePiece);
      __syncthreads();  // cleared words
      if (fast) {
        // kWideKeys survivors per lane at a time, their hash chains interleaved;
        // a lane past the end adds 0
        for (int64_t i0 = p0 + threadIdx.x; i0 < p1;
             i0 += kWideKeys * kBuildThreads) {
          uint64_t xs[kWideKeys];
          bool ok[kWideKeys];
          bool wide_key = false;
#pragma unroll
          for (int u = 0; u < kWideKeys; ++u) {
            const int64_t i = i0 + u * kBuildThreads;
            ok[u] = i < p1;
            xs[u] = ok[u] ? x[i] : 0;
          }
#pragma unroll
          for (int u = 0; u < kWideKeys; ++u)
            wide_key = wide_key || (xs[u] >> 32) != 0;
          if (!__any(wide_key)) {
            int32_t sign[kWideKeys];
            uint32_t bk[kWideKeys];
            hash_many_pow2_auto<kWideKeys>(xs, sd, bm.mask, sign, bk);
            // one range holds every bucket: the half is bit 0 of the bucket
#pragma unroll
            for (int u = 0; u < kWideKeys; ++u)
              atomicAdd(&pairs[bk[u] >> 1],
                        ok[u] ? (uint32_t)sign[u] << ((bk[u] & 1u) << 4) : 0u);
          } else {
#pragma unroll
            for (int u = 0; u < kWideKeys; ++u) {
              if (!ok[u]) continue;
              int32_t sign;
              uint32_t bk;
              if ((xs[u] >> 32) == 0)
                hash_xi_h<true>(xs[u], sd, bm, sign, bk);
              else
                hash_xi_h<false>(xs[u], sd, bm, sign, bk);
              atomicAdd(&pairs[bk >> 1], (uint32_t)sign << ((bk & 1u) << 4));
            }
          }
        }
      } else {
        // four survivors per lane at a time: their hash chains interleave
        for (int64_t i0 = p0 + threadIdx.x; i0 < p1; i0 += 4 * kBuildThreads) {
          uint64_t xs[4];
          bool ok[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * kBuildThreads;
            ok[u] = i < p1;
            xs[u] = ok[u] ? x[i] : 0;
          }
          bool wide_key = false;
#pragma unroll
          for (int u = 0; u < 4; ++u) wide_key = wide_key || (xs[u] >> 32) != 0;
          int32_t sign[4];
          uint32_t bk[4];
          if (!__any(wide_key)) {
#pragma unroll
            for (int u = 0; u < 4; ++u) hash_xi_h<true>(xs[u], sd, bm, sign[u], bk[u]);
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if ((xs[u] >> 32) == 0)
                hash_xi_h<true>(xs[u], sd, bm, sign[u], bk[u]);
              else
                hash_xi_h<false>(xs[u], sd, bm, sign[u], bk[u]);
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int jj = (int)bk[u] - lo;
            if (ok[u] && jj >= 0 && (int)bk[u] < hi)
              atomicAdd(&pairs[jj >> 1],
                        (jj & 1) ? (uint32_t)sign[u] << 16 : (uint32_t)sign[u]);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kWidePairsPerLane; ++i) {
        const int wi = threadIdx.x + i * kBuildThreads;
        if (wi < nwords) {
          const uint32_t word = pairs[wi];
          const int32_t l16 = (int32_t)(int16_t)(word & 0xFFFFu);
          acc[2 * i] += l16;
          acc[2 * i + 1] += (int32_t)(word - (uint32_t)l16) >> 16;
          pairs[wi] = 0;
        }
      }
    }
    int32_t *dst = slab + ((int64_t)k * n_slices + sl) * w + lo;
#pragma unroll
    for (int i = 0; i < kWidePairsPerLane; ++i) {
      const int wi = threadIdx.x + i * kBuildThreads;
      if (2 * wi < hi - lo) dst[2 * wi] = acc[2 * i];
      if (2 * wi + 1 < hi - lo) dst[2 * wi + 1] = acc[2 * i + 1];
    }
  }
}

hipError_t launch_wide_compact(const BuildParams &P, uint64_t *surv,
                               int64_t cap, void *count, int64_t row_begin,
                               int64_t row_end, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL(wide_compact_kernel, dim3(n_blocks), dim3(kBuildThreads),
                     0, st, P, surv, cap,
                     reinterpret_cast<unsigned long long *>(count), row_begin,
                     row_end);
  return hipGetLastError();
}

hipError_t launch_wide_hash(const uint64_t *surv, const FlushCtl &fc,
                            const void *seeds, const BucketMod &bm, int d,
                            int n_slices, int ranges, int chunks,
                            int32_t *slab, int n_cu, hipStream_t st) {
  const int w = (int)bm.w;
  const int wr = (w + ranges - 1) / ranges;
  if (wr > kWideRange) return hipErrorInvalidValue;  // 16-bit pairs, 128 KiB
  const size_t lds = (size_t)((wr + 1) / 2) * 4;
  // one workgroup per CU (128 KiB of LDS each), whole XCD shares
  const int items = n_slices * ranges * chunks;
  const int grid = (std::min(items, std::max(kXcds, n_cu)) + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(wide_hash_kernel, dim3(grid),
                     dim3(kBuildThreads), lds, st, surv, fc,
                     reinterpret_cast<const RowSeeds *>(seeds), bm, d,
                     n_slices, ranges, chunks, slab);
  return hipGetLastError();
}

// counters[s][row][j] = (accumulate ? counters : 0) + sum over chunks of
// slab[chunk][s * d + row][j]: one thread per counter, chunks summed in
// order (integer sums: exact and order-independent anyway).
struct CounterList {
  void *p[kMaxSketches];
};

__global__ void slab_reduce_kernel(const int32_t *__restrict__ slab,
                                   int64_t chunks, int32_t n_slices, int32_t d,
                                   int32_t w, CounterList cl,
                                   int32_t counter_bits, int32_t accumulate,
                                   FlushCtl fc, int32_t vec4) {
  // two-phase builds: a flush reduces only the chunks wide_hash_kernel
  // filled, and its last workgroup empties the survivor buffer
  if (fc.count) {
    const int64_t n = (int64_t)*fc.count;
    if (!flush_due(fc, n)) return;
    chunks = active_chunks(n, chunks);
  }
  const int64_t total = (int64_t)n_slices * w;
  if (vec4) {
    // four consecutive counters of one sketch row per lane: 16-byte loads
    // of the slab (eight chunk rows in flight) and of the counters
    const int64_t total4 = total / 4;
    const int4 *slab4 = reinterpret_cast<const int4 *>(slab);
    for (int64_t k4 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         k4 < total4; k4 += (int64_t)gridDim.x * blockDim.x) {
      int64_t a[4] = {0, 0, 0, 0};
      int64_t c = 0;
      for (; c + 8 <= chunks; c += 8) {
        int4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = slab4[(c + u) * total4 + k4];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a[0] += v[u].x;
          a[1] += v[u].y;
          a[2] += v[u].z;
          a[3] += v[u].w;
        }
      }
      for (; c < chunks; ++c) {
        const int4 v = slab4[c * total4 + k4];
        a[0] += v.x;
        a[1] += v.y;
        a[2] += v.z;
        a[3] += v.w;
      }
      const int64_t k = 4 * k4;
      const int gs = (int)(k / w);
      const int j = (int)(k - (int64_t)gs * w);
      const int s = gs / d, row = gs - s * d;
      const size_t idx = (size_t)row * w + j;  // a multiple of 4
      if (counter_bits == 32) {
        int4 *g = reinterpret_cast<int4 *>(reinterpret_cast<int32_t *>(cl.p[s]) + idx);
        int4 o = accumulate ? *g : make_int4(0, 0, 0, 0);
        o.x += (int32_t)a[0];
        o.y += (int32_t)a[1];
        o.z += (int32_t)a[2];
        o.w += (int32_t)a[3];
        *g = o;
      } else {
        longlong2 *g = reinterpret_cast<longlong2 *>(reinterpret_cast<int64_t *>(cl.p[s]) + idx);
        longlong2 o0 = accumulate ? g[0] : make_longlong2(0, 0);
        longlong2 o1 = accumulate ? g[1] : make_longlong2(0, 0);
        o0.x += a[0];
        o0.y += a[1];
        o1.x += a[2];
        o1.y += a[3];
        g[0] = o0;
        g[1] = o1;
      }
    }
  }
  for (int64_t k = vec4 ? total : blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
       k < total; k += (int64_t)gridDim.x * blockDim.x) {
    // eight chunk rows in flight per lane
    int64_t a8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t c = 0;
    for (; c + 8 <= chunks; c += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a8[u] += slab[(c + u) * total + k];
    }
    for (; c < chunks; ++c) a8[0] += slab[c * total + k];
    int64_t acc = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += a8[u];
    const int gs = (int)(k / w);
    const int j = (int)(k - (int64_t)gs * w);
    const int s = gs / d, row = gs - s * d;
    const size_t idx = (size_t)row * w + j;
    if (counter_bits == 32) {
      int32_t *g = reinterpret_cast<int32_t *>(cl.p[s]);
      g[idx] = (accumulate ? g[idx] : 0) + (int32_t)acc;
    } else {
      int64_t *g = reinterpret_cast<int64_t *>(cl.p[s]);
      g[idx] = (accumulate ? g[idx] : 0) + acc;
    }
  }
  if (fc.count) {
    // every workgroup has read the count before it takes a ticket; the
    // last one resets the count (and the ticket) for the next batch
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      const unsigned t = atomicAdd(fc.ticket, 1u);
      if (t == gridDim.x - 1) {
        atomicExch(fc.count, 0ull);
        atomicExch(fc.ticket, 0u);
      }
    }
  }
}

hipError_t launch_slab_reduce(const int32_t *slab, int64_t chunks,
                              int n_slices, int d, int w,
                              void *const *counters, int n_sketches,
                              int counter_bits, int accumulate,
                              const FlushCtl &fc, hipStream_t st) {
  CounterList cl;
  // 16-byte vector path: rows of a multiple of 4 counters, every counter
  // array 16-byte aligned (the slab is)
  int vec4 = (w % 4) == 0;
  for (int s = 0; s < kMaxSketches; ++s) {
    cl.p[s] = s < n_sketches ? counters[s] : nullptr;
    if (s < n_sketches && (reinterpret_cast<uintptr_t>(counters[s]) & 15)) vec4 = 0;
  }
  const int64_t total = (int64_t)n_slices * w;
  int64_t blocks = (total / (vec4 ? 4 : 1) + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(slab_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     st, slab, chunks, n_slices, d, w, cl, counter_bits,
                     accumulate, fc, vec4);
  return hipGetLastError();
}

// Seeds of the two-phase build's slices to device memory, written by a
// kernel from its arguments (no host staging buffer).
__global__ void store_seeds_kernel(SeedBlock b, RowSeeds *__restrict__ dst) {
  const int i = threadIdx.x;
  if (i < b.n) dst[b.first + i] = b.s[i];
}

hipError_t launch_store_seeds(const RowSeeds *src, int n, RowSeeds *dst,
                              hipStream_t st) {
  for (int a = 0; a < n; a += kSeedBlock) {
    SeedBlock b;
    b.first = a;
    b.n = std::min(kSeedBlock, n - a);
    for (int k = 0; k < b.n; ++k) b.s[k] = src[a + k];
    hipLaunchKernelGGL(store_seeds_kernel, dim3(1), dim3(kSeedBlock), 0, st, b,
                       dst);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// zero-fill used instead of hipMemsetAsync so that callers may capture the
// build in a HIP graph
__global__ void fill_zero_kernel(uint32_t *p, int64_t n_words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// several regions zeroed by one launch (grid.y walks the regions)
__global__ void fill_zero_list_kernel(ZeroSpans z) {
  for (int k = blockIdx.y; k < z.n; k += gridDim.y) {
    uint32_t *p = reinterpret_cast<uint32_t *>(z.p[k]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
         i < z.words[k]; i += (int64_t)gridDim.x * blockDim.x)
      p[i] = 0;
  }
}

hipError_t launch_fill_zero_list(const ZeroSpans &z, hipStream_t st) {
  if (z.n <= 0) return hipSuccess;
  int64_t most = 1;
  for (int k = 0; k < z.n; ++k) most = std::max(most, z.words[k]);
  int64_t blocks = (most + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_zero_list_kernel, dim3((unsigned)blocks, (unsigned)z.n),
                     dim3(256), 0, st, z);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t st) {
  const int64_t words = bytes / 4;
  if (words <= 0) return hipSuccess;
  int64_t blocks = (words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     st, reinterpret_cast<uint32_t *>(p), words);
  return hipGetLastError();
}

hipError_t launch_scan_sketch(const BuildParams &P, int n_blocks,
                              size_t lds_bytes, hipStream_t st) {
  // P.n_blocks pairs, padded to whole rounds of the XCDs
  const int grid = (n_blocks + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL(scan_sketch_kernel,
                     dim3((unsigned)grid), dim3(kBuildThreads), lds_bytes,
                     st, P);
  return hipGetLastError();
}


}  // namespace compass
