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
//  * Rows are read in coalesced 4-byte columns, 4096 rows per tile
//    (1024 lanes x 4).  Predicates are evaluated per row; survivors are
//    compacted with a wave ballot + mbcnt prefix into an LDS queue of row
//    offsets, so hashing runs on dense waves even at 0.1% selectivity.
//  * Each survivor's key is turned into its field element once per sketch;
//    the d row hashes then use wave-uniform seeds (scalar registers) and a
//    fire-and-forget ds_add into LDS.
//  * The merge pass adds each non-zero LDS partial into the global counters
//    with one integer atomic; integer addition is order-independent, so the
//    result is bit-exact whatever the schedule (Section 2: sketches of
//    partitions add up to the sketch of the whole).
//  * Block -> (chunk, group) with the group varying fastest, so the groups
//    that re-read one chunk's columns are dispatched together and share it
//    through the Infinity Cache.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
  __device__ int slice_sketch(int sl) const { return P.slice_sketch[sl]; }
  __device__ int slice_row(int sl) const { return P.slice_row[sl]; }
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
  const int gi = blockIdx.x % ngroups;
  const int64_t chunk = blockIdx.x / ngroups;
  const int sb = P.group_begin[gi];
  const int se = P.group_begin[gi + 1];
  const int ns = se - sb;
  const int w = (int)P.bm.w;
  int32_t *cnt = lds;                       // ns * w partial counters
  int32_t *queue = lds + (size_t)ns * w;    // kBuildTile row offsets

  for (int i = threadIdx.x; i < ns * w; i += kBuildThreads) cnt[i] = 0;
  __syncthreads();
  const int64_t row0 = chunk * P.rows_per_chunk;
  const int64_t row1 = min(row0 + P.rows_per_chunk, P.n_rows);
  const uint64_t sel = scan_rows(job, row0, row1, sb, se, cnt, queue, &s_qn);
  merge_slices(job, sb, se, cnt);
  if (P.count_selected && gi == 0 && threadIdx.x == 0 && sel)
    atomicAdd(reinterpret_cast<unsigned long long *>(P.n_selected),
              (unsigned long long)sel);
}

// Sketch rows too wide for LDS (w * 4 > the LDS budget, e.g. w = 65536):
// the same fused scan + compaction, with every (survivor, slice) hash
// update going straight to the global counters as one integer atomic.  The
// counters of such sketches (d x w x 8 bytes, a few MB each) stay resident in
// the L2 / Infinity Cache, and at the selective predicates this is meant
// for, HBM traffic is the predicate columns.  Work of a tile is flattened
// to (survivor, slice) tasks so that a handful of survivors still keeps
// every lane busy; the slice seeds are staged in LDS.
struct DirectJob {
  const BuildParams &P;
  __device__ int n_preds() const { return P.n_preds; }
  __device__ const PredDev &pred(int q) const { return P.preds[q]; }
};

__global__ __launch_bounds__(kBuildThreads) void scan_direct_kernel(
    const BuildParams P, const RowSeeds *__restrict__ seeds, int32_t n_slices,
    int32_t d) {
  extern __shared__ int32_t lds[];
  __shared__ int32_t s_qn;
  RowSeeds *sd = reinterpret_cast<RowSeeds *>(lds);
  int32_t *queue = lds + (n_slices * sizeof(RowSeeds) + 3) / 4;
  for (int i = threadIdx.x; i < n_slices; i += kBuildThreads) sd[i] = seeds[i];
  __syncthreads();
  const DirectJob job{P};
  const int64_t row0 = (int64_t)blockIdx.x * P.rows_per_chunk;
  const int64_t row1 = min(row0 + P.rows_per_chunk, P.n_rows);
  uint64_t sel = 0;
  const int w = (int)P.bm.w;
  for (int64_t base = row0; base < row1; base += kBuildTile) {
    const int nt = (int)min((int64_t)kBuildTile, row1 - base);
    const int qn = compact_tile<DirectJob, kBuildRowsPerThread>(
        job, base, nt, P.n_preds, queue, &s_qn);
    sel += (uint64_t)qn;
    const int tasks = qn * n_slices;
    for (int t = threadIdx.x; t < tasks; t += kBuildThreads) {
      const int q = t / n_slices;
      const int sl = t - q * n_slices;
      const int s = sl / d, i = sl - s * d;
      const int64_t row = base + (P.n_preds ? queue[q] : q);
      const uint64_t x = load_field(P.keys[s], row);
      int32_t sign;
      uint32_t b;
      if ((x >> 32) == 0)
        hash_xi_h<true>(x, sd[sl], P.bm, sign, b);
      else
        hash_xi_h<false>(x, sd[sl], P.bm, sign, b);
      const size_t idx = (size_t)i * w + b;
      if (P.counter_bits == 32)
        atomicAdd(reinterpret_cast<int32_t *>(P.counters[s]) + idx, sign);
      else
        atomicAdd(reinterpret_cast<unsigned long long *>(P.counters[s]) + idx,
                  (unsigned long long)(int64_t)sign);
    }
    __syncthreads();  // queue and s_qn are reused by the next tile
  }
  if (P.count_selected && threadIdx.x == 0 && sel)
    atomicAdd(reinterpret_cast<unsigned long long *>(P.n_selected),
              (unsigned long long)sel);
}

hipError_t launch_scan_direct(const BuildParams &P, const void *seeds,
                              int n_slices, int d, int n_blocks,
                              hipStream_t st) {
  const size_t lds = ((size_t)n_slices * sizeof(RowSeeds) + 3) / 4 * 4 +
                     (size_t)kBuildTile * 4;
  hipLaunchKernelGGL(scan_direct_kernel, dim3((unsigned)n_blocks),
                     dim3(kBuildThreads), lds, st, P,
                     reinterpret_cast<const RowSeeds *>(seeds), n_slices, d);
  return hipGetLastError();
}

// zero-fill used instead of hipMemsetAsync so that callers may capture the
// build in a HIP graph
__global__ void fill_zero_kernel(uint32_t *p, int64_t n_words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
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
  hipLaunchKernelGGL(scan_sketch_kernel,
                     dim3((unsigned)n_blocks), dim3(kBuildThreads), lds_bytes,
                     st, P);
  return hipGetLastError();
}


}  // namespace compass
