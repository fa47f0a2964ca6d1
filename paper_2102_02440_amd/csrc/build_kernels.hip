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

namespace compass {

__device__ __forceinline__ bool eval_pred(const PredDev &p, int64_t row) {
  if (p.dtype == kDtF32) {
    const float v = reinterpret_cast<const float *>(p.col)[row];
    if (p.kind == kPredPoint) return v == p.lo.f;
    return (v >= p.lo.f) & (v <= p.hi.f);
  }
  const int32_t v = reinterpret_cast<const int32_t *>(p.col)[row];
  if (p.kind == kPredPoint) return v == p.lo.i;
  if (p.kind == kPredRange) return (v >= p.lo.i) & (v <= p.hi.i);
  // subset: dictionary code must lie in [0, domain) and have its bit set
  if (v < 0 || (int64_t)v >= p.domain) return false;
  const uint64_t word = p.bitmap[v >> 6];
  return (word >> (v & 63)) & 1ull;
}

__device__ __forceinline__ uint64_t load_field(const KeyDev &k, int64_t row) {
  if (k.dtype == kDtI32) {
    const int32_t v = reinterpret_cast<const int32_t *>(k.col)[row];
    return v >= 0 ? (uint64_t)v : key_field((int64_t)v);
  }
  const int64_t v = reinterpret_cast<const int64_t *>(k.col)[row];
  return key_field(v);
}

template <int kRowsPerThread>
__global__ __launch_bounds__(kBuildThreads) void scan_sketch_kernel(
    const BuildParams P) {
  extern __shared__ int32_t lds[];
  __shared__ int32_t s_qn;
  __shared__ unsigned long long s_sel;

  const int ngroups = P.n_groups;
  const int gi = blockIdx.x % ngroups;
  const int64_t chunk = blockIdx.x / ngroups;
  const int sb = P.group_begin[gi];
  const int se = P.group_begin[gi + 1];
  const int ns = se - sb;
  const int w = (int)P.bm.w;
  int32_t *cnt = lds;                       // ns * w partial counters
  int32_t *queue = lds + (size_t)ns * w;    // kTile row offsets

  for (int i = threadIdx.x; i < ns * w; i += kBuildThreads) cnt[i] = 0;
  if (threadIdx.x == 0) s_sel = 0;

  const int64_t row0 = chunk * P.rows_per_chunk;
  const int64_t row1 = min(row0 + P.rows_per_chunk, P.n_rows);
  const bool dense = (P.n_preds == 0);
  constexpr int kTile = kBuildThreads * kRowsPerThread;
  __syncthreads();

  for (int64_t base = row0; base < row1; base += kTile) {
    const int nt = (int)min((int64_t)kTile, row1 - base);
    int qn;
    if (dense) {
      qn = nt;
    } else {
      if (threadIdx.x == 0) s_qn = 0;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k) {
        const int r = threadIdx.x + k * kBuildThreads;
        bool pass = r < nt;
        if (pass) {
          for (int q = 0; q < P.n_preds; ++q) {
            if (!eval_pred(P.preds[q], base + r)) {
              pass = false;
              break;
            }
          }
        }
        const uint64_t ballot = __ballot(pass);
        const int lane = __lane_id();
        const uint32_t before = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(ballot >> 32),
            __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
        const int total = __popcll(ballot);
        int off = 0;
        if (lane == 0 && total) off = atomicAdd(&s_qn, total);
        off = __shfl(off, 0);
        if (pass) queue[off + before] = r;
      }
      __syncthreads();
      qn = s_qn;
    }
    if (threadIdx.x == 0) s_sel += (unsigned long long)qn;

    // survivors handled by this thread: entries threadIdx.x + k * threads
    int ridx[kRowsPerThread];
    bool valid[kRowsPerThread];
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) {
      const int q = threadIdx.x + k * kBuildThreads;
      valid[k] = q < qn;
      ridx[k] = valid[k] ? (dense ? q : queue[q]) : 0;
    }
    uint64_t x[kRowsPerThread];
    int cur_sketch = -1;
    for (int sl = sb; sl < se; ++sl) {
      const int s = P.slice_sketch[sl];
      if (s != cur_sketch) {
        cur_sketch = s;
#pragma unroll
        for (int k = 0; k < kRowsPerThread; ++k)
          x[k] = valid[k] ? load_field(P.keys[s], base + ridx[k]) : 0;
      }
      const RowSeeds sd = P.seeds[sl];
      int32_t *c = cnt + (size_t)(sl - sb) * w;
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k) {
        if (!valid[k]) continue;
        int32_t sign;
        uint32_t b;
        if ((x[k] >> 32) == 0)
          hash_xi_h<true>(x[k], sd, P.bm, sign, b);
        else
          hash_xi_h<false>(x[k], sd, P.bm, sign, b);
        atomicAdd(&c[b], sign);
      }
    }
    __syncthreads();  // queue and s_qn are reused by the next tile
  }

  // merge pass: LDS partials -> global counters (non-zero buckets only)
  for (int l = 0; l < ns; ++l) {
    const int sl = sb + l;
    const int s = P.slice_sketch[sl];
    const int row = P.slice_row[sl];
    const int32_t *c = cnt + (size_t)l * w;
    if (P.counter_bits == 32) {
      int32_t *g = reinterpret_cast<int32_t *>(P.counters[s]) + (size_t)row * w;
      for (int j = threadIdx.x; j < w; j += kBuildThreads) {
        const int32_t v = c[j];
        if (v) atomicAdd(&g[j], v);
      }
    } else {
      unsigned long long *g =
          reinterpret_cast<unsigned long long *>(P.counters[s]) +
          (size_t)row * w;
      for (int j = threadIdx.x; j < w; j += kBuildThreads) {
        const int32_t v = c[j];
        if (v) atomicAdd(&g[j], (unsigned long long)(int64_t)v);
      }
    }
  }
  if (P.count_selected && gi == 0 && threadIdx.x == 0 && s_sel)
    atomicAdd(reinterpret_cast<unsigned long long *>(P.n_selected), s_sel);
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
  hipLaunchKernelGGL(scan_sketch_kernel<kBuildRowsPerThread>,
                     dim3((unsigned)n_blocks), dim3(kBuildThreads), lds_bytes,
                     st, P);
  return hipGetLastError();
}


}  // namespace compass
