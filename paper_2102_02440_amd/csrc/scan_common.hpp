// scan_common.hpp -- the per-chunk body of the fused selection scan +
// Fast-AGMS sketch update, shared by the one-table kernel and the batched
// persistent kernel.  A "job view" J supplies the table's predicates, key
// columns, slice -> (sketch, row) mapping, seeds and counters.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "build_params.hpp"
#include "device_math.hpp"

namespace compass {

// predicate columns are int32 or float32: their 32-bit patterns.  Rows of
// a tile are read through the tile's first row (a wave-uniform pointer)
// and a 32-bit lane offset, so no 64-bit address per row stays live; the
// loads are streaming (nontemporal): each column word is read once.
__device__ __forceinline__ const uint32_t *pred_tile(const PredDev &p,
                                                    int64_t base) {
  return reinterpret_cast<const uint32_t *>(p.col) + base;
}

// pass[k] &= (row k satisfies p) for the R rows of a lane.  The
// predicate's kind and type are the same for every row, so they are
// dispatched once; each row is then a few compares with no branch (a
// subset reads its bitmap word at a clamped index, then masks).
template <int R>
__device__ __forceinline__ void and_pred(const PredDev &p,
                                         const uint32_t (&raw)[R],
                                         bool (&pass)[R]) {
  const int32_t kind = p.kind;
  if (p.dtype == kDtF32) {
    const float lo = p.lo.f, hi = p.hi.f;
    if (kind == kPredPoint) {
#pragma unroll
      for (int k = 0; k < R; ++k) pass[k] = pass[k] & (__uint_as_float(raw[k]) == lo);
    } else {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const float v = __uint_as_float(raw[k]);
        pass[k] = pass[k] & (v >= lo) & (v <= hi);
      }
    }
    return;
  }
  const int32_t lo = p.lo.i, hi = p.hi.i;
  if (kind == kPredPoint) {
#pragma unroll
    for (int k = 0; k < R; ++k) pass[k] = pass[k] & ((int32_t)raw[k] == lo);
  } else if (kind == kPredRange) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int32_t v = (int32_t)raw[k];
      pass[k] = pass[k] & (v >= lo) & (v <= hi);
    }
  } else if (p.domain <= 0) {  // subset of an empty domain
#pragma unroll
    for (int k = 0; k < R; ++k) pass[k] = false;
  } else {
    // dictionary code in [0, domain) with its bit set; the bitmap is read
    // as 32-bit words (bit c of the 64-bit words is bit c & 31 of 32-bit
    // word c >> 5), and out-of-domain codes read word 0, then are masked
    // (four rows at a time, so that few words are live at once)
    const int64_t dom = p.domain;
    const uint32_t *bm32 = reinterpret_cast<const uint32_t *>(p.bitmap);
#pragma unroll
    for (int h = 0; h < R; h += 4) {
      uint32_t word[4];
      bool in[4];
#pragma unroll
      for (int u = 0; u < 4 && h + u < R; ++u) {
        const int32_t v = (int32_t)raw[h + u];
        in[u] = (v >= 0) & ((int64_t)v < dom);
        word[u] = bm32[in[u] ? (v >> 5) : 0];
      }
#pragma unroll
      for (int u = 0; u < 4 && h + u < R; ++u)
        pass[h + u] = pass[h + u] & in[u] &
                      (((word[u] >> (raw[h + u] & 31u)) & 1u) != 0);
      __asm__ volatile("" ::: "memory");  // the next four loads stay below
    }
  }
}

__device__ __forceinline__ uint64_t field_of_raw(int64_t v) {
  return (v >= 0 && (uint64_t)v < kP61) ? (uint64_t)v : key_field(v);
}

__device__ __forceinline__ uint64_t load_field(const KeyDev &k, int64_t row) {
  if (k.dtype == kDtI32) {
    const int32_t v = reinterpret_cast<const int32_t *>(k.col)[row];
    return v >= 0 ? (uint64_t)v : key_field((int64_t)v);
  }
  const int64_t v = reinterpret_cast<const int64_t *>(k.col)[row];
  return key_field(v);
}

// Field elements of the keys of rows base + ridx[k] (every such row lies in
// the table): all loads are issued before the first is used.
template <int R>
__device__ __forceinline__ void load_fields(const KeyDev &kd, int64_t base,
                                            const int (&ridx)[R],
                                            uint64_t (&x)[R]) {
  if (kd.dtype == kDtI32) {
    int32_t raw[R];
#pragma unroll
    for (int k = 0; k < R; ++k)
      raw[k] = reinterpret_cast<const int32_t *>(kd.col)[base + ridx[k]];
#pragma unroll
    for (int k = 0; k < R; ++k)
      x[k] = raw[k] >= 0 ? (uint64_t)raw[k] : key_field((int64_t)raw[k]);
  } else {
    int64_t raw[R];
#pragma unroll
    for (int k = 0; k < R; ++k)
      raw[k] = reinterpret_cast<const int64_t *>(kd.col)[base + ridx[k]];
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = key_field(raw[k]);
  }
}

// First predicate's raw column values of the tile's rows (0 past nt): a
// caller can issue these loads for the next tile before it compacts the
// current one.
template <class J, int kRowsPerThread>
__device__ __forceinline__ void load_first_pred(const J &job, int64_t base,
                                                int nt,
                                                uint32_t (&cur)[kRowsPerThread]) {
  const uint32_t *t = pred_tile(job.pred(0), base);
  uint32_t lane = threadIdx.x;
  __asm__("" : "+v"(lane));  // per call: no per-row addresses kept live
#pragma unroll
  for (int k = 0; k < kRowsPerThread; ++k) {
    const uint32_t r = lane + k * kBuildThreads;
    cur[k] = (int)r < nt ? __builtin_nontemporal_load(t + r) : 0u;
  }
}

// compact_tile with the first predicate's values already loaded (by
// load_first_pred for the same tile); n_preds >= 1.
template <class J, int kRowsPerThread>
__device__ int compact_tile_loaded(const J &job, int64_t base, int nt,
                                   int n_preds, int32_t *queue, int32_t *s_qn,
                                   int start, int bias,
                                   uint32_t (&cur)[kRowsPerThread]) {
  if (threadIdx.x == 0) *s_qn = start;
  // predicate q + 1 is loaded before predicate q is evaluated
  uint32_t nxt[kRowsPerThread];
  bool pass[kRowsPerThread];
#pragma unroll
  for (int k = 0; k < kRowsPerThread; ++k)
    pass[k] = (int)threadIdx.x + k * kBuildThreads < nt;
  for (int q = 0; q < n_preds; ++q) {
    if (q + 1 < n_preds) {
      const uint32_t *t = pred_tile(job.pred(q + 1), base);
      uint32_t lane = threadIdx.x;
      __asm__("" : "+v"(lane));
#pragma unroll
      for (int k = 0; k < kRowsPerThread; ++k) {
        const uint32_t r = lane + k * kBuildThreads;
        nxt[k] = (int)r < nt ? __builtin_nontemporal_load(t + r) : 0u;
      }
    }
    and_pred<kRowsPerThread>(job.pred(q), cur, pass);
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) cur[k] = nxt[k];
  }
  __syncthreads();  // s_qn initialised
#pragma unroll
  for (int k = 0; k < kRowsPerThread; ++k) {
    const int r = threadIdx.x + k * kBuildThreads;
    const uint64_t ballot = __ballot(pass[k]);
    const int lane = __lane_id();
    const uint32_t before = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(ballot >> 32),
        __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
    const int total = __popcll(ballot);
    int off = 0;
    if (lane == 0 && total) off = atomicAdd(s_qn, total);
    off = __shfl(off, 0);
    if (pass[k]) queue[off + before] = r + bias;
  }
  __syncthreads();
  return *s_qn;
}

// Compacts the qualifying rows of tile [base, base + nt) into `queue`
// (entries start .. start + count - 1, each the row offset plus `bias`;
// unordered: the sums do not depend on order) and returns start + their
// number.  Each predicate column is loaded for all of the thread's rows,
// and before it is evaluated the next one is loaded too, so loads overlap
// instead of waiting on the previous predicate's outcome.  With no
// predicates every row qualifies; the queue is then not used and nt is
// returned.  Every thread of the block must call it.
template <class J, int kRowsPerThread>
__device__ int compact_tile(const J &job, int64_t base, int nt, int n_preds,
                            int32_t *queue, int32_t *s_qn, int start = 0,
                            int bias = 0) {
  if (n_preds == 0) return nt;
  uint32_t cur[kRowsPerThread];
  load_first_pred<J, kRowsPerThread>(job, base, nt, cur);
  return compact_tile_loaded<J, kRowsPerThread>(job, base, nt, n_preds, queue,
                                                s_qn, start, bias, cur);
}

// Scans rows [row0, row1) of job J into the LDS partial counters `cnt` of
// slices [sb, se) (slice sl at cnt + (sl - sb) * w), in tiles of
// kBuildThreads * kRowsPerThread rows.  Returns, in thread 0, the number of
// qualifying rows.  `queue` holds a tile's row offsets (unused, and may be
// null, when the job has no predicates); `s_qn` is a shared counter.  Every
// thread of the block must call it.
template <class J, int kRowsPerThread = kBuildRowsPerThread>
__device__ uint64_t scan_rows(const J &job, int64_t row0, int64_t row1,
                              int sb, int se, int32_t *cnt, int32_t *queue,
                              int32_t *s_qn, RowSink sink = RowSink{}) {
  __shared__ unsigned long long s_roff;
  constexpr int kTile = kBuildThreads * kRowsPerThread;
  // the slice range is the same in every lane: say so, so that the slice
  // tables and seeds are read with scalar loads and the per-slice branches
  // stay uniform
  sb = __builtin_amdgcn_readfirstlane(sb);
  se = __builtin_amdgcn_readfirstlane(se);
  const int w = (int)job.bm().w;
  const int n_preds = job.n_preds();
  const bool dense = (n_preds == 0);
  uint64_t sel = 0;
  // Dense tables: the keys of the group's first sketch for the next tile
  // are loaded while the current tile is hashed (software prefetch).  They
  // are kept as raw 32-bit words (no sign extension at the load, which
  // would make the load wait at once).
  const int s_first = job.slice_sketch(sb);
  const KeyDev kd_first = job.key(s_first);
  const bool first_i32 = kd_first.dtype == kDtI32;
  uint32_t pre_lo[kRowsPerThread], pre_hi[kRowsPerThread];
  bool have_pre = false;
  for (int64_t base = row0; base < row1; base += kTile) {
    const int nt = (int)min((int64_t)kTile, row1 - base);
    const int qn = compact_tile<J, kRowsPerThread>(job, base, nt, n_preds,
                                                   queue, s_qn);
    sel += (uint64_t)qn;
    if (sink.out) {  // selection output: one reservation per tile
      if (threadIdx.x == 0)
        s_roff = qn ? atomicAdd(sink.count, (unsigned long long)qn) : 0ull;
      __syncthreads();
      const int64_t off = (int64_t)s_roff;
      for (int q = threadIdx.x; q < qn; q += kBuildThreads)
        if (off + q < sink.cap)
          sink.out[off + q] = sink.row_base + base + (dense ? q : queue[q]);
    }

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
    int x_wide = -1;  // wave-uniform: -1 = not yet decided for these keys
    const bool full_tile = qn == kTile;  // every lane has all its rows
    if (dense) {
      if (!have_pre) load_fields<kRowsPerThread>(kd_first, base, ridx, x);
      if (have_pre) {
#pragma unroll
        for (int k = 0; k < kRowsPerThread; ++k) {
          const int64_t raw =
              first_i32 ? (int64_t)(int32_t)pre_lo[k]
                        : (int64_t)(((uint64_t)pre_hi[k] << 32) | pre_lo[k]);
          x[k] = field_of_raw(raw);
        }
      }
      cur_sketch = s_first;
      const int64_t nb = base + kTile;
      const int nt2 = (int)max((int64_t)0, min((int64_t)kTile, row1 - nb));
      if (first_i32) {
        const uint32_t *col = reinterpret_cast<const uint32_t *>(kd_first.col);
#pragma unroll
        for (int k = 0; k < kRowsPerThread; ++k) {
          const int q = threadIdx.x + k * kBuildThreads;
          pre_lo[k] = q < nt2 ? col[nb + q] : 0u;
          pre_hi[k] = 0u;
        }
      } else {
        const uint64_t *col = reinterpret_cast<const uint64_t *>(kd_first.col);
#pragma unroll
        for (int k = 0; k < kRowsPerThread; ++k) {
          const int q = threadIdx.x + k * kBuildThreads;
          const uint64_t v = q < nt2 ? col[nb + q] : 0ull;
          pre_lo[k] = (uint32_t)v;
          pre_hi[k] = (uint32_t)(v >> 32);
        }
      }
      have_pre = true;
    }
    for (int sl0 = sb; sl0 < se; ++sl0) {
      const int sl = __builtin_amdgcn_readfirstlane(sl0);
      const int s = job.slice_sketch(sl);
      if (s != cur_sketch) {
        cur_sketch = s;
        // rows of invalid entries are row `base` (in the table); their
        // values are never used
        load_fields<kRowsPerThread>(job.key(s), base, ridx, x);
        x_wide = -1;
      }
      const RowSeeds sd = job.seeds(sl);
      const BucketMod bm = job.bm();
      int32_t *c = cnt + (size_t)(sl - sb) * w;
      // one uniform branch when no key of the wave needs the 61-bit path
      // (every non-negative int32 key); decided once per key load:
      // x_wide 0 = every key below 2^31, 2 = below 2^32, 1 = wider
      if (x_wide < 0) {
        bool wide_key = false, big_key = false;
#pragma unroll
        for (int k = 0; k < kRowsPerThread; ++k) {
          wide_key = wide_key || (valid[k] && (x[k] >> 32) != 0);
          big_key = big_key || (valid[k] && (x[k] >> 31) != 0);
        }
        x_wide = __any(wide_key) ? 1 : (__any(big_key) ? 2 : 0);
      }
      if (x_wide != 1) {
        // branch-free hashes (the lane's chains interleave), then the adds;
        // a lane without a row adds 0, so no hash sits under a branch
        int32_t sign[kRowsPerThread];
        uint32_t b[kRowsPerThread];
        if (bm.pow2 && x_wide == 0) {
          hash_many_pow2<kRowsPerThread, true>(x, sd, bm.mask, sign, b);
        } else if (bm.pow2) {
          hash_many_pow2<kRowsPerThread>(x, sd, bm.mask, sign, b);
        } else {
#pragma unroll
          for (int k = 0; k < kRowsPerThread; ++k)
            hash_xi_h<true>(x[k], sd, bm, sign[k], b[k]);
        }
        if (full_tile) {
#pragma unroll
          for (int k = 0; k < kRowsPerThread; ++k) atomicAdd(&c[b[k]], sign[k]);
        } else {
#pragma unroll
          for (int k = 0; k < kRowsPerThread; ++k)
            atomicAdd(&c[b[k]], valid[k] ? sign[k] : 0);
        }
      } else {
#pragma unroll
        for (int k = 0; k < kRowsPerThread; ++k) {
          if (!valid[k]) continue;
          int32_t sign;
          uint32_t b;
          if ((x[k] >> 32) == 0)
            hash_xi_h<true>(x[k], sd, bm, sign, b);
          else
            hash_xi_h<false>(x[k], sd, bm, sign, b);
          atomicAdd(&c[b], sign);
        }
      }
    }
    __syncthreads();  // queue and s_qn are reused by the next tile
  }
  return sel;
}

// Adds the non-zero LDS partials of slices [sb, se) into the job's global
// counters (integer atomics: order-independent, hence exact).
template <class J>
__device__ void merge_slices(const J &job, int sb, int se,
                             const int32_t *cnt) {
  const int w = (int)job.bm().w;
  for (int sl = sb; sl < se; ++sl) {
    const int s = job.slice_sketch(sl);
    const int row = job.slice_row(sl);
    const int32_t *c = cnt + (size_t)(sl - sb) * w;
    if (job.counter_bits() == 32) {
      int32_t *g = reinterpret_cast<int32_t *>(job.counters(s)) + (size_t)row * w;
      for (int j = threadIdx.x; j < w; j += kBuildThreads) {
        const int32_t v = c[j];
        if (v) atomicAdd(&g[j], v);
      }
    } else {
      unsigned long long *g =
          reinterpret_cast<unsigned long long *>(job.counters(s)) +
          (size_t)row * w;
      for (int j = threadIdx.x; j < w; j += kBuildThreads) {
        const int32_t v = c[j];
        if (v) atomicAdd(&g[j], (unsigned long long)(int64_t)v);
      }
    }
  }
}

}  // namespace compass
