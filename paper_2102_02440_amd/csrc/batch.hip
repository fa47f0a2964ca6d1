// batch.hip -- every attribute sketch of many tables (of many queries) in
// one persistent, graph-captured launch.
//
// The batch is cut into work items (table job, row range, slice group).
// A fixed grid of persistent workgroups pulls items from a device-side
// counter until the list is exhausted (every workgroup reaches the exit:
// the counter only grows), so uneven filtered sizes (10k..36M rows, 0.1%..
// 100% selectivity) balance dynamically.  Items are ordered largest first.
// Each item runs the same fused scan + LDS-private sketch + merge body as the
// one-table kernel.  Plan creation captures "zero counters + reset queue +
// persistent kernel" in a hipGraph; a launch is one hipGraphLaunch.
//
// The tile parameters (rows per item, LDS budget per workgroup, persistent
// workgroups per CU) come from a small autotuner: it times every candidate
// on the batch itself and caches the winner per (gfx arch, shape class).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <errno.h>
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "build_params.hpp"
#include "build_plan.hpp"
#include "compass.h"
#include "device_math.hpp"
#include "scan_common.hpp"

namespace compass {

struct BatchJob {
  int64_t n_rows;
  int64_t *n_selected;
  int32_t n_preds;
  int32_t n_sketch;
  int32_t d;
  int32_t counter_bits;
  int32_t seed_base;   // first RowSeeds of this job (slice sl -> seed_base + sl)
  int32_t pad;
  BucketMod bm;
  PredDev preds[kMaxPreds];
  KeyDev keys[kMaxSketches];
  void *counters[kMaxSketches];
};

struct BatchItem {
  int64_t row0, row1;
  int32_t job;
  int32_t slice_begin, slice_end;
  int32_t count_selected;
};

struct ZeroRegion {
  void *p;
  int64_t words;
};

// Job view over the device-resident job and seed tables.  They are read-only
// while the kernel runs and every lane reads the same entry, so they are
// read through the constant address space (scalar loads, uniform values).
typedef const __attribute__((address_space(4))) BatchJob KJob;
typedef const __attribute__((address_space(4))) BatchItem KItem;
typedef const __attribute__((address_space(4))) RowSeeds KSeeds;

struct GlobalJob {
  KJob *J;
  KSeeds *seed_arr;
  __device__ int n_preds() const { return J->n_preds; }
  __device__ PredDev pred(int q) const {
    PredDev p;
    p.col = J->preds[q].col;
    p.bitmap = J->preds[q].bitmap;
    p.domain = J->preds[q].domain;
    p.kind = J->preds[q].kind;
    p.dtype = J->preds[q].dtype;
    p.lo.i = J->preds[q].lo.i;
    p.hi.i = J->preds[q].hi.i;
    return p;
  }
  __device__ KeyDev key(int s) const {
    KeyDev k;
    k.col = J->keys[s].col;
    k.dtype = J->keys[s].dtype;
    k.pad = 0;
    return k;
  }
  __device__ int slice_sketch(int sl) const { return sl / J->d; }
  __device__ int slice_row(int sl) const { return sl % J->d; }
  __device__ RowSeeds seeds(int sl) const {
    KSeeds &x = seed_arr[J->seed_base + sl];
    return RowSeeds{x.a0, x.a1, x.a2, x.a3, x.b0, x.b1};
  }
  __device__ BucketMod bm() const {
    BucketMod m;
    m.w = J->bm.w;
    m.mask = J->bm.mask;
    m.r32 = J->bm.r32;
    m.pow2 = J->bm.pow2;
    m.inv = J->bm.inv;
    return m;
  }
  __device__ int counter_bits() const { return J->counter_bits; }
  __device__ void *counters(int s) const { return J->counters[s]; }
  __device__ int64_t *n_selected() const { return J->n_selected; }
};

__global__ __launch_bounds__(kBuildThreads) void batch_scan_kernel(
    const BatchJob *jobs, const BatchItem *items, int32_t n_items,
    int32_t *queue, const RowSeeds *seeds) {
  extern __shared__ int32_t lds[];
  __shared__ int32_t s_qn;
  __shared__ int32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n_items) break;  // uniform across the workgroup
    KItem &KI = ((KItem *)items)[it];
    BatchItem I;
    I.row0 = KI.row0;
    I.row1 = KI.row1;
    I.job = KI.job;
    I.slice_begin = KI.slice_begin;
    I.slice_end = KI.slice_end;
    I.count_selected = KI.count_selected;
    const GlobalJob job{(KJob *)jobs + I.job, (KSeeds *)seeds};
    const int w = (int)job.bm().w;
    const int ns = I.slice_end - I.slice_begin;
    int32_t *cnt = lds;
    int32_t *queue_rows = lds + (size_t)ns * w;
    for (int i = threadIdx.x; i < ns * w; i += kBuildThreads) cnt[i] = 0;
    __syncthreads();
    const uint64_t sel = scan_rows(job, I.row0, I.row1, I.slice_begin,
                                   I.slice_end, cnt, queue_rows, &s_qn);
    merge_slices(job, I.slice_begin, I.slice_end, cnt);
    if (I.count_selected && threadIdx.x == 0 && sel)
      atomicAdd(reinterpret_cast<unsigned long long *>(job.n_selected()),
                (unsigned long long)sel);
    __syncthreads();  // LDS is reused by the next item
  }
}

// ---------------------------------------------------------------------
// jobs with predicates: two phases over segments (a row range of one job
// whose survivors' key field elements fit its own region of the plan's
// survivor arena; segments of one round share the arena, rounds run one
// after another)
// ---------------------------------------------------------------------
struct BatchSeg {
  int64_t row0, row1;
  uint64_t *surv;              // [n_sketch][row1 - row0] field elements
  unsigned long long *count;   // survivors written so far
  int32_t job;
  int32_t chunks;              // hashing chunks at most (all rows surviving)
};

struct CompactItem {
  int64_t row0, row1;          // table rows, inside the segment
  int32_t seg;
  int32_t pad;
};

struct HashItem {
  int32_t seg;
  int32_t slice;
  int32_t chunk;
  int32_t pad;
};

typedef const __attribute__((address_space(4))) BatchSeg KSeg;
typedef const __attribute__((address_space(4))) CompactItem KCItem;
typedef const __attribute__((address_space(4))) HashItem KHItem;

constexpr int kBatchQueue = 16384;       // survivors buffered in LDS
// compaction tiles of eight rows per lane: more predicate loads in flight
constexpr int kBatchRows = 8;
constexpr int kBatchTile = kBuildThreads * kBatchRows;
static_assert(kBatchQueue >= 2 * kBatchTile, "a tile fits after a partial queue");
constexpr int64_t kBatchChunk = 1 << 20;  // survivors per hashing chunk
constexpr int kBatchPiece = 32767;        // survivors per 16-bit fold
constexpr int kBatchPairsPerLane = 16;    // 32768 buckets / 2 / 1024 lanes

// Phase A: one workgroup per compact item compacts its tiles (predicates
// evaluated once per row) into an LDS queue of survivor offsets and, when
// the queue is nearly full or the item ends, reserves space in the
// segment's region with one atomic and gathers the key field element of
// every (sketch, survivor) pair.
__global__ __launch_bounds__(kBuildThreads) void batch_compact_kernel(
    const BatchJob *jobs, const BatchSeg *segs, const CompactItem *items) {
  __shared__ int32_t queue[kBatchQueue];
  __shared__ int32_t s_qn;
  __shared__ unsigned long long s_off;
  KCItem &it = ((KCItem *)items)[blockIdx.x];
  const int64_t r0 = it.row0, r1 = it.row1;
  KSeg &sg = ((KSeg *)segs)[it.seg];
  const GlobalJob job{(KJob *)jobs + sg.job, nullptr};
  const int64_t seg_rows = sg.row1 - sg.row0;
  const int n_preds = job.n_preds();
  const int n_sketch = job.J->n_sketch;
  uint64_t sel = 0;
  int qtot = 0;  // block-uniform
  // the first predicate of the next tile is loaded while this one is
  // compacted (jobs here have at least one predicate)
  uint32_t pre[kBatchRows];
  load_first_pred<GlobalJob, kBatchRows>(
      job, r0, (int)min((int64_t)kBatchTile, r1 - r0), pre);
  for (int64_t base = r0; base < r1; base += kBatchTile) {
    const int nt = (int)min((int64_t)kBatchTile, r1 - base);
    uint32_t cur[kBatchRows];
#pragma unroll
    for (int k = 0; k < kBatchRows; ++k) cur[k] = pre[k];
    const int64_t nb = base + kBatchTile;
    if (nb < r1)
      load_first_pred<GlobalJob, kBatchRows>(
          job, nb, (int)min((int64_t)kBatchTile, r1 - nb), pre);
    qtot = compact_tile_loaded<GlobalJob, kBatchRows>(
        job, base, nt, n_preds, queue, &s_qn, qtot, (int)(base - r0), cur);
    const bool last = base + kBatchTile >= r1;
    if (qtot > kBatchQueue - kBatchTile || (last && qtot > 0)) {
      __syncthreads();  // queue complete
      if (threadIdx.x == 0) s_off = atomicAdd(sg.count, (unsigned long long)qtot);
      __syncthreads();
      const int64_t off = (int64_t)s_off;
      for (int s = 0; s < n_sketch; ++s) {
        const KeyDev kd = job.key(s);
        uint64_t *dst = sg.surv + (int64_t)s * seg_rows + off;
        for (int q0 = threadIdx.x; q0 < qtot; q0 += 4 * kBuildThreads) {
          uint64_t v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * kBuildThreads;
            v[u] = q < qtot ? load_field(kd, r0 + queue[q]) : 0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * kBuildThreads;
            if (q < qtot) dst[q] = v[u];
          }
        }
      }
      sel += (uint64_t)qtot;
      qtot = 0;
    }
    __syncthreads();  // queue, s_qn and s_off are reused
  }
  if (threadIdx.x == 0 && sel)
    atomicAdd(reinterpret_cast<unsigned long long *>(job.n_selected()),
              (unsigned long long)sel);
}

// chunks of a segment's survivors that carry work: at least kBatchChunk
// survivors each, at most the planned number
__device__ __forceinline__ int64_t batch_active_chunks(int64_t n,
                                                       int64_t chunks) {
  const int64_t need = (n + kBatchChunk - 1) / kBatchChunk;
  return need < 1 ? 1 : (need < chunks ? need : chunks);
}

// Phase B: one workgroup per (segment, slice, chunk) hashes its chunk of the
// segment's survivors for one sketch row into two 16-bit counters per LDS
// word (+-1 to the low half, +-65536 to the word for the high half; exact
// while both halves stay within [-32767, 32767], so survivors are taken
// kBatchPiece at a time and folded into int32 registers), then adds its
// non-zero counters to the job's counters (zeroed by the plan's first node).
__global__ __launch_bounds__(kBuildThreads) void batch_hash_kernel(
    const BatchJob *jobs, const BatchSeg *segs, const HashItem *items,
    const RowSeeds *seeds) {
  extern __shared__ uint32_t pairs[];
  KHItem &it = ((KHItem *)items)[blockIdx.x];
  KSeg &sg = ((KSeg *)segs)[it.seg];
  const int64_t n = (int64_t)*sg.count;
  const int64_t act = batch_active_chunks(n, sg.chunks);
  if (it.chunk >= act) return;  // uniform: no survivors for this chunk
  const GlobalJob job{(KJob *)jobs + sg.job, (KSeeds *)seeds};
  const BucketMod bm = job.bm();
  const int w = (int)bm.w;  // <= 2 * kBatchPairsPerLane * kBuildThreads
  const int nwords = (w + 1) / 2;
  const int sl = it.slice;
  const int s = job.slice_sketch(sl), row = job.slice_row(sl);
  const RowSeeds sd = job.seeds(sl);
  const int64_t seg_rows = sg.row1 - sg.row0;
  const uint64_t *x = sg.surv + (int64_t)s * seg_rows;
  const int64_t a = n * it.chunk / act, b = n * (it.chunk + 1) / act;
  for (int j = threadIdx.x; j < nwords; j += kBuildThreads) pairs[j] = 0;
  int32_t acc[2 * kBatchPairsPerLane];
#pragma unroll
  for (int i = 0; i < 2 * kBatchPairsPerLane; ++i) acc[i] = 0;
  for (int64_t p0 = a; p0 < b; p0 += kBatchPiece) {
    const int64_t p1 = min(b, p0 + (int64_t)kBatchPiece);
    __syncthreads();  // cleared words
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
      if (!__any(wide_key) && bm.pow2) {
        // interleaved chains; a lane past the end adds 0
        hash_many_pow2_auto<4>(xs, sd, bm.mask, sign, bk);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          atomicAdd(&pairs[bk[u] >> 1],
                    ok[u] ? (uint32_t)sign[u] << ((bk[u] & 1u) << 4) : 0u);
        continue;
      }
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
      for (int u = 0; u < 4; ++u)
        if (ok[u])
          atomicAdd(&pairs[bk[u] >> 1],
                    (bk[u] & 1) ? (uint32_t)sign[u] << 16 : (uint32_t)sign[u]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kBatchPairsPerLane; ++i) {
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
  // integer atomics: order-independent, hence exact
  const size_t rbase = (size_t)row * w;
#pragma unroll
  for (int i = 0; i < kBatchPairsPerLane; ++i) {
    const int wi = threadIdx.x + i * kBuildThreads;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * wi + h;
      const int32_t v = acc[2 * i + h];
      if (j < w && v != 0) {
        if (job.counter_bits() == 32)
          atomicAdd(reinterpret_cast<int32_t *>(job.counters(s)) + rbase + j, v);
        else
          atomicAdd(reinterpret_cast<unsigned long long *>(job.counters(s)) +
                        rbase + j,
                    (unsigned long long)(int64_t)v);
      }
    }
  }
}

// Phase B for rows of at most kBatchNarrowW buckets: one int32 LDS counter
// per bucket (a chunk holds at most kBatchChunk survivors, far inside int32),
// so there is no piece folding and no register copy of the counters, and
// two workgroups fit a CU.  Same items and result as batch_hash_kernel.
constexpr int kBatchNarrowW = 16384;  // 64 KiB of int32 counters
__global__ __launch_bounds__(kBuildThreads) void batch_hash32_kernel(
    const BatchJob *jobs, const BatchSeg *segs, const HashItem *items,
    const RowSeeds *seeds) {
  extern __shared__ int32_t cnt32[];
  KHItem &it = ((KHItem *)items)[blockIdx.x];
  KSeg &sg = ((KSeg *)segs)[it.seg];
  const int64_t n = (int64_t)*sg.count;
  const int64_t act = batch_active_chunks(n, sg.chunks);
  if (it.chunk >= act) return;  // uniform: no survivors for this chunk
  const GlobalJob job{(KJob *)jobs + sg.job, (KSeeds *)seeds};
  const BucketMod bm = job.bm();
  const int w = (int)bm.w;  // <= kBatchNarrowW
  const int sl = it.slice;
  const int s = job.slice_sketch(sl), row = job.slice_row(sl);
  const RowSeeds sd = job.seeds(sl);
  const int64_t seg_rows = sg.row1 - sg.row0;
  const uint64_t *x = sg.surv + (int64_t)s * seg_rows;
  const int64_t a = n * it.chunk / act, b = n * (it.chunk + 1) / act;
  for (int j = threadIdx.x; j < w; j += kBuildThreads) cnt32[j] = 0;
  __syncthreads();
  for (int64_t i0 = a + threadIdx.x; i0 < b; i0 += 4 * kBuildThreads) {
    uint64_t xs[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + u * kBuildThreads;
      ok[u] = i < b;
      xs[u] = ok[u] ? x[i] : 0;
    }
    bool wide_key = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) wide_key = wide_key || (xs[u] >> 32) != 0;
    int32_t sign[4];
    uint32_t bk[4];
    if (!__any(wide_key) && bm.pow2) {
      // interleaved chains; a lane past the end adds 0
      hash_many_pow2_auto<4>(xs, sd, bm.mask, sign, bk);
#pragma unroll
      for (int u = 0; u < 4; ++u) atomicAdd(&cnt32[bk[u]], ok[u] ? sign[u] : 0);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!ok[u]) continue;
        if ((xs[u] >> 32) == 0)
          hash_xi_h<true>(xs[u], sd, bm, sign[u], bk[u]);
        else
          hash_xi_h<false>(xs[u], sd, bm, sign[u], bk[u]);
        atomicAdd(&cnt32[bk[u]], sign[u]);
      }
    }
  }
  __syncthreads();
  // integer atomics: order-independent, hence exact
  const size_t rbase = (size_t)row * w;
  for (int j = threadIdx.x; j < w; j += kBuildThreads) {
    const int32_t v = cnt32[j];
    if (v == 0) continue;
    if (job.counter_bits() == 32)
      atomicAdd(reinterpret_cast<int32_t *>(job.counters(s)) + rbase + j, v);
    else
      atomicAdd(reinterpret_cast<unsigned long long *>(job.counters(s)) + rbase + j,
                (unsigned long long)(int64_t)v);
  }
}

__global__ void zero_regions_kernel(const ZeroRegion *r, int32_t n) {
  for (int k = blockIdx.y; k < n; k += gridDim.y) {
    uint32_t *p = reinterpret_cast<uint32_t *>(r[k].p);
    const int64_t words = r[k].words;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
      p[i] = 0;
  }
}

}  // namespace compass

using namespace compass;

// ---------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------
namespace compass {
void set_last_error(const std::string &s);
}

static compass_status bfail(compass_status s, const std::string &msg) {
  compass::set_last_error(msg);
  return s;
}

#define BHIP(expr)                                                           \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return bfail(COMPASS_E_HIP,                                            \
                   std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

struct compass_batch_plan_s {
  int device = 0;
  int counter_bits = 32;
  std::vector<BatchJob> jobs;
  std::vector<RowSeeds> seeds;
  std::vector<ZeroRegion> zeros;
  std::vector<int64_t> job_rows;
  std::vector<int32_t> job_slices;
  std::vector<int32_t> job_w;
  compass_tune tune{};
  // device copies
  char *dmem = nullptr;
  size_t dbytes = 0;
  BatchJob *d_jobs = nullptr;
  BatchItem *d_items = nullptr;
  RowSeeds *d_seeds = nullptr;
  ZeroRegion *d_zeros = nullptr;
  int32_t *d_queue = nullptr;
  int32_t n_items = 0;
  size_t lds = 0;
  int grid = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n_cu = 0;
  size_t lds_limit = 0;   // LDS one workgroup may allocate on the device
  // jobs with predicates: segments, rounds and the items of both phases
  struct Round {
    size_t c0, c1, h0, h1, g0, g1;  // g: hash items of narrow rows
  };
  std::vector<BatchSeg> segs;        // surv = arena offset until uploaded
  std::vector<size_t> seg_arena_off;
  std::vector<CompactItem> citems;
  std::vector<HashItem> hitems;
  std::vector<HashItem> gitems;      // rows of at most kBatchNarrowW buckets
  std::vector<Round> rounds;
  size_t arena_bytes = 0;
  char *arena = nullptr;
  size_t hash_lds = 0;
  size_t hash32_lds = 0;
  BatchSeg *d_segs = nullptr;
  CompactItem *d_citems = nullptr;
  HashItem *d_hitems = nullptr;
  HashItem *d_gitems = nullptr;
  unsigned long long *d_counts = nullptr;
};

// Jobs with predicates take two phases (compaction of the survivors' key
// field elements, then hashing them per sketch row by many workgroups), so
// their predicates are evaluated once instead of once per slice group.
// Their rows are cut into segments whose worst-case survivor regions (every
// row surviving) fit the arena; segments are packed into rounds that share
// the arena and run one after another.
static void plan_two_phase(compass_batch_plan_s &pl) {
  // arena bytes: 8 GiB, or COMPASS_BATCH_ARENA_BYTES (at least one tile of
  // every job's keys; smaller arenas give more rounds and segments)
  size_t kArenaMax = (size_t)8 << 30;
  if (const char *e = getenv("COMPASS_BATCH_ARENA_BYTES")) {
    const long long v = atoll(e);
    if (v > 0) kArenaMax = (size_t)v;
  }
  constexpr int64_t kCompactRows = 64 * kBuildTile;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  pl.segs.clear();
  pl.seg_arena_off.clear();
  pl.citems.clear();
  pl.hitems.clear();
  pl.gitems.clear();
  pl.rounds.clear();
  pl.arena_bytes = 0;
  pl.hash_lds = 0;
  pl.hash32_lds = 0;
  size_t used = 0;
  compass_batch_plan_s::Round cur{0, 0, 0, 0, 0, 0};
  for (size_t j = 0; j < pl.jobs.size(); ++j) {
    const BatchJob &J = pl.jobs[j];
    const int64_t n = pl.job_rows[j];
    if (J.n_preds == 0 || n == 0) continue;
    const bool narrow = pl.job_w[j] <= kBatchNarrowW;
    if (narrow)
      pl.hash32_lds = std::max(pl.hash32_lds, (size_t)pl.job_w[j] * 4);
    else
      pl.hash_lds = std::max(pl.hash_lds, (size_t)((pl.job_w[j] + 1) / 2) * 4);
    const int64_t max_rows = std::max<int64_t>(
        kBuildTile, (int64_t)(kArenaMax / (8 * (size_t)J.n_sketch)) /
                        kBuildTile * kBuildTile);
    for (int64_t r0 = 0; r0 < n; r0 += max_rows) {
      const int64_t r1 = std::min(n, r0 + max_rows);
      const size_t bytes = al((size_t)(r1 - r0) * J.n_sketch * 8);
      if (used > 0 && used + bytes > kArenaMax) {  // close the round
        cur.c1 = pl.citems.size();
        cur.h1 = pl.hitems.size();
        cur.g1 = pl.gitems.size();
        pl.rounds.push_back(cur);
        cur = {pl.citems.size(), 0, pl.hitems.size(), 0, pl.gitems.size(), 0};
        used = 0;
      }
      BatchSeg sg;
      memset(&sg, 0, sizeof sg);
      sg.row0 = r0;
      sg.row1 = r1;
      sg.job = (int32_t)j;
      sg.chunks = (int32_t)((r1 - r0 + kBatchChunk - 1) / kBatchChunk);
      const int32_t si = (int32_t)pl.segs.size();
      pl.segs.push_back(sg);
      pl.seg_arena_off.push_back(used);
      used += bytes;
      pl.arena_bytes = std::max(pl.arena_bytes, used);
      for (int64_t a = r0; a < r1; a += kCompactRows)
        pl.citems.push_back(CompactItem{a, std::min(r1, a + kCompactRows), si, 0});
      const int S = pl.job_slices[j];
      for (int sl = 0; sl < S; ++sl)
        for (int k = 0; k < sg.chunks; ++k)
          (narrow ? pl.gitems : pl.hitems).push_back(HashItem{si, sl, k, 0});
    }
  }
  if (!pl.segs.empty()) {
    cur.c1 = pl.citems.size();
    cur.h1 = pl.hitems.size();
    cur.g1 = pl.gitems.size();
    pl.rounds.push_back(cur);
  }
}

static BucketMod bmod(uint32_t w) {
  BucketMod m;
  m.w = w;
  m.pow2 = (w & (w - 1)) == 0;
  m.mask = w - 1;
  m.r32 = (uint32_t)((1ull << 32) % w);
  m.inv = 1.0 / (double)w;
  return m;
}

// Work items for a tuning choice; returns the LDS bytes per workgroup.
static size_t make_items(const compass_batch_plan_s &pl, const compass_tune &t,
                         std::vector<BatchItem> &items) {
  items.clear();
  size_t lds_max = 0;
  for (size_t j = 0; j < pl.jobs.size(); ++j) {
    const int64_t n = pl.job_rows[j];
    const int S = pl.job_slices[j];
    const int w = pl.job_w[j];
    if (n == 0 || S == 0) continue;
    if (pl.jobs[j].n_preds > 0) continue;  // two-phase (plan_two_phase)
    const int per_max = std::max(1, std::min<int>(
        (int)(std::min<size_t>(t.lds_budget, kLdsBudget) / ((size_t)w * 4)),
        kMaxLaunchSlices));
    const int ng = (S + per_max - 1) / per_max;
    int64_t rpi = std::max<int64_t>(kBuildTile, t.rows_per_item);
    rpi = (rpi + kBuildTile - 1) / kBuildTile * kBuildTile;
    for (int g = 0; g < ng; ++g) {
      const int sb = (int)((int64_t)S * g / ng);
      const int se = (int)((int64_t)S * (g + 1) / ng);
      lds_max = std::max(lds_max, (size_t)(se - sb) * w * 4);
      for (int64_t r = 0; r < n; r += rpi) {
        BatchItem it;
        it.row0 = r;
        it.row1 = std::min(n, r + rpi);
        it.job = (int32_t)j;
        it.slice_begin = sb;
        it.slice_end = se;
        it.count_selected = (g == 0) ? 1 : 0;
        items.push_back(it);
      }
    }
  }
  // largest first (rows x slices)
  std::stable_sort(items.begin(), items.end(),
                   [&](const BatchItem &a, const BatchItem &b) {
                     const double ca = (double)(a.row1 - a.row0) *
                                       (1 + (a.slice_end - a.slice_begin));
                     const double cb = (double)(b.row1 - b.row0) *
                                       (1 + (b.slice_end - b.slice_begin));
                     return ca > cb;
                   });
  // jobs without predicates only: the row queue is never used
  return lds_max;
}

static compass_status upload_plan(compass_batch_plan_s &pl,
                                  const std::vector<BatchItem> &items) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t b_jobs = al(sizeof(BatchJob) * pl.jobs.size());
  const size_t b_items = al(sizeof(BatchItem) * std::max<size_t>(1, items.size()));
  const size_t b_seeds = al(sizeof(RowSeeds) * std::max<size_t>(1, pl.seeds.size()));
  const size_t b_zero = al(sizeof(ZeroRegion) * (pl.zeros.size() + 2));
  const size_t b_queue = 256;
  const size_t b_segs = al(sizeof(BatchSeg) * std::max<size_t>(1, pl.segs.size()));
  const size_t b_cit = al(sizeof(CompactItem) * std::max<size_t>(1, pl.citems.size()));
  const size_t b_hit = al(sizeof(HashItem) * std::max<size_t>(1, pl.hitems.size()));
  const size_t b_git = al(sizeof(HashItem) * std::max<size_t>(1, pl.gitems.size()));
  const size_t b_cnt = al(8 * std::max<size_t>(1, pl.segs.size()));
  const size_t total = b_jobs + b_items + b_seeds + b_zero + b_queue + b_segs +
                       b_cit + b_hit + b_git + b_cnt;
  if (total > pl.dbytes) {
    if (pl.dmem) BHIP(hipFree(pl.dmem));
    pl.dmem = nullptr;
    BHIP(hipMalloc(&pl.dmem, total));
    pl.dbytes = total;
  }
  size_t off = 0;
  pl.d_jobs = reinterpret_cast<BatchJob *>(pl.dmem + off); off += b_jobs;
  pl.d_items = reinterpret_cast<BatchItem *>(pl.dmem + off); off += b_items;
  pl.d_seeds = reinterpret_cast<RowSeeds *>(pl.dmem + off); off += b_seeds;
  pl.d_zeros = reinterpret_cast<ZeroRegion *>(pl.dmem + off); off += b_zero;
  pl.d_queue = reinterpret_cast<int32_t *>(pl.dmem + off); off += b_queue;
  pl.d_segs = reinterpret_cast<BatchSeg *>(pl.dmem + off); off += b_segs;
  pl.d_citems = reinterpret_cast<CompactItem *>(pl.dmem + off); off += b_cit;
  pl.d_hitems = reinterpret_cast<HashItem *>(pl.dmem + off); off += b_hit;
  pl.d_gitems = reinterpret_cast<HashItem *>(pl.dmem + off); off += b_git;
  pl.d_counts = reinterpret_cast<unsigned long long *>(pl.dmem + off);
  if (pl.arena_bytes > 0 && !pl.arena) BHIP(hipMalloc(&pl.arena, pl.arena_bytes));
  std::vector<BatchSeg> sg = pl.segs;
  for (size_t k = 0; k < sg.size(); ++k) {
    sg[k].surv = reinterpret_cast<uint64_t *>(pl.arena + pl.seg_arena_off[k]);
    sg[k].count = pl.d_counts + k;
  }
  if (!sg.empty())
    BHIP(hipMemcpy(pl.d_segs, sg.data(), sizeof(BatchSeg) * sg.size(),
                   hipMemcpyHostToDevice));
  if (!pl.citems.empty())
    BHIP(hipMemcpy(pl.d_citems, pl.citems.data(),
                   sizeof(CompactItem) * pl.citems.size(), hipMemcpyHostToDevice));
  if (!pl.hitems.empty())
    BHIP(hipMemcpy(pl.d_hitems, pl.hitems.data(),
                   sizeof(HashItem) * pl.hitems.size(), hipMemcpyHostToDevice));
  if (!pl.gitems.empty())
    BHIP(hipMemcpy(pl.d_gitems, pl.gitems.data(),
                   sizeof(HashItem) * pl.gitems.size(), hipMemcpyHostToDevice));
  std::vector<ZeroRegion> z = pl.zeros;
  z.push_back(ZeroRegion{pl.d_queue, 1});
  if (!pl.segs.empty())
    z.push_back(ZeroRegion{pl.d_counts, 2 * (int64_t)pl.segs.size()});
  BHIP(hipMemcpy(pl.d_jobs, pl.jobs.data(), sizeof(BatchJob) * pl.jobs.size(),
                 hipMemcpyHostToDevice));
  if (!items.empty())
    BHIP(hipMemcpy(pl.d_items, items.data(), sizeof(BatchItem) * items.size(),
                   hipMemcpyHostToDevice));
  if (!pl.seeds.empty())
    BHIP(hipMemcpy(pl.d_seeds, pl.seeds.data(),
                   sizeof(RowSeeds) * pl.seeds.size(), hipMemcpyHostToDevice));
  BHIP(hipMemcpy(pl.d_zeros, z.data(), sizeof(ZeroRegion) * z.size(),
                 hipMemcpyHostToDevice));
  pl.n_items = (int32_t)items.size();
  return COMPASS_OK;
}

static void enqueue(const compass_batch_plan_s &pl, hipStream_t st) {
  const int nz = (int)pl.zeros.size() + 1 + (pl.segs.empty() ? 0 : 1);
  hipLaunchKernelGGL(zero_regions_kernel, dim3(16, std::min(nz, 65535)),
                     dim3(256), 0, st, pl.d_zeros, nz);
  if (pl.n_items > 0)
    hipLaunchKernelGGL(batch_scan_kernel, dim3(pl.grid), dim3(kBuildThreads),
                       pl.lds, st, pl.d_jobs, pl.d_items, pl.n_items,
                       pl.d_queue, pl.d_seeds);
  for (const auto &r : pl.rounds) {
    if (r.c1 > r.c0)
      hipLaunchKernelGGL(batch_compact_kernel, dim3((unsigned)(r.c1 - r.c0)),
                         dim3(kBuildThreads), 0, st, pl.d_jobs, pl.d_segs,
                         pl.d_citems + r.c0);
    if (r.g1 > r.g0)
      hipLaunchKernelGGL(batch_hash32_kernel, dim3((unsigned)(r.g1 - r.g0)),
                         dim3(kBuildThreads), pl.hash32_lds, st, pl.d_jobs,
                         pl.d_segs, pl.d_gitems + r.g0, pl.d_seeds);
    if (r.h1 > r.h0)
      hipLaunchKernelGGL(batch_hash_kernel, dim3((unsigned)(r.h1 - r.h0)),
                         dim3(kBuildThreads), pl.hash_lds, st, pl.d_jobs,
                         pl.d_segs, pl.d_hitems + r.h0, pl.d_seeds);
  }
}

static std::string cache_path() {
  const char *p = getenv("COMPASS_AUTOTUNE_CACHE");
  if (p && *p) return p;
  const char *h = getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/compass_autotune.txt";
}

// shape class: arch, counter width, and a coarse histogram of the jobs
static std::string shape_key(const compass_batch_plan_s &pl,
                             const char *arch) {
  std::map<std::string, int64_t> h;
  int64_t rows = 0;
  for (size_t j = 0; j < pl.jobs.size(); ++j) {
    std::ostringstream k;
    k << "w" << pl.job_w[j] << "d" << pl.jobs[j].d
      << (pl.jobs[j].n_preds ? "s" : "x");
    h[k.str()] += 1;
    rows += pl.job_rows[j];
  }
  std::ostringstream o;
  o << arch << "|c" << pl.counter_bits << "|r"
    << (int)std::log2((double)std::max<int64_t>(1, rows)) << "|j"
    << (int)std::log2((double)std::max<size_t>(1, pl.jobs.size()));
  for (auto &kv : h)
    o << "|" << kv.first << ":"
      << (int)std::log2((double)std::max<int64_t>(1, kv.second));
  return o.str();
}

static bool cache_lookup(const std::string &key, compass_tune *t) {
  std::ifstream f(cache_path());
  std::string k;
  long long rpi;
  int lb, bpc;
  while (f >> k >> rpi >> lb >> bpc) {
    if (k == key) {
      t->rows_per_item = rpi;
      t->lds_budget = lb;
      t->blocks_per_cu = bpc;
      return true;
    }
  }
  return false;
}

// Creates every missing directory of `dir` in this process (mkdir(2) per
// path component; no child process).  Returns false with errno set.
static bool make_dirs(const std::string &dir) {
  for (size_t i = 1; i <= dir.size(); ++i) {
    if (i < dir.size() && dir[i] != '/') continue;
    const std::string part = dir.substr(0, i);
    if (mkdir(part.c_str(), 0755) != 0 && errno != EEXIST) return false;
  }
  return true;
}

// Appends the winner to the cache file.  A cache that cannot be written
// does not fail plan creation (the plan is complete either way); the
// reason is left in compass_last_error() and false is returned.
static bool cache_store(const std::string &key, const compass_tune &t) {
  const std::string p = cache_path();
  const size_t slash = p.rfind('/');
  if (slash != std::string::npos && slash > 0 && !make_dirs(p.substr(0, slash))) {
    bfail(COMPASS_OK, "autotune cache not written: cannot create the "
                      "directory of " + p + ": " + strerror(errno));
    return false;
  }
  std::ofstream f(p, std::ios::app);
  if (f)
    f << key << " " << (long long)t.rows_per_item << " " << t.lds_budget << " "
      << t.blocks_per_cu << "\n";
  if (!f) {
    bfail(COMPASS_OK, "autotune cache not written: cannot write " + p);
    return false;
  }
  return true;
}

// Every kernel of the plan fits the LDS one workgroup may allocate:
// dynamic (from the plan) plus static (from the compiled kernel).  Checked
// before anything of the plan is launched.
static compass_status check_lds(const compass_batch_plan_s &pl) {
  struct K {
    const void *fn;
    size_t dyn;
    const char *name;
  } ks[] = {
      {reinterpret_cast<const void *>(batch_scan_kernel), pl.lds, "batch_scan"},
      {reinterpret_cast<const void *>(batch_compact_kernel), 0, "batch_compact"},
      {reinterpret_cast<const void *>(batch_hash32_kernel), pl.hash32_lds,
       "batch_hash32"},
      {reinterpret_cast<const void *>(batch_hash_kernel), pl.hash_lds, "batch_hash"},
  };
  for (const K &k : ks) {
    hipFuncAttributes at;
    BHIP(hipFuncGetAttributes(&at, k.fn));
    if (!lds_fits(k.dyn, at.sharedSizeBytes, pl.lds_limit)) {
      char msg[256];
      snprintf(msg, sizeof msg, "%s needs %zu + %zu bytes of LDS, above the "
               "%zu a workgroup may allocate", k.name, k.dyn,
               (size_t)at.sharedSizeBytes, pl.lds_limit);
      return bfail(COMPASS_E_UNSUPPORTED, msg);
    }
  }
  return COMPASS_OK;
}

static compass_status apply_tune(compass_batch_plan_s &pl,
                                 const compass_tune &t) {
  std::vector<BatchItem> items;
  pl.lds = make_items(pl, t, items);
  compass_status s = check_lds(pl);
  if (s != COMPASS_OK) return s;
  s = upload_plan(pl, items);
  if (s != COMPASS_OK) return s;
  int bpc = std::max(1, t.blocks_per_cu);
  if (pl.lds * bpc > 160 * 1024) bpc = 1;
  pl.grid = std::max(1, pl.n_cu * bpc);
  pl.tune = t;
  return COMPASS_OK;
}

static compass_status autotune(compass_batch_plan_s &pl, hipStream_t st,
                               compass_tune *best_out) {
  const int64_t rpis[] = {65536, 262144, 1048576};
  const int32_t budgets[] = {65536, 131072};
  const int32_t bpcs[] = {1, 2};
  hipEvent_t a, b;
  BHIP(hipEventCreate(&a));
  BHIP(hipEventCreate(&b));
  float best = 1e30f;
  compass_tune bt{};
  compass_status last_fail = COMPASS_OK;
  std::string last_msg;
  for (int64_t rpi : rpis)
    for (int32_t lb : budgets)
      for (int32_t bpc : bpcs) {
        if ((size_t)lb * bpc > 144 * 1024) continue;
        compass_tune t{rpi, lb, bpc};
        bool fits = true;
        for (int w : pl.job_w)
          if ((size_t)w * 4 > (size_t)lb) fits = false;
        if (!fits) continue;
        compass_status s = apply_tune(pl, t);
        if (s != COMPASS_OK) {
          last_fail = s;
          last_msg = compass_last_error();
          continue;
        }
        enqueue(pl, st);  // warm
        BHIP(hipEventRecord(a, st));
        enqueue(pl, st);
        BHIP(hipEventRecord(b, st));
        BHIP(hipEventSynchronize(b));
        float ms = 0;
        BHIP(hipEventElapsedTime(&ms, a, b));
        if (ms < best) {
          best = ms;
          bt = t;
        }
      }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (best >= 1e30f)
    return last_fail != COMPASS_OK ? bfail(last_fail, last_msg)
                                   : bfail(COMPASS_E_UNSUPPORTED, "no tile fits");
  compass::set_last_error("");
  *best_out = bt;
  return COMPASS_OK;
}

extern "C" compass_status compass_batch_plan_create(
    const compass_build_job *jobs, int32_t n_jobs, int32_t counter_bits,
    const compass_tune *tune, hipStream_t stream, compass_batch_plan *out) {
  compass::set_last_error("");
  if (!out || (n_jobs > 0 && !jobs))
    return bfail(COMPASS_E_ARG, "null pointer argument");
  *out = nullptr;
  if (n_jobs < 0) return bfail(COMPASS_E_ARG, "n_jobs < 0");
  if (counter_bits != 32 && counter_bits != 64)
    return bfail(COMPASS_E_ARG, "counter_bits must be 32 or 64");
  compass_batch_plan_s *pl = new compass_batch_plan_s();
  pl->counter_bits = counter_bits;
  auto cleanup = [&](compass_status s) {
    if (pl->dmem) (void)hipFree(pl->dmem);
    if (pl->arena) (void)hipFree(pl->arena);
    delete pl;
    return s;
  };
  for (int j = 0; j < n_jobs; ++j) {
    const compass_build_job &J = jobs[j];
    char msg[256];
    if (J.n_rows < 0 || J.n_rows >= (1ll << 47) ||
        (counter_bits == 32 && J.n_rows > 0x7FFFFFFFll)) {
      snprintf(msg, sizeof msg, "job %d: n_rows out of range", j);
      return cleanup(bfail(COMPASS_E_RANGE, msg));
    }
    if (J.d < 1 || J.d > 32 || J.w < 1 || J.w > (1 << 20) ||
        J.n_sketches < 1 || J.n_sketches > kMaxSketches || J.n_preds < 0 ||
        J.n_preds > kMaxPreds || !J.sketches || !J.n_selected ||
        (J.n_preds > 0 && !J.preds)) {
      snprintf(msg, sizeof msg, "job %d: bad d/w/sketches/predicates", j);
      return cleanup(bfail(COMPASS_E_ARG, msg));
    }
    if ((size_t)J.w * 4 > kLdsBudget) {
      snprintf(msg, sizeof msg, "job %d: w=%d exceeds the LDS budget", j, J.w);
      return cleanup(bfail(COMPASS_E_UNSUPPORTED, msg));
    }
    BatchJob b;
    memset(&b, 0, sizeof b);
    b.n_rows = J.n_rows;
    b.n_selected = J.n_selected;
    b.n_preds = J.n_preds;
    b.n_sketch = J.n_sketches;
    b.d = J.d;
    b.counter_bits = counter_bits;
    b.seed_base = (int32_t)pl->seeds.size();
    b.bm = bmod((uint32_t)J.w);
    for (int q = 0; q < J.n_preds; ++q) {
      const compass_pred &p = J.preds[q];
      if (p.col < 0 || p.col >= J.n_pred_cols || !J.pred_cols ||
          (J.n_rows > 0 && !J.pred_cols[p.col]) || p.kind < 0 || p.kind > 2 ||
          (p.dtype != COMPASS_I32 && p.dtype != COMPASS_F32) ||
          (p.kind == COMPASS_PRED_SUBSET &&
           (p.dtype != COMPASS_I32 || !p.bitmap || p.domain < 0))) {
        snprintf(msg, sizeof msg, "job %d predicate %d is invalid", j, q);
        return cleanup(bfail(COMPASS_E_ARG, msg));
      }
      PredDev &d = b.preds[q];
      d.col = J.pred_cols[p.col];
      d.bitmap = p.bitmap;
      d.domain = p.domain;
      d.kind = p.kind;
      d.dtype = p.dtype;
      memcpy(&d.lo, &p.lo, 4);
      memcpy(&d.hi, &p.hi, 4);
    }
    for (int s = 0; s < J.n_sketches; ++s) {
      const compass_sketch_spec &k = J.sketches[s];
      if (!k.seeds || !k.counters || (J.n_rows > 0 && !k.key_col) ||
          (k.key_dtype != COMPASS_I32 && k.key_dtype != COMPASS_I64)) {
        snprintf(msg, sizeof msg, "job %d sketch %d is invalid", j, s);
        return cleanup(bfail(COMPASS_E_ARG, msg));
      }
      for (int i = 0; i < J.d; ++i) {
        const uint64_t *sd = k.seeds + 6 * i;
        for (int c = 0; c < 6; ++c)
          if (sd[c] >= kP61) {
            snprintf(msg, sizeof msg, "job %d sketch %d: seed not below p", j, s);
            return cleanup(bfail(COMPASS_E_ARG, msg));
          }
        pl->seeds.push_back(RowSeeds{sd[0], sd[1], sd[2], sd[3], sd[4], sd[5]});
      }
      b.keys[s].col = k.key_col;
      b.keys[s].dtype = k.key_dtype;
      b.counters[s] = k.counters;
      pl->zeros.push_back(ZeroRegion{
          k.counters, (int64_t)J.d * J.w * (counter_bits / 8) / 4});
    }
    pl->zeros.push_back(ZeroRegion{J.n_selected, 2});
    pl->jobs.push_back(b);
    pl->job_rows.push_back(J.n_rows);
    pl->job_slices.push_back(J.n_sketches * J.d);
    pl->job_w.push_back(J.w);
  }
  hipDeviceProp_t prop;
  if (hipGetDevice(&pl->device) != hipSuccess ||
      hipGetDeviceProperties(&prop, pl->device) != hipSuccess)
    return cleanup(bfail(COMPASS_E_HIP, "device query failed"));
  pl->n_cu = prop.multiProcessorCount;
  // LDS per workgroup: the device's, or a smaller COMPASS_LDS_LIMIT_BYTES
  // (lets a test force the guard without launching anything)
  pl->lds_limit = prop.sharedMemPerBlock;
  if (const char *e = getenv("COMPASS_LDS_LIMIT_BYTES")) {
    const long long v = atoll(e);
    if (v > 0 && (size_t)v < pl->lds_limit) pl->lds_limit = (size_t)v;
  }
  if (pl->jobs.empty()) {
    *out = pl;
    return COMPASS_OK;
  }
  plan_two_phase(*pl);
  compass_tune t{};
  if (tune) t = *tune;
  const std::string key = shape_key(*pl, prop.gcnArchName);
  if (t.rows_per_item <= 0 || t.lds_budget <= 0 || t.blocks_per_cu <= 0) {
    compass_tune found{};
    if (cache_lookup(key, &found)) {
      t = found;
    } else {
      compass_status s = autotune(*pl, stream, &found);
      if (s != COMPASS_OK) return cleanup(s);
      t = found;
      (void)cache_store(key, t);  // a failure is reported, not fatal
    }
  }
  compass_status s = apply_tune(*pl, t);
  if (s != COMPASS_OK) return cleanup(s);
  // capture zeroing + persistent kernel on a private stream (capture does
  // not execute anything; the graph is launched on the caller's stream)
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
    return cleanup(bfail(COMPASS_E_HIP, "hipStreamCreate failed"));
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) !=
      hipSuccess) {
    (void)hipStreamDestroy(cap);
    return cleanup(bfail(COMPASS_E_HIP, "hipStreamBeginCapture failed"));
  }
  enqueue(*pl, cap);
  const hipError_t ce = hipStreamEndCapture(cap, &pl->graph);
  (void)hipStreamDestroy(cap);
  if (ce != hipSuccess)
    return cleanup(bfail(COMPASS_E_HIP, "hipStreamEndCapture failed"));
  if (hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) !=
      hipSuccess) {
    (void)hipGraphDestroy(pl->graph);
    return cleanup(bfail(COMPASS_E_HIP, "hipGraphInstantiate failed"));
  }
  *out = pl;
  return COMPASS_OK;
}

extern "C" compass_status compass_batch_plan_launch(compass_batch_plan pl,
                                                    hipStream_t stream) {
  if (!pl) return bfail(COMPASS_E_ARG, "null plan");
  if (pl->jobs.empty()) return COMPASS_OK;
  BHIP(hipGraphLaunch(pl->exec, stream));
  return COMPASS_OK;
}

extern "C" compass_status compass_batch_plan_info(compass_batch_plan pl,
                                                  compass_tune *tune,
                                                  int32_t *n_items,
                                                  int32_t *grid) {
  if (!pl) return bfail(COMPASS_E_ARG, "null plan");
  if (tune) *tune = pl->tune;
  if (n_items) *n_items = pl->n_items;
  if (grid) *grid = pl->grid;
  return COMPASS_OK;
}

extern "C" compass_status compass_batch_plan_destroy(compass_batch_plan pl) {
  if (!pl) return COMPASS_OK;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->dmem) (void)hipFree(pl->dmem);
  if (pl->arena) (void)hipFree(pl->arena);
  delete pl;
  return COMPASS_OK;
}
