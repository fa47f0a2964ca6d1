// api.hip -- host side of the C ABI declared in include/compass.h.
//
// Validation, work decomposition and launch sequencing for the fused
// selection + sketch build and for the merged-sketch estimates.  All GPU
// work goes to the caller's stream; nothing here computes a sketch or an
// estimate on the host.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "build_params.hpp"
#include "build_plan.hpp"
#include "compass.h"
#include "estimate_buffers.hpp"
#include "estimate_params.hpp"
#include "generic_params.hpp"
#include "partition_params.hpp"
#include "agms_params.hpp"

namespace compass {
// kernels (build_kernels.hip, estimate_kernels.hip)
hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t st);
hipError_t launch_fill_zero_list(const ZeroSpans &z, hipStream_t st);
hipError_t launch_scan_sketch(const BuildParams &P, int n_blocks,
                              size_t lds_bytes, hipStream_t st);
hipError_t launch_wide_compact(const BuildParams &P, uint64_t *surv,
                               int64_t cap, void *count, int64_t row_begin,
                               int64_t row_end, int n_blocks, hipStream_t st);
hipError_t launch_wide_hash(const uint64_t *surv, const FlushCtl &fc,
                            const void *seeds, const BucketMod &bm, int d,
                            int n_slices, int ranges, int chunks,
                            int32_t *slab, int n_cu, hipStream_t st);
hipError_t launch_slab_reduce(const int32_t *slab, int64_t chunks,
                              int n_slices, int d, int w,
                              void *const *counters, int n_sketches,
                              int counter_bits, int accumulate,
                              const FlushCtl &fc, hipStream_t st);
hipError_t launch_store_seeds(const RowSeeds *src, int n, RowSeeds *dst,
                              hipStream_t st);
hipError_t launch_sort_rows(const SortJob *jobs, int n_jobs,
                            ResolveArgs R, const EstBuffers &B,
                            hipStream_t st);
hipError_t launch_node_merge(const NodeTask *tasks, int n, int max_L,
                             const EstBuffers &B, int stage_bytes,
                             hipStream_t st);
hipError_t launch_node(const NodeTask *tasks, int n, const EstBuffers &B,
                       hipStream_t st);
hipError_t launch_node1(const NodeTask *tasks, int n, const EstBuffers &B,
                        hipStream_t st);
hipError_t launch_apex_prep(const NodeTask *tasks, int n, int Lmax_apex,
                            const EstBuffers &B, hipStream_t st);
hipError_t launch_tri_order(const TriTask *tasks, int n, const EstBuffers &B,
                            hipStream_t st);
hipError_t launch_tri_lane(const TriTask *tasks, int n, const TriGroup *groups,
                           int n_groups, int zblocks,
                           const EstBuffers &B, hipStream_t st);
hipError_t launch_gen_contract(const GenArgs &A, const EstBuffers &B,
                               int n_blocks, int fp64, hipStream_t st);
hipError_t launch_finish(const SubplanTask *sps, int n, const EstBuffers &B,
                         const double *approx, uint64_t *row_est, double *est,
                         int32_t *flags, int32_t n_tables, hipStream_t st);
hipError_t launch_scan2d(const BuildParams &P, const KdDims &kx, int n_blocks,
                         hipStream_t st);
hipError_t launch_tensor_level(const TensorArgs &A, int n_tasks, int max_blocks,
                               hipStream_t st);
hipError_t launch_tensor_finish(const u128 *partial, int n_chunks, int d,
                                const int64_t *n_sel, int n_tables,
                                uint64_t *row_est, double *est, int32_t *flags,
                                hipStream_t st);
hipError_t launch_scan2d_binned(const BuildParams &P, const Bin2dArgs &a,
                                const KdDims &kx,
                                int accumulate, hipStream_t st);
hipError_t launch_chain3(const ChainArgs &a, uint64_t *row_est, double *est,
                         int32_t *flags, hipStream_t st);
hipError_t launch_agms_build(const AgmsParams &P, int n_blocks, hipStream_t st);
hipError_t launch_agms_estimate(const AgmsEstArgs &a, uint64_t *row_sums,
                                double *est, int32_t *flag, hipStream_t st);
}  // namespace compass

using namespace compass;

// ---------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------
static thread_local std::string g_err;

static compass_status fail(compass_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

namespace compass {
void set_last_error(const std::string &s) { g_err = s; }
}  // namespace compass

#define HIP_OK(expr)                                                       \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail(COMPASS_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

// ---------------------------------------------------------------------
// per-device state: scratch memory, pinned staging ring, kernel attrs
// ---------------------------------------------------------------------
struct DeviceState {
  // scratch memory per stream: calls on different streams of one device
  // never share it, so they may be in flight at the same time
  struct Scratch {
    void *p = nullptr;
    size_t bytes = 0;
  };
  std::map<hipStream_t, Scratch> scratch;
  static constexpr int kRing = 4;
  void *pinned[kRing] = {};
  size_t pinned_bytes[kRing] = {};
  hipEvent_t pinned_done[kRing] = {};
  bool pinned_used[kRing] = {};
  int ring_next = 0;
  bool attrs_set = false;
  int n_cu = 256;
};

static std::mutex g_mu;
static std::map<int, DeviceState> g_dev;

static compass_status device_state(DeviceState **out) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  DeviceState &ds = g_dev[dev];
  if (!ds.attrs_set) {
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    ds.n_cu = prop.multiProcessorCount;
    for (int i = 0; i < DeviceState::kRing; ++i)
      HIP_OK(hipEventCreateWithFlags(&ds.pinned_done[i],
                                     hipEventDisableTiming));
    ds.attrs_set = true;
  }
  *out = &ds;
  return COMPASS_OK;
}

// Scratch of at least `bytes` for work on `stream` (grown, never shrunk,
// until compass_release).  Growing waits for the device first: the old
// buffer may still be in use by work already enqueued.
static compass_status ensure_scratch(DeviceState *ds, hipStream_t stream,
                                     size_t bytes, void **out) {
  DeviceState::Scratch &sc = ds->scratch[stream];
  if (bytes > sc.bytes) {
    if (sc.p) {
      HIP_OK(hipDeviceSynchronize());
      HIP_OK(hipFree(sc.p));
      sc.p = nullptr;
    }
    const size_t want = std::max(bytes, sc.bytes * 2);
    sc.bytes = 0;
    HIP_OK(hipMalloc(&sc.p, want));
    sc.bytes = want;
  }
  *out = sc.p;
  return COMPASS_OK;
}

// copies `bytes` of host data to `dst` (device) asynchronously through a
// pinned staging buffer that is reused only once its copy has completed
static compass_status upload(DeviceState *ds, void *dst, const void *src,
                             size_t bytes, hipStream_t st) {
  if (bytes == 0) return COMPASS_OK;
  const int k = ds->ring_next;
  ds->ring_next = (k + 1) % DeviceState::kRing;
  if (ds->pinned_used[k]) HIP_OK(hipEventSynchronize(ds->pinned_done[k]));
  if (ds->pinned_bytes[k] < bytes) {
    if (ds->pinned[k]) HIP_OK(hipHostFree(ds->pinned[k]));
    ds->pinned[k] = nullptr;
    size_t want = std::max(bytes, (size_t)65536);
    HIP_OK(hipHostMalloc(&ds->pinned[k], want, hipHostMallocDefault));
    ds->pinned_bytes[k] = want;
  }
  memcpy(ds->pinned[k], src, bytes);
  HIP_OK(hipMemcpyAsync(dst, ds->pinned[k], bytes, hipMemcpyHostToDevice, st));
  HIP_OK(hipEventRecord(ds->pinned_done[k], st));
  ds->pinned_used[k] = true;
  return COMPASS_OK;
}

// ---------------------------------------------------------------------
// kernel timing (HIP events around each launch, on the launch stream)
// ---------------------------------------------------------------------
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;
// set while an entry point that must not allocate runs: no timing events
static bool g_prof_suppressed = false;
static std::vector<std::string> g_prof_sel;  // empty: every kernel

struct ProfScope {
  ProfRec rec;
  bool on;
  hipStream_t st;
  ProfScope(const char *name, hipStream_t s)
      : on(g_prof_on && !g_prof_suppressed), st(s) {
    if (on && !g_prof_sel.empty())
      on = std::find(g_prof_sel.begin(), g_prof_sel.end(), name) != g_prof_sel.end();
    if (!on) return;
    rec.name = name;
    (void)hipEventCreate(&rec.a);
    (void)hipEventCreate(&rec.b);
    (void)hipEventRecord(rec.a, st);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(rec.b, st);
    g_prof.push_back(rec);
  }
};

extern "C" compass_status compass_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof_on = on != 0;
  return COMPASS_OK;
}

// Synchronises the recorded events and returns, for kernel `name`, the
// number of launches and their total time in milliseconds; then forgets
// every record of that name.
extern "C" compass_status compass_profile_select(const char *names) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof_sel.clear();
  if (!names) return COMPASS_OK;
  std::string cur;
  for (const char *c = names;; ++c) {
    if (*c == ',' || *c == 0) {
      if (!cur.empty()) g_prof_sel.push_back(cur);
      cur.clear();
      if (*c == 0) break;
    } else {
      cur += *c;
    }
  }
  return COMPASS_OK;
}
extern "C" compass_status compass_profile_take(const char *name,
                                               int64_t *count,
                                               double *total_ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  *count = 0;
  *total_ms = 0;
  std::vector<ProfRec> keep;
  for (auto &r : g_prof) {
    if (r.name != name) {
      keep.push_back(r);
      continue;
    }
    HIP_OK(hipEventSynchronize(r.b));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
    *count += 1;
    *total_ms += ms;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.swap(keep);
  return COMPASS_OK;
}

// ---------------------------------------------------------------------
// compass_sketch_build
// ---------------------------------------------------------------------
static BucketMod make_bucket_mod(uint32_t w) {
  BucketMod m;
  m.w = w;
  m.pow2 = (w & (w - 1)) == 0;
  m.mask = w - 1;
  m.r32 = (uint32_t)((1ull << 32) % w);
  m.inv = 1.0 / (double)w;
  return m;
}

static int dtype_size(int dt) { return dt == COMPASS_I64 ? 8 : 4; }

// Validates the predicates of one scan and copies them into the kernel
// parameters.
static compass_status fill_preds(BuildParams &base, int64_t n_rows,
                                 const void *const *pred_cols,
                                 int32_t n_pred_cols, const compass_pred *preds,
                                 int32_t n_preds) {
  for (int i = 0; i < n_preds; ++i) {
    const compass_pred &p = preds[i];
    if (p.col < 0 || p.col >= n_pred_cols ||
        (n_rows > 0 && !pred_cols[p.col]))
      return fail(COMPASS_E_ARG, "predicate %d: bad column index %d", i,
                  p.col);
    if (p.kind < COMPASS_PRED_POINT || p.kind > COMPASS_PRED_SUBSET)
      return fail(COMPASS_E_ARG, "predicate %d: bad kind %d", i, p.kind);
    if (p.dtype != COMPASS_I32 && p.dtype != COMPASS_F32)
      return fail(COMPASS_E_ARG, "predicate %d: dtype must be I32 or F32", i);
    if (p.kind == COMPASS_PRED_SUBSET &&
        (p.dtype != COMPASS_I32 || !p.bitmap || p.domain < 0))
      return fail(COMPASS_E_ARG, "predicate %d: subset needs I32 codes, a "
                  "bitmap and a domain >= 0", i);
    PredDev &q = base.preds[i];
    q.col = pred_cols ? pred_cols[p.col] : nullptr;
    q.bitmap = p.bitmap;
    q.domain = p.domain;
    q.kind = p.kind;
    q.dtype = p.dtype;
    memcpy(&q.lo, &p.lo, 4);
    memcpy(&q.hi, &p.hi, 4);
  }
  return COMPASS_OK;
}

// Where a build's scratch comes from: the pool of the calling stream, or a
// fixed device region (the entry point that allocates nothing).
struct Arena {
  DeviceState *ds = nullptr;   // pooled
  hipStream_t stream = 0;
  char *fixed = nullptr;       // fixed region, fixed_bytes long
  size_t fixed_bytes = 0;
  // called once the arguments are valid, before any GPU work: sets up the
  // fixed region and the CU count
  compass_status (*prepare)(Arena *, int *n_cu) = nullptr;
  compass_status get(size_t bytes, void **out) const {
    if (fixed) {
      if (bytes > fixed_bytes)
        return fail(COMPASS_E_RANGE, "build needs %zu bytes of scratch, the "
                    "fixed region holds %zu", bytes, fixed_bytes);
      *out = fixed;
      return COMPASS_OK;
    }
    return ensure_scratch(ds, stream, bytes, out);
  }
};

// Scratch the pooled two-phase build may take: survivor buffer (8 bytes
// per sketch per buffered survivor) + slab + seeds.
static size_t pooled_two_phase_budget() {
  size_t b = ((size_t)17) << 29;  // 8.5 GiB
  if (const char *e = getenv("COMPASS_TWO_PHASE_BYTES")) {
    const long long v = atoll(e);
    if (v > 0) b = (size_t)v;
  }
  return b;
}

// Two-phase build (tables with predicates, and rows too wide for LDS
// partials): batches of rows are compacted into the survivor buffer
// (their keys' field elements, per sketch); the buffer is hashed into LDS
// counters over bucket ranges and reduced into the counters only when the
// next batch might not fit it, and after the last batch.  `zs` holds the
// regions the call clears first; the buffer's count and ticket join them.
static compass_status build_two_phase(const BuildParams &base,
                                      const compass_sketch_spec *sketches,
                                      int n_sketches, int d, int w,
                                      int counter_bits, int64_t n_rows,
                                      ZeroSpans zs, int n_cu, bool serial,
                                      const Arena &ar, hipStream_t stream) {
  const int S = n_sketches * d;
  int64_t cap_env = 0;
  if (const char *e = getenv("COMPASS_SURVIVOR_CAP_ROWS")) cap_env = atoll(e);
  const size_t budget = ar.fixed ? ar.fixed_bytes : pooled_two_phase_budget();
  const TwoPhasePlan pl = plan_two_phase(n_rows, n_sketches, d, w, n_cu, budget,
                                         cap_env, kBuildTile, sizeof(RowSeeds));
  if (!pl.ok)
    return fail(COMPASS_E_RANGE, "two-phase build of %d sketches x d=%d x "
                "w=%d does not fit %zu bytes of scratch", n_sketches, d, w,
                budget);
  void *scr;
  compass_status st = ar.get(pl.total_bytes, &scr);
  if (st != COMPASS_OK) return st;
  char *c = reinterpret_cast<char *>(scr);
  RowSeeds *dseeds = reinterpret_cast<RowSeeds *>(c);
  unsigned long long *count =
      reinterpret_cast<unsigned long long *>(c + pl.seeds_bytes);
  unsigned int *ticket = reinterpret_cast<unsigned int *>(c + pl.seeds_bytes + 8);
  uint64_t *surv = reinterpret_cast<uint64_t *>(c + pl.seeds_bytes + pl.ctl_bytes);
  int32_t *wslab = reinterpret_cast<int32_t *>(c + pl.seeds_bytes + pl.ctl_bytes +
                                               pl.surv_bytes);
  RowSeeds sd[kMaxSketches * 32];  // S <= 16 sketches x 32 rows
  for (int s = 0; s < n_sketches; ++s)
    for (int i = 0; i < d; ++i) {
      const uint64_t *p = sketches[s].seeds + 6 * i;
      sd[s * d + i] = RowSeeds{p[0], p[1], p[2], p[3], p[4], p[5]};
    }
  HIP_OK(launch_store_seeds(sd, S, dseeds, stream));
  {
    ProfScope ps("fill_zero", stream);
    zs.add(count, 16);  // count and ticket
    HIP_OK(launch_fill_zero_list(zs, stream));
  }
  BuildParams P = base;
  P.count_selected = 1;
  P.n_groups = n_sketches;
  void *cp[kMaxSketches];
  for (int s = 0; s < n_sketches; ++s) cp[s] = sketches[s].counters;
  for (int64_t r0 = 0; r0 < n_rows; r0 += pl.batch) {
    const int64_t r1 = std::min(n_rows, r0 + pl.batch);
    const int64_t tiles = (r1 - r0 + kBuildTile - 1) / kBuildTile;
    {
      ProfScope ps("wide_compact", stream);
      HIP_OK(launch_wide_compact(P, surv, pl.cap, count, r0, r1,
                                 serial ? 1 : (int)std::min<int64_t>(tiles, 2ll * n_cu),
                                 stream));
    }
    FlushCtl fc;
    memset(&fc, 0, sizeof fc);
    fc.count = count;
    fc.ticket = ticket;
    fc.cap = pl.cap;
    fc.need = r1 < n_rows ? std::min(pl.batch, n_rows - r1) : 0;
    fc.force = r1 >= n_rows;
    {
      ProfScope ps("wide_hash", stream);
      HIP_OK(launch_wide_hash(surv, fc, dseeds, base.bm, d, S, pl.ranges,
                              pl.chunks, wslab, n_cu, stream));
    }
    {
      ProfScope ps("slab_reduce", stream);
      HIP_OK(launch_slab_reduce(wslab, pl.chunks, S, d, w, cp, n_sketches,
                                counter_bits, 1, fc, stream));
    }
  }
  return COMPASS_OK;
}

// The pooled arena of the current device and `stream`, and its CU count.
static compass_status pooled_arena(hipStream_t stream, Arena *ar, int *n_cu) {
  DeviceState *ds;
  compass_status st = device_state(&ds);
  if (st != COMPASS_OK) return st;
  ar->ds = ds;
  ar->stream = stream;
  *n_cu = ds->n_cu;
  return COMPASS_OK;
}

static compass_status sketch_build_impl(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *sketches, int32_t n_sketches, int32_t d,
    int32_t w, int32_t counter_bits, int32_t accumulate, int64_t *n_selected,
    const RowSink &sink, const Arena *fixed, int fixed_n_cu,
    hipStream_t stream) {
  if (n_rows < 0 || n_rows >= (1ll << 47))
    return fail(COMPASS_E_RANGE, "n_rows %lld outside [0, 2^47)",
                (long long)n_rows);
  if (d < 1 || d > 32) return fail(COMPASS_E_ARG, "d=%d outside [1, 32]", d);
  if (w < 1 || w > (1 << 20))
    return fail(COMPASS_E_ARG, "w=%d outside [1, 2^20]", w);
  if (counter_bits != 32 && counter_bits != 64)
    return fail(COMPASS_E_ARG, "counter_bits must be 32 or 64");
  if (counter_bits == 32 && n_rows > 0x7FFFFFFFll)
    return fail(COMPASS_E_RANGE, "int32 counters need n_rows < 2^31");
  if (n_sketches < 1 || n_sketches > kMaxSketches)
    return fail(COMPASS_E_ARG, "n_sketches=%d outside [1, %d]", n_sketches,
                kMaxSketches);
  if (n_preds < 0 || n_preds > kMaxPreds)
    return fail(COMPASS_E_ARG, "n_preds=%d outside [0, %d]", n_preds,
                kMaxPreds);
  if (!sketches || !n_selected || (n_preds > 0 && !preds))
    return fail(COMPASS_E_ARG, "null pointer argument");
  if (n_preds > 0 && n_rows > 0 && !pred_cols)
    return fail(COMPASS_E_ARG, "null predicate column array");

  BuildParams base;
  memset(&base, 0, sizeof(base));
  base.n_rows = n_rows;
  base.n_preds = n_preds;
  base.counter_bits = counter_bits;
  base.n_selected = n_selected;
  base.bm = make_bucket_mod((uint32_t)w);
  base.sink = sink;
  compass_status st0 = fill_preds(base, n_rows, pred_cols, n_pred_cols, preds, n_preds);
  if (st0 != COMPASS_OK) return st0;
  for (int s = 0; s < n_sketches; ++s) {
    const compass_sketch_spec &k = sketches[s];
    if (!k.seeds || !k.counters || (n_rows > 0 && !k.key_col))
      return fail(COMPASS_E_ARG, "sketch %d: null pointer", s);
    if (k.key_dtype != COMPASS_I32 && k.key_dtype != COMPASS_I64)
      return fail(COMPASS_E_ARG, "sketch %d: key dtype must be I32 or I64", s);
    for (int i = 0; i < 6 * d; ++i)
      if (k.seeds[i] >= kP61)
        return fail(COMPASS_E_ARG, "sketch %d: seed %d is not below 2^61-1",
                    s, i);
    base.keys[s].col = k.key_col;
    base.keys[s].dtype = k.key_dtype;
    base.counters[s] = k.counters;
  }
  (void)dtype_size;
  compass_status st;
  // scratch: the calling stream's pool, or the caller's fixed region
  Arena ar;
  int n_cu = fixed_n_cu;
  if (fixed) {
    ar = *fixed;
    if (ar.prepare) {
      st = ar.prepare(&ar, &n_cu);
      if (st != COMPASS_OK) return st;
    }
  } else {
    st = pooled_arena(stream, &ar, &n_cu);
    if (st != COMPASS_OK) return st;
  }
  // serial mode (COMPASS_SERIAL=1, for debugging): one chunk per slice
  // group and single-workgroup compaction and hashing, so that no two
  // workgroups combine partial counters; its results must equal the
  // default launch's bit for bit (integer sums do not depend on order)
  const char *ser = getenv("COMPASS_SERIAL");
  const bool serial = ser && atoi(ser) != 0;
  if (serial) n_cu = 1;

  // Two phases (compaction of the survivors' keys, then hashing them) for
  // rows too wide for LDS-private partials, and for every table with
  // predicates: the predicates are then evaluated once (not once per slice
  // group), and the hashing reads only survivors, many workgroups at a
  // time.  Tables without predicates take the fused scan.
  const bool wide = (size_t)w * 4 > kLdsBudget;
  const bool two_phase = wide || n_preds > 0;
  // what an overwriting call clears first, in one launch: the selected
  // count and the selection output's count, and the counters unless the
  // fused scan's reduction overwrites them (the two-phase build adds into
  // them; an empty table launches nothing else).  The two-phase build adds
  // its survivor buffer's count to the same launch.
  ZeroSpans zs;
  memset(&zs, 0, sizeof zs);
  if (!accumulate) {
    if (two_phase || n_rows == 0)
      for (int s = 0; s < n_sketches; ++s)
        zs.add(sketches[s].counters, (int64_t)d * w * (counter_bits / 8));
    zs.add(n_selected, 8);
    if (sink.out) zs.add(sink.count, 8);
  }
  if (n_rows == 0) {
    if (zs.n > 0) {
      ProfScope ps("fill_zero", stream);
      HIP_OK(launch_fill_zero_list(zs, stream));
    }
    return COMPASS_OK;
  }
  if (two_phase)
    return build_two_phase(base, sketches, n_sketches, d, w, counter_bits,
                           n_rows, zs, n_cu, serial, ar, stream);

  // slice groups: consecutive (sketch, row) slices whose int32 partials fit
  // the LDS budget; among the group sizes that fit, prefer one that splits
  // the slices into equal groups (every workgroup then does equal work)
  // (the fused scan builds tables without predicates: no row queue; the
  // queue of one kScanTile is kept for a caller of the fused path with
  // predicates, inside the CU's 160 KiB with a margin for static LDS)
  const size_t queue_bytes = n_preds > 0 ? (size_t)kScanTile * 4 : 0;
  const size_t partial_budget =
      std::min<size_t>(kLdsBudget, 160 * 1024 - 1024 - queue_bytes);
  const int S = n_sketches * d;
  const int per_max = (int)std::min<size_t>(partial_budget / ((size_t)w * 4),
                                            (size_t)kMaxLaunchSlices);
  int per_group = std::min(per_max, S);
  {
    int best_waste = 1 << 30;
    for (int g = per_group; g >= std::max(1, (per_group + 1) / 2); --g) {
      const int ng = (S + g - 1) / g;
      const int waste = ng * g - S;
      if (waste < best_waste) {
        best_waste = waste;
        per_group = g;
      }
      if (waste == 0) break;
    }
  }
  const int n_groups_total = (S + per_group - 1) / per_group;

  // chunks: two whole waves of the resident workgroup slots, else one
  // (whole waves, so that no slot runs one more workgroup than the others),
  // with at least eight tiles per workgroup, which keeps zeroing and
  // writing back its LDS partials small next to its scan; a table too small
  // for one full wave at eight tiles gets fewer chunks.  Each chunk writes
  // its partial counters to a slab (summed by one reduction kernel), which
  // is cheap next to the scan: bound the slab to 1 GiB (or to the fixed
  // scratch region).  A chunk never exceeds INT32_MAX rows (its partials
  // are int32), so very long tables get more chunks than that bound.
  const size_t lds_block = (size_t)per_group * w * 4 + queue_bytes;
  const int per_cu = std::max(1, std::min(2, (int)((160 * 1024) / (lds_block + 1024))));
  const int64_t slots = (int64_t)n_cu * per_cu;
  const int64_t tiles = (n_rows + kScanTile - 1) / kScanTile;
  int64_t chunks = 1;
  for (int waves = 2; waves >= 1; --waves) {
    const int64_t c = std::max<int64_t>(1, waves * slots / n_groups_total);
    if (tiles / c >= 8 || waves == 1) {
      chunks = std::min(c, std::max<int64_t>(1, tiles / 8));
      break;
    }
  }
  const size_t slab_row = (size_t)S * w * 4;
  const size_t slab_cap = ar.fixed ? ar.fixed_bytes : ((size_t)1 << 30);
  if (slab_row > slab_cap)
    return fail(COMPASS_E_RANGE, "one chunk's partial counters (%zu bytes) "
                "exceed the scratch", slab_row);
  chunks = std::min<int64_t>(chunks, std::max<size_t>(1, slab_cap / slab_row));
  if (serial) chunks = 1;
  const int64_t rows_per_chunk = fused_rows_per_chunk(n_rows, chunks, kScanTile);
  chunks = (n_rows + rows_per_chunk - 1) / rows_per_chunk;
  base.rows_per_chunk = rows_per_chunk;
  void *slab;
  st = ar.get((size_t)chunks * slab_row, &slab);
  if (st != COMPASS_OK) return st;
  base.slab = reinterpret_cast<int32_t *>(slab);
  base.d = d;
  base.n_slices_total = S;
  if (zs.n > 0) {
    ProfScope ps("fill_zero", stream);
    HIP_OK(launch_fill_zero_list(zs, stream));
  }

  // launches: as many whole groups as the kernel-argument seed table holds
  int slice = 0;
  bool first = true;
  while (slice < S) {
    BuildParams P = base;
    int ls = 0, ng = 0;
    P.slice_base = slice;
    P.group_begin[0] = 0;
    while (slice < S && ng < kMaxLaunchGroups) {
      const int gs = std::min(per_group, S - slice);
      if (ls + gs > kMaxLaunchSlices) break;
      for (int q = 0; q < gs; ++q) {
        const int gsl = slice + q;
        const int s = gsl / d, i = gsl % d;
        const uint64_t *sd = sketches[s].seeds + 6 * i;
        P.seeds[ls + q] = RowSeeds{sd[0], sd[1], sd[2], sd[3], sd[4], sd[5]};
      }
      ls += gs;
      slice += gs;
      ++ng;
      P.group_begin[ng] = ls;
    }
    P.n_groups = ng;
    P.count_selected = first ? 1 : 0;
    first = false;
    int max_group = 0;
    for (int g = 0; g < ng; ++g)
      max_group = std::max(max_group, P.group_begin[g + 1] - P.group_begin[g]);
    const size_t lds = (size_t)max_group * w * 4 + queue_bytes;
    const int64_t blocks = chunks * ng;
    if (blocks > 0x7FFFFFF0)
      return fail(COMPASS_E_RANGE, "too many workgroups");
    P.n_blocks = (int32_t)blocks;
    ProfScope ps("scan_sketch", stream);
    HIP_OK(launch_scan_sketch(P, (int)blocks, lds, stream));
  }
  {
    void *cp[kMaxSketches];
    for (int s = 0; s < n_sketches; ++s) cp[s] = sketches[s].counters;
    FlushCtl none;
    memset(&none, 0, sizeof none);
    ProfScope ps("slab_reduce", stream);
    HIP_OK(launch_slab_reduce(base.slab, chunks, S, d, w, cp, n_sketches,
                              counter_bits, accumulate, none, stream));
  }
  return COMPASS_OK;
}

extern "C" compass_status compass_sketch_build(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *sketches, int32_t n_sketches, int32_t d,
    int32_t w, int32_t counter_bits, int32_t accumulate, int64_t *n_selected,
    hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  return sketch_build_impl(n_rows, pred_cols, n_pred_cols, preds, n_preds,
                           sketches, n_sketches, d, w, counter_bits, accumulate,
                           n_selected, RowSink{}, nullptr, 0, stream);
}

extern "C" compass_status compass_sketch_build_select(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *sketches, int32_t n_sketches, int32_t d,
    int32_t w, int32_t counter_bits, int32_t accumulate, int64_t *n_selected,
    int64_t *rows_out, int64_t rows_cap, int64_t *rows_count, int64_t row_base,
    hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  if (!rows_count || (rows_cap > 0 && !rows_out) || rows_cap < 0)
    return fail(COMPASS_E_ARG, "selection output: null pointer or negative "
                "capacity");
  if (row_base < 0 || row_base >= (1ll << 47))
    return fail(COMPASS_E_RANGE, "row_base outside [0, 2^47)");
  RowSink sink;
  sink.out = rows_cap > 0 ? rows_out : nullptr;
  sink.cap = rows_cap;
  sink.count = reinterpret_cast<unsigned long long *>(rows_count);
  sink.row_base = row_base;
  if (!sink.out) {
    // nothing can be written, but the count is still kept
    sink.out = reinterpret_cast<int64_t *>(rows_count);
    sink.cap = 0;
  }
  return sketch_build_impl(n_rows, pred_cols, n_pred_cols, preds, n_preds,
                           sketches, n_sketches, d, w, counter_bits, accumulate,
                           n_selected, sink, nullptr, 0, stream);
}

// ---------------------------------------------------------------------
// compass_sketch_build_noalloc: the same build with a fixed scratch region
// ---------------------------------------------------------------------
// One region per device, held until the process ends.  In host code
// `scratch` names a host-side stand-in: kernels get the device address
// taken with hipGetSymbolAddress on the device itself.
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

struct NoAllocDevice {
  char *ptr = nullptr;  // device address of this device's `scratch`
  int n_cu = 0;
};
static std::map<int, NoAllocDevice> g_noalloc;

// The current device's region: its device address is looked up once per
// device, on the first call there, with that device current.
static compass_status noalloc_prepare(Arena *ar, int *n_cu) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  NoAllocDevice &na = g_noalloc[dev];
  if (!na.ptr) {
    void *p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(COMPASS_E_HIP, "no device address for the scratch region");
    int cus = 0;
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    na.ptr = reinterpret_cast<char *>(p);
    na.n_cu = cus;
  }
  ar->fixed = na.ptr;
  *n_cu = na.n_cu;
  return COMPASS_OK;
}

extern "C" compass_status compass_sketch_build_noalloc(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *sketches, int32_t n_sketches, int32_t d,
    int32_t w, int32_t counter_bits, int32_t accumulate, int64_t *n_selected,
    hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  Arena ar;
  ar.fixed_bytes = kNoAllocScratchBytes;
  ar.stream = stream;
  ar.prepare = noalloc_prepare;
  g_prof_suppressed = true;
  const compass_status st = sketch_build_impl(
      n_rows, pred_cols, n_pred_cols, preds, n_preds, sketches, n_sketches, d, w,
      counter_bits, accumulate, n_selected, RowSink{}, &ar, 0, stream);
  g_prof_suppressed = false;
  return st;
}

// ---------------------------------------------------------------------
// compass_estimate: host planning
// ---------------------------------------------------------------------
namespace {

struct PlanNode {
  int table;
  int parent = -1;        // node index
  int parent_edge = -1;
  std::vector<int> children;       // node indices
  std::vector<int> child_edges;
  int cut_edge = -1;
  int height = 0;
};

struct Planner {
  const compass_join_graph *g;
  int d, w;
  std::vector<NodeTask> tasks;
  std::vector<int> task_level;
  std::vector<TriTask> tris;
  std::vector<std::array<int32_t, 9>> tri_key;  // what a sweep group shares
  std::vector<SubplanTask> sps;
  int n_msg_slots = 0, n_x_slots = 0, n_prep_slots = 0, n_partial_slots = 0;
  int Lmax = 0, Lprep = 0;
  std::vector<char> side_used;   // sides read in sorted order
  // generic contraction (any shape; fp64 evaluation of uncertified ones)
  std::vector<GenNode> gnodes;
  std::vector<GenPlan> gplans;
  std::vector<GenBlock> gblocks[2];   // [fp64]
  int64_t glists_len = 0;             // merged list entries, all blocks
  int64_t gmsg_len = 0;               // values (16 bytes each)
  int n_approx_slots = 0;
  // message tasks by subtree: shared by every sub-plan that needs them
  std::map<std::string, int> msg_task;

  int side_of(int table, int e) const {
    return 2 * e + (g->edge_u[e] == table ? 0 : 1);
  }
};

}  // namespace

// Work bounds of the generic contraction: list elements walked over all
// assignments and rows, and message scratch of one plan.
constexpr double kGenWorkCap = 68719476736.0;  // 2^36 element steps
constexpr size_t kGenMsgCap = (size_t)256 << 20;     // exact plans
constexpr size_t kGenMsgCapFp64 = (size_t)64 << 20;  // fp64 plans

// Plans the generic contraction of sub-plan `mask` (index spi): a BFS
// spanning tree from its lowest table (edges in id order), the other edges
// conditioned.  fp64: the approximate evaluation run when the 128-bit
// values are not certified.  Returns false when the shape or its work
// exceeds the bounds (then nothing is added).
static bool plan_generic(Planner &pl, uint64_t mask, int spi, bool fp64,
                         int *out_slot, int *n_slots) {
  const compass_join_graph *g = pl.g;
  const int w = pl.w, d = pl.d;
  std::vector<int> tabs, edges;
  for (int t = 0; t < g->n_tables; ++t)
    if (mask >> t & 1ull) tabs.push_back(t);
  for (int e = 0; e < g->n_edges; ++e)
    if ((mask >> g->edge_u[e] & 1ull) && (mask >> g->edge_v[e] & 1ull))
      edges.push_back(e);
  if (tabs.size() < 2) return false;
  std::vector<int> node_of(g->n_tables, -1), table_of, parent_edge, parent;
  std::vector<char> tree(g->n_edges, 0);
  table_of.push_back(tabs[0]);
  parent_edge.push_back(-1);
  parent.push_back(-1);
  node_of[tabs[0]] = 0;
  for (size_t h = 0; h < table_of.size(); ++h) {
    const int t = table_of[h];
    for (int e : edges) {
      int other;
      if (g->edge_u[e] == t) other = g->edge_v[e];
      else if (g->edge_v[e] == t) other = g->edge_u[e];
      else continue;
      if (node_of[other] >= 0) continue;
      node_of[other] = (int)table_of.size();
      table_of.push_back(other);
      parent_edge.push_back(e);
      parent.push_back((int)h);
      tree[e] = 1;
    }
  }
  const int nn = (int)table_of.size();
  if (nn != (int)tabs.size() || nn > 64) return false;
  std::vector<int> cuts;
  for (int e : edges)
    if (!tree[e]) cuts.push_back(e);
  if ((int)cuts.size() > kGenMaxCut) return false;
  double n_assign = 1;
  for (size_t k = 0; k < cuts.size(); ++k) n_assign *= w;
  // nodes in post-order (reverse BFS order: children before parents)
  std::vector<GenNode> nodes(nn);
  std::vector<int> msg_of(nn, -1);
  int n_msgs = 0;
  for (int a = 1; a < nn; ++a) msg_of[a] = n_msgs++;
  int64_t list_len = 0;
  std::vector<int> post;
  for (int a = nn - 1; a >= 0; --a) post.push_back(a);
  std::vector<char> dynamic(nn, 0);
  for (int a : post) {
    GenNode &N = nodes[a];
    memset(&N, 0, sizeof N);
    const int t = table_of[a];
    N.parent_side = a == 0 ? -1 : pl.side_of(t, parent_edge[a]);
    N.parent_eid = a == 0 ? -1 : parent_edge[a];
    N.msg = msg_of[a];
    for (int c = 1; c < nn; ++c) {
      if (parent[c] != a) continue;
      if (N.n_child >= kGenMaxGroups) return false;
      N.c_side[N.n_child] = pl.side_of(t, parent_edge[c]);
      N.c_eid[N.n_child] = parent_edge[c];
      N.c_msg[N.n_child] = msg_of[c];
      dynamic[a] |= dynamic[c];
      ++N.n_child;
    }
    for (size_t k = 0; k < cuts.size(); ++k) {
      const int e = cuts[k];
      if (g->edge_u[e] != t && g->edge_v[e] != t) continue;
      if (N.n_fixed >= kGenMaxGroups) return false;
      N.f_side[N.n_fixed] = pl.side_of(t, e);
      N.f_eid[N.n_fixed] = e;
      N.f_cut[N.n_fixed] = (int)k;
      ++N.n_fixed;
      dynamic[a] = 1;
    }
    N.is_static = !dynamic[a];
    N.list_off = (int)list_len;
    N.list_len = (N.n_child + (a != 0)) * w;
    list_len += N.list_len;
  }
  if (n_assign * (double)list_len * d > kGenWorkCap) return false;
  // J blocks: enough workgroups to fill the device, message scratch bounded
  const size_t per_block = (size_t)std::max(1, n_msgs) * w * 16;
  int64_t blocks = (int64_t)std::min<double>(n_assign, std::max(1, 2048 / d));
  const size_t cap = fp64 ? kGenMsgCapFp64 : kGenMsgCap;
  blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)(cap / (per_block * d))));
  GenPlan P;
  memset(&P, 0, sizeof P);
  P.node0 = (int)pl.gnodes.size();
  P.n_nodes = nn;
  P.n_msgs = n_msgs;
  P.n_cut = (int)cuts.size();
  P.n_assign = (int64_t)n_assign;
  P.lists_off = pl.glists_len;
  P.msg_off = pl.gmsg_len;
  P.n_blocks = (int)blocks;
  P.sp = spi;
  P.fp64 = fp64 ? 1 : 0;
  if (fp64) {
    P.out_slot = pl.n_approx_slots;
    pl.n_approx_slots += (int)blocks;
  } else {
    P.out_slot = pl.n_partial_slots;
    pl.n_partial_slots += (int)blocks;
  }
  *out_slot = P.out_slot;
  *n_slots = (int)blocks;
  const int plan_idx = (int)pl.gplans.size();
  P.lists_len = (int)list_len;
  for (int a : post) {
    const GenNode &N = nodes[a];
    // the merge reads every list of the node in sorted order (the fp64
    // plans' sides too: sorting them only when some sub-plan is not
    // certified would need the certificates first, which costs more than
    // the sorts it saves)
    for (int c = 0; c < N.n_child; ++c) pl.side_used[N.c_side[c]] = 1;
    if (N.parent_side >= 0) pl.side_used[N.parent_side] = 1;
    pl.gnodes.push_back(N);
  }
  for (int b = 0; b < blocks; ++b) pl.gblocks[fp64 ? 1 : 0].push_back(GenBlock{plan_idx, b});
  pl.gplans.push_back(P);
  pl.glists_len += (int64_t)blocks * d * list_len;
  pl.gmsg_len += (int64_t)blocks * d * n_msgs * w;
  return true;
}

// A sub-plan the triangle-specialised path does not evaluate: the generic
// contraction if it fits its bounds, else flagged unsupported.
static void plan_other_shape(Planner &pl, SubplanTask &sp, uint64_t mask, int spi) {
  int slot = 0, n = 0;
  if (plan_generic(pl, mask, spi, false, &slot, &n)) {
    sp.type = kSpGeneric;
    sp.x_slot = slot;
    sp.n_partials = n;
  } else {
    sp.type = kSpUnsupported;
  }
}

// Builds the rooted spanning tree of one sub-plan and its node tasks.
static compass_status plan_subplan(Planner &pl, uint64_t mask, int spi) {
  const compass_join_graph *g = pl.g;
  SubplanTask sp;
  memset(&sp, 0, sizeof(sp));
  sp.mask = mask;
  sp.approx_slot = -1;
  std::vector<int> tabs, edges;
  for (int t = 0; t < g->n_tables; ++t)
    if (mask >> t & 1ull) tabs.push_back(t);
  for (int e = 0; e < g->n_edges; ++e)
    if ((mask >> g->edge_u[e] & 1ull) && (mask >> g->edge_v[e] & 1ull))
      edges.push_back(e);
  sp.n_tables = (int)tabs.size();
  sp.n_edges = (int)edges.size();
  if (tabs.size() == 1) {
    sp.type = kSpSingle;
    sp.single_table = tabs[0];
    pl.sps.push_back(sp);
    return COMPASS_OK;
  }
  // BFS spanning tree from the lowest table, edges in id order
  std::map<int, int> node_of;
  std::vector<PlanNode> base;
  base.push_back(PlanNode());
  base[0].table = tabs[0];
  node_of[tabs[0]] = 0;
  std::vector<char> base_tree(g->n_edges, 0);
  for (size_t head = 0; head < base.size(); ++head) {
    const int t = base[head].table;
    for (int e : edges) {
      int other;
      if (g->edge_u[e] == t)
        other = g->edge_v[e];
      else if (g->edge_v[e] == t)
        other = g->edge_u[e];
      else
        continue;
      if (node_of.count(other)) continue;
      PlanNode nd;
      nd.table = other;
      node_of[other] = (int)base.size();
      base_tree[e] = 1;
      base.push_back(nd);
    }
  }
  if (base.size() != tabs.size())
    return fail(COMPASS_E_GRAPH, "sub-plan %d (mask 0x%llx) is not connected",
                spi, (unsigned long long)mask);
  std::vector<int> cuts;
  for (int e : edges)
    if (!base_tree[e]) cuts.push_back(e);

  const int nn = (int)base.size();
  auto build_adj = [&](const std::vector<char> &tree) {
    std::vector<std::vector<std::pair<int, int>>> adj(nn);
    for (int e : edges) {
      if (!tree[e]) continue;
      const int a = node_of[g->edge_u[e]], b = node_of[g->edge_v[e]];
      adj[a].push_back({b, e});
      adj[b].push_back({a, e});
    }
    return adj;
  };
  const auto base_adj = build_adj(base_tree);

  // Roots to plan.  A tree is rooted at its lowest table.  A triangle may
  // cut any of its three edges (the estimate is the same number); the
  // apex (the vertex opposite the cut) should have as few children as
  // possible, so every triangle vertex of fewest sub-plan edges is a
  // candidate.  All candidates are planned; on the device the one whose
  // table has the fewest selected rows runs and the others' blocks return
  // at once (fewer rows give smaller counters with fewer distinct
  // magnitudes, hence fewer and longer same-child runs in the sweep).
  std::vector<int> cand;
  int apex = -1, cut0 = -1;
  if (cuts.size() > 1) {
    plan_other_shape(pl, sp, mask, spi);
    pl.sps.push_back(sp);
    return COMPASS_OK;
  }
  if (cuts.size() == 1) {
    cut0 = cuts[0];
    const int cu = node_of[g->edge_u[cut0]], cv = node_of[g->edge_v[cut0]];
    // apex: a common tree neighbour of both endpoints (a triangle)
    bool direct = false;
    for (auto &pa : base_adj[cu]) {
      if (pa.first == cv) direct = true;
      for (auto &pb : base_adj[cv])
        if (pa.first == pb.first) apex = pa.first;
    }
    if (direct || apex < 0) {
      plan_other_shape(pl, sp, mask, spi);
      pl.sps.push_back(sp);
      return COMPASS_OK;
    }
    auto degree = [&](int node) {
      int k = 0;
      for (int e : edges)
        k += g->edge_u[e] == base[node].table || g->edge_v[e] == base[node].table;
      return k;
    };
    const int dmin = std::min(degree(apex), std::min(degree(cu), degree(cv)));
    for (int x : {apex, cu, cv})
      if (degree(x) == dmin) cand.push_back(x);
    std::sort(cand.begin(), cand.end(), [&](int x, int y) {
      return base[x].table < base[y].table;
    });
  } else {
    cand.push_back(0);
  }

  // orient every candidate; drop those with a node beyond kMaxChild children
  struct Oriented {
    std::vector<PlanNode> nodes;
    std::vector<int> order;
    int root, cut_e, cut_u, cut_v;
  };
  std::vector<Oriented> ors;
  for (int root : cand) {
    Oriented o;
    o.nodes = base;
    o.root = root;
    o.cut_e = cut0;
    std::vector<char> tree = base_tree;
    if (cut0 >= 0 && root != apex) {
      // cut the triangle edge opposite `root` instead
      const int cu = node_of[g->edge_u[cut0]], cv = node_of[g->edge_v[cut0]];
      const int other = root == cu ? cv : cu;
      int new_cut = -1;
      for (auto &p : base_adj[apex])
        if (p.first == other) new_cut = p.second;
      tree[cut0] = 1;
      tree[new_cut] = 0;
      o.cut_e = new_cut;
    }
    const auto adj = build_adj(tree);
    o.cut_u = o.cut_v = -1;
    if (o.cut_e >= 0) {
      o.cut_u = node_of[g->edge_u[o.cut_e]];
      o.cut_v = node_of[g->edge_v[o.cut_e]];
    }
    std::vector<char> seen(nn, 0);
    o.order.push_back(root);
    seen[root] = 1;
    for (size_t h = 0; h < o.order.size(); ++h) {
      const int a = o.order[h];
      std::vector<std::pair<int, int>> nb = adj[a];
      std::sort(nb.begin(), nb.end(),
                [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
                  return x.second < y.second;
                });
      for (auto &p : nb) {
        if (seen[p.first]) continue;
        seen[p.first] = 1;
        o.nodes[p.first].parent = a;
        o.nodes[p.first].parent_edge = p.second;
        o.nodes[a].children.push_back(p.first);
        o.nodes[a].child_edges.push_back(p.second);
        o.order.push_back(p.first);
      }
    }
    if (o.cut_e >= 0) {
      o.nodes[o.cut_u].cut_edge = o.cut_e;
      o.nodes[o.cut_v].cut_edge = o.cut_e;
    }
    bool fits = true;
    for (int k = nn - 1; k >= 0; --k) {
      PlanNode &nd = o.nodes[o.order[k]];
      for (int c : nd.children)
        nd.height = std::max(nd.height, o.nodes[c].height + 1);
      if ((int)nd.children.size() > kMaxChild) fits = false;
    }
    if (fits) ors.push_back(std::move(o));
  }
  if (ors.empty()) {
    plan_other_shape(pl, sp, mask, spi);
    pl.sps.push_back(sp);
    return COMPASS_OK;
  }
  TaskGuard gd;
  memset(&gd, 0, sizeof(gd));
  gd.n = (int)ors.size();
  for (size_t k = 0; k < ors.size(); ++k) gd.tab[k] = base[ors[k].root].table;

  for (size_t ko = 0; ko < ors.size(); ++ko) {
    Oriented &o = ors[ko];
    std::vector<PlanNode> &nodes = o.nodes;
    const int root = o.root, cut_e = o.cut_e, cut_u = o.cut_u, cut_v = o.cut_v;
    gd.self = (int)ko;
    // tasks: every non-root node emits a message slot; cut endpoints also a
    // cut-constant slot.  A leaf's message and cut constants are its own
    // counters (slot -1 - side: read in place, no task).  A message whose
    // subtree (tables, edges, cut edges) another sub-plan already planned
    // is the same array: its slots are shared and no task is added.
    std::vector<int> msg_slot(nn, -1), cmsg_slot(nn, -1);
    std::vector<std::string> key(nn);
    for (int k = nn - 1; k >= 0; --k) {
      const int a = o.order[k];
      PlanNode &nd = nodes[a];
      if (a != root) {
        std::vector<std::string> ck;
        for (size_t c = 0; c < nd.children.size(); ++c) ck.push_back(key[nd.children[c]]);
        std::sort(ck.begin(), ck.end());
        key[a] = "(" + std::to_string(nd.table) + "," + std::to_string(nd.parent_edge) +
                 "," + std::to_string(nd.cut_edge) + ":";
        for (auto &x : ck) key[a] += x;
        key[a] += ")";
        if (nd.children.empty()) {
          msg_slot[a] = -1 - pl.side_of(nd.table, nd.parent_edge);
          if (nd.cut_edge >= 0) cmsg_slot[a] = -1 - pl.side_of(nd.table, nd.cut_edge);
          continue;
        }
        auto it = pl.msg_task.find(key[a]);
        if (it != pl.msg_task.end()) {
          NodeTask &S = pl.tasks[it->second];
          msg_slot[a] = S.msg_slot;
          cmsg_slot[a] = S.cmsg_slot;
          // shared by rootings of different guards: always computed
          if (memcmp(&S.guard, &gd, sizeof(gd)) != 0) S.guard.n = 0;
          continue;
        }
        msg_slot[a] = pl.n_msg_slots++;
        if (nd.cut_edge >= 0) cmsg_slot[a] = pl.n_msg_slots++;
        pl.msg_task[key[a]] = (int)pl.tasks.size();
      }
      NodeTask T;
      memset(&T, 0, sizeof(T));
      T.guard = gd;
      T.m = (int)nd.children.size();
      T.parent_side = -1;
      T.cut_side = -1;
      T.msg_slot = msg_slot[a];
      T.cmsg_slot = cmsg_slot[a];
      for (int c = 0; c < T.m; ++c) {
        const int e = nd.child_edges[c];
        T.child_side[c] = pl.side_of(nd.table, e);
        T.child_eid[c] = e;
        T.child_msg[c] = msg_slot[nd.children[c]];
        T.child_cut[c] = -1;
        pl.side_used[T.child_side[c]] = 1;
      }
      // a one-child node reads its query lists (parent, cut) by bucket; a
      // merged node reads every list in sorted order
      int nl = T.m;
      if (a != root) {
        T.parent_side = pl.side_of(nd.table, nd.parent_edge);
        T.parent_eid = nd.parent_edge;
        if (T.m >= 2) pl.side_used[T.parent_side] = 1;
        ++nl;
      }
      if (nd.cut_edge >= 0) {
        T.cut_side = pl.side_of(nd.table, nd.cut_edge);
        T.cut_eid = nd.cut_edge;
        if (T.m >= 2) pl.side_used[T.cut_side] = 1;
        ++nl;
      }
      if (a != root) {
        T.mode = kModeMessage;
      } else if (cut_e < 0) {
        T.mode = kModeTreeRoot;
        T.out_slot = pl.n_x_slots++;
        sp.type = kSpTree;
        sp.x_slot = T.out_slot;
      } else {
        T.mode = kModeTriRootPrep;
        T.out_slot = pl.n_prep_slots++;
        for (int c = 0; c < T.m; ++c) {
          const int ch = nd.children[c];
          if (ch == cut_u) T.child_cut[c] = 0;
          if (ch == cut_v) T.child_cut[c] = 1;
        }
        pl.Lprep = std::max(pl.Lprep, T.m * pl.w);
        TriTask tr;
        memset(&tr, 0, sizeof(tr));
        tr.guard = gd;
        tr.prep_slot = T.out_slot;
        tr.L = T.m * pl.w;
        tr.m = T.m;
        tr.cut_eid = cut_e;
        tr.cut_side[0] = pl.side_of(nodes[cut_u].table, cut_e);
        tr.cut_side[1] = pl.side_of(nodes[cut_v].table, cut_e);
        tr.cut_cmsg[0] = cmsg_slot[cut_u];
        tr.cut_cmsg[1] = cmsg_slot[cut_v];
        for (int c = 0; c < T.m; ++c) {
          if (nd.children[c] == cut_u) {
            tr.cut_child[0] = c;
            tr.cut_peid[0] = nd.child_edges[c];
          }
          if (nd.children[c] == cut_v) {
            tr.cut_child[1] = c;
            tr.cut_peid[1] = nd.child_edges[c];
          }
          // tables of the child's subtree (bounds for narrow arithmetic)
          uint64_t sub = 0;
          std::vector<int> stack{nd.children[c]};
          while (!stack.empty()) {
            const int x = stack.back();
            stack.pop_back();
            sub |= 1ull << nodes[x].table;
            for (int y : nodes[x].children) stack.push_back(y);
          }
          tr.child_tables[c] = sub;
        }
        tr.root_table = nd.table;
        const int zb = (pl.w + kLaneThreads - 1) / kLaneThreads;
        // every candidate writes the same partial sums (only one runs)
        if (ko == 0) {
          sp.type = kSpTriangle;
          sp.x_slot = pl.n_partial_slots;
          sp.n_partials = zb;
          pl.n_partial_slots += zb;
        }
        tr.partial_slot = sp.x_slot;
        T.tri = (int)pl.tris.size();
        pl.tris.push_back(tr);
        pl.tri_key.push_back({tr.root_table, T.m, T.child_side[0],
                              T.m > 1 ? T.child_side[1] : -1, tr.cut_eid,
                              tr.cut_side[0], tr.cut_side[1], tr.cut_child[0],
                              tr.cut_child[1]});
      }
      if (T.m > 0) pl.Lmax = std::max(pl.Lmax, nl * pl.w);
      pl.tasks.push_back(T);
      pl.task_level.push_back(nd.height);
    }
  }
  pl.sps.push_back(sp);
  return COMPASS_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

extern "C" compass_status compass_estimate(const compass_join_graph *g,
                                           const uint64_t *masks,
                                           int32_t n_subplans,
                                           compass_i128 *row_est, double *est,
                                           int32_t *flags,
                                           hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  if (!g || !masks || !est || !flags)
    return fail(COMPASS_E_ARG, "null pointer argument");
  if (n_subplans < 0) return fail(COMPASS_E_ARG, "n_subplans < 0");
  if (n_subplans == 0) return COMPASS_OK;
  if (g->n_tables < 1 || g->n_tables > 64)
    return fail(COMPASS_E_RANGE, "n_tables=%d outside [1, 64]", g->n_tables);
  if (g->n_edges < 0 || g->n_edges > 64)
    return fail(COMPASS_E_RANGE, "n_edges=%d outside [0, 64]", g->n_edges);
  if (g->d < 1 || g->d > 32)
    return fail(COMPASS_E_ARG, "d=%d outside [1, 32]", g->d);
  if (g->w < 1 || g->w > kMaxEstimateW)
    return fail(COMPASS_E_UNSUPPORTED, "w=%d outside [1, %d]", g->w,
                kMaxEstimateW);
  if (g->counter_bits != 32 && g->counter_bits != 64)
    return fail(COMPASS_E_ARG, "counter_bits must be 32 or 64");
  if (!g->n_selected || (g->n_edges > 0 && (!g->edge_u || !g->edge_v ||
                                            !g->sketch)))
    return fail(COMPASS_E_ARG, "null graph array");
  for (int e = 0; e < g->n_edges; ++e) {
    if (g->edge_u[e] < 0 || g->edge_u[e] >= g->n_tables || g->edge_v[e] < 0 ||
        g->edge_v[e] >= g->n_tables || g->edge_u[e] == g->edge_v[e])
      return fail(COMPASS_E_GRAPH, "edge %d has bad endpoints", e);
    if (!g->sketch[2 * e] || !g->sketch[2 * e + 1])
      return fail(COMPASS_E_GRAPH, "edge %d lacks a sketch", e);
  }
  const uint64_t all =
      g->n_tables == 64 ? ~0ull : ((1ull << g->n_tables) - 1);
  for (int i = 0; i < n_subplans; ++i)
    if (masks[i] == 0 || (masks[i] & ~all))
      return fail(COMPASS_E_GRAPH, "sub-plan %d: mask 0x%llx is empty or "
                  "names a missing table", i, (unsigned long long)masks[i]);

  Planner pl;
  pl.g = g;
  pl.d = g->d;
  pl.w = g->w;
  pl.side_used.assign(2 * g->n_edges, 0);
  for (int i = 0; i < n_subplans; ++i) {
    compass_status s = plan_subplan(pl, masks[i], i);
    if (s != COMPASS_OK) return s;
  }
  // an fp64 evaluation of every multi-table sub-plan, run on the device
  // only when its 128-bit values cannot be certified
  for (int i = 0; i < n_subplans; ++i) {
    SubplanTask &sp = pl.sps[i];
    if (sp.n_tables < 2 || sp.type == kSpUnsupported) continue;
    int slot = 0, n = 0;
    if (plan_generic(pl, masks[i], i, true, &slot, &n)) {
      sp.approx_slot = slot;
      sp.n_approx = n;
    }
  }

  DeviceState *ds;
  compass_status st = device_state(&ds);
  if (st != COMPASS_OK) return st;

  // sort jobs
  std::vector<SortJob> sort_jobs;
  for (int s = 0; s < 2 * g->n_edges; ++s)
    if (pl.side_used[s]) {
      SortJob j;
      memset(&j, 0, sizeof j);
      j.counters = g->sketch[s];
      j.side = s;
      sort_jobs.push_back(j);
    }
  // levels
  int max_level = 0;
  for (int lv : pl.task_level) max_level = std::max(max_level, lv);
  std::vector<std::vector<NodeTask>> levels(max_level + 1);
  for (size_t k = 0; k < pl.tasks.size(); ++k)
    levels[pl.task_level[k]].push_back(pl.tasks[k]);
  // a level is launched in groups of node tasks whose merge scratch
  // (merged list + records per sketch row) stays within kNodeScratchBytes;
  // groups run one after another on the stream and reuse the slots
  const int d = g->d, w = g->w;
  const size_t per_task =
      (size_t)d * std::max(1, pl.Lmax) * (sizeof(uint32_t) + sizeof(NodeRec));
  const size_t group_tasks = std::min<size_t>(
      kMaxGridZ, std::max<size_t>(1, kNodeScratchBytes / per_task));
  size_t max_level_tasks = 0;
  std::vector<NodeTask> flat;
  std::vector<size_t> level_off;
  // within a level: one-child nodes, other nodes, triangle apexes, so that
  // every kernel of a group is launched over its own tasks only
  auto kind = [](const NodeTask &t) {
    return t.mode == kModeTriRootPrep ? 2 : (t.m == 1 ? 0 : 1);
  };
  for (auto &lv : levels) {
    std::stable_sort(lv.begin(), lv.end(),
                     [&](const NodeTask &a, const NodeTask &b) {
                       return kind(a) < kind(b);
                     });
    for (size_t k = 0; k < lv.size(); ++k)
      lv[k].scratch_slot = (int)(k % group_tasks);
    level_off.push_back(flat.size());
    flat.insert(flat.end(), lv.begin(), lv.end());
    max_level_tasks = std::max(max_level_tasks, std::min(lv.size(), group_tasks));
  }
  // scratch layout
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t o_sides = carve(sizeof(void *) * std::max(1, 2 * g->n_edges));
  const size_t o_jobs = carve(sizeof(SortJob) * std::max<size_t>(1, sort_jobs.size()));
  const size_t o_tasks = carve(sizeof(NodeTask) * std::max<size_t>(1, flat.size()));
  const size_t o_tris = carve(sizeof(TriTask) * std::max<size_t>(1, pl.tris.size()));
  // two-child sweep groups: triangle tasks of the same apex structure, in
  // order of first appearance, kTriGroupMax at most per group
  std::vector<TriGroup> tgroups;
  {
    std::map<std::array<int32_t, 9>, int> open;  // key -> group being filled
    for (size_t t = 0; t < pl.tris.size(); ++t) {
      if (pl.tris[t].m != 2) continue;
      auto it = open.find(pl.tri_key[t]);
      if (it == open.end() || tgroups[it->second].n == kTriGroupMax) {
        TriGroup gr;
        memset(&gr, 0, sizeof gr);
        tgroups.push_back(gr);
        open[pl.tri_key[t]] = (int)tgroups.size() - 1;
        it = open.find(pl.tri_key[t]);
      }
      TriGroup &gr = tgroups[it->second];
      gr.member[gr.n++] = (int)t;
    }
  }
  const size_t o_tgroups = carve(sizeof(TriGroup) * std::max<size_t>(1, tgroups.size()));
  const size_t o_sps = carve(sizeof(SubplanTask) * pl.sps.size());
  const size_t o_sorted = carve(sizeof(uint64_t) * 2 * g->n_edges * d * (size_t)w);
  const size_t o_msg = carve(16ull * pl.n_msg_slots * d * (size_t)w);
  const size_t o_merged = carve(4ull * max_level_tasks * d * (size_t)std::max(1, pl.Lmax));
  const size_t o_nrec = carve(sizeof(NodeRec) * max_level_tasks * d *
                              (size_t)std::max(1, pl.Lmax));
  const size_t o_n1tot = carve(16ull * 2 * kN1MaxChunks * max_level_tasks * d);
  const size_t o_xout = carve(16ull * std::max(1, pl.n_x_slots) * d);
  const size_t np = std::max(1, pl.n_prep_slots);
  const size_t lp = std::max(1, pl.Lprep);
  const size_t o_prep = carve(sizeof(TriElem) * np * d * lp);
  const size_t o_prepn = carve(sizeof(TriElemN) * np * d * lp);
  const size_t o_prepz = carve(sizeof(int32_t) * np * d);
  const size_t o_tkey = carve(sizeof(uint32_t) * np * d * lp);
  const size_t o_tpre = carve(sizeof(TriPre) * np * d *
                              ((lp + kOrderTile - 1) / kOrderTile) *
                              (kOrderTile + 1));
  const size_t o_tseg = carve(sizeof(int32_t) * np * d * (kFastSegs + 1));
  const int pcap = std::min((int)lp, kOrderCap) + 1;
  const size_t o_tpiece = carve(sizeof(TriPiece) * np * d * (size_t)pcap);
  const size_t o_tsegp = carve(sizeof(int32_t) * np * d * (kFastSegs + 1));
  const size_t o_part = carve(16ull * std::max(1, pl.n_partial_slots) * d);
  const size_t o_gnodes = carve(sizeof(GenNode) * std::max<size_t>(1, pl.gnodes.size()));
  const size_t o_gplans = carve(sizeof(GenPlan) * std::max<size_t>(1, pl.gplans.size()));
  const size_t o_gblk0 = carve(sizeof(GenBlock) * std::max<size_t>(1, pl.gblocks[0].size()));
  const size_t o_gblk1 = carve(sizeof(GenBlock) * std::max<size_t>(1, pl.gblocks[1].size()));
  const size_t o_glists = carve(4ull * std::max<int64_t>(1, pl.glists_len));
  const size_t o_gmsg = carve(16ull * std::max<int64_t>(1, pl.gmsg_len));
  const size_t o_approx = carve(8ull * std::max(1, pl.n_approx_slots) * d);
  void *scratch;
  st = ensure_scratch(ds, stream, off, &scratch);
  if (st != COMPASS_OK) return st;
  char *base = reinterpret_cast<char *>(scratch);

  // one staging upload of every host-built table
  std::vector<char> host(o_sorted, 0);
  memcpy(host.data() + o_sides, g->sketch, sizeof(void *) * 2 * g->n_edges);
  if (!sort_jobs.empty())
    memcpy(host.data() + o_jobs, sort_jobs.data(), sizeof(SortJob) * sort_jobs.size());
  if (!flat.empty())
    memcpy(host.data() + o_tasks, flat.data(), sizeof(NodeTask) * flat.size());
  if (!pl.tris.empty())
    memcpy(host.data() + o_tris, pl.tris.data(), sizeof(TriTask) * pl.tris.size());
  if (!tgroups.empty())
    memcpy(host.data() + o_tgroups, tgroups.data(), sizeof(TriGroup) * tgroups.size());
  memcpy(host.data() + o_sps, pl.sps.data(), sizeof(SubplanTask) * pl.sps.size());
  st = upload(ds, base, host.data(), o_sorted, stream);
  if (st != COMPASS_OK) return st;
  if (!pl.gplans.empty()) {
    // the generic plans' tables (between o_gnodes and o_glists)
    std::vector<char> gh(o_glists - o_gnodes, 0);
    memcpy(gh.data(), pl.gnodes.data(), sizeof(GenNode) * pl.gnodes.size());
    memcpy(gh.data() + (o_gplans - o_gnodes), pl.gplans.data(),
           sizeof(GenPlan) * pl.gplans.size());
    if (!pl.gblocks[0].empty())
      memcpy(gh.data() + (o_gblk0 - o_gnodes), pl.gblocks[0].data(),
             sizeof(GenBlock) * pl.gblocks[0].size());
    if (!pl.gblocks[1].empty())
      memcpy(gh.data() + (o_gblk1 - o_gnodes), pl.gblocks[1].data(),
             sizeof(GenBlock) * pl.gblocks[1].size());
    st = upload(ds, base + o_gnodes, gh.data(), gh.size(), stream);
    if (st != COMPASS_OK) return st;
  }

  EstBuffers B;
  memset(&B, 0, sizeof(B));
  B.sides = reinterpret_cast<const void *const *>(base + o_sides);
  B.n_sel = g->n_selected;
  B.sorted = reinterpret_cast<const uint64_t *>(base + o_sorted);
  B.msg = reinterpret_cast<u128 *>(base + o_msg);
  B.merged = reinterpret_cast<uint32_t *>(base + o_merged);
  B.nrec = reinterpret_cast<NodeRec *>(base + o_nrec);
  B.n1tot = reinterpret_cast<u128 *>(base + o_n1tot);
  B.xout = reinterpret_cast<u128 *>(base + o_xout);
  B.prep = reinterpret_cast<TriElem *>(base + o_prep);
  B.prepn = reinterpret_cast<TriElemN *>(base + o_prepn);
  B.prep_z = reinterpret_cast<int32_t *>(base + o_prepz);
  B.tkey = reinterpret_cast<uint32_t *>(base + o_tkey);
  B.tpre = reinterpret_cast<TriPre *>(base + o_tpre);
  B.tseg = reinterpret_cast<int32_t *>(base + o_tseg);
  B.tpiece = reinterpret_cast<TriPiece *>(base + o_tpiece);
  B.tsegp = reinterpret_cast<int32_t *>(base + o_tsegp);
  B.Pcap = pcap;
  B.partial = reinterpret_cast<u128 *>(base + o_part);
  B.counter_bits = g->counter_bits;
  B.d = d;
  B.w = w;
  B.Lmax = std::max(1, pl.Lmax);
  B.Lprep = (int)lp;

  {
    // the row sorts, with every task's guard resolved alongside
    ResolveArgs R;
    memset(&R, 0, sizeof R);
    R.tasks = reinterpret_cast<NodeTask *>(base + o_tasks);
    R.tris = reinterpret_cast<TriTask *>(base + o_tris);
    R.n = (int)flat.size();
    R.n_tri = (int)pl.tris.size();
    ProfScope ps("sort_rows", stream);
    HIP_OK(launch_sort_rows(reinterpret_cast<const SortJob *>(base + o_jobs),
                            (int)sort_jobs.size(), R, B, stream));
  }
  const NodeTask *dtasks = reinterpret_cast<const NodeTask *>(base + o_tasks);
  for (size_t lv = 0; lv < levels.size(); ++lv) {
    if (levels[lv].empty()) continue;
    // LDS for the staged merge: the level's widest node, if it fits
    int stage = 0;
    if (g->counter_bits == 32) {
      for (const NodeTask &t : levels[lv]) {
        if (t.m < 2) continue;  // only multi-child nodes are merged
        const int nl = t.m + (t.parent_side >= 0) + (t.cut_side >= 0);
        const int need = nl * w * 4;
        if (need <= kNodeStageBytes) stage = std::max(stage, need);
      }
    }
    ProfScope ps("node", stream);
    for (size_t g0 = 0; g0 < levels[lv].size(); g0 += group_tasks) {
      const size_t ng = std::min(group_tasks, levels[lv].size() - g0);
      int n_kind[3] = {0, 0, 0};
      int apex_L = 0, merge_L = 0;
      for (size_t k = g0; k < g0 + ng; ++k) {
        const NodeTask &t = levels[lv][k];
        const int nl = t.m + (t.parent_side >= 0) + (t.cut_side >= 0);
        ++n_kind[kind(t)];
        if (t.m >= 2) merge_L = std::max(merge_L, nl * w);
        if (t.mode == kModeTriRootPrep) apex_L = std::max(apex_L, t.m * w);
      }
      const NodeTask *dt = dtasks + level_off[lv] + g0;
      const NodeTask *d1 = dt + n_kind[0], *d2 = d1 + n_kind[1];
      if (n_kind[1] + n_kind[2] > 0)
        HIP_OK(launch_node_merge(d1, n_kind[1] + n_kind[2], merge_L, B, stage,
                                 stream));
      if (n_kind[1] > 0) HIP_OK(launch_node(d1, n_kind[1], B, stream));
      if (n_kind[0] > 0) HIP_OK(launch_node1(dt, n_kind[0], B, stream));
      if (n_kind[2] > 0)
        HIP_OK(launch_apex_prep(d2, n_kind[2], apex_L, B, stream));
    }
  }
  if (!pl.tris.empty()) {
    ProfScope ps("tri_order", stream);
    HIP_OK(launch_tri_order(reinterpret_cast<const TriTask *>(base + o_tris),
                            (int)pl.tris.size(), B, stream));
  }
  if (!pl.tris.empty()) {
    ProfScope ps("tri_lane", stream);
    HIP_OK(launch_tri_lane(reinterpret_cast<const TriTask *>(base + o_tris),
                           (int)pl.tris.size(),
                           reinterpret_cast<const TriGroup *>(base + o_tgroups),
                           (int)tgroups.size(),
                           (w + kLaneThreads - 1) / kLaneThreads, B, stream));
  }
  if (!pl.gplans.empty()) {
    GenArgs A;
    memset(&A, 0, sizeof A);
    A.nodes = reinterpret_cast<const GenNode *>(base + o_gnodes);
    A.plans = reinterpret_cast<const GenPlan *>(base + o_gplans);
    A.lists = reinterpret_cast<uint32_t *>(base + o_glists);
    A.msg = base + o_gmsg;
    A.partial = B.partial;
    A.approx = reinterpret_cast<double *>(base + o_approx);
    A.sps = reinterpret_cast<const SubplanTask *>(base + o_sps);
    A.n_tables = g->n_tables;
    ProfScope ps("generic", stream);
    A.blocks = reinterpret_cast<const GenBlock *>(base + o_gblk0);
    HIP_OK(launch_gen_contract(A, B, (int)pl.gblocks[0].size(), 0, stream));
    A.blocks = reinterpret_cast<const GenBlock *>(base + o_gblk1);
    HIP_OK(launch_gen_contract(A, B, (int)pl.gblocks[1].size(), 1, stream));
  }
  {
    ProfScope ps("finish", stream);
    HIP_OK(launch_finish(reinterpret_cast<const SubplanTask *>(base + o_sps),
                         (int)pl.sps.size(), B,
                         reinterpret_cast<const double *>(base + o_approx),
                         reinterpret_cast<uint64_t *>(row_est), est, flags,
                         g->n_tables, stream));
  }
  return COMPASS_OK;
}

// ---------------------------------------------------------------------
// sketch partitioning (Section 5.1)
// ---------------------------------------------------------------------
// Tiles of the binned two-dimensional build: R = 2^r rows of one sketch
// row's matrix, R * w2 int32 counters.  R grows to fill a 64 KiB tile (no
// further than w1 needs), then, while there are more than kBinMaxBins tiles,
// up to kBinTileWords counters.  -1: no tiling fits (the atomic scan is
// used).
static int bin2d_shift(int d, int w1, int w2) {
  if (w2 > kBinTileWords) return -1;
  int rs = 0;
  while (((int64_t)w2 << (rs + 1)) <= kBinTileWords / 2 && (1 << rs) < w1) ++rs;
  auto bins = [&](int r) { return (int64_t)d * ((w1 + (1 << r) - 1) >> r); };
  while (bins(rs) > kBinMaxBins && ((int64_t)w2 << (rs + 1)) <= kBinTileWords)
    ++rs;
  if (bins(rs) > kBinMaxBins) return -1;
  return rs;
}

// The binned build in batches of rows whose records (4 bytes per selected
// row and sketch row) fit the record budget (1 GiB, or
// COMPASS_2D_RECORD_BYTES); every batch after the first adds to the
// counters.
static compass_status sketch_build_2d_binned(const BuildParams &P,
                                             const KdDims &kx,
                                             DeviceState *ds, int64_t n_rows,
                                             int d, int w1, int w2, int r_shift,
                                             int accumulate, hipStream_t stream) {
  int64_t budget = (int64_t)1 << 30;
  if (const char *e = getenv("COMPASS_2D_RECORD_BYTES")) {
    const long long v = atoll(e);
    if (v > 0) budget = v;
  }
  const int64_t batch = std::max<int64_t>(
      kBuildTile, budget / (4 * (int64_t)d) / kBuildTile * kBuildTile);
  Bin2dArgs a;
  memset(&a, 0, sizeof(a));
  a.d = d;
  a.w1 = w1;
  a.w2 = w2;
  a.r_shift = r_shift;
  a.nbr = (w1 + (1 << r_shift) - 1) >> r_shift;
  a.n_bins = d * a.nbr;
  // blocks of the scan: two per CU when their LDS (histogram + row queue)
  // allows it
  const size_t scan_lds = (size_t)((a.n_bins + 3) & ~3) * 4 + (size_t)kBuildTile * 4;
  const int64_t per_cu = scan_lds <= 80 * 1024 ? 2 : 1;
  const int64_t rows_max = std::min<int64_t>(n_rows, batch);
  const int64_t tiles_max = (rows_max + kBuildTile - 1) / kBuildTile;
  const int64_t blocks_max = std::min<int64_t>(tiles_max, per_cu * ds->n_cu);
  const int64_t rpb_max = (tiles_max + blocks_max - 1) / blocks_max * kBuildTile;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_rec = al((size_t)blocks_max * rpb_max * d * 4);
  const size_t b_cnt = al((size_t)blocks_max * 4);
  const size_t b_hist = al((size_t)blocks_max * a.n_bins * 4);
  const size_t b_tot = al((size_t)a.n_bins * 4);
  const size_t b_start = al((size_t)(a.n_bins + 1) * 4);
  const size_t b_sorted = al((size_t)rows_max * d * 2);
  void *scr;
  compass_status st = ensure_scratch(
      ds, stream, b_rec + b_cnt + b_hist + b_tot + b_start + b_sorted, &scr);
  if (st != COMPASS_OK) return st;
  char *c = reinterpret_cast<char *>(scr);
  a.rec = reinterpret_cast<uint32_t *>(c); c += b_rec;
  a.rec_count = reinterpret_cast<int32_t *>(c); c += b_cnt;
  a.hist = reinterpret_cast<int32_t *>(c); c += b_hist;
  a.bin_total = reinterpret_cast<int32_t *>(c); c += b_tot;
  a.bin_start = reinterpret_cast<int32_t *>(c); c += b_start;
  a.sorted = reinterpret_cast<uint16_t *>(c);
  if (!accumulate) {
    ProfScope ps("fill_zero", stream);
    HIP_OK(launch_fill_zero(P.n_selected, 8, stream));
  }
  for (int64_t b0 = 0; b0 < n_rows; b0 += batch) {
    const int64_t b1 = std::min(n_rows, b0 + batch);
    const int64_t tiles = (b1 - b0 + kBuildTile - 1) / kBuildTile;
    const int64_t blocks = std::min<int64_t>(tiles, per_cu * ds->n_cu);
    a.rows_per_block = (tiles + blocks - 1) / blocks * kBuildTile;
    a.n_blocks = (int32_t)((b1 - b0 + a.rows_per_block - 1) / a.rows_per_block);
    a.row0 = b0;
    a.row1 = b1;
    ProfScope ps("scan2d", stream);
    HIP_OK(launch_scan2d_binned(P, a, kx, (accumulate || b0 > 0) ? 1 : 0,
                                stream));
  }
  return COMPASS_OK;
}

// Partitioned sketch of k = 2 .. 4 joins: the second dimension of the
// binned (or atomic) two-dimensional build is the flattened index of joins
// 2 .. k.
static compass_status sketch_build_kd_impl(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *const *spec, int32_t k, int32_t d,
    const int32_t *w, int32_t counter_bits, int32_t accumulate, void *counters,
    int64_t *n_selected, hipStream_t stream) {
  if (n_rows < 0 || n_rows >= (1ll << 47))
    return fail(COMPASS_E_RANGE, "n_rows %lld outside [0, 2^47)",
                (long long)n_rows);
  if (k < 2 || k > 4) return fail(COMPASS_E_ARG, "k=%d outside [2, 4]", k);
  if (d < 1 || d > kMaxLaunchSlices / k)
    return fail(COMPASS_E_ARG, "d=%d outside [1, %d] for %d joins", d,
                kMaxLaunchSlices / k, k);
  int64_t total = 1;
  for (int m = 0; m < k; ++m) {
    if (w[m] < 1 || w[m] > (1 << 20))
      return fail(COMPASS_E_ARG, "w%d=%d outside [1, 2^20]", m + 1, w[m]);
    total *= w[m];
    if (total > ((int64_t)1 << 28))
      return fail(COMPASS_E_ARG, "the widths' product exceeds 2^28");
  }
  if (counter_bits != 32 && counter_bits != 64)
    return fail(COMPASS_E_ARG, "counter_bits must be 32 or 64");
  if (counter_bits == 32 && n_rows > 0x7FFFFFFFll)
    return fail(COMPASS_E_RANGE, "int32 counters need n_rows < 2^31");
  if (n_preds < 0 || n_preds > kMaxPreds)
    return fail(COMPASS_E_ARG, "n_preds=%d outside [0, %d]", n_preds,
                kMaxPreds);
  if (!counters || !n_selected || (n_preds > 0 && !preds))
    return fail(COMPASS_E_ARG, "null pointer argument");
  if (n_preds > 0 && n_rows > 0 && !pred_cols)
    return fail(COMPASS_E_ARG, "null predicate column array");
  BuildParams P;
  memset(&P, 0, sizeof(P));
  P.n_rows = n_rows;
  P.n_preds = n_preds;
  P.counter_bits = counter_bits;
  P.n_selected = n_selected;
  P.count_selected = 1;
  P.d = d;
  P.bm1 = make_bucket_mod((uint32_t)w[0]);
  P.bm = make_bucket_mod((uint32_t)w[1]);
  KdDims kx;
  memset(&kx, 0, sizeof kx);
  kx.kd = k;
  kx.w3 = k > 2 ? w[2] : 1;
  kx.w4 = k > 3 ? w[3] : 1;
  kx.bm3 = make_bucket_mod((uint32_t)kx.w3);
  kx.bm4 = make_bucket_mod((uint32_t)kx.w4);
  compass_status st = fill_preds(P, n_rows, pred_cols, n_pred_cols, preds, n_preds);
  if (st != COMPASS_OK) return st;
  for (int s = 0; s < k; ++s) {
    if (!spec[s]) return fail(COMPASS_E_ARG, "key %d: null pointer", s);
    const compass_sketch_spec &ks = *spec[s];
    if (!ks.seeds || (n_rows > 0 && !ks.key_col))
      return fail(COMPASS_E_ARG, "key %d: null pointer", s);
    if (ks.key_dtype != COMPASS_I32 && ks.key_dtype != COMPASS_I64)
      return fail(COMPASS_E_ARG, "key %d: dtype must be I32 or I64", s);
    for (int i = 0; i < 6 * d; ++i)
      if (ks.seeds[i] >= kP61)
        return fail(COMPASS_E_ARG, "key %d: seed %d is not below 2^61-1", s, i);
    P.keys[s].col = ks.key_col;
    P.keys[s].dtype = ks.key_dtype;
    for (int i = 0; i < d; ++i) {
      const uint64_t *q = ks.seeds + 6 * i;
      P.seeds[s * d + i] = RowSeeds{q[0], q[1], q[2], q[3], q[4], q[5]};
    }
  }
  P.counters[0] = counters;
  DeviceState *ds;
  st = device_state(&ds);
  if (st != COMPASS_OK) return st;
  const int w1 = w[0];
  const int64_t wrest = total / w1;
  const int r_shift = wrest <= kBinTileWords ? bin2d_shift(d, w1, (int)wrest) : -1;
  if (r_shift >= 0 && n_rows > 0)
    return sketch_build_2d_binned(P, kx, ds, n_rows, d, w1, (int)wrest, r_shift,
                                  accumulate, stream);
  if (!accumulate) {
    ProfScope ps("fill_zero", stream);
    HIP_OK(launch_fill_zero(counters, (int64_t)d * total * (counter_bits / 8),
                            stream));
    HIP_OK(launch_fill_zero(n_selected, 8, stream));
  }
  if (n_rows == 0) return COMPASS_OK;
  const int64_t tiles = (n_rows + kBuildTile - 1) / kBuildTile;
  ProfScope ps("scan2d", stream);
  HIP_OK(launch_scan2d(P, kx, (int)std::min<int64_t>(tiles, 4ll * ds->n_cu),
                       stream));
  return COMPASS_OK;
}

extern "C" compass_status compass_sketch_build_2d(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *first, const compass_sketch_spec *second,
    int32_t d, int32_t w1, int32_t w2, int32_t counter_bits,
    int32_t accumulate, void *counters, int64_t *n_selected,
    hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  const compass_sketch_spec *spec[2] = {first, second};
  const int32_t w[2] = {w1, w2};
  return sketch_build_kd_impl(n_rows, pred_cols, n_pred_cols, preds, n_preds,
                              spec, 2, d, w, counter_bits, accumulate,
                              counters, n_selected, stream);
}

extern "C" compass_status compass_sketch_build_kd(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *joins, int32_t k, int32_t d, const int32_t *w,
    int32_t counter_bits, int32_t accumulate, void *counters,
    int64_t *n_selected, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  if (!joins || !w) return fail(COMPASS_E_ARG, "null pointer argument");
  if (k < 2 || k > 4) return fail(COMPASS_E_ARG, "k=%d outside [2, 4]", k);
  const compass_sketch_spec *spec[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int m = 0; m < k; ++m) spec[m] = joins + m;
  return sketch_build_kd_impl(n_rows, pred_cols, n_pred_cols, preds, n_preds,
                              spec, k, d, w, counter_bits, accumulate,
                              counters, n_selected, stream);
}

extern "C" compass_status compass_estimate_chain3(
    const void *a, const void *p, const void *b, int32_t counter_bits,
    int32_t d, int32_t w1, int32_t w2, const int64_t *n_a, const int64_t *n_p,
    const int64_t *n_b, compass_i128 *row_est, double *est, int32_t *flags,
    hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  if (!a || !p || !b || !n_a || !n_p || !n_b || !est || !flags)
    return fail(COMPASS_E_ARG, "null pointer argument");
  if (d < 1 || d > 32) return fail(COMPASS_E_ARG, "d=%d outside [1, 32]", d);
  if (w1 < 1 || w2 < 1 || w1 > (1 << 20) || w2 > 16384 ||
      (int64_t)w1 * w2 > ((int64_t)1 << 28))
    return fail(COMPASS_E_ARG, "w1=%d in [1, 2^20], w2=%d in [1, 16384], "
                "product at most 2^28", w1, w2);
  if (counter_bits != 32 && counter_bits != 64)
    return fail(COMPASS_E_ARG, "counter_bits must be 32 or 64");
  DeviceState *ds;
  compass_status st = device_state(&ds);
  if (st != COMPASS_OK) return st;
  const int nblk = (w1 + kChainRows - 1) / kChainRows;
  void *scr;
  st = ensure_scratch(ds, stream, (size_t)d * nblk * 16, &scr);
  if (st != COMPASS_OK) return st;
  ChainArgs c;
  c.A = a;
  c.P = p;
  c.B = b;
  c.n_a = n_a;
  c.n_p = n_p;
  c.n_b = n_b;
  c.partial = reinterpret_cast<u128 *>(scr);
  c.counter_bits = counter_bits;
  c.d = d;
  c.w1 = w1;
  c.w2 = w2;
  ProfScope ps("chain3", stream);
  HIP_OK(launch_chain3(c, reinterpret_cast<uint64_t *>(row_est), est, flags,
                       stream));
  return COMPASS_OK;
}

extern "C" compass_status compass_estimate_partitioned(
    const compass_tensor_graph *g, compass_i128 *row_est, double *est,
    int32_t *flags, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  if (!g || !est || !flags) return fail(COMPASS_E_ARG, "null pointer argument");
  const int nt = g->n_tables, ne = g->n_edges, d = g->d;
  if (nt < 2 || nt > 64)
    return fail(COMPASS_E_RANGE, "n_tables=%d outside [2, 64]", nt);
  if (ne != nt - 1)
    return fail(COMPASS_E_GRAPH, "%d edges for %d tables: not a tree", ne, nt);
  if (d < 1 || d > 32) return fail(COMPASS_E_ARG, "d=%d outside [1, 32]", d);
  if (g->counter_bits != 32 && g->counter_bits != 64)
    return fail(COMPASS_E_ARG, "counter_bits must be 32 or 64");
  if (!g->edge_u || !g->edge_v || !g->width || !g->tensor || !g->n_selected)
    return fail(COMPASS_E_ARG, "null graph array");
  std::vector<std::vector<int>> inc(nt);
  for (int e = 0; e < ne; ++e) {
    const int u = g->edge_u[e], v = g->edge_v[e];
    if (u < 0 || u >= nt || v < 0 || v >= nt || u == v)
      return fail(COMPASS_E_GRAPH, "edge %d has bad endpoints", e);
    if (g->width[e] < 1 || g->width[e] > (1 << 20))
      return fail(COMPASS_E_ARG, "edge %d: width %d outside [1, 2^20]", e,
                  g->width[e]);
    inc[u].push_back(e);
    inc[v].push_back(e);
  }
  for (int t = 0; t < nt; ++t) {
    if (!g->tensor[t]) return fail(COMPASS_E_ARG, "table %d: null tensor", t);
    if ((int)inc[t].size() > kTensorMaxDims)
      return fail(COMPASS_E_UNSUPPORTED, "table %d has %d joins (at most %d)",
                  t, (int)inc[t].size(), kTensorMaxDims);
  }
  // rooted at table 0: parents, depths (a tree: every table reached once)
  std::vector<int> parent(nt, -2), pedge(nt, -1), depth(nt, 0), order{0};
  parent[0] = -1;
  for (size_t h = 0; h < order.size(); ++h) {
    const int t = order[h];
    for (int e : inc[t]) {
      const int o = g->edge_u[e] == t ? g->edge_v[e] : g->edge_u[e];
      if (parent[o] != -2) continue;
      parent[o] = t;
      pedge[o] = e;
      depth[o] = depth[t] + 1;
      order.push_back(o);
    }
  }
  if ((int)order.size() != nt)
    return fail(COMPASS_E_GRAPH, "the join graph is not connected");
  // tasks: every table but the leaves (their messages are their counters)
  std::vector<int> slot(nt, -1);
  int n_slots = 0, w_max = 1, max_depth = 0;
  for (int e = 0; e < ne; ++e) w_max = std::max(w_max, (int)g->width[e]);
  for (int t = 1; t < nt; ++t)
    if (inc[t].size() > 1) slot[t] = n_slots++;
  std::vector<std::vector<TensorTask>> levels;
  for (int t = 0; t < nt; ++t) max_depth = std::max(max_depth, depth[t]);
  levels.resize(max_depth + 1);
  int root_chunks = 1;
  for (int t = 0; t < nt; ++t) {
    if (t != 0 && inc[t].size() == 1) continue;  // leaf
    std::vector<int> dims = inc[t];
    std::sort(dims.begin(), dims.end());
    TensorTask T;
    memset(&T, 0, sizeof T);
    T.tensor = g->tensor[t];
    T.n_dims = (int)dims.size();
    T.parent_dim = -1;
    int64_t size = 1;
    for (int k = T.n_dims - 1; k >= 0; --k) {
      T.width[k] = g->width[dims[k]];
      T.stride[k] = size;
      size *= T.width[k];
      if (size > ((int64_t)1 << 28))
        return fail(COMPASS_E_ARG, "table %d: tensor of more than 2^28 "
                    "entries per row", t);
    }
    T.size = size;
    for (int k = 0; k < T.n_dims; ++k) {
      const int e = dims[k];
      if (e == pedge[t]) {
        T.parent_dim = k;
        continue;
      }
      const int c = g->edge_u[e] == t ? g->edge_v[e] : g->edge_u[e];
      if (inc[c].size() == 1) {
        T.child_msg[k] = -1 - c;
        T.leaf[k] = g->tensor[c];
      } else {
        T.child_msg[k] = slot[c];
      }
    }
    T.out_slot = slot[t];
    if (t == 0) {
      T.n_chunks = (int)((size + kTensorChunk - 1) / kTensorChunk);
      root_chunks = T.n_chunks;
    }
    levels[depth[t]].push_back(T);
  }
  DeviceState *ds;
  compass_status st = device_state(&ds);
  if (st != COMPASS_OK) return st;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t o_tasks = carve(sizeof(TensorTask) * nt);
  const size_t o_msg = carve(16ull * std::max(1, n_slots) * d * w_max);
  const size_t o_part = carve(16ull * d * root_chunks);
  void *scratch;
  st = ensure_scratch(ds, stream, off, &scratch);
  if (st != COMPASS_OK) return st;
  char *base = reinterpret_cast<char *>(scratch);
  std::vector<TensorTask> flat;
  std::vector<std::pair<size_t, size_t>> range;  // per level: [first, count)
  for (int lv = max_depth; lv >= 0; --lv) {
    range.push_back({flat.size(), levels[lv].size()});
    flat.insert(flat.end(), levels[lv].begin(), levels[lv].end());
  }
  st = upload(ds, base + o_tasks, flat.data(), sizeof(TensorTask) * flat.size(),
              stream);
  if (st != COMPASS_OK) return st;
  TensorArgs A;
  memset(&A, 0, sizeof A);
  A.msg = reinterpret_cast<u128 *>(base + o_msg);
  A.partial = reinterpret_cast<u128 *>(base + o_part);
  A.counter_bits = g->counter_bits;
  A.d = d;
  A.w_max = w_max;
  ProfScope ps("tensor_tree", stream);
  for (auto &r : range) {
    if (r.second == 0) continue;
    int per_row = 1;
    for (size_t k = r.first; k < r.first + r.second; ++k) {
      const TensorTask &T = flat[k];
      per_row = std::max(per_row, T.parent_dim < 0 ? T.n_chunks
                                                   : T.width[T.parent_dim]);
    }
    A.tasks = reinterpret_cast<const TensorTask *>(base + o_tasks) + r.first;
    HIP_OK(launch_tensor_level(A, (int)r.second, d * per_row, stream));
  }
  HIP_OK(launch_tensor_finish(A.partial, root_chunks, d, g->n_selected, nt,
                              reinterpret_cast<uint64_t *>(row_est), est, flags,
                              stream));
  return COMPASS_OK;
}

// ---------------------------------------------------------------------
// AGMS baseline (Section 4.1)
// ---------------------------------------------------------------------
extern "C" compass_status compass_agms_build(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *joins, int32_t n_joins, int32_t r, int32_t b,
    int32_t accumulate, int64_t *counters, int64_t *n_selected,
    hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  if (n_rows < 0 || n_rows >= (1ll << 47))
    return fail(COMPASS_E_RANGE, "n_rows %lld outside [0, 2^47)",
                (long long)n_rows);
  if (n_joins < 1 || n_joins > kAgmsMaxJoins)
    return fail(COMPASS_E_ARG, "n_joins=%d outside [1, %d]", n_joins,
                kAgmsMaxJoins);
  if (r < 1 || r > 64 || b < 1 || r * b > kAgmsMaxCounters)
    return fail(COMPASS_E_ARG, "r=%d in [1, 64], b=%d, r*b at most %d", r, b,
                kAgmsMaxCounters);
  if (n_preds < 0 || n_preds > kMaxPreds)
    return fail(COMPASS_E_ARG, "n_preds=%d outside [0, %d]", n_preds,
                kMaxPreds);
  if (!joins || !counters || !n_selected || (n_preds > 0 && !preds))
    return fail(COMPASS_E_ARG, "null pointer argument");
  if (n_preds > 0 && n_rows > 0 && !pred_cols)
    return fail(COMPASS_E_ARG, "null predicate column array");
  BuildParams bp;
  memset(&bp, 0, sizeof(bp));
  compass_status st = fill_preds(bp, n_rows, pred_cols, n_pred_cols, preds, n_preds);
  if (st != COMPASS_OK) return st;
  const int K = r * b;
  AgmsParams P;
  memset(&P, 0, sizeof(P));
  P.n_rows = n_rows;
  P.n_preds = n_preds;
  P.n_joins = n_joins;
  P.K = K;
  P.count_selected = 1;
  P.n_selected = n_selected;
  P.counters = counters;
  memcpy(P.preds, bp.preds, sizeof(P.preds));
  std::vector<RowSeeds> sd((size_t)n_joins * K);
  for (int e = 0; e < n_joins; ++e) {
    const compass_sketch_spec &k = joins[e];
    if (!k.seeds || (n_rows > 0 && !k.key_col))
      return fail(COMPASS_E_ARG, "join %d: null pointer", e);
    if (k.key_dtype != COMPASS_I32 && k.key_dtype != COMPASS_I64)
      return fail(COMPASS_E_ARG, "join %d: key dtype must be I32 or I64", e);
    for (int c = 0; c < K; ++c) {
      const uint64_t *q = k.seeds + 6 * (size_t)c;
      for (int z = 0; z < 4; ++z)
        if (q[z] >= kP61)
          return fail(COMPASS_E_ARG, "join %d: seed of basic sketch %d is not "
                      "below 2^61-1", e, c);
      sd[(size_t)e * K + c] = RowSeeds{q[0], q[1], q[2], q[3], 0, 0};
    }
    P.keys[e].col = k.key_col;
    P.keys[e].dtype = k.key_dtype;
  }
  DeviceState *ds;
  st = device_state(&ds);
  if (st != COMPASS_OK) return st;
  void *scr;
  const size_t bytes = sizeof(RowSeeds) * sd.size();
  st = ensure_scratch(ds, stream, bytes, &scr);
  if (st != COMPASS_OK) return st;
  st = upload(ds, scr, sd.data(), bytes, stream);
  if (st != COMPASS_OK) return st;
  P.seeds = reinterpret_cast<const RowSeeds *>(scr);
  if (!accumulate) {
    ProfScope ps("fill_zero", stream);
    HIP_OK(launch_fill_zero(counters, (int64_t)K * 8, stream));
    HIP_OK(launch_fill_zero(n_selected, 8, stream));
  }
  if (n_rows == 0) return COMPASS_OK;
  const int64_t tiles = (n_rows + kBuildTile - 1) / kBuildTile;
  const int64_t blocks = std::min<int64_t>(tiles, 4ll * ds->n_cu);
  P.rows_per_chunk = (tiles + blocks - 1) / blocks * kBuildTile;
  const int64_t chunks = (n_rows + P.rows_per_chunk - 1) / P.rows_per_chunk;
  ProfScope ps("agms_build", stream);
  HIP_OK(launch_agms_build(P, (int)chunks, stream));
  return COMPASS_OK;
}

extern "C" compass_status compass_agms_estimate(
    const int64_t *const *sketches, const int64_t *const *n_selected,
    int32_t n_tables, int32_t r, int32_t b, compass_i128 *row_sums,
    double *est, int32_t *flag, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err.clear();
  if (n_tables < 1 || n_tables > 16)
    return fail(COMPASS_E_ARG, "n_tables=%d outside [1, 16]", n_tables);
  if (r < 1 || r > 64 || b < 1 || r * b > kAgmsMaxCounters)
    return fail(COMPASS_E_ARG, "r=%d in [1, 64], b=%d, r*b at most %d", r, b,
                kAgmsMaxCounters);
  if (!sketches || !n_selected || !est || !flag)
    return fail(COMPASS_E_ARG, "null pointer argument");
  AgmsEstArgs a;
  memset(&a, 0, sizeof(a));
  for (int t = 0; t < n_tables; ++t) {
    if (!sketches[t] || !n_selected[t])
      return fail(COMPASS_E_ARG, "table %d: null pointer", t);
    a.sk[t] = sketches[t];
    a.n_sel[t] = n_selected[t];
  }
  a.n_tables = n_tables;
  a.r = r;
  a.b = b;
  DeviceState *ds;
  compass_status st = device_state(&ds);
  if (st != COMPASS_OK) return st;
  ProfScope ps("agms_estimate", stream);
  HIP_OK(launch_agms_estimate(a, reinterpret_cast<uint64_t *>(row_sums), est,
                              flag, stream));
  return COMPASS_OK;
}

extern "C" compass_status compass_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) return COMPASS_OK;
  DeviceState &ds = it->second;
  HIP_OK(hipDeviceSynchronize());
  for (auto &kv : ds.scratch)
    if (kv.second.p) HIP_OK(hipFree(kv.second.p));
  ds.scratch.clear();

  for (int k = 0; k < DeviceState::kRing; ++k) {
    if (ds.pinned[k]) HIP_OK(hipHostFree(ds.pinned[k]));
    ds.pinned[k] = nullptr;
    ds.pinned_bytes[k] = 0;
    ds.pinned_used[k] = false;
  }
  return COMPASS_OK;
}

extern "C" const char *compass_last_error(void) { return g_err.c_str(); }

extern "C" const char *compass_version(void) { return "compass-gfx950 0.1.0"; }
