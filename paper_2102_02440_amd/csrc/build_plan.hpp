// build_plan.hpp -- host-side work decomposition of the sketch builds.
//
// Plain integer arithmetic with no HIP dependency, so the host tests can
// compile and check it on a machine without a GPU.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

namespace compass {

// Rows of one chunk of the fused scan.  A workgroup adds at most one +-1
// per row of its chunk to an int32 LDS partial and writes that partial to
// an int32 slab, so a chunk never exceeds INT32_MAX rows (rounded down to
// whole tiles); the chunk count grows instead.  Returns rows per chunk
// (a multiple of `tile`, >= tile) for the wanted number of chunks.
inline int64_t fused_rows_per_chunk(int64_t n_rows, int64_t chunks, int64_t tile) {
  if (chunks < 1) chunks = 1;
  int64_t r = (n_rows + chunks - 1) / chunks;
  r = (r + tile - 1) / tile * tile;
  const int64_t most = (int64_t)INT32_MAX / tile * tile;
  if (r > most) r = most;
  if (r < tile) r = tile;
  return r;
}

// Whether a kernel's LDS (static + dynamic) fits what one workgroup may
// allocate on the device.
inline bool lds_fits(size_t dynamic_bytes, size_t static_bytes, size_t limit) {
  return dynamic_bytes + static_bytes <= limit;
}

// Plan of the two-phase build (survivor compaction, then hashing of the
// buffered survivors into LDS counters, then a slab reduction).
//
// Rows are compacted in batches of `batch` rows; the buffer holds `cap`
// survivors per sketch.  After a batch the buffer is flushed (hashed and
// reduced into the counters, then emptied) only if the next batch might not
// fit, so selective scans hash once per build.  cap >= 2 * batch unless one
// batch covers the whole table.
struct TwoPhasePlan {
  int64_t cap = 0;        // survivors per sketch the buffer holds
  int64_t batch = 0;      // rows per compaction launch
  int32_t chunks = 1;     // survivor chunks per slice in one flush
  int32_t ranges = 1;     // bucket ranges of at most 65536 per slice
  size_t seeds_bytes = 0, ctl_bytes = 0, surv_bytes = 0, slab_bytes = 0;
  size_t total_bytes = 0; // seeds | count, ticket | survivors | slab
  bool ok = false;
};

inline size_t plan_align(size_t x) { return (x + 255) & ~(size_t)255; }

// n_cu: compute units (one hashing workgroup per CU: 128 KiB of LDS);
// budget: bytes of scratch the plan may use; cap_rows_max: an upper bound
// on the buffer's survivors (0 = none).  The survivor chunk count is picked
// so that the workgroups of a flush fill whole waves of the CUs as far as
// the slab (chunks x slices x w int32) stays within a quarter of the budget.
inline TwoPhasePlan plan_two_phase(int64_t n_rows, int n_sketches, int d,
                                   int w, int n_cu, size_t budget,
                                   int64_t cap_rows_max, int64_t tile,
                                   int seed_bytes_per_slice) {
  TwoPhasePlan p;
  const int S = n_sketches * d;
  p.ranges = (w + 65535) / 65536;
  const size_t slab_row = (size_t)S * w * 4;
  p.seeds_bytes = plan_align((size_t)S * seed_bytes_per_slice);
  p.ctl_bytes = 256;
  const int items1 = S * p.ranges;
  int best_c = 1;
  double best_eff = 0.0;
  const int c_max = std::max(1, 4 * n_cu / std::max(1, items1));
  for (int c = 1; c <= c_max; ++c) {
    if ((size_t)c * slab_row > budget / 4 && c > 1) break;
    const int64_t items = (int64_t)items1 * c;
    const int64_t waves = (items + n_cu - 1) / n_cu;
    const double eff = (double)items / (double)(waves * n_cu);
    // more chunks only for a clearly better fill (each costs a slab row)
    if (eff > best_eff + 0.02) {
      best_eff = eff;
      best_c = c;
    }
  }
  p.chunks = best_c;
  p.slab_bytes = plan_align((size_t)p.chunks * slab_row);
  const size_t fixed = p.seeds_bytes + p.ctl_bytes + p.slab_bytes;
  if (fixed >= budget) return p;
  const int64_t worst = (n_rows + tile - 1) / tile * tile;
  int64_t cap = (int64_t)((budget - fixed) / (8 * (size_t)n_sketches)) / tile * tile;
  if (cap_rows_max > 0) cap = std::min(cap, std::max(tile, cap_rows_max / tile * tile));
  if (cap >= worst) {
    p.cap = std::max<int64_t>(worst, tile);
    p.batch = p.cap;
  } else {
    p.cap = cap;
    p.batch = cap / 2 / tile * tile;
    if (p.batch < tile) return p;  // too small for one tile per batch
  }
  p.surv_bytes = plan_align((size_t)p.cap * 8 * n_sketches);
  p.total_bytes = fixed + p.surv_bytes;
  p.ok = p.total_bytes <= budget;
  return p;
}

}  // namespace compass
