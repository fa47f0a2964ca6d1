// build_params.hpp -- kernel-argument layout of the fused scan + sketch build.
#pragma once
#include <stdint.h>

#include "device_math.hpp"

namespace compass {

constexpr int kBuildThreads = 1024;
constexpr int kXcds = 8;  // MI355X: accelerator complex dies, one L2 each
constexpr int kBuildRowsPerThread = 4;
constexpr int kBuildTile = kBuildThreads * kBuildRowsPerThread;
// the one-table fused scan (tables without predicates) takes longer tiles:
// twice the independent hash chains per lane
constexpr int kScanRowsPerThread = 8;
constexpr int kScanTile = kBuildThreads * kScanRowsPerThread;
constexpr int kMaxPreds = 8;
constexpr int kMaxSketches = 16;
constexpr int kMaxLaunchSlices = 48;   // slices whose seeds ride in kernargs
constexpr int kMaxLaunchGroups = 16;
constexpr size_t kLdsBudget = 128 * 1024;  // partial counters per workgroup

enum { kDtI32 = 0, kDtF32 = 1, kDtI64 = 2 };
enum { kPredPoint = 0, kPredRange = 1, kPredSubset = 2 };

union Scalar32 {
  int32_t i;
  float f;
};

struct PredDev {
  const void *col;
  const uint64_t *bitmap;
  int64_t domain;
  int32_t kind;
  int32_t dtype;
  Scalar32 lo, hi;
};

// Optional materialisation of the selection output (the qualifying row
// indices) next to the sketches: rows go to out[count ...] while below cap.
struct RowSink {
  int64_t *out;                  // nullptr: not materialised
  int64_t cap;
  unsigned long long *count;     // device: rows seen so far (all calls)
  int64_t row_base;              // added to every row index
};

struct KeyDev {
  const void *col;
  int32_t dtype;
  int32_t pad;
};

// One launch covers n_groups slice groups; group g owns launch-local
// slices [group_begin[g], group_begin[g+1]).
// regions zeroed by one launch (word counts: 4-byte words)
constexpr int kMaxZeroSpans = kMaxSketches + 3;
struct ZeroSpans {
  void *p[kMaxZeroSpans];
  int64_t words[kMaxZeroSpans];
  int32_t n;
  int32_t pad;
  void add(void *q, int64_t bytes) {
    p[n] = q;
    words[n] = bytes / 4;
    ++n;
  }
};

struct BuildParams {
  int64_t n_rows;
  int64_t rows_per_chunk;
  int32_t n_preds;
  int32_t n_groups;
  int32_t counter_bits;
  int32_t count_selected;
  int64_t *n_selected;
  int32_t *slab;        // [chunk][sketch * d + row][w] partial counters
  int32_t d;
  int32_t n_slices_total;  // n_sketches * d of the call (slab row count)
  int32_t n_blocks;     // (chunk, slice group) pairs of a fused-scan launch
  int32_t pad_nb;
  BucketMod bm;
  BucketMod bm1;        // first dimension of a partitioned sketch (w1)
  PredDev preds[kMaxPreds];
  KeyDev keys[kMaxSketches];
  void *counters[kMaxSketches];
  int32_t slice_base;   // launch-local slice l is the call's slice
                        // slice_base + l = sketch * d + row
  int32_t group_begin[kMaxLaunchGroups + 1];  // 32-bit: scalar loads
  RowSeeds seeds[kMaxLaunchSlices];
  RowSink sink;         // written by the workgroups of slice group 0 only
};

static_assert(sizeof(BuildParams) <= 4096, "kernel arguments must stay small");

// Survivor buffer of the two-phase build and when to empty it: the hashing
// and the slab reduction after a batch run only when `force` is set or
// count + need > cap (the next batch of `need` rows might not fit); the
// reduction's last workgroup then sets count (and ticket) back to 0.
struct FlushCtl {
  unsigned long long *count;   // survivors in the buffer (device)
  unsigned int *ticket;        // workgroups of the reduction done (device)
  int64_t cap;                 // survivors the buffer holds per sketch
  int64_t need;                // rows of the next batch
  int32_t force;
  int32_t pad;
};

// A run of slice seeds written to device memory by one small launch.
constexpr int kSeedBlock = 64;
struct SeedBlock {
  int32_t first, n;
  RowSeeds s[kSeedBlock];
};
static_assert(sizeof(SeedBlock) <= 4096, "kernel arguments must stay small");

}  // namespace compass
