// partition_params.hpp -- arguments of the two-dimensional build and of the
// three-table chain estimate.
#pragma once
#include <stdint.h>

#include "device_math.hpp"

namespace compass {

constexpr int kChainRows = 32;  // rows of the two-dimensional sketch per block

struct ChainArgs {
  const void *A, *P, *B;        // d x w1, d x w1 x w2, d x w2 counters
  const int64_t *n_a, *n_p, *n_b;  // device: selected rows of the 3 tables
  u128 *partial;                // [d][ceil(w1 / kChainRows)] block sums
  int32_t counter_bits, d, w1, w2;
};

// Binned two-dimensional build (see partition.hip): a tile is R = 2^r_shift
// consecutive j1 rows of one sketch row's w1 x w2 matrix (R * w2 <=
// kBinTileWords int32 counters in LDS); tiles are numbered i * nbr + j1 / R.
constexpr int kBinTileWords = 32768;   // 128 KiB of int32 per tile
constexpr int kBinMaxBins = 32768;     // per-block histograms in LDS (128 KiB)

// Joins beyond the second of a partitioned sketch (k = 3 or 4 joins):
// their dimensions are flattened into the second one, which then has width
// w2 * w3 * w4 (w3 = w4 = 1 when absent); the sign of an update is the
// product over every join.
struct KdDims {
  BucketMod bm3, bm4;
  int32_t kd;   // joins: 2, 3 or 4
  int32_t w3, w4;
  int32_t pad;
};

// Estimate from partitioned sketches over a tree of tables (Section 5.1):
// table t's counters form, per sketch row, a tensor with one dimension per
// incident edge (edges in increasing id, row-major).  One task per table,
// processed children first: a non-root table sends its parent, for every
// bucket j of the parent edge, the sum over its tensor's slice at j of the
// entry times its children's messages at the entry's other indices; the
// root sums its whole tensor that way, in chunks.
constexpr int kTensorMaxDims = 4;
constexpr int kTensorThreads = 256;
constexpr int kTensorChunk = 4096;   // root entries summed by one workgroup

struct TensorTask {
  const void *tensor;           // d x prod(widths)
  int32_t n_dims;
  int32_t parent_dim;           // -1: the root
  int32_t width[kTensorMaxDims];
  int64_t stride[kTensorMaxDims];
  int64_t size;                 // entries per sketch row
  int32_t child_msg[kTensorMaxDims];  // per dimension: message slot, -1 - leaf
                                      // table (its counters), or unused
  const void *leaf[kTensorMaxDims];   // a leaf child's counters (d x width)
  int32_t out_slot;             // message slot (non-root)
  int32_t n_chunks;             // root: chunks of kTensorChunk entries
};

struct TensorArgs {
  const TensorTask *tasks;
  u128 *msg;                    // [slot][row][w_max]
  u128 *partial;                // [row][root chunk]
  int32_t counter_bits, d, w_max, pad;
};

struct Bin2dArgs {
  int32_t d, w1, w2, r_shift;
  int32_t nbr, n_bins, n_blocks, pad;
  int64_t row0, row1;            // rows of this batch
  int64_t rows_per_block;        // a multiple of kBuildTile
  uint32_t *rec;                 // per block rows_per_block * d records
  int32_t *rec_count;            // [n_blocks]
  int32_t *hist;                 // [n_blocks][n_bins]: counts, then offsets
  int32_t *bin_total;            // [n_bins]
  int32_t *bin_start;            // [n_bins + 1]
  uint16_t *sorted;              // records grouped by tile
};

}  // namespace compass
