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
