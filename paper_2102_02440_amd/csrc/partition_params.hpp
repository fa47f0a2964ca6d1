// partition_params.hpp -- arguments of the three-table chain estimate.
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

}  // namespace compass
