// estimate_buffers.hpp -- device scratch views of one compass_estimate call.
#pragma once
#include <stdint.h>

#include "device_math.hpp"

namespace compass {

struct EstBuffers {
  const void *const *sides;   // [2 * n_edges] counter arrays (d x w)
  const int64_t *n_sel;       // [n_tables]
  const uint64_t *sorted;     // [side][row][w] keys (|v| << 16 | j)
  u128 *msg;                  // [slot][row][w]
  uint32_t *merged;           // [scratch slot][row][Lmax]
  u128 *xout;                 // [slot][row]
  uint32_t *prep_meta;        // [prep slot][row][Lprep]
  int64_t *prep_v;
  u128 *prep_mu;
  uint64_t *prep_key;
  u128 *partial;              // [slot][row]
  int32_t counter_bits;
  int32_t d;
  int32_t w;
  int32_t Lmax;
  int32_t Lprep;
  int32_t pad;
};

}  // namespace compass
