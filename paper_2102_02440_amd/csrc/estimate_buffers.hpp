// estimate_buffers.hpp -- device scratch views of one compass_estimate call.
#pragma once
#include <stdint.h>

#include "device_math.hpp"

namespace compass {

// One element of a triangle apex's merged list, read by every lane of the
// sweep with wave-uniform scalar loads (48 bytes: one x8 + one x4 load).
struct TriElem {
  int64_t v;        // the apex's counter on the child's edge
  uint64_t key;     // kappa of the child's own bucket (cut children only)
  u128 mu;          // the child's unconditioned message
  uint32_t child;   // child slot
  uint32_t pad[3];
};

struct EstBuffers {
  const void *const *sides;   // [2 * n_edges] counter arrays (d x w)
  const int64_t *n_sel;       // [n_tables]
  const uint64_t *sorted;     // [side][row][w] keys (|v| << 16 | j)
  u128 *msg;                  // [slot][row][w]
  uint32_t *merged;           // [scratch slot][row][Lmax]
  u128 *xout;                 // [slot][row]
  TriElem *prep;              // [prep slot][row][Lprep]
  u128 *partial;              // [slot][row]
  int32_t counter_bits;
  int32_t d;
  int32_t w;
  int32_t Lmax;
  int32_t Lprep;
  int32_t pad;
};

}  // namespace compass
