// certificate.hpp -- when a sub-plan's 128-bit row values are the true
// integers.
#pragma once
#include <stdint.h>

#include "device_math.hpp"
#include "estimate_params.hpp"

namespace compass {

// |X_i| <= prod over the sub-plan's tables of n_sel, times w^(edges -
// tables) when positive (each bucket row sums to at most n_sel in absolute
// value, and a one-to-one assignment of tables to incident edges factorises
// the bound).  Certified when that bound is below 2^127, or when a table
// selected no row (then every X_i is 0).
__device__ inline bool subplan_certified(const SubplanTask &S,
                                         const int64_t *n_sel, int n_tables,
                                         int w) {
  const u128 lim = (u128)1 << 127;
  u128 b = 1;
  bool ok = true;
  for (int t = 0; t < n_tables && ok; ++t) {
    if (!((S.mask >> t) & 1ull)) continue;
    const int64_t ns = n_sel[t];
    const u128 f = ns < 0 ? 0 : (u128)ns;
    if (f == 0) return true;
    // b * f > 2^127 stops the product (no 128-bit division)
    u128 prod;
    if (__builtin_mul_overflow(b, f, &prod) || prod > lim) ok = false;
    else b = prod;
  }
  for (int k = 0; k < S.n_edges - S.n_tables && ok; ++k) {
    u128 prod;
    if (__builtin_mul_overflow(b, (u128)w, &prod) || prod > lim) ok = false;
    else b = prod;
  }
  return ok && b < lim;
}

}  // namespace compass
