// bitonic.hpp -- ascending bitonic sort of 64-bit keys held in LDS by one
// workgroup.
//
// Each wave owns kB = 64 * R consecutive keys (positions wave * kB + lane +
// 64 r, r < R) and keeps them in registers.  A compare-exchange stage
// pairs position i with i ^ j; it stays inside the wave when j < kB (for
// j <= 32 by lane shuffles, for 64 <= j < kB between the lane's own
// registers), so only stages with j >= kB go through LDS between block
// barriers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace compass {

// Sorts keys[0, n) ascending; n a power of two, kB <= n <= NT * R.  Every
// thread of the workgroup must call it; keys lives in LDS.
template <int NT, int R>
__device__ __forceinline__ void bitonic_sort_lds(unsigned long long *keys,
                                                 int n) {
  constexpr int kB = 64 * R;
  const int lane = (int)threadIdx.x & 63;
  const int base = ((int)threadIdx.x >> 6) * kB + lane;
  const bool mine = base < n;  // whole waves
  unsigned long long x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = mine ? keys[base + 64 * r] : 0ull;
  for (int k = 2; k <= n; k <<= 1) {
    int j = k >> 1;
    if (j >= kB) {
      if (mine) {
#pragma unroll
        for (int r = 0; r < R; ++r) keys[base + 64 * r] = x[r];
      }
      __syncthreads();
      for (; j >= kB; j >>= 1) {
        for (int t = threadIdx.x; t < (n >> 1); t += NT) {
          const int i = 2 * t - (t & (j - 1));
          const unsigned long long a = keys[i], b = keys[i + j];
          if ((a > b) == ((i & k) == 0)) {
            keys[i] = b;
            keys[i + j] = a;
          }
        }
        __syncthreads();
      }
      if (mine) {
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = keys[base + 64 * r];
      }
    }
    if (!mine) continue;
    for (; j >= 64; j >>= 1) {
      const int jr = j >> 6;  // register distance of the pair
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r & jr) continue;
        const unsigned long long lo = x[r] < x[r + jr] ? x[r] : x[r + jr];
        const unsigned long long hi = x[r] < x[r + jr] ? x[r + jr] : x[r];
        const bool asc = ((base + 64 * r) & k) == 0;
        x[r] = asc ? lo : hi;
        x[r + jr] = asc ? hi : lo;
      }
    }
    for (; j >= 1; j >>= 1) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const unsigned long long y = __shfl_xor(x[r], j);
        const int e = base + 64 * r;
        // the smaller key stays at the lower position of an ascending pair
        // (bit k clear) and at the upper position of a descending one
        const bool keep_min = ((e & k) == 0) == ((e & j) == 0);
        x[r] = keep_min ? (x[r] < y ? x[r] : y) : (x[r] < y ? y : x[r]);
      }
    }
  }
  __syncthreads();
  if (mine) {
#pragma unroll
    for (int r = 0; r < R; ++r) keys[base + 64 * r] = x[r];
  }
  __syncthreads();
}

}  // namespace compass
