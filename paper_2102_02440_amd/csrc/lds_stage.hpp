// lds_stage.hpp -- copies of global arrays into LDS with many loads in
// flight per lane.
//
// A plain `for (i = lane; i < n; i += lanes) lds[i] = f(src[i])` loop
// compiles to load, wait, store per trip: every trip pays the full memory
// latency.  Here each lane first issues U loads (indexes clamped into
// [0, n), so the loads need no branch), then waits once and stores the
// values that are in range.
#pragma once
#include <hip/hip_runtime.h>

namespace compass {

template <int NT, int U, typename TS, typename TD, typename F>
__device__ __forceinline__ void stage_lds(TD *dst, const TS *src, int n, F f) {
  if (n <= 0) return;
  for (int b = 0; b < n; b += NT * U) {
    TS r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = b + u * NT + (int)threadIdx.x;
      r[u] = src[i < n ? i : n - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = b + u * NT + (int)threadIdx.x;
      if (i < n) dst[i] = f(r[u]);
    }
  }
}

struct StageCopy {
  template <typename T>
  __device__ __forceinline__ T operator()(T x) const { return x; }
};

// the magnitude field (|v|, below 2^32 for int32 counters) of a sort key
// (|v| << 16 | bucket)
struct StageMag {
  __device__ __forceinline__ uint32_t operator()(uint64_t k) const {
    return (uint32_t)(k >> 16);
  }
};

}  // namespace compass
