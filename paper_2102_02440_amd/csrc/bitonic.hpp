// bitonic.hpp -- ascending bitonic sort of 64-bit keys held in LDS by one
// workgroup.
//
// Each wave owns kB = 64 * R consecutive keys (positions wave * kB + lane +
// 64 r, r < R) and keeps them in registers.  A compare-exchange stage
// pairs position i with i ^ j; it stays inside the wave when j < kB (for
// j <= 32 across lanes, for 64 <= j < kB between the lane's own
// registers), so only stages with j >= kB go through LDS between block
// barriers.
//
// The cross-lane stages are unrolled, so that every partner exchange is a
// fixed lane pattern: DPP row moves for j = 1, 2 (quad permutes) and 8 (a
// rotation by half a row), ds_swizzle for j = 4 and 16 (xor within 32
// lanes), ds_bpermute for j = 32.  The keep-the-smaller decision of a
// lane, ((i & k) == 0) == ((i & j) == 0), is a fixed lane mask per stage,
// and the exchange is one 64-bit compare and two selects.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace compass {

namespace bitonic_detail {

// the 32-bit value of lane (lane ^ (1 << LJ)); LJ < 6
template <int LJ>
__device__ __forceinline__ int partner32(int v, int bperm_addr) {
  if constexpr (LJ == 0) {
    return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  } else if constexpr (LJ == 1) {
    return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  } else if constexpr (LJ == 2) {
    return __builtin_amdgcn_ds_swizzle(v, (4 << 10) | 0x1F);  // xor 4
  } else if constexpr (LJ == 3) {
    return __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false);  // row_ror 8
  } else if constexpr (LJ == 4) {
    return __builtin_amdgcn_ds_swizzle(v, (16 << 10) | 0x1F);  // xor 16
  } else {
    return __builtin_amdgcn_ds_bpermute(bperm_addr, v);  // xor 32
  }
}

template <int LJ>
__device__ __forceinline__ unsigned long long partner64(unsigned long long v,
                                                        int bperm_addr) {
  const int lo = partner32<LJ>((int)(uint32_t)v, bperm_addr);
  const int hi = partner32<LJ>((int)(uint32_t)(v >> 32), bperm_addr);
  return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

// keep x or take its partner y: the smaller when keep_min, else the larger
__device__ __forceinline__ unsigned long long exch(unsigned long long x,
                                                   unsigned long long y,
                                                   bool keep_min) {
  return (x < y) == keep_min ? x : y;
}

// the cross-lane stages j = 2^LJ, ..., 1 of merge size k (all in registers)
template <int R, int LJ>
__device__ __forceinline__ void lane_stages(unsigned long long (&x)[R], int k,
                                            int base, int bperm_addr) {
  if constexpr (LJ >= 0) {
    const int lane = base & 63;
    const bool lj = (lane >> LJ) & 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const unsigned long long y = partner64<LJ>(x[r], bperm_addr);
      const bool lk = ((base + 64 * r) & k) != 0;
      x[r] = exch(x[r], y, lk == lj);
    }
    lane_stages<R, LJ - 1>(x, k, base, bperm_addr);
  }
}

}  // namespace bitonic_detail

// Sorts keys[0, n) ascending; n a power of two, kB <= n <= NT * R.  Every
// thread of the workgroup must call it; keys lives in LDS.
template <int NT, int R>
__device__ __forceinline__ void bitonic_sort_lds(unsigned long long *keys,
                                                 int n) {
  using namespace bitonic_detail;
  constexpr int kB = 64 * R;
  constexpr int kLogMax = __builtin_ctz(NT * R);
  const int lane = (int)threadIdx.x & 63;
  const int base = ((int)threadIdx.x >> 6) * kB + lane;
  const int bperm_addr = (lane ^ 32) << 2;
  // whole waves (n is a multiple of kB): a uniform branch
  const bool mine = __builtin_amdgcn_readfirstlane(base < n ? 1 : 0) != 0;
  unsigned long long x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = mine ? keys[base + 64 * r] : 0ull;
#pragma unroll
  for (int lk = 1; lk <= kLogMax; ++lk) {
    const int k = 1 << lk;
    if (k > n) break;  // uniform
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
    // register stages 64 <= j < kB: pairs (r, r + j / 64) of the lane
#pragma unroll
    for (int lj = kLogMax; lj >= 6; --lj) {
      const int jj = 1 << lj;
      if (jj >= kB || jj > j) continue;
      const int jr = jj >> 6;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r & jr) continue;
        const bool asc = ((base + 64 * r) & k) == 0;  // uniform
        const bool swap = (x[r] > x[r + jr]) == asc;
        const unsigned long long a = x[r], b = x[r + jr];
        x[r] = swap ? b : a;
        x[r + jr] = swap ? a : b;
      }
    }
    // cross-lane stages j = min(k / 2, 32), ..., 1
    switch (lk) {
      case 1: lane_stages<R, 0>(x, k, base, bperm_addr); break;
      case 2: lane_stages<R, 1>(x, k, base, bperm_addr); break;
      case 3: lane_stages<R, 2>(x, k, base, bperm_addr); break;
      case 4: lane_stages<R, 3>(x, k, base, bperm_addr); break;
      case 5: lane_stages<R, 4>(x, k, base, bperm_addr); break;
      default: lane_stages<R, 5>(x, k, base, bperm_addr); break;
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
