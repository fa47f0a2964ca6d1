// agms.hip -- the AGMS baseline (Section 4.1) that Fast-AGMS improves on.
//
//  agms_build_kernel  fused selection scan; for every qualifying row, every
//                     one of the K = r * b basic sketches adds the product
//                     over the table's joins of that join's +-1 variable of
//                     the row's key (the composed sketch of a table in a
//                     multi-way join).  A tile's survivors are compacted
//                     (the same ballot compaction as the Fast-AGMS scan) and
//                     their key field elements staged in LDS; lane (c, part)
//                     owns basic sketch c (its seeds in registers) and every
//                     parts-th survivor, reading keys by LDS broadcast.  The
//                     cost is K sign evaluations per join per row -- the
//                     update cost that makes AGMS impractical (Section 4.1.4).
//  agms_estimate      basic estimate (i, j) = product of the tables' counters;
//                     exact 128-bit row sums, averages over b, median over r.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "agms_params.hpp"
#include "device_math.hpp"
#include "scan_common.hpp"

namespace compass {

struct AgmsJob {
  const AgmsParams &P;
  __device__ int n_preds() const { return P.n_preds; }
  __device__ const PredDev &pred(int q) const { return P.preds[q]; }
};

// +-1 variable of one field element under one basic sketch's seeds
// (the lanes of a wave mostly share the key: the width test is nearly
// always uniform)
__device__ __forceinline__ int32_t agms_xi(uint64_t x, const RowSeeds &s) {
  uint64_t v;
  if ((x >> 31) == 0) {
    const uint32_t x32 = (uint32_t)x;
    v = madd61_x31(s.a3, x32, s.a2);
    v = madd61_x31(v, x32, s.a1);
    v = madd61_x31(v, x32, s.a0);
  } else if ((x >> 32) == 0) {
    const uint32_t x32 = (uint32_t)x;
    v = madd61_x32(s.a3, x32, s.a2);
    v = madd61_x32(v, x32, s.a1);
    v = madd61_x32(v, x32, s.a0);
  } else {
    v = madd61_x61(s.a3, x, s.a2);
    v = madd61_x61(v, x, s.a1);
    v = madd61_x61(v, x, s.a0);
  }
  // parity as add-with-carry plus bit extract, then doubled | 1
  uint32_t lr = low_of_residue(v);
  __asm__("" : "+v"(lr));
  int32_t par = __builtin_amdgcn_sbfe((int32_t)lr, 0, 1);
  __asm__("" : "+v"(par));
  return (int32_t)((uint32_t)par << 1) | 1;
}

__global__ __launch_bounds__(kBuildThreads) void agms_build_kernel(
    const AgmsParams P) {
  extern __shared__ uint64_t xs[];  // [join][kBuildTile] survivor keys
  __shared__ int32_t queue[kBuildTile];
  __shared__ int32_t s_qn;
  __shared__ int64_t red[kBuildThreads];
  const AgmsJob job{P};
  const int K = P.K;
  const int parts = kBuildThreads / K;
  const int c = threadIdx.x % K;
  const int part = threadIdx.x / K;  // parts .. : idle lanes
  const bool lane_on = part < parts;
  RowSeeds sd[kAgmsMaxJoins];
#pragma unroll
  for (int e = 0; e < kAgmsMaxJoins; ++e)
    if (e < P.n_joins && lane_on) sd[e] = P.seeds[(size_t)e * K + c];
  int64_t acc = 0;
  uint64_t sel = 0;
  const int64_t row0 = (int64_t)blockIdx.x * P.rows_per_chunk;
  const int64_t row1 = min(row0 + P.rows_per_chunk, P.n_rows);
  for (int64_t base = row0; base < row1; base += kBuildTile) {
    const int nt = (int)min((int64_t)kBuildTile, row1 - base);
    const int qn = compact_tile<AgmsJob, kBuildRowsPerThread>(
        job, base, nt, P.n_preds, queue, &s_qn);
    sel += (uint64_t)qn;
    for (int e = 0; e < P.n_joins; ++e)
      for (int q = threadIdx.x; q < qn; q += kBuildThreads)
        xs[(size_t)e * kBuildTile + q] =
            load_field(P.keys[e], base + (P.n_preds ? queue[q] : q));
    __syncthreads();
    if (lane_on) {
      for (int q = part; q < qn; q += parts) {
        int32_t prod = 1;
#pragma unroll
        for (int e = 0; e < kAgmsMaxJoins; ++e)
          if (e < P.n_joins) prod *= agms_xi(xs[(size_t)e * kBuildTile + q], sd[e]);
        acc += prod;
      }
    }
    __syncthreads();  // xs, queue and s_qn are reused by the next tile
  }
  red[threadIdx.x] = lane_on ? acc : 0;
  __syncthreads();
  if (threadIdx.x < K) {
    int64_t t = 0;
    for (int p = 0; p < parts; ++p) t += red[p * K + threadIdx.x];
    if (t) atomicAdd(reinterpret_cast<unsigned long long *>(P.counters + threadIdx.x),
                     (unsigned long long)t);
  }
  if (P.count_selected && threadIdx.x == 0 && sel)
    atomicAdd(reinterpret_cast<unsigned long long *>(P.n_selected),
              (unsigned long long)sel);
}

hipError_t launch_agms_build(const AgmsParams &P, int n_blocks,
                             hipStream_t st) {
  const size_t lds = (size_t)P.n_joins * kBuildTile * 8;
  hipLaunchKernelGGL(agms_build_kernel, dim3(n_blocks), dim3(kBuildThreads),
                     lds, st, P);
  return hipGetLastError();
}

__global__ void agms_estimate_kernel(AgmsEstArgs a, uint64_t *row_sums,
                                     double *est, int32_t *flag) {
  __shared__ double avg[64];
  const int r = a.r, b = a.b;
  for (int i = threadIdx.x; i < r; i += blockDim.x) {
    u128 sum = 0;
    for (int j = 0; j < b; ++j) {
      u128 x = 1;
      for (int t = 0; t < a.n_tables; ++t)
        x = mul_u128(x, s64_to_u128(a.sk[t][(size_t)i * b + j]));
      sum += x;
    }
    if (row_sums) {
      row_sums[2 * i] = (uint64_t)sum;
      row_sums[2 * i + 1] = (uint64_t)(sum >> 64);
    }
    avg[i] = i128_to_double(sum) / (double)b;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = 1; i < r; ++i) {  // insertion sort of r <= 64 averages
    const double v = avg[i];
    int k = i - 1;
    while (k >= 0 && avg[k] > v) {
      avg[k + 1] = avg[k];
      --k;
    }
    avg[k + 1] = v;
  }
  *est = (r & 1) ? avg[r / 2] : (avg[r / 2 - 1] + avg[r / 2]) * 0.5;
  const u128 lim = (u128)1 << 127;
  u128 p = 1;
  bool ok = true;
  for (int t = 0; t < a.n_tables && ok; ++t) {
    const int64_t n = *a.n_sel[t];
    const u128 f = (u128)(n < 0 ? 0 : n);
    if (f == 0) {
      p = 0;
      break;
    }
    if (p > lim / f) ok = false; else p *= f;
  }
  *flag = ok && p < lim ? 1 : 0;
}

hipError_t launch_agms_estimate(const AgmsEstArgs &a, uint64_t *row_sums,
                                double *est, int32_t *flag, hipStream_t st) {
  hipLaunchKernelGGL(agms_estimate_kernel, dim3(1), dim3(64), 0, st, a,
                     row_sums, est, flag);
  return hipGetLastError();
}

}  // namespace compass
