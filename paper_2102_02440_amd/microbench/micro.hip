// micro.hip -- roofline probes for gfx950: VALU rates of 32-bit ops and
// v_mad_u64_u32, the sketch hash rate, LDS atomic rate, HBM stream read and
// global atomic rate.  Every index is bounded by its buffer.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <string>
#include <vector>
#include "../csrc/device_math.hpp"

#define CK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

__global__ void k_add32(uint32_t* out, int iters) {
  uint32_t a = threadIdx.x, b = blockIdx.x, c = a ^ 0x1234, d = b + 7;
  uint32_t e = a + 1, f = b + 2, g = a * 3, h = b * 5;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      a = a + b; c = c ^ d; e = e + f; g = g ^ h;
      b = b + c; d = d ^ e; f = f + g; h = h ^ a;
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = a ^ b ^ c ^ d ^ e ^ f ^ g ^ h;
}

__global__ void k_mad64(uint64_t* out, int iters) {
  uint64_t a = threadIdx.x, b = blockIdx.x + 1, c = a + 3, d = b + 5;
  uint32_t x = threadIdx.x * 2654435761u, y = blockIdx.x * 40503u + 1;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      a = (uint64_t)(uint32_t)a * x + (uint32_t)(b >> 13);
      b = (uint64_t)(uint32_t)b * y + (uint32_t)(c >> 11);
      c = (uint64_t)(uint32_t)c * x + (uint32_t)(d >> 7);
      d = (uint64_t)(uint32_t)d * y + (uint32_t)(a >> 5);
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = a ^ b ^ c ^ d;
}

__global__ void k_hash(uint32_t* out, int iters, compass::RowSeeds s, compass::BucketMod m) {
  uint64_t x = (blockIdx.x * blockDim.x + threadIdx.x) & 0x7fffffff;
  uint32_t acc = 0;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int32_t sg; uint32_t b;
      compass::hash_xi_h<true>(x + k, s, m, sg, b);
      acc += b + sg;
    }
    x += 7;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void k_lds_atomic(uint32_t* out, int iters, int w, int hot) {
  extern __shared__ int32_t c[];
  for (int i = threadIdx.x; i < w; i += blockDim.x) c[i] = 0;
  __syncthreads();
  uint32_t h = (blockIdx.x * blockDim.x + threadIdx.x) * 2654435761u;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      h = h * 1664525u + 1013904223u;
      uint32_t idx = hot ? ((h >> 28) & 3) : ((h >> 8) & (w - 1));
      atomicAdd(&c[idx], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = c[0];
}

__global__ void k_stream(const uint4* __restrict__ in, size_t n, uint32_t* out) {
  uint32_t acc = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    uint4 v = in[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x12345678) out[0] = acc;
}

__global__ void k_gatomic(int32_t* c, size_t w, int iters) {
  uint32_t h = (blockIdx.x * blockDim.x + threadIdx.x) * 2654435761u + 17;
  for (int i = 0; i < iters; ++i) {
    h = h * 1664525u + 1013904223u;
    size_t idx = ((size_t)h * 7919u) % w;
    atomicAdd(&c[idx], 1);
  }
}

__global__ void k_copy(const uint4 *__restrict__ in, uint4 *__restrict__ out,
                       size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = in[i];
}

// Gather probes: out[i] = in[idx(i)] for about 1% of the positions of an
// 8 GiB array of 8-byte values, in increasing order (like the survivors of
// a 1%-selective scan), read three ways: plain loads, nontemporal loads and
// system-scope relaxed atomic loads.  idx(i) = 100 i + h(i) mod 100 <
// 100 n_idx <= the array's length (checked on the host).
__device__ __host__ inline uint64_t gather_idx(uint64_t i) {
  return 100 * i + ((i * 2654435761ull) >> 7) % 100;
}

__global__ void k_gather_plain(const uint64_t *__restrict__ in, uint64_t n_idx,
                               uint64_t *__restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_idx;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = in[gather_idx(i)];
}

__global__ void k_gather_nt(const uint64_t *__restrict__ in, uint64_t n_idx,
                            uint64_t *__restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_idx;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = __builtin_nontemporal_load(in + gather_idx(i));
}

__global__ void k_gather_sys(const uint64_t *__restrict__ in, uint64_t n_idx,
                             uint64_t *__restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_idx;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = __hip_atomic_load(in + gather_idx(i), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
}

static int gather_probe() {
  const uint64_t n = (uint64_t)1 << 30;  // 8 GiB of uint64
  const uint64_t n_idx = n / 100;
  if (gather_idx(n_idx - 1) >= n) {
    printf("gather index out of range\n");
    return 1;
  }
  uint64_t *in, *out;
  CK(hipMalloc(&in, n * 8));
  CK(hipMalloc(&out, n_idx * 8));
  CK(hipMemset(in, 3, n * 8));
  CK(hipDeviceSynchronize());
  hipEvent_t a, b;
  CK(hipEventCreate(&a));
  CK(hipEventCreate(&b));
  const char *names[3] = {"plain", "nontemporal", "system-scope"};
  for (int rep = 0; rep < 2; ++rep)
    for (int v = 0; v < 3; ++v) {
      CK(hipEventRecord(a));
      if (v == 0) hipLaunchKernelGGL(k_gather_plain, dim3(2048), dim3(256), 0, 0, in, n_idx, out);
      if (v == 1) hipLaunchKernelGGL(k_gather_nt, dim3(2048), dim3(256), 0, 0, in, n_idx, out);
      if (v == 2) hipLaunchKernelGGL(k_gather_sys, dim3(2048), dim3(256), 0, 0, in, n_idx, out);
      CK(hipEventRecord(b));
      CK(hipEventSynchronize(b));
      float ms;
      CK(hipEventElapsedTime(&ms, a, b));
      printf("gather %s: %llu values of 8 bytes at 1%% density in %.3f ms\n",
             names[v], (unsigned long long)n_idx, ms);
    }
  return 0;
}

// `micro copy`: one plain copy of exactly 1 GiB (read 1 GiB, write 1 GiB),
// the calibration kernel for the FETCH_SIZE / WRITE_SIZE counters.
static int copy_probe() {
  const size_t bytes = (size_t)1 << 30, n = bytes / 16;
  uint4 *a, *b;
  CK(hipMalloc(&a, bytes));
  CK(hipMalloc(&b, bytes));
  CK(hipMemset(a, 1, bytes));
  CK(hipDeviceSynchronize());
  hipLaunchKernelGGL(k_copy, dim3(256 * 16), dim3(256), 0, 0, a, b, n);
  CK(hipDeviceSynchronize());
  printf("copied %zu bytes\n", bytes);
  return 0;
}

int main(int argc, char **argv) {
  if (argc > 1 && std::string(argv[1]) == "copy") return copy_probe();
  if (argc > 1 && std::string(argv[1]) == "gather") return gather_probe();
  hipDeviceProp_t p; CK(hipGetDeviceProperties(&p, 0));
  printf("device %s CUs %d clock %d kHz l2 %d bytes sharedPerBlock %zu maxSharedPerMP %zu\n", p.name, p.multiProcessorCount, p.clockRate, p.l2CacheSize, p.sharedMemPerBlock, p.maxSharedMemoryPerMultiProcessor);
  hipEvent_t a, b; CK(hipEventCreate(&a)); CK(hipEventCreate(&b));
  float ms;
  const int blocks = 256 * 8, threads = 256;
  uint64_t* o64; CK(hipMalloc(&o64, (size_t)blocks * threads * 8));
  uint32_t* o32 = (uint32_t*)o64;
  int iters = 2000;
  // add32: 16*8 ops per iter
  hipLaunchKernelGGL(k_add32, dim3(blocks), dim3(threads), 0, 0, o32, 10); CK(hipDeviceSynchronize());
  CK(hipEventRecord(a)); hipLaunchKernelGGL(k_add32, dim3(blocks), dim3(threads), 0, 0, o32, iters); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&ms, a, b));
  double ops = (double)blocks * threads * iters * 16 * 8;
  printf("M1a add/xor32: %.1f Gop/s (lane-ops)\n", ops / ms / 1e6);
  hipLaunchKernelGGL(k_mad64, dim3(blocks), dim3(threads), 0, 0, o64, 10); CK(hipDeviceSynchronize());
  CK(hipEventRecord(a)); hipLaunchKernelGGL(k_mad64, dim3(blocks), dim3(threads), 0, 0, o64, iters); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&ms, a, b));
  ops = (double)blocks * threads * iters * 16 * 4;
  printf("M1b mad_u64_u32 (+shift): %.1f Gmad/s\n", ops / ms / 1e6);
  compass::RowSeeds s{123456789ull, 987654321ull, 555555555555ull, 77777777777ull, 31337ull, 2305843009213693000ull};
  compass::BucketMod m{8192, 8191, 0, 1, 1.0 / 8192};
  hipLaunchKernelGGL(k_hash, dim3(blocks), dim3(threads), 0, 0, o32, 10, s, m); CK(hipDeviceSynchronize());
  CK(hipEventRecord(a)); hipLaunchKernelGGL(k_hash, dim3(blocks), dim3(threads), 0, 0, o32, 500, s, m); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&ms, a, b));
  ops = (double)blocks * threads * 500 * 4;
  printf("M1c hash (xi+h, x<2^32): %.1f Ghash/s\n", ops / ms / 1e6);
  for (int hot = 0; hot < 2; ++hot) {
    int w = 8192;
    hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(threads), w * 4, 0, o32, 10, w, hot); CK(hipDeviceSynchronize());
    CK(hipEventRecord(a)); hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(threads), w * 4, 0, o32, 1000, w, hot); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&ms, a, b));
    ops = (double)blocks * threads * 1000 * 8;
    printf("M2 LDS atomic add (%s): %.1f Gatomic/s\n", hot ? "4 hot addresses" : "uniform 8192", ops / ms / 1e6);
  }
  size_t bytes = (size_t)4 << 30;
  uint4* big; CK(hipMalloc(&big, bytes)); CK(hipMemset(big, 1, bytes));
  size_t n = bytes / 16;
  for (int rep = 0; rep < 3; ++rep) {
    CK(hipEventRecord(a)); hipLaunchKernelGGL(k_stream, dim3(256 * 16), dim3(256), 0, 0, big, n, o32); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&ms, a, b));
    printf("M3 stream read 4 GiB: %.1f GB/s\n", bytes / ms / 1e6);
  }
  int32_t* cnt; size_t w = 35u << 20; CK(hipMalloc(&cnt, w * 4)); CK(hipMemset(cnt, 0, w * 4));
  CK(hipEventRecord(a)); hipLaunchKernelGGL(k_gatomic, dim3(256 * 16), dim3(256), 0, 0, cnt, w / 4, 1000); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&ms, a, b));
  printf("M4 global atomic add (int32, 35 MiB region): %.1f Gatomic/s\n", 256.0 * 16 * 256 * 1000 / ms / 1e6);
  CK(hipEventRecord(a)); hipLaunchKernelGGL(k_gatomic, dim3(256 * 16), dim3(256), 0, 0, cnt, (size_t)(2u << 20) / 4, 1000); CK(hipEventRecord(b)); CK(hipEventSynchronize(b)); CK(hipEventElapsedTime(&ms, a, b));
  printf("M4 global atomic add (int32, 2 MiB region): %.1f Gatomic/s\n", 256.0 * 16 * 256 * 1000 / ms / 1e6);
  return 0;
}
