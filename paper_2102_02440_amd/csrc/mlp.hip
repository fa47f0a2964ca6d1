// mlp.hip -- learned correction of sketch estimates (gfx950 kernels).
//
// A small MLP (n_in -> H -> ... -> H -> 1, ReLU) maps per-row sketch
// estimates, selected sizes and sub-plan shape to a correction of the log
// cardinality: y = ln(1 + max(raw, 0)) + net(x), so the zero network is the
// raw median estimate, which stays the fallback.  Weights are kept in fp32
// (master, Adam state) and in bfloat16 (the copy the products read); every
// layer rounds its input activations to bfloat16 and accumulates in fp32.
//
// Kernels (tiny dense layers: H <= 64, so plain FP32 FMA over LDS tiles; a
// matrix-core tile would sit idle at these shapes):
//   mlp_fwd_kernel     8 samples per workgroup (64 workgroups per 512-sample
//                      batch); layer weights staged in LDS;
//                      saves rounded inputs and pre-activations for training
//   mlp_bwd_kernel     per-workgroup partial gradients (deterministic slab)
//   mlp_reduce_adam_kernel  sums the slab in a fixed order, then Adam on
//                      the fp32 masters and the bfloat16 copy
//   mlp_features_kernel  sub-plan features from the 128-bit row estimates
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <cmath>
#include <string>
#include <vector>

#include "compass.h"
#include "device_math.hpp"

namespace compass {

constexpr int kMlpMaxDim = 64;
constexpr int kMlpMaxLayers = 8;
constexpr int kMlpTile = 8;        // samples per workgroup
constexpr int kMlpThreads = 256;

struct MlpShape {
  int32_t n_layers;                  // weight layers (hidden + output)
  int32_t dim[kMlpMaxLayers + 1];    // dim[0] = n_in ... dim[n_layers] = 1
  int32_t woff[kMlpMaxLayers];       // offset of W_l in the flat parameters
  int32_t boff[kMlpMaxLayers];       // offset of b_l
  int32_t n_params;
};

__device__ __forceinline__ float bf16_to_f(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

// round-to-nearest-even to bfloat16 (finite inputs)
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

__device__ __forceinline__ float round_bf16(float f) {
  return bf16_to_f(f_to_bf16(f));
}

// Forward pass of up to kMlpTile samples.  act: [layer][sample][kMlpMaxDim]
// rounded layer inputs, pre: [layer][sample][kMlpMaxDim] pre-activations
// (both only when `save`).  Sample s reads row idx[s] of x and base (row s
// when idx is null).
__global__ __launch_bounds__(kMlpThreads) void mlp_fwd_kernel(
    MlpShape S, const uint16_t *__restrict__ wb, const float *__restrict__ p,
    const float *__restrict__ x, const float *__restrict__ base,
    const int32_t *__restrict__ idx, int32_t n, float *__restrict__ y,
    float *__restrict__ act, float *__restrict__ pre, int32_t save) {
  __shared__ float a[kMlpTile][kMlpMaxDim + 1];
  __shared__ float z[kMlpTile][kMlpMaxDim + 1];
  __shared__ float W[kMlpMaxDim][kMlpMaxDim + 1];
  __shared__ float bb[kMlpMaxDim];
  const int s0 = blockIdx.x * kMlpTile;
  const int n_in = S.dim[0];
  for (int k = threadIdx.x; k < kMlpTile * n_in; k += kMlpThreads) {
    const int s = k / n_in, i = k % n_in;
    if (s0 + s < n) {
      const size_t r = idx ? (size_t)idx[s0 + s] : (size_t)(s0 + s);
      a[s][i] = round_bf16(x[r * n_in + i]);
    } else {
      a[s][i] = 0.f;
    }
  }
  for (int l = 0; l < S.n_layers; ++l) {
    const int di = S.dim[l], dout = S.dim[l + 1];
    for (int k = threadIdx.x; k < dout * di; k += kMlpThreads)
      W[k / di][k % di] = bf16_to_f(wb[S.woff[l] + k]);
    for (int k = threadIdx.x; k < dout; k += kMlpThreads) bb[k] = p[S.boff[l] + k];
    __syncthreads();
    if (save) {
      for (int k = threadIdx.x; k < kMlpTile * di; k += kMlpThreads) {
        const int s = k / di, i = k % di;
        if (s0 + s < n)
          act[((size_t)l * n + s0 + s) * kMlpMaxDim + i] = a[s][i];
      }
    }
    for (int k = threadIdx.x; k < kMlpTile * dout; k += kMlpThreads) {
      const int s = k / dout, o = k % dout;
      float acc = 0.f;
      for (int i = 0; i < di; ++i) acc = fmaf(a[s][i], W[o][i], acc);
      z[s][o] = acc + bb[o];
    }
    __syncthreads();
    const bool last = (l == S.n_layers - 1);
    for (int k = threadIdx.x; k < kMlpTile * dout; k += kMlpThreads) {
      const int s = k / dout, o = k % dout;
      const float v = z[s][o];
      if (save && s0 + s < n) pre[((size_t)l * n + s0 + s) * kMlpMaxDim + o] = v;
      if (!last) a[s][o] = round_bf16(v > 0.f ? v : 0.f);
    }
    __syncthreads();
  }
  for (int s = threadIdx.x; s < kMlpTile; s += kMlpThreads)
    if (s0 + s < n) y[s0 + s] = base[idx ? idx[s0 + s] : s0 + s] + z[s][0];
}

// Backward pass: dL/dy = 2 (y - t) / n; partial gradients of this
// workgroup's samples go to slab[blockIdx.x][param]; loss partial too.
// Sample s's target is t[idx[s]] (t[s] when idx is null).
__global__ __launch_bounds__(kMlpThreads) void mlp_bwd_kernel(
    MlpShape S, const uint16_t *__restrict__ wb, const float *__restrict__ y,
    const float *__restrict__ t, const int32_t *__restrict__ idx, int32_t n,
    const float *__restrict__ act,
    const float *__restrict__ pre, float *__restrict__ slab,
    float *__restrict__ loss_part) {
  __shared__ float dz[kMlpTile][kMlpMaxDim + 1];
  __shared__ float da[kMlpTile][kMlpMaxDim + 1];
  __shared__ float ar[kMlpTile][kMlpMaxDim + 1];
  __shared__ float W[kMlpMaxDim][kMlpMaxDim + 1];
  __shared__ float red[kMlpThreads];
  const int s0 = blockIdx.x * kMlpTile;
  float* part = slab + (size_t)blockIdx.x * S.n_params;
  float lsum = 0.f;
  for (int s = threadIdx.x; s < kMlpTile; s += kMlpThreads) {
    float g = 0.f;
    if (s0 + s < n) {
      const float r = y[s0 + s] - t[idx ? idx[s0 + s] : s0 + s];
      g = 2.f * r / (float)n;
      lsum += r * r;
    }
    dz[s][0] = g;
  }
  red[threadIdx.x] = lsum;
  __syncthreads();
  for (int off = kMlpThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
  for (int l = S.n_layers - 1; l >= 0; --l) {
    const int di = S.dim[l], dout = S.dim[l + 1];
    for (int k = threadIdx.x; k < kMlpTile * di; k += kMlpThreads) {
      const int s = k / di, i = k % di;
      ar[s][i] = (s0 + s < n) ? act[((size_t)l * n + s0 + s) * kMlpMaxDim + i] : 0.f;
    }
    for (int k = threadIdx.x; k < dout * di; k += kMlpThreads)
      W[k / di][k % di] = bf16_to_f(wb[S.woff[l] + k]);
    __syncthreads();
    // dW[o][i] = sum_s dz[s][o] ar[s][i]; db[o] = sum_s dz[s][o]
    for (int k = threadIdx.x; k < dout * di; k += kMlpThreads) {
      const int o = k / di, i = k % di;
      float acc = 0.f;
      for (int s = 0; s < kMlpTile; ++s) acc = fmaf(dz[s][o], ar[s][i], acc);
      part[S.woff[l] + k] = acc;
    }
    for (int o = threadIdx.x; o < dout; o += kMlpThreads) {
      float acc = 0.f;
      for (int s = 0; s < kMlpTile; ++s) acc += dz[s][o];
      part[S.boff[l] + o] = acc;
    }
    if (l > 0) {
      // da[s][i] = sum_o dz[s][o] W[o][i]; dz_prev = da * (pre_prev > 0)
      for (int k = threadIdx.x; k < kMlpTile * di; k += kMlpThreads) {
        const int s = k / di, i = k % di;
        float acc = 0.f;
        for (int o = 0; o < dout; ++o) acc = fmaf(dz[s][o], W[o][i], acc);
        const float zp =
            (s0 + s < n) ? pre[((size_t)(l - 1) * n + s0 + s) * kMlpMaxDim + i] : 0.f;
        da[s][i] = zp > 0.f ? acc : 0.f;
      }
      __syncthreads();
      for (int k = threadIdx.x; k < kMlpTile * di; k += kMlpThreads) {
        const int s = k / di, i = k % di;
        dz[s][i] = da[s][i];
      }
    }
    __syncthreads();
  }
}

// Gradient = sum of the workgroups' partials (in workgroup order, eight
// partials' loads in flight per lane), then, when `adam`, the Adam update
// of the same parameter (fp32 master, moments, bfloat16 copy).  Lane 0 of
// workgroup 0 also sums the loss partials.
__global__ void mlp_reduce_adam_kernel(
    const float *__restrict__ slab, int32_t parts, int32_t n_params,
    float *__restrict__ g, const float *__restrict__ loss_part,
    float *__restrict__ loss, float inv_n, int32_t adam, float *__restrict__ p,
    float *__restrict__ m, float *__restrict__ v, uint16_t *__restrict__ wb,
    float lr, float b1, float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && loss) {
    float acc = 0.f;
    for (int b = 0; b < parts; ++b) acc += loss_part[b];
    *loss = acc * inv_n;  // mean squared error
  }
  if (k >= n_params) return;
  constexpr int kU = 8;
  float acc = 0.f;
  for (int b0 = 0; b0 < parts; b0 += kU) {
    float t[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      t[u] = b0 + u < parts ? slab[(size_t)(b0 + u) * n_params + k] : 0.f;
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (b0 + u < parts) acc += t[u];
  }
  g[k] = acc;
  if (!adam) return;
  const float mk = b1 * m[k] + (1.f - b1) * acc;
  const float vk = b2 * v[k] + (1.f - b2) * acc * acc;
  m[k] = mk;
  v[k] = vk;
  const float pk = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  p[k] = pk;
  wb[k] = f_to_bf16(pk);
}

__global__ void mlp_to_bf16_kernel(const float *__restrict__ p,
                                   uint16_t *__restrict__ wb, int32_t n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) wb[k] = f_to_bf16(p[k]);
}

// The query's join graph in kernel arguments (edge endpoints).
struct FeatGraph {
  int32_t n_edges;
  uint8_t u[64], v[64];
};

// Shape of the sub-plan `m` (its tables and the edges between them):
// number of tables, number of edges, diameter (longest shortest path, in
// edges), largest degree, independent cycles (edges - tables + 1).
__device__ void subplan_shape(const FeatGraph &g, uint64_t m, float out[5]) {
  int ne = 0;
  int deg_max = 0;
  const int nt = __popcll(m);
  for (int e = 0; e < g.n_edges; ++e)
    ne += ((m >> g.u[e]) & (m >> g.v[e]) & 1ull) ? 1 : 0;
  int diam = 0;
  for (uint64_t rest = m; rest; rest &= rest - 1) {
    const int t = __ffsll((long long)rest) - 1;
    int deg = 0;
    for (int e = 0; e < g.n_edges; ++e)
      if ((m >> g.u[e]) & (m >> g.v[e]) & 1ull)
        deg += (g.u[e] == t) + (g.v[e] == t);
    deg_max = deg > deg_max ? deg : deg_max;
    // breadth-first levels from t over the sub-plan's edges
    uint64_t seen = 1ull << t, frontier = seen;
    int depth = 0;
    while (true) {
      uint64_t next = 0;
      for (int e = 0; e < g.n_edges; ++e) {
        if (!((m >> g.u[e]) & (m >> g.v[e]) & 1ull)) continue;
        if ((frontier >> g.u[e]) & 1ull) next |= 1ull << g.v[e];
        if ((frontier >> g.v[e]) & 1ull) next |= 1ull << g.u[e];
      }
      next &= ~seen;
      if (!next) break;
      seen |= next;
      frontier = next;
      ++depth;
    }
    diam = depth > diam ? depth : diam;
  }
  out[0] = (float)nt;
  out[1] = (float)ne;
  out[2] = (float)diam;
  out[3] = (float)deg_max;
  out[4] = (float)(ne - nt + 1);
}

// Sub-plan features: 7 order statistics (positions round(k (d-1) / 6)) of
// slog(X_i) = sign * ln(1 + |X_i|) over the sorted row estimates; log2(1 +
// n_sel) of the sub-plan's tables, descending, first 8, zero padded; the 5
// shape statistics of subplan_shape.  base = ln(1 + max(est, 0)).
__global__ void mlp_features_kernel(const u128 *__restrict__ rows, int32_t d,
                                    const double *__restrict__ est,
                                    const uint64_t *__restrict__ masks,
                                    const int64_t *__restrict__ n_sel,
                                    int32_t n_tables, FeatGraph g,
                                    int32_t n, float *__restrict__ x,
                                    float *__restrict__ base) {
  const int sp = blockIdx.x * blockDim.x + threadIdx.x;
  if (sp >= n) return;
  double v[32];
  for (int i = 0; i < d; ++i) {
    const double r = i128_to_double(rows[(size_t)sp * d + i]);
    v[i] = r;
  }
  for (int a = 1; a < d; ++a) {  // sort ascending (by the exact doubles)
    const double t = v[a];
    int b = a - 1;
    while (b >= 0 && v[b] > t) {
      v[b + 1] = v[b];
      --b;
    }
    v[b + 1] = t;
  }
  float *xo = x + (size_t)sp * 20;
  for (int k = 0; k < 7; ++k) {
    const int pos = (int)((k * (d - 1) + 3) / 6);  // round(k (d-1) / 6)
    const double r = v[pos];
    const double s = r < 0 ? -log1p(-r) : log1p(r);
    xo[k] = (float)s;
  }
  double ls[64];
  int cnt = 0;
  const uint64_t m = masks[sp];
  for (int t = 0; t < n_tables; ++t)
    if ((m >> t) & 1ull) ls[cnt++] = log2(1.0 + (double)n_sel[t]);
  for (int k = 0; k < 8 && k < cnt; ++k) {  // 8 largest, descending
    int best = k;
    for (int j = k + 1; j < cnt; ++j)
      if (ls[j] > ls[best]) best = j;
    const double tmp = ls[k];
    ls[k] = ls[best];
    ls[best] = tmp;
  }
  for (int k = 0; k < 8; ++k) xo[7 + k] = k < cnt ? (float)ls[k] : 0.f;
  float sh[5];
  subplan_shape(g, m, sh);
  for (int k = 0; k < 5; ++k) xo[15 + k] = sh[k];
  const double e = est[sp];
  base[sp] = (float)log1p(e > 0 ? e : 0.0);
}

}  // namespace compass

using namespace compass;

namespace compass {
void set_last_error(const std::string &s);
}

static compass_status mfail(compass_status s, const std::string &m) {
  compass::set_last_error(m);
  return s;
}

#define MHIP(expr)                                                        \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return mfail(COMPASS_E_HIP,                                         \
                   std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

struct compass_mlp_s {
  MlpShape S;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t *wb = nullptr;
  float *act = nullptr, *pre = nullptr, *slab = nullptr, *loss_part = nullptr;
  float *y = nullptr;
  int32_t cap = 0;     // samples the training buffers hold
  int64_t step = 0;
};

extern "C" compass_status compass_mlp_create(int32_t n_in, int32_t hidden,
                                             int32_t n_hidden_layers,
                                             const float *init,
                                             compass_mlp *out) {
  if (!out || !init) return mfail(COMPASS_E_ARG, "null pointer argument");
  if (n_in < 1 || n_in > kMlpMaxDim || hidden < 1 || hidden > kMlpMaxDim ||
      n_hidden_layers < 1 || n_hidden_layers + 1 > kMlpMaxLayers)
    return mfail(COMPASS_E_ARG, "MLP shape outside [1, 64] x [1, 7] layers");
  compass_mlp_s *M = new compass_mlp_s();
  MlpShape &S = M->S;
  memset(&S, 0, sizeof S);
  S.n_layers = n_hidden_layers + 1;
  S.dim[0] = n_in;
  for (int l = 1; l <= n_hidden_layers; ++l) S.dim[l] = hidden;
  S.dim[S.n_layers] = 1;
  int off = 0;
  for (int l = 0; l < S.n_layers; ++l) {
    S.woff[l] = off;
    off += S.dim[l] * S.dim[l + 1];
    S.boff[l] = off;
    off += S.dim[l + 1];
  }
  S.n_params = off;
  const size_t b = sizeof(float) * off;
  auto bad = [&](hipError_t e) {
    if (e != hipSuccess) {
      delete M;
      return true;
    }
    return false;
  };
  if (bad(hipMalloc(&M->p, b)) || bad(hipMalloc(&M->m, b)) ||
      bad(hipMalloc(&M->v, b)) || bad(hipMalloc(&M->g, b)) ||
      bad(hipMalloc(&M->wb, sizeof(uint16_t) * off)))
    return mfail(COMPASS_E_HIP, "hipMalloc failed");
  MHIP(hipMemcpy(M->p, init, b, hipMemcpyHostToDevice));
  MHIP(hipMemset(M->m, 0, b));
  MHIP(hipMemset(M->v, 0, b));
  MHIP(hipMemset(M->g, 0, b));
  hipLaunchKernelGGL(mlp_to_bf16_kernel, dim3((off + 255) / 256), dim3(256), 0,
                     0, M->p, M->wb, off);
  MHIP(hipGetLastError());
  MHIP(hipDeviceSynchronize());
  *out = M;
  return COMPASS_OK;
}

extern "C" int64_t compass_mlp_n_params(compass_mlp M) {
  return M ? M->S.n_params : 0;
}

extern "C" int64_t compass_mlp_adam_steps(compass_mlp M) {
  return M ? (int64_t)M->step : 0;
}

extern "C" compass_status compass_mlp_forward(compass_mlp M, const float *x,
                                              const float *base, int32_t n,
                                              float *y, hipStream_t st) {
  if (!M || (n > 0 && (!x || !base || !y)) || n < 0)
    return mfail(COMPASS_E_ARG, "bad argument");
  if (n == 0) return COMPASS_OK;
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3((n + kMlpTile - 1) / kMlpTile),
                     dim3(kMlpThreads), 0, st, M->S, M->wb, M->p, x, base,
                     (const int32_t *)nullptr, n, y, nullptr, nullptr, 0);
  MHIP(hipGetLastError());
  return COMPASS_OK;
}

// One Adam step on samples idx[0..n) of (x, base, target) (rows 0..n when
// idx is null); grows the activation buffers when n exceeds them.
static compass_status train_batch(compass_mlp M, const float *x,
                                  const float *base, const float *target,
                                  const int32_t *idx, int32_t n, float lr,
                                  float *loss, hipStream_t st) {
  const int blocks = (n + kMlpTile - 1) / kMlpTile;
  if (n > M->cap) {
    (void)hipDeviceSynchronize();
    (void)hipFree(M->act);
    (void)hipFree(M->pre);
    (void)hipFree(M->slab);
    (void)hipFree(M->loss_part);
    (void)hipFree(M->y);
    M->act = M->pre = M->slab = M->loss_part = M->y = nullptr;
    const size_t per = (size_t)M->S.n_layers * n * kMlpMaxDim * sizeof(float);
    MHIP(hipMalloc(&M->act, per));
    MHIP(hipMalloc(&M->pre, per));
    MHIP(hipMalloc(&M->slab, (size_t)blocks * M->S.n_params * sizeof(float)));
    MHIP(hipMalloc(&M->loss_part, (size_t)blocks * sizeof(float)));
    MHIP(hipMalloc(&M->y, (size_t)n * sizeof(float)));
    M->cap = n;
  }
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3(blocks), dim3(kMlpThreads), 0, st,
                     M->S, M->wb, M->p, x, base, idx, n, M->y, M->act, M->pre, 1);
  hipLaunchKernelGGL(mlp_bwd_kernel, dim3(blocks), dim3(kMlpThreads), 0, st,
                     M->S, M->wb, M->y, target, idx, n, M->act, M->pre, M->slab,
                     M->loss_part);
  const int np = M->S.n_params;
  if (lr > 0.f) M->step += 1;  // a gradient-only call is not an Adam step
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)M->step);
  const float c2 = 1.f - powf(b2, (float)M->step);
  hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((np + 255) / 256), dim3(256),
                     0, st, M->slab, blocks, np, M->g, M->loss_part, loss,
                     1.f / (float)n, lr > 0.f ? 1 : 0, M->p, M->m, M->v, M->wb,
                     lr, b1, b2, 1e-8f, c1, c2);
  MHIP(hipGetLastError());
  return COMPASS_OK;
}

extern "C" compass_status compass_mlp_train_step(compass_mlp M, const float *x,
                                                 const float *base,
                                                 const float *target, int32_t n,
                                                 float lr, float *loss,
                                                 hipStream_t st) {
  if (!M || !x || !base || !target || n < 1)
    return mfail(COMPASS_E_ARG, "bad argument");
  return train_batch(M, x, base, target, nullptr, n, lr, loss, st);
}

extern "C" compass_status compass_mlp_train_epoch(
    compass_mlp M, const float *x, const float *base, const float *target,
    const int32_t *idx, int32_t n_batches, int32_t batch, float lr,
    float *losses, hipStream_t st) {
  if (!M || !x || !base || !target || !idx || !losses || n_batches < 0 ||
      batch < 1 || lr <= 0.f)
    return mfail(COMPASS_E_ARG, "bad argument");
  for (int32_t k = 0; k < n_batches; ++k) {
    const compass_status s = train_batch(M, x, base, target,
                                         idx + (int64_t)k * batch, batch, lr,
                                         losses + k, st);
    if (s != COMPASS_OK) return s;
  }
  return COMPASS_OK;
}

// what: 0 parameters, 1 last gradients, 2 Adam first moments, 3 second
extern "C" compass_status compass_mlp_read(compass_mlp M, int32_t what,
                                           float *host_out) {
  if (!M || !host_out || what < 0 || what > 3)
    return mfail(COMPASS_E_ARG, "bad argument");
  const float *src = what == 0 ? M->p : what == 1 ? M->g : what == 2 ? M->m : M->v;
  MHIP(hipDeviceSynchronize());
  MHIP(hipMemcpy(host_out, src, sizeof(float) * M->S.n_params,
                 hipMemcpyDeviceToHost));
  return COMPASS_OK;
}

extern "C" compass_status compass_mlp_write(compass_mlp M, const float *params,
                                            const float *adam_m,
                                            const float *adam_v, int64_t step) {
  if (!M || !params) return mfail(COMPASS_E_ARG, "bad argument");
  const size_t b = sizeof(float) * M->S.n_params;
  MHIP(hipDeviceSynchronize());
  MHIP(hipMemcpy(M->p, params, b, hipMemcpyHostToDevice));
  if (adam_m) MHIP(hipMemcpy(M->m, adam_m, b, hipMemcpyHostToDevice));
  if (adam_v) MHIP(hipMemcpy(M->v, adam_v, b, hipMemcpyHostToDevice));
  M->step = step;
  hipLaunchKernelGGL(mlp_to_bf16_kernel, dim3((M->S.n_params + 255) / 256),
                     dim3(256), 0, 0, M->p, M->wb, M->S.n_params);
  MHIP(hipGetLastError());
  MHIP(hipDeviceSynchronize());
  return COMPASS_OK;
}

extern "C" compass_status compass_mlp_destroy(compass_mlp M) {
  if (!M) return COMPASS_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(M->p);
  (void)hipFree(M->m);
  (void)hipFree(M->v);
  (void)hipFree(M->g);
  (void)hipFree(M->wb);
  (void)hipFree(M->act);
  (void)hipFree(M->pre);
  (void)hipFree(M->slab);
  (void)hipFree(M->loss_part);
  (void)hipFree(M->y);
  delete M;
  return COMPASS_OK;
}

extern "C" compass_status compass_mlp_features(
    const compass_i128 *row_est, int32_t d, const double *est,
    const uint64_t *masks, const int64_t *n_selected, int32_t n_tables,
    int32_t n_edges, const int32_t *edge_u, const int32_t *edge_v, int32_t n,
    float *x, float *base, hipStream_t st) {
  if (n < 0 || d < 1 || d > 32 || n_tables < 1 || n_tables > 64 ||
      n_edges < 0 || n_edges > 64)
    return mfail(COMPASS_E_ARG, "bad feature arguments");
  if (n_edges > 0 && (!edge_u || !edge_v))
    return mfail(COMPASS_E_ARG, "null edge array");
  FeatGraph g;
  memset(&g, 0, sizeof g);
  g.n_edges = n_edges;
  for (int e = 0; e < n_edges; ++e) {
    if (edge_u[e] < 0 || edge_u[e] >= n_tables || edge_v[e] < 0 ||
        edge_v[e] >= n_tables || edge_u[e] == edge_v[e])
      return mfail(COMPASS_E_GRAPH, "edge with bad endpoints");
    g.u[e] = (uint8_t)edge_u[e];
    g.v[e] = (uint8_t)edge_v[e];
  }
  if (n == 0) return COMPASS_OK;
  if (!row_est || !est || !masks || !n_selected || !x || !base)
    return mfail(COMPASS_E_ARG, "null pointer argument");
  hipLaunchKernelGGL(mlp_features_kernel, dim3((n + 127) / 128), dim3(128), 0, st,
                     reinterpret_cast<const u128 *>(row_est), d, est, masks,
                     n_selected, n_tables, g, n, x, base);
  MHIP(hipGetLastError());
  return COMPASS_OK;
}
