// generic.hip -- contraction of any connected sub-plan (gfx950).
//
// What is computed (Section 5.1 contraction with the Section 5.2 min-abs
// merge, applied to any number of joins): for sketch row i,
//   X_i = sum over bucket assignments of the sub-plan's edges of the
//         product over its tables of the table's merged counter,
// the merged counter being the incident bucket of smallest |value| (ties
// to the lower edge id).  The triangle-specialised path covers trees plus
// one triangle; this one covers every shape: the edges outside a spanning
// tree are conditioned (their bucket fixed, J), the tree is contracted
// bottom-up for every assignment J, and the w^k results are added.
//
// Contraction of one node.  Its elements are the parent edge's buckets
// (queries), each child edge's buckets weighted by the child's message, and
// one element per conditioned edge at the node (weight 1).  In the order
// kappa = (|value|, edge id, bucket), the merged value of a choice is its
// first element, so
//   M(q) = value(q) * prod_g W_g(after q) + B(q),
//   B(q) = sum over weighted elements z before q of
//          value(z) * weight(z) * prod_{g != group(z)} W_g(after z),
// with W_g(after k) = the weight of group g's elements after k.  One
// workgroup merges the node's lists into kappa order (the sort kernels'
// per-side keys, merged by binary searches), then walks the merged list
// tile by tile; block scans give the per-group prefix weights and the
// prefix of the terms.
//
// The arithmetic is a template parameter: 128-bit two's complement (the
// exact row values of shapes the fast path does not evaluate) or double
// (an approximate evaluation of sub-plans whose 128-bit values cannot be
// certified).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "certificate.hpp"
#include "device_math.hpp"
#include "estimate_buffers.hpp"
#include "estimate_params.hpp"
#include "generic_params.hpp"

namespace compass {


template <typename T>
struct Ar;

template <>
struct Ar<u128> {
  static __device__ __forceinline__ u128 of(int64_t v) { return s64_to_u128(v); }
  static __device__ __forceinline__ u128 mul(u128 a, u128 b) { return mul_u128(a, b); }
  static __device__ __forceinline__ u128 up(u128 v, int off) {
    const uint64_t lo = __shfl_up((unsigned long long)(uint64_t)v, off, 64);
    const uint64_t hi = __shfl_up((unsigned long long)(uint64_t)(v >> 64), off, 64);
    return ((u128)hi << 64) | lo;
  }
};

template <>
struct Ar<double> {
  static __device__ __forceinline__ double of(int64_t v) { return (double)v; }
  static __device__ __forceinline__ double mul(double a, double b) { return a * b; }
  static __device__ __forceinline__ double up(double v, int off) {
    return __shfl_up(v, off, 64);
  }
};

__device__ __forceinline__ int64_t gen_counter(const EstBuffers &B, int side,
                                               int row, int j) {
  const size_t idx = (size_t)row * B.w + j;
  if (B.counter_bits == 32)
    return reinterpret_cast<const int32_t *>(B.sides[side])[idx];
  return reinterpret_cast<const int64_t *>(B.sides[side])[idx];
}

__device__ __forceinline__ uint64_t uabs64(int64_t v) {
  return v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
}

// kappa order: (|value|, edge id, bucket)
__device__ __forceinline__ bool kappa_less(uint64_t av, int ae, int aj,
                                           uint64_t bv, int be, int bj) {
  if (av != bv) return av < bv;
  if (ae != be) return ae < be;
  return aj < bj;
}

// number of keys (|v| << 16 | j, ascending) below thr
__device__ __forceinline__ int gen_lower_bound(const uint64_t *a, int n,
                                               uint64_t thr) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < thr) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Merged kappa order of one node's lists, written by the workgroup: element
// i of list a (the side's sorted keys, ascending |v| then bucket) lands at
// i plus, for every other list b of the node, the number of b's elements
// of smaller kappa (|v_b| < |v|, or |v_b| == |v| with b's edge id below
// a's).
__device__ void gen_merge_node(const EstBuffers &B, const GenNode &N, int row,
                               uint32_t *list) {
  const int w = B.w;
  const int nl = N.n_child + (N.parent_side >= 0 ? 1 : 0);
  for (int idx = threadIdx.x; idx < nl * w; idx += blockDim.x) {
    const int a = idx / w, i = idx - a * w;
    const bool par = a == N.n_child;
    const int side = par ? N.parent_side : N.c_side[a];
    const int eid = par ? N.parent_eid : N.c_eid[a];
    const uint32_t code = par ? kGenQuery : (uint32_t)a;
    const uint64_t key = B.sorted[((size_t)side * B.d + row) * w + i];
    const uint64_t av = key >> 16;
    int pos = i;
    for (int b = 0; b < nl; ++b) {
      if (b == a) continue;
      const bool pb = b == N.n_child;
      const int sb = pb ? N.parent_side : N.c_side[b];
      const int eb = pb ? N.parent_eid : N.c_eid[b];
      const uint64_t *kb = B.sorted + ((size_t)sb * B.d + row) * w;
      pos += gen_lower_bound(kb, w, (av + (eb < eid ? 1 : 0)) << 16);
    }
    list[pos] = (code << 16) | (uint32_t)(key & 0xFFFFu);
  }
}

// inclusive scan over the workgroup (kGenThreads lanes); returns the
// prefix and the total; wsum: 4 values of LDS
template <typename T>
__device__ __forceinline__ T gen_block_scan(T x, T *wsum, T &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = Ar<T>::up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kGenThreads / 64; ++k) {
    if (k < wave) before += wsum[k];
    all += wsum[k];
  }
  __syncthreads();
  total = all;
  return x + before;
}

// One node for one assignment J (digits in s_J).  Writes the node's
// message (non-root) and its total to s_tot[msg], or returns the root's
// value (thread 0).
template <typename T>
__device__ T gen_node(const GenArgs &A, const EstBuffers &B, const GenNode &N,
                      const uint32_t *list, T *msgs, int row,
                      const int64_t *s_J, T *s_tot, T *s_wsum, T *s_fterm,
                      T (*s_fP)[kGenMaxGroups], int *s_fpos, int64_t *s_fv,
                      int *s_fdone) {
  const int w = B.w;
  const int L = N.list_len;
  const int nc = N.n_child, nf = N.n_fixed;
  // conditioned elements: value, and their position among the list's
  // elements (number of elements of smaller kappa)
  if ((int)threadIdx.x < nf) {
    const int f = threadIdx.x;
    const int jf = (int)s_J[N.f_cut[f]];
    const int64_t v = gen_counter(B, N.f_side[f], row, jf);
    const uint64_t av = uabs64(v);
    const int ef = N.f_eid[f];
    int lo = 0, hi = L;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const uint32_t code = list[mid] >> 16;
      const int jm = (int)(list[mid] & 0xFFFFu);
      const int side = code == kGenQuery ? N.parent_side : N.c_side[code];
      const int em = code == kGenQuery ? N.parent_eid : N.c_eid[code];
      if (kappa_less(uabs64(gen_counter(B, side, row, jm)), em, jm, av, ef, jf))
        lo = mid + 1;
      else
        hi = mid;
    }
    s_fpos[f] = lo;
    s_fv[f] = v;
    s_fdone[f] = 0;
  }
  __syncthreads();
  T tot[kGenMaxGroups];
  T carry[kGenMaxGroups];
#pragma unroll
  for (int g = 0; g < kGenMaxGroups; ++g) {
    tot[g] = g < nc ? s_tot[N.c_msg[g]] : (T)0;
    carry[g] = 0;
  }
  T carry_below = 0;
  T msg_total = 0;
  // the conditioned element f's own kappa against f2's
  auto f_before = [&](int f2, int f) {
    const uint64_t a2 = uabs64(s_fv[f2]), a = uabs64(s_fv[f]);
    return kappa_less(a2, N.f_eid[f2], (int)s_J[N.f_cut[f2]], a, N.f_eid[f],
                      (int)s_J[N.f_cut[f]]);
  };
  for (int b0 = 0; b0 < L; b0 += kGenThreads) {
    const int e = b0 + threadIdx.x;
    const bool in = e < L;
    int code = kGenQuery, j = 0;
    int64_t v = 0;
    T wt = 0;
    if (in) {
      const uint32_t c = list[e];
      code = (int)(c >> 16);
      j = (int)(c & 0xFFFFu);
      const int side = code == kGenQuery ? N.parent_side : N.c_side[code];
      v = gen_counter(B, side, row, j);
      if (code != (int)kGenQuery) wt = msgs[(size_t)N.c_msg[code] * w + j];
    }
    // prefix weight of every child group up to and including e
    T P[kGenMaxGroups];
#pragma unroll
    for (int g = 0; g < kGenMaxGroups; ++g) {
      if (g >= nc) {
        P[g] = 0;
        continue;
      }
      T tg;
      const T s = gen_block_scan<T>(in && code == g ? wt : (T)0, s_wsum, tg);
      P[g] = carry[g] + s;
      carry[g] += tg;
    }
    // conditioned elements that rank inside this tile (position p in
    // [b0, b0 + tile)): the child groups' weights before p ...
    for (int f = 0; f < nf; ++f) {
      const int p = s_fpos[f];
      if (p < b0 || p >= b0 + kGenThreads) continue;
      if (p == b0) {
        if (threadIdx.x == 0) {
          // weights before the tile: lane 0's inclusive prefix minus its
          // own weight
          for (int g = 0; g < nc; ++g)
            s_fP[f][g] = P[g] - (in && code == g ? wt : (T)0);
        }
      } else if (e == p - 1) {
        for (int g = 0; g < nc; ++g) s_fP[f][g] = P[g];
      }
    }
    __syncthreads();
    // ... and their terms
    if ((int)threadIdx.x < nf) {
      const int f = threadIdx.x;
      const int p = s_fpos[f];
      if (p >= b0 && p < b0 + kGenThreads) {
        T term = Ar<T>::of(s_fv[f]);
        for (int g = 0; g < nc; ++g) term = Ar<T>::mul(term, tot[g] - s_fP[f][g]);
        for (int f2 = 0; f2 < nf; ++f2)
          if (f2 != f && f_before(f2, f)) term = 0;
        s_fterm[f] = term;
        s_fdone[f] = 1;
      }
    }
    __syncthreads();
    // this element's factors: every child group's weight after it, and the
    // conditioned elements after it (weight 1) or before it (weight 0)
    bool fixed_after = true;
    T fixed_below = 0;
    for (int f = 0; f < nf; ++f) {
      const int p = s_fpos[f];
      if (p <= e) {
        fixed_after = false;
        if (p >= b0) fixed_below += s_fterm[f];
      }
    }
    T term = 0, prod = 0;
    if (in) {
      if (code == (int)kGenQuery) {
        prod = Ar<T>::of(v);
        for (int g = 0; g < nc; ++g) prod = Ar<T>::mul(prod, tot[g] - P[g]);
        if (!fixed_after) prod = 0;
      } else {
        term = Ar<T>::mul(Ar<T>::of(v), wt);
        for (int g = 0; g < nc; ++g)
          if (g != code) term = Ar<T>::mul(term, tot[g] - P[g]);
        if (!fixed_after) term = 0;
      }
    }
    T tile_terms;
    const T incl = gen_block_scan<T>(term, s_wsum, tile_terms);
    const T below = carry_below + (incl - term) + fixed_below;
    if (in && code == (int)kGenQuery) {
      const T m = prod + below;
      msgs[(size_t)N.msg * w + j] = m;
      msg_total += m;
    }
    // carry: this tile's terms and the conditioned terms placed in it
    T fixed_tile = 0;
    for (int f = 0; f < nf; ++f) {
      const int p = s_fpos[f];
      if (p >= b0 && p < b0 + kGenThreads) fixed_tile += s_fterm[f];
    }
    carry_below += tile_terms + fixed_tile;
  }
  // conditioned elements after every list element that no tile held
  // (position L at a tile boundary)
  __syncthreads();
  if ((int)threadIdx.x < nf) {
    const int f = threadIdx.x;
    if (!s_fdone[f]) {
      T term = Ar<T>::of(s_fv[f]);
      for (int g = 0; g < nc; ++g) term = Ar<T>::mul(term, tot[g] - carry[g]);
      for (int f2 = 0; f2 < nf; ++f2)
        if (f2 != f && f_before(f2, f)) term = 0;
      s_fterm[f] = term;
      s_fdone[f] = 2;
    }
  }
  __syncthreads();
  for (int f = 0; f < nf; ++f)
    if (s_fdone[f] == 2) carry_below += s_fterm[f];
  if (N.parent_side >= 0) {
    T t;
    (void)gen_block_scan<T>(msg_total, s_wsum, t);
    if (threadIdx.x == 0) s_tot[N.msg] = t;
    __syncthreads();
    return 0;
  }
  return carry_below;
}

// One workgroup per (plan, J block, row): every assignment J of the block,
// the plan's nodes bottom-up; the block's sum of root values to its slot.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void gen_contract_kernel(GenArgs A,
                                                                  EstBuffers B) {
  __shared__ T s_tot[64];
  __shared__ T s_wsum[kGenThreads / 64];
  __shared__ T s_fterm[kGenMaxGroups];
  __shared__ T s_fP[kGenMaxGroups][kGenMaxGroups];
  __shared__ int s_fpos[kGenMaxGroups];
  __shared__ int64_t s_fv[kGenMaxGroups];
  __shared__ int s_fdone[kGenMaxGroups];
  __shared__ int64_t s_J[kGenMaxCut];
  const GenBlock blk = A.blocks[blockIdx.x];
  const GenPlan P = A.plans[blk.plan];
  const int row = blockIdx.y;
  const int w = B.w;
  if (P.fp64 && subplan_certified(A.sps[P.sp], B.n_sel, A.n_tables, w)) return;
  const int64_t per = (P.n_assign + P.n_blocks - 1) / P.n_blocks;
  const int64_t J0 = (int64_t)blk.jb * per;
  const int64_t J1 = J0 + per < P.n_assign ? J0 + per : P.n_assign;
  uint32_t *list = A.lists + P.lists_off +
                   ((size_t)row * P.n_blocks + blk.jb) * (size_t)P.lists_len;
  T *msgs = reinterpret_cast<T *>(A.msg) +
            (size_t)P.msg_off +
            ((size_t)row * P.n_blocks + blk.jb) * (size_t)P.n_msgs * w;
  // every node's lists in kappa order (this block's own copy)
  for (int k = 0; k < P.n_nodes; ++k) {
    const GenNode &N = A.nodes[P.node0 + k];
    gen_merge_node(B, N, row, list + N.list_off);
  }
  __syncthreads();
  T acc = 0;
  for (int64_t J = J0; J < J1; ++J) {
    if (threadIdx.x == 0) {
      int64_t r = J;
      for (int k = 0; k < P.n_cut; ++k) {
        s_J[k] = r % w;
        r /= w;
      }
    }
    __syncthreads();
    for (int k = 0; k < P.n_nodes; ++k) {
      const GenNode &N = A.nodes[P.node0 + k];
      if (N.is_static && J != J0) continue;  // its message does not depend on J
      const T r = gen_node<T>(A, B, N, list + N.list_off, msgs, row, s_J, s_tot,
                              s_wsum, s_fterm, s_fP, s_fpos, s_fv, s_fdone);
      if (N.parent_side < 0) acc += r;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const size_t slot = ((size_t)P.out_slot + blk.jb) * B.d + row;
    if (P.fp64)
      A.approx[slot] = (double)acc;
    else
      A.partial[slot] = (u128)acc;
  }
}

hipError_t launch_gen_contract(const GenArgs &A, const EstBuffers &B,
                               int n_blocks, int fp64, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(gen_contract_kernel<double>, dim3(n_blocks, B.d),
                       dim3(kGenThreads), 0, st, A, B);
  else
    hipLaunchKernelGGL(gen_contract_kernel<u128>, dim3(n_blocks, B.d),
                       dim3(kGenThreads), 0, st, A, B);
  return hipGetLastError();
}

}  // namespace compass
