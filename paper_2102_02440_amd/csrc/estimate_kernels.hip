// estimate_kernels.hip -- merged-sketch join-size estimates on gfx950.
//
// What is computed (Section 4.2.1 two-way estimate and median; Section 5.1
// contraction; Section 5.2 min-abs sketch merging, generalised iteratively):
// for a connected sub-plan C and sketch row i,
//   X_i = sum over bucket assignments iota of C's induced edges of
//         prod over tables t in C of merged_t(iota),
// merged_t = the incident bucket of smallest |value|, ties to the lower
// edge id.  X_i is exact modulo 2^128.
//
// How (our exact re-association of that sum, never materialising tensors):
// order every bucket element of a table by kappa = (|value|, edge id); the
// merged value is the element of smallest kappa.  On a rooted spanning tree
// the message of table t to its parent for parent bucket j is
//   M(j) = x_j * prod_c A_c(kappa_j) + G(kappa_j)
// with A_c(k) = sum of child-c message values over child-c elements of
// kappa > k and G(k) = sum over child elements z of kappa < k of
// v_z * mu_z * prod_{c' != c(z)} A_c'(kappa_z).  A node therefore needs its
// incident bucket lists merged by kappa and two scans over the merged list.
//
// Kernels:
//  sort_rows_kernel    the w buckets of each (sketch, row) sorted by
//                      (|v|, j): an LSD radix sort in LDS, one workgroup a
//                      row (its trailing workgroups resolve the guards);
//  node_merge_kernel   k-way merge of a node's sorted lists by rank (binary
//                      search), many workgroups per (tree node, row);
//  node_kernel         one workgroup per (tree node, row): block-wide scans
//                      of 128-bit A and G over the merged records, emitting
//                      the node's message (or the root's X);
//  node1_*             nodes with one child (prefix sums + binary search);
//  apex_prep_kernel, tri_order_kernel (with the segment bounds),
//  tri_fast_kernel     two-child triangle apexes: run-ordered sweeps by
//                      binary search, several sub-plans per workgroup;
//  tri_lane_kernel     other triangles: one lane per bucket J of the cut edge.
//                      Fixing J turns each cut endpoint's message into
//                      "M(j) if its parent-edge element ranks below the
//                      fixed element, else the constant C(J)", so every
//                      lane streams the apex's merged list (wave-uniform
//                      scalar loads) with O(1) state.
//  finish_kernel       per sub-plan: gathers X_i, median over rows,
//                      round-to-nearest-even double, exactness certificate.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_math.hpp"
#include "estimate_params.hpp"
#include "estimate_buffers.hpp"
#include "certificate.hpp"
#include "lds_stage.hpp"
#include "bitonic.hpp"

namespace compass {



__device__ __forceinline__ int64_t counter_at(const EstBuffers &B, int side,
                                              int row, int j) {
  const size_t idx = (size_t)row * B.w + j;
  if (B.counter_bits == 32)
    return reinterpret_cast<const int32_t *>(B.sides[side])[idx];
  return reinterpret_cast<const int64_t *>(B.sides[side])[idx];
}

__device__ __forceinline__ const uint64_t *sorted_of(const EstBuffers &B,
                                                     int side, int row) {
  return B.sorted + ((size_t)side * B.d + row) * B.w;
}

__device__ __forceinline__ u128 *msg_of(const EstBuffers &B, int slot,
                                        int row) {
  return B.msg + ((size_t)slot * B.d + row) * B.w;
}

// A child's message (or cut constant) at bucket j: slot >= 0 is a computed
// message array; a leaf's message is its own counter on that edge, read in
// place (slot = -1 - side).
__device__ __forceinline__ u128 child_msg_at(const EstBuffers &B, int slot,
                                             int row, int j) {
  if (slot >= 0) return msg_of(B, slot, row)[j];
  return s64_to_u128(counter_at(B, -1 - slot, row, j));
}

// number of keys < thr in a sorted array
__device__ __forceinline__ int lower_bound_u64(const uint64_t *a, int n,
                                               uint64_t thr) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < thr)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Whether this rooting of a sub-plan is the one that runs: among the
// planned candidates, the one whose table has the fewest selected rows
// (ties: the earlier candidate).
__device__ __forceinline__ bool guard_on(int n, int self, int t0, int t1,
                                         int t2, const int64_t *n_sel) {
  if (n <= 1) return true;
  const int tab[3] = {t0, t1, t2};
  int best = 0;
  int64_t nb = n_sel[t0];
  for (int k = 1; k < n; ++k) {
    const int64_t v = n_sel[tab[k]];
    if (v < nb) {
      nb = v;
      best = k;
    }
  }
  return best == self;
}
#define COMPASS_GUARD_ON(G, NSEL) \
  guard_on((G).n, (G).self, (G).tab[0], (G).tab[1], (G).tab[2], (NSEL))

// Workgroup placement.  A launch covers Q = tasks x sketch rows (task, row)
// pairs of X chunks each, on a 1-D grid; workgroups go to the 8 XCDs in
// turn by linear id and every XCD has its own L2.  xcd = 1 (Q >= 8): the
// grid has 8 X ceil(Q / 8) workgroups and all chunks of pair q run on XCD
// q % 8, so that data they share (a staged sorted row, a list the chunks
// gather from) stays in one L2; xcd = 0: chunk-major (X Q workgroups, a
// pair's chunks spread over every XCD).
struct GridMap {
  int32_t X, Q, d, xcd;
};
struct GridPos {
  int c, row, task;
  bool ok;
};
__device__ __forceinline__ GridPos grid_pos(const GridMap &m) {
  GridPos g;
  const int i = blockIdx.x;
  int q;
  if (m.xcd) {
    const int k = i >> 3;
    q = (i & 7) + 8 * (k / m.X);
    g.c = k % m.X;
  } else {
    q = i / m.X;
    g.c = i % m.X;
  }
  g.ok = q < m.Q;
  g.row = q % m.d;
  g.task = q / m.d;
  return g;
}

// |v| saturated below 2^47 (every sketch built from < 2^47 rows satisfies
// this; saturation only keeps sort keys well-formed for foreign input)
__device__ __forceinline__ uint64_t abs_u64(int64_t v) {
  const uint64_t a = v < 0 ? 0ull - (uint64_t)v : (uint64_t)v;
  return a < (1ull << 47) ? a : (1ull << 47) - 1;
}

// ---------------------------------------------------------------------
// sort of each (sketch side, row) by (|v|, j): grid (n_jobs, d, chunks);
// jobs[blockIdx.x / d] = sketch side, blockIdx.x % d = row
// ---------------------------------------------------------------------
// sort_rows_kernel: one workgroup per (sketch side, row) sorts the row's w
// keys (|v| << 16 | j) ascending: an LSD radix sort on |v|, four bits a
// pass, as many passes as the row's largest |v| needs.  The keys start in
// j order and every pass is stable, so equal |v| stay in j order, which is
// the order of the full keys.  Thread t holds the consecutive keys
// [t kpt, (t + 1) kpt) (kpt = ceil(w / kSortThreads)), so thread order is
// key order.  A pass: each thread counts its keys per digit (4-bit fields
// of one 64-bit word), the counts are scanned over the workgroup (16-bit
// fields, two per 32-bit word, wave scans by DPP row shifts and
// broadcasts, then over the waves), and each key goes to its digit's base
// plus the count of equal digits before it.
__device__ void resolve_task(const ResolveArgs &R, int i, const EstBuffers &B);

// inclusive scan over the 64 lanes of a wave (32-bit words of two 16-bit
// fields that never carry into each other)
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr 1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr 2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr 4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr 8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast 15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast 31
  return x;
}

// 4-bit digit counts (one nibble per digit) -> word k = count(2k) | count(2k+1) << 16
__device__ __forceinline__ uint32_t nibbles_to_word(uint64_t c, int k) {
  const uint32_t b = (uint32_t)(c >> (8 * k)) & 0xFFu;  // digits 2k, 2k + 1
  return (b & 0xFu) | ((b >> 4) << 16);
}

// The guard resolution (resolve_task) rides along as the last R.blocks
// workgroups, which need none of the sort: its dependent loads then
// overlap the sort instead of adding a launch.
template <int KPT>  // keys per thread at most (8 or kSortKpt)
__global__ __launch_bounds__(kSortThreads) void sort_rows_kernel(
    const SortJob *jobs, EstBuffers B, int n_pairs, ResolveArgs R) {
  if ((int)blockIdx.x >= n_pairs) {
    resolve_task(R, ((int)blockIdx.x - n_pairs) * kSortThreads + (int)threadIdx.x, B);
    return;
  }
  // LDS: the keys by position, one pad entry after every 16 so that the
  // threads' consecutive runs of keys fall on different banks, then the
  // digit starts of the pass (16-bit, two digits a word, [word][thread];
  // before the first pass: the wave maxima), then the scan's scratch and
  // the waves' digit bases.  The largest rows (KPT = 16) fill the LDS with
  // the keys unpadded and the starts; their scratch and bases take the
  // keys' space before each scatter.
  extern __shared__ __align__(16) uint64_t sk[];
  constexpr int kWaves = kSortThreads / 64;
  const int w = B.w;
  const int kpt = (w + kSortThreads - 1) / kSortThreads;  // uniform, <= KPT
  constexpr bool kPad = KPT <= 8;  // also: the scan scratch after the starts
  const int nsk = kpt * kSortThreads + (kPad ? kpt * kSortThreads / 16 : 0);
  uint32_t *runtab = reinterpret_cast<uint32_t *>(sk + nsk);  // [8][threads]
  auto at = [](int p) { return kPad ? p + (p >> 4) : p; };
  uint32_t *scr = kPad ? runtab + 8 * kSortThreads
                       : reinterpret_cast<uint32_t *>(sk);  // [kWaves][8]
  uint32_t *wbase = scr + kWaves * 8;                       // [kWaves][8]
  const SortJob &job = jobs[blockIdx.x / B.d];
  const int side = job.side;
  const int row = (int)blockIdx.x % B.d;
  const int t = (int)threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int p0 = t * kpt;
  uint64_t key[KPT];
  uint64_t mx = 0;
  {
    // the row's keys, loaded coalesced (all of a lane's loads in flight
    // together) into LDS, then each thread's consecutive run from there
    int64_t v[KPT];
    const size_t rb = (size_t)row * w;
    if (B.counter_bits == 32) {
      const int32_t *src = reinterpret_cast<const int32_t *>(job.counters) + rb;
#pragma unroll
      for (int i = 0; i < KPT; ++i) {
        const int j = t + i * kSortThreads;
        v[i] = j < w ? src[j] : 0;
      }
    } else {
      const int64_t *src = reinterpret_cast<const int64_t *>(job.counters) + rb;
#pragma unroll
      for (int i = 0; i < KPT; ++i) {
        const int j = t + i * kSortThreads;
        v[i] = j < w ? src[j] : 0;
      }
    }
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int j = t + i * kSortThreads;
      const uint64_t a = abs_u64(v[i]);
      if (j < w) sk[at(j)] = (a << 16) | (uint64_t)(uint32_t)j;
      mx = a > mx ? a : mx;
    }
  }
  // passes: the bits of the row's largest |v|, four at a time
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  uint64_t *wmax = reinterpret_cast<uint64_t *>(runtab);  // free until a pass
  if (lane == 0) wmax[wave] = mx;
  __syncthreads();
  mx = 0;
  for (int k = 0; k < kWaves; ++k) mx = wmax[k] > mx ? wmax[k] : mx;
#pragma unroll
  for (int i = 0; i < KPT; ++i)
    if (i < kpt && p0 + i < w) key[i] = sk[at(p0 + i)];
  const int bits = mx ? 64 - __builtin_clzll(mx) : 0;
  const int passes = (bits + 3) / 4;
  for (int pass = 0; pass < passes; ++pass) {
    const int sh = 16 + 4 * pass;
    // my keys' digit counts (at most 8 keys a nibble word)
    uint64_t ca = 0, cb = 0;
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      if (i >= kpt || p0 + i >= w) continue;
      const uint64_t inc = 1ull << (4 * (int)((key[i] >> sh) & 15));
      if (i < 8) ca += inc; else cb += inc;
    }
    // scan of the counts over the workgroup: 8 words of two digits
    uint32_t cnt[8], incl[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cnt[k] = nibbles_to_word(ca, k) + (KPT > 8 ? nibbles_to_word(cb, k) : 0u);
      incl[k] = wave_scan_incl(cnt[k]);
    }
    if (!kPad) __syncthreads();  // the previous pass's reads of sk are done
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < 8; ++k) scr[wave * 8 + k] = incl[k];
    }
    __syncthreads();
    if (wave == 0) {  // uniform
      // lane q < kWaves: wave q's totals; per word the earlier waves'
      // counts, the workgroup totals and the digit bases (exclusive prefix
      // of the totals over the 16 digits), summed into each wave's base
      uint32_t run = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t x = lane < kWaves ? scr[lane * 8 + k] : 0u;
        const uint32_t wi = wave_scan_incl(x);
        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)wi, kWaves - 1);
        const uint32_t lo = b & 0xFFFFu, hi = b >> 16;
        const uint32_t basew = run | ((run + lo) << 16);
        run += lo + hi;
        if (lane < kWaves) wbase[lane * 8 + k] = basew + wi - x;
      }
    }
    __syncthreads();
    // my first position per digit
#pragma unroll
    for (int k = 0; k < 8; ++k)
      runtab[k * kSortThreads + t] = wbase[wave * 8 + k] + incl[k] - cnt[k];
    if (!kPad) __syncthreads();  // the bases (in the keys' space) are read
    // scatter: digit start + equal digits earlier in my keys
    const uint16_t *start16 = reinterpret_cast<const uint16_t *>(runtab);
    uint64_t seen = 0;  // running nibble counts (the last increment may carry)
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      if (i >= kpt || p0 + i >= w) continue;
      const int dg = (int)((key[i] >> sh) & 15);
      const int pos = (int)start16[((dg >> 1) * kSortThreads + t) * 2 + (dg & 1)] +
                      (int)((seen >> (4 * dg)) & 15);
      seen += 1ull << (4 * dg);
      sk[at(pos)] = key[i];
    }
    __syncthreads();
    if (pass + 1 < passes) {
#pragma unroll
      for (int i = 0; i < KPT; ++i)
        if (i < kpt && p0 + i < w) key[i] = sk[at(p0 + i)];
    }
  }
  // the sorted row (in LDS by position: the loads' order when no pass ran),
  // stored coalesced
  uint64_t *out = const_cast<uint64_t *>(sorted_of(B, side, row));
#pragma unroll
  for (int i = 0; i < KPT; ++i) {
    const int j = t + i * kSortThreads;
    if (j < w) out[j] = sk[at(j)];
  }
}

// ---------------------------------------------------------------------
// block scans over kNodeThreads 128-bit values
// ---------------------------------------------------------------------
__device__ u128 block_scan_incl(u128 v, u128 *sh, bool suffix) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kNodeThreads; off <<= 1) {
    u128 add = 0;
    if (suffix) {
      if (t + off < kNodeThreads) add = sh[t + off];
    } else {
      if (t >= off) add = sh[t - off];
    }
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const u128 r = sh[t];
  __syncthreads();
  return r;
}

struct ListRef {
  int side;
  int eid;
};

// list a of a node (a may differ across lanes: read through global memory
// rather than indexing a register copy of the task)
__device__ __forceinline__ ListRef list_of(const NodeTask *T, int a) {
  ListRef r;
  if (a < T->m) {
    r.side = T->child_side[a];
    r.eid = T->child_eid[a];
  } else if (a == T->m && T->parent_side >= 0) {
    r.side = T->parent_side;
    r.eid = T->parent_eid;
  } else {
    r.side = T->cut_side;
    r.eid = T->cut_eid;
  }
  return r;
}

// ---------------------------------------------------------------------
// merge of a node's lists (nodes with two or more children): grid
// (tasks, d, chunks of kMergeChunk elements), kMergeThreads lanes
// ---------------------------------------------------------------------
// k-way merge by rank: the position of an element is its index in its own
// list plus the number of elements of smaller kappa in every other list
// (ties in |v| go to the lower edge id), so every element is placed on its
// own and a node's merge spreads over many workgroups.  With int32
// counters every |v| < 2^32: the lists' sorted magnitudes are staged in LDS
// as 32-bit values and the rank searches run there.  Each element's record
// (list, bucket, counter, child message) is gathered here once.
__global__ __launch_bounds__(kMergeThreads) void node_merge_kernel(
    const NodeTask *tasks, EstBuffers B, int32_t stage_bytes, GridMap gm) {
  const GridPos gp = grid_pos(gm);
  if (!gp.ok) return;
  const NodeTask *Tg = tasks + gp.task;
  const NodeTask T = *Tg;
  if (T.m < 2 || !T.guard.on) return;  // uniform
  const int row = gp.row;
  const int w = B.w;
  const int m = T.m;
  const int nl = m + (T.parent_side >= 0) + (T.cut_side >= 0);
  const int L = nl * w;
  const int e_lo = gp.c * kMergeChunk;
  if (e_lo >= L) return;
  const int e_hi = min(L, e_lo + kMergeChunk);
  uint32_t *merged =
      B.merged + ((size_t)T.scratch_slot * B.d + row) * (size_t)B.Lmax;
  NodeRec *rec = B.nrec + ((size_t)T.scratch_slot * B.d + row) * (size_t)B.Lmax;
  extern __shared__ uint32_t mags[];  // nl * w when staged
  __shared__ int32_t s_side[kMaxChild + 2], s_eid[kMaxChild + 2],
      s_msg[kMaxChild + 2];
  if ((int)threadIdx.x < nl) {
    const ListRef lr = list_of(Tg, threadIdx.x);
    s_side[threadIdx.x] = lr.side;
    s_eid[threadIdx.x] = lr.eid;
    s_msg[threadIdx.x] = (int)threadIdx.x < m ? Tg->child_msg[threadIdx.x] : 0;
  }
  __syncthreads();
  const bool staged = B.counter_bits == 32 &&
                      (size_t)nl * w * 4 <= (size_t)stage_bytes;
  // a chunk inside one list needs no rank in that list (its own index)
  const int own = e_lo / w == (e_hi - 1) / w ? e_lo / w : -1;
  if (staged) {
    for (int a = 0; a < nl; ++a)
      if (a != own)
        stage_lds<kMergeThreads, 8>(mags + (size_t)a * w,
                                    sorted_of(B, s_side[a], row), w, StageMag());
    __syncthreads();
    // kMergeU elements per lane at a time: their rank searches run in
    // lockstep (uniform trip count), so the LDS probes overlap
    constexpr int kMergeU = kMergeChunk / kMergeThreads;
    {
      const int e0 = e_lo + (int)threadIdx.x;
      int a[kMergeU], pos[kMergeU];
      uint32_t j[kMergeU];
      uint64_t absv[kMergeU];
      bool ok[kMergeU];
#pragma unroll
      for (int u = 0; u < kMergeU; ++u) {
        const int e = e0 + u * kMergeThreads;
        ok[u] = e < e_hi;
        const int ee = ok[u] ? e : e_lo;
        a[u] = ee / w;
        const int k = ee - a[u] * w;
        const uint64_t key = sorted_of(B, s_side[a[u]], row)[k];
        absv[u] = key >> 16;
        j[u] = (uint32_t)(key & 0xFFFF);
        pos[u] = k;
      }
      for (int b = 0; b < nl; ++b) {
        if (b == own) continue;  // uniform
        const uint32_t *mb = mags + (size_t)b * w;
        const int eb = s_eid[b];
        uint64_t t[kMergeU];
        int base[kMergeU];
#pragma unroll
        for (int u = 0; u < kMergeU; ++u) {
          t[u] = absv[u] + (eb < s_eid[a[u]] ? 1 : 0);  // count |v_b| < t
          base[u] = 0;
        }
        int n = w;
        while (n > 1) {
          const int half = n >> 1;
#pragma unroll
          for (int u = 0; u < kMergeU; ++u)
            base[u] = (uint64_t)mb[base[u] + half] < t[u] ? base[u] + half : base[u];
          n -= half;
        }
#pragma unroll
        for (int u = 0; u < kMergeU; ++u) {
          const int r = base[u] + ((uint64_t)mb[base[u]] < t[u] ? 1 : 0);
          if (b != a[u]) pos[u] += r;
        }
      }
      NodeRec r[kMergeU];
#pragma unroll
      for (int u = 0; u < kMergeU; ++u) {
        r[u].v = counter_at(B, s_side[a[u]], row, (int)j[u]);
        r[u].mu = a[u] < m ? child_msg_at(B, s_msg[a[u]], row, (int)j[u]) : (u128)0;
        r[u].aj = ((uint32_t)a[u] << 16) | j[u];
        r[u].pad = 0;
      }
#pragma unroll
      for (int u = 0; u < kMergeU; ++u) {
        if (!ok[u]) continue;
        merged[pos[u]] = r[u].aj;
        rec[pos[u]] = r[u];
      }
    }
  } else {
    for (int e = e_lo + (int)threadIdx.x; e < e_hi; e += kMergeThreads) {
      const int a = e / w;
      const int k = e - a * w;
      const uint64_t key = sorted_of(B, s_side[a], row)[k];
      const uint64_t absv = key >> 16;
      const uint32_t j = (uint32_t)(key & 0xFFFF);
      int pos = k;
      for (int b = 0; b < nl; ++b) {
        if (b == a) continue;
        const uint64_t t = absv + (s_eid[b] < s_eid[a] ? 1 : 0);  // count |v_b| < t
        pos += lower_bound_u64(sorted_of(B, s_side[b], row), w, t << 16);
      }
      NodeRec r;
      r.v = counter_at(B, s_side[a], row, (int)j);
      r.mu = a < m ? child_msg_at(B, s_msg[a], row, (int)j) : (u128)0;
      r.aj = ((uint32_t)a << 16) | j;
      r.pad = 0;
      merged[pos] = r.aj;
      rec[pos] = r;
    }
  }
}

// product of the A of every child but `a` (a >= M: of every child)
template <int M>
__device__ __forceinline__ u128 times_others(u128 t, const u128 *A, int a) {
  if (M == 1) return a >= M ? mul_u128(t, A[0]) : t;
  if (M == 2 && a < M) return mul_u128(t, a ? A[0] : A[1]);
#pragma unroll
  for (int c = 0; c < M; ++c)
    if (c != a) t = mul_u128(t, A[c]);
  return t;
}

// The three sweeps of a node with M children over its merged records, each
// thread taking a contiguous segment: the segment totals of every child's
// messages (suffix-scanned into A at the segment start), the running term
// sum G (prefix-scanned), and the emitted message and cut constants.
template <int M>
__device__ void node_sweeps(const NodeTask &T, const NodeRec *rec, int L,
                            int row, const EstBuffers &B, u128 *sh) {
  // records loaded together (fewer with more children: registers)
  constexpr int kSweepU = M <= 2 ? 4 : (M == 3 ? 2 : 1);
  const int has_parent = T.parent_side >= 0;
  const int seg = (L + kNodeThreads - 1) / kNodeThreads;
  const int s0 = min(L, (int)threadIdx.x * seg);
  const int s1 = min(L, s0 + seg);

  u128 tot[M];
#pragma unroll
  for (int c = 0; c < M; ++c) tot[c] = 0;
  for (int p0 = s0; p0 < s1; p0 += kSweepU) {
    NodeRec rr[kSweepU];
#pragma unroll
    for (int u = 0; u < kSweepU; ++u)
      if (p0 + u < s1) rr[u] = rec[p0 + u];
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) {
      if (p0 + u >= s1) break;
      const int a = (int)(rr[u].aj >> 16);
#pragma unroll
      for (int c = 0; c < M; ++c)
        if (c == a) tot[c] += rr[u].mu;
    }
  }
  u128 A0[M];  // A at the start of my segment (inclusive)
#pragma unroll
  for (int c = 0; c < M; ++c) A0[c] = block_scan_incl(tot[c], sh, true);

  u128 A[M];
#pragma unroll
  for (int c = 0; c < M; ++c) A[c] = A0[c];
  u128 gl = 0;
  for (int p0 = s0; p0 < s1; p0 += kSweepU) {
    NodeRec rr[kSweepU];
#pragma unroll
    for (int u = 0; u < kSweepU; ++u)
      if (p0 + u < s1) rr[u] = rec[p0 + u];
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) {
      if (p0 + u >= s1) break;
      const NodeRec &r = rr[u];
      const int a = (int)(r.aj >> 16);
      if (a >= M) continue;
      gl += times_others<M>(mul_s64_u128(r.v, r.mu), A, a);
#pragma unroll
      for (int c = 0; c < M; ++c)
        if (c == a) A[c] -= r.mu;
    }
  }
  const u128 gincl = block_scan_incl(gl, sh, false);

  if (T.mode == kModeTreeRoot) {
    if (threadIdx.x == kNodeThreads - 1)
      B.xout[(size_t)T.out_slot * B.d + row] = gincl;
    return;
  }

  // emit the message (parent list) and cut constants (cut list)
  u128 G = gincl - gl;
#pragma unroll
  for (int c = 0; c < M; ++c) A[c] = A0[c];
  u128 *Mo = has_parent ? msg_of(B, T.msg_slot, row) : nullptr;
  u128 *Co = T.cut_side >= 0 ? msg_of(B, T.cmsg_slot, row) : nullptr;
  for (int p0 = s0; p0 < s1; p0 += kSweepU) {
    NodeRec rr[kSweepU];
#pragma unroll
    for (int u = 0; u < kSweepU; ++u)
      if (p0 + u < s1) rr[u] = rec[p0 + u];
#pragma unroll
    for (int u = 0; u < kSweepU; ++u) {
      if (p0 + u >= s1) break;
      const NodeRec &r = rr[u];
      const int a = (int)(r.aj >> 16);
      const int j = (int)(r.aj & 0xFFFF);
      if (a < M) {
        G += times_others<M>(mul_s64_u128(r.v, r.mu), A, a);
#pragma unroll
        for (int c = 0; c < M; ++c)
          if (c == a) A[c] -= r.mu;
      } else {
        const u128 p = times_others<M>(s64_to_u128(r.v), A, a);
        const bool is_parent = has_parent && a == M;
        (is_parent ? Mo : Co)[j] = p + G;
      }
    }
  }
}

__global__ __launch_bounds__(kNodeThreads) void node_kernel(
    const NodeTask *tasks, EstBuffers B) {
  __shared__ u128 sh[kNodeThreads];
  const NodeTask *Tg = tasks + blockIdx.x;
  const NodeTask T = *Tg;
  if (!T.guard.on) return;  // uniform
  const int row = blockIdx.y;
  const int w = B.w;
  const int m = T.m;
  const int has_parent = T.parent_side >= 0;
  const int has_cut = T.cut_side >= 0;
  const int nl = m + has_parent + has_cut;

  // one child: node1_prefix_kernel / node1_emit_kernel; leaves have no
  // task (their messages are their counters)
  if (m < 2) return;

  const int L = nl * w;
  NodeRec *rec = B.nrec + ((size_t)T.scratch_slot * B.d + row) * (size_t)B.Lmax;
  // the merged records come from node_merge_kernel
  if (T.mode == kModeTriRootPrep) return;  // apex_prep_kernel

  switch (m) {
    case 2: node_sweeps<2>(T, rec, L, row, B, sh); break;
    case 3: node_sweeps<3>(T, rec, L, row, B, sh); break;
    case 4: node_sweeps<4>(T, rec, L, row, B, sh); break;
    case 5: node_sweeps<5>(T, rec, L, row, B, sh); break;
    default: node_sweeps<kMaxChild>(T, rec, L, row, B, sh); break;
  }
}

// ---------------------------------------------------------------------
// nodes with one child: grid (tasks, d, chunks), kN1Threads lanes
// ---------------------------------------------------------------------
// With a single child c the message of the node for a query element q
// (a bucket of the parent list or of the cut list) is
//   M(q) = s_q * A(kappa_q) + G(kappa_q),
// A = sum of the child's messages over child elements of larger kappa,
// G = sum of v * mu over child elements of smaller kappa.  The child's
// elements are already sorted by |v| (sort_rows_kernel), and kappa_z <
// kappa_q exactly when |v_z| < |s_q| + [eid_c < eid_q]: so with prefix sums
// of mu and v * mu in that order, M(q) is one binary search and one read.
// node1_prefix_kernel: chunk-local exclusive prefix sums (and chunk
// totals); node1_emit_kernel: the messages (or, at a tree root, X).
__device__ __forceinline__ u128 *n1_prefix(const EstBuffers &B, int slot,
                                           int row) {
  return reinterpret_cast<u128 *>(B.nrec +
                                  ((size_t)slot * B.d + row) * (size_t)B.Lmax);
}
__device__ __forceinline__ u128 *n1_total(const EstBuffers &B, int slot,
                                          int row) {
  return B.n1tot + ((size_t)slot * B.d + row) * (2 * kN1MaxChunks);
}

// 128-bit value of lane (lane - off), or 0 below lane off
__device__ __forceinline__ u128 shfl_up_u128(u128 v, int off) {
  const int lane = (int)threadIdx.x & 63;
  u128 r = 0;
#pragma unroll
  for (int k = 3; k >= 0; --k)
    r = (r << 32) | (uint32_t)__shfl_up((int)(uint32_t)(v >> (32 * k)), off);
  return lane >= off ? r : (u128)0;
}

__global__ __launch_bounds__(kN1Threads) void node1_prefix_kernel(
    const NodeTask *tasks, EstBuffers B, GridMap gm) {
  const GridPos gp = grid_pos(gm);
  if (!gp.ok) return;
  __shared__ u128 sh_m[kN1Threads / 64], sh_x[kN1Threads / 64];
  const NodeTask &T = tasks[gp.task];
  if (T.m != 1 || !T.guard.on) return;
  const int row = gp.row;
  const int w = B.w;
  const int c0 = gp.c * kN1Chunk;
  if (c0 >= w) return;
  const int cside = T.child_side[0];
  const int cmsg = T.child_msg[0];
  const uint64_t *srt = sorted_of(B, cside, row);
  u128 pm[kN1Per], px[kN1Per];
  const int k0 = c0 + threadIdx.x * kN1Per;
#pragma unroll
  for (int u = 0; u < kN1Per; ++u) {
    pm[u] = px[u] = 0;
    const int k = k0 + u;
    if (k < w) {
      const int j = (int)(srt[k] & 0xFFFF);
      const u128 mu = child_msg_at(B, cmsg, row, j);
      pm[u] = mu;
      px[u] = mul_s64_u128(counter_at(B, cside, row, j), mu);
    }
  }
  u128 tm = 0, tx = 0;
#pragma unroll
  for (int u = 0; u < kN1Per; ++u) {
    tm += pm[u];
    tx += px[u];
  }
  // inclusive block scans of the thread sums: within the waves by
  // shuffles, then the earlier waves' totals
  u128 im = tm, ix = tx;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    im += shfl_up_u128(im, off);
    ix += shfl_up_u128(ix, off);
  }
  const int wave = (int)threadIdx.x >> 6;
  if (((int)threadIdx.x & 63) == 63) {
    sh_m[wave] = im;
    sh_x[wave] = ix;
  }
  __syncthreads();
  u128 bm = 0, bx = 0;  // the earlier waves' totals, and the block's
#pragma unroll
  for (int k = 0; k < kN1Threads / 64; ++k) {
    if (k < wave) {
      bm += sh_m[k];
      bx += sh_x[k];
    }
  }
  u128 em = bm + im - tm, ex = bx + ix - tx;
  u128 *P = n1_prefix(B, T.scratch_slot, row);
  // a tree root (no parent or cut list) needs the chunk totals only
  const bool queries = T.parent_side >= 0 || T.cut_side >= 0;
#pragma unroll
  for (int u = 0; u < kN1Per; ++u) {
    const int k = k0 + u;
    if (queries && k < w) {
      P[2 * (size_t)k] = em;
      P[2 * (size_t)k + 1] = ex;
    }
    em += pm[u];
    ex += px[u];
  }
  if (threadIdx.x == kN1Threads - 1) {
    u128 *tot = n1_total(B, T.scratch_slot, row);
    tot[2 * gp.c] = bm + im;
    tot[2 * gp.c + 1] = bx + ix;
  }
}

__global__ __launch_bounds__(kN1Threads) void node1_emit_kernel(
    const NodeTask *tasks, EstBuffers B, GridMap gm) {
  const GridPos gp = grid_pos(gm);
  if (!gp.ok) return;
  extern __shared__ uint32_t smag[];  // the child's sorted |v| (int32 counters)
  __shared__ u128 soff[2 * kN1MaxChunks + 2];
  const NodeTask &T = tasks[gp.task];
  if (T.m != 1 || !T.guard.on) return;
  const int row = gp.row;
  const int w = B.w;
  const int has_parent = T.parent_side >= 0;
  const int nq = has_parent + (T.cut_side >= 0);
  const int nch = (w + kN1Chunk - 1) / kN1Chunk;
  const u128 *tot = n1_total(B, T.scratch_slot, row);
  if (nq == 0) {  // tree root: X = G(+inf)
    if (gp.c == 0 && threadIdx.x == 0) {
      u128 x = 0;
      for (int c = 0; c < nch; ++c) x += tot[2 * c + 1];
      B.xout[(size_t)T.out_slot * B.d + row] = x;
    }
    return;
  }
  const int e0 = gp.c * kN1Chunk;
  if (e0 >= nq * w) return;
  const int cside = T.child_side[0];
  const uint64_t *srt = sorted_of(B, cside, row);
  const bool staged = B.counter_bits == 32;
  if (staged) stage_lds<kN1Threads, 8>(smag, srt, w, StageMag());
  if (threadIdx.x < 64) {
    // chunk offsets: lane c loads chunk c's totals, an exclusive scan over
    // the lanes (nch <= kN1MaxChunks <= 64)
    const int c = (int)threadIdx.x;
    const u128 tm = c < nch ? tot[2 * c] : (u128)0;
    const u128 tx = c < nch ? tot[2 * c + 1] : (u128)0;
    u128 im = tm, ix = tx;
#pragma unroll
    for (int off = 1; off < kN1MaxChunks; off <<= 1) {
      im += shfl_up_u128(im, off);
      ix += shfl_up_u128(ix, off);
    }
    if (c < nch) {
      soff[2 * c] = im - tm;
      soff[2 * c + 1] = ix - tx;
    }
    if (c == nch - 1) {
      soff[2 * nch] = im;  // totals: the prefix at r = w
      soff[2 * nch + 1] = ix;
    }
  }
  __syncthreads();
  const u128 *P = n1_prefix(B, T.scratch_slot, row);
  const u128 tot_m = soff[2 * nch];
  int r[kN1Per], qi[kN1Per], qa[kN1Per];
  int64_t sv[kN1Per];
  uint64_t t[kN1Per];
  bool ok[kN1Per];
#pragma unroll
  for (int u = 0; u < kN1Per; ++u) {
    const int e = e0 + threadIdx.x + u * kN1Threads;
    ok[u] = e < nq * w;
    const int ee = ok[u] ? e : 0;
    qa[u] = ee / w;
    qi[u] = ee - qa[u] * w;
    const bool par = has_parent && qa[u] == 0;
    const int qside = par ? T.parent_side : T.cut_side;
    const int qeid = par ? T.parent_eid : T.cut_eid;
    sv[u] = counter_at(B, qside, row, qi[u]);
    t[u] = abs_u64(sv[u]) + (T.child_eid[0] < qeid ? 1 : 0);
  }
  if (staged) {
    int base[kN1Per];
#pragma unroll
    for (int u = 0; u < kN1Per; ++u) base[u] = 0;
    int n = w;
    while (n > 1) {
      const int half = n >> 1;
#pragma unroll
      for (int u = 0; u < kN1Per; ++u)
        base[u] = (uint64_t)smag[base[u] + half] < t[u] ? base[u] + half : base[u];
      n -= half;
    }
#pragma unroll
    for (int u = 0; u < kN1Per; ++u)
      r[u] = base[u] + ((uint64_t)smag[base[u]] < t[u] ? 1 : 0);
  } else {
#pragma unroll
    for (int u = 0; u < kN1Per; ++u) r[u] = lower_bound_u64(srt, w, t[u] << 16);
  }
#pragma unroll
  for (int u = 0; u < kN1Per; ++u) {
    if (!ok[u]) continue;
    u128 pm, px;
    if (r[u] == w) {
      pm = tot_m;
      px = soff[2 * nch + 1];
    } else {
      const int c = r[u] / kN1Chunk;
      pm = soff[2 * c] + P[2 * (size_t)r[u]];
      px = soff[2 * c + 1] + P[2 * (size_t)r[u] + 1];
    }
    const bool par = has_parent && qa[u] == 0;
    u128 *out = msg_of(B, par ? T.msg_slot : T.cmsg_slot, row);
    out[qi[u]] = mul_s64_u128(sv[u], tot_m - pm) + px;
  }
}

// min(a * b, 2^63) for a <= 2^63, b < 2^63
__device__ __forceinline__ u128 sat_mul63(u128 a, uint64_t b) {
  const u128 r = a * (u128)b;
  const u128 cap = (u128)1 << 63;
  return r > cap ? cap : r;
}

typedef const __attribute__((address_space(4))) TriTask ConstTask;
typedef const __attribute__((address_space(4))) TriElemN ConstElemN;
typedef const __attribute__((address_space(4))) TriPre ConstPre;

enum { kTriFast = 0, kTriNarrow = 1, kTriWide = 2 };

// Arithmetic of one triangle task (the same in every lane and block).
// Narrow arithmetic is exact when: every message value of child c is
// bounded by B_c = prod of n_sel over c's subtree (the L1 norm of a sketch
// row is at most n_sel), each A_c by (w + 1) B_c, and the apex's counters by
// n_sel(apex); when all of these stay below 2^62, messages and A are int64
// and only the running sum G needs 128 bits.  The compact two-child sweep
// also needs every table's n_sel below 2^30 (counters, keys and thresholds
// then fit 32 bits).
__device__ int tri_path(ConstTask &T, const EstBuffers &B) {
  bool narrow = true, small = true;
  const u128 lim = (u128)1 << 62;
  const int64_t nr = B.n_sel[T.root_table];
  const uint64_t nroot = nr < 0 ? 0 : (uint64_t)nr;
  small = nroot < (1ull << 30);
  for (int c = 0; c < T.m; ++c) {
    u128 bc = 1;
    for (uint64_t s = T.child_tables[c]; s; s &= s - 1) {
      const int64_t ns = B.n_sel[__builtin_ctzll(s)];
      const uint64_t f = ns < 0 ? 0 : (uint64_t)ns;
      small = small && f < (1ull << 30);
      bc = sat_mul63(bc, f);
    }
    if (bc * (u128)(B.w + 1) >= lim || bc * (u128)nroot >= lim) narrow = false;
  }
  if (!narrow) return kTriWide;
  return small && T.m == 2 ? kTriFast : kTriNarrow;
}

// Every task's guard (and a triangle's arithmetic path) resolved once per
// estimate into guard.on, so that the later launches test one field of the
// task they load anyway instead of re-reading the selected-row counts.
// Index i: triangle tasks first, then node tasks.
__device__ void resolve_task(const ResolveArgs &R, int i, const EstBuffers &B) {
  if (i < R.n_tri) {
    TriTask &T = R.tris[i];
    const bool on = COMPASS_GUARD_ON(T.guard, B.n_sel);
    T.guard.on = on ? 1 + tri_path(*(ConstTask *)&T, B) : 0;
  } else if (i < R.n_tri + R.n) {
    NodeTask &T = R.tasks[i - R.n_tri];
    int on = COMPASS_GUARD_ON(T.guard, B.n_sel) ? 1 : 0;
    if (on && T.mode == kModeTriRootPrep && T.m == 2 &&
        tri_path(*(ConstTask *)(R.tris + T.tri), B) == kTriFast)
      on |= 2;
    T.guard.on = on;
  }
}


// ---------------------------------------------------------------------
// triangle apex preparation: grid (tasks, d, chunks of kPrepChunk)
// ---------------------------------------------------------------------
// From the apex's merged records: the element list the sweeps read (its
// child, counter, message, and the kappa of the child's own bucket), the
// length of the zero-counter prefix and, for two-child apexes, each
// element's same-child run [run_lo, run_hi].
__device__ __forceinline__ int rec_child(const uint32_t *merged, int p) {
  return (int)(merged[p] >> 16);
}

// block-wide inclusive max-scan (forward) and min-scan (from the end) of
// one int per thread, kPrepThreads lanes: shuffles within the waves, then
// the earlier (later) waves' totals from LDS
__device__ __forceinline__ void prep_scans(int &mx, int &mn, int *wtot) {
  constexpr int kW = kPrepThreads / 64;
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int a = __shfl_up(mx, off);
    const int b = __shfl_down(mn, off);
    if (lane >= off) mx = max(mx, a);
    if (lane + off < 64) mn = min(mn, b);
  }
  if (lane == 63) wtot[wave] = mx;
  if (lane == 0) wtot[kW + wave] = mn;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kW; ++k) {
    if (k < wave) mx = max(mx, wtot[k]);
    if (k > wave) mn = min(mn, wtot[kW + k]);
  }
}

// block max / min of one int per thread (all threads get it); red holds
// 2 * waves ints and must not be in use by a previous call still read
__device__ __forceinline__ int block_max(int v, int *red) {
  constexpr int kW = kPrepThreads / 64;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  if (((int)threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  v = red[0];
#pragma unroll
  for (int k = 1; k < kW; ++k) v = max(v, red[k]);
  return v;
}

__global__ __launch_bounds__(kPrepThreads) void apex_prep_kernel(
    const NodeTask *tasks, EstBuffers B, GridMap gm) {
  const GridPos gp = grid_pos(gm);
  if (!gp.ok) return;
  constexpr int kW = kPrepThreads / 64;
  __shared__ int s_tot[2 * kW], s_red[4][kW];
  const NodeTask &T = tasks[gp.task];
  if (T.mode != kModeTriRootPrep || !T.guard.on) return;
  const int row = gp.row;
  const int m = T.m;
  const int L = m * B.w;  // an apex has no parent or cut list
  const int p0 = gp.c * kPrepChunk;
  if (p0 >= L) return;
  const int p1 = min(L, p0 + kPrepChunk);
  const NodeRec *rec =
      B.nrec + ((size_t)T.scratch_slot * B.d + row) * (size_t)B.Lmax;
  const uint32_t *mg =
      B.merged + ((size_t)T.scratch_slot * B.d + row) * (size_t)B.Lmax;
  const size_t slot_row = (size_t)T.out_slot * B.d + row;
  TriElem *out = B.prep + slot_row * (size_t)B.Lprep;
  TriElemN *outn = B.prepn + slot_row * (size_t)B.Lprep;
  // the two-child sweep reads the compact elements only, the general one
  // the full elements only
  const bool fast = (T.guard.on & 2) != 0;
  const int q0 = p0 + threadIdx.x * kPrepPer;  // my positions [q0, q0 + kPrepPer)
  // my records, the children around them, then the own-bucket counters
  NodeRec nr[kPrepPer];
  int ch[kPrepPer + 2];  // children of q0 - 1 .. q0 + kPrepPer (-1: none)
#pragma unroll
  for (int u = 0; u < kPrepPer; ++u) nr[u] = rec[min(q0 + u, p1 - 1)];
#pragma unroll
  for (int u = 0; u < kPrepPer + 2; ++u) {
    const int q = q0 - 1 + u;
    ch[u] = (q >= 0 && q < L) ? rec_child(mg, q) : -1;
  }
  const int64_t vprev = q0 > 0 && q0 - 1 < L ? rec[q0 - 1].v : 0;
  uint64_t own[kPrepPer];
#pragma unroll
  for (int u = 0; u < kPrepPer; ++u) {
    const int a = (int)(nr[u].aj >> 16);
    const int j = (int)(nr[u].aj & 0xFFFF);
    own[u] = 0;
    // kappa of the child's own bucket on the edge to the apex
    if (q0 + u < p1 && T.child_cut[a] >= 0)
      own[u] = abs_u64(counter_at(B, T.child_side[a] ^ 1, row, j));
  }
  int last_start = -1, first_end = L;
#pragma unroll
  for (int u = 0; u < kPrepPer; ++u) {
    const int pos = q0 + u;
    if (pos >= p1) break;
    const int a = (int)(nr[u].aj >> 16);
    // the list is ascending in |v|: its zero counters form a prefix, and
    // they add nothing to the sweep (it ends there)
    const int64_t vp = u == 0 ? vprev : nr[u - 1].v;
    if (nr[u].v != 0) {
      if (pos == 0 || vp == 0) B.prep_z[slot_row] = pos;
    } else if (pos == L - 1) {
      B.prep_z[slot_row] = L;
    }
    if (!fast) {
      TriElem e;
      e.v = nr[u].v;
      e.mu = nr[u].mu;
      e.key = T.child_cut[a] >= 0 ? (own[u] << 7) | (uint64_t)T.child_eid[a] : 0;
      e.child = (uint32_t)a;
      e.pad[0] = e.pad[1] = e.pad[2] = 0;
      out[pos] = e;
    }
    if (ch[u] != a) last_start = pos;
    if (first_end == L && ch[u + 2] != a) first_end = pos;
  }
  if (!fast) return;  // uniform
  // run starts and ends: the latest start at or before each of my
  // positions, the earliest end at or after; the run holding the chunk's
  // first (last) position may start (end) in an earlier (later) chunk:
  // searched kPrepThreads * kPrepPer positions at a time (uniform loops)
  int cur = last_start, nxt = first_end;
  prep_scans(cur, nxt, s_tot);
  int prev = -1, next = L;
  int it = 0;
  for (int base = p0 - 1; base >= 0; base -= kPrepThreads * kPrepPer, ++it) {
    int f = -1;
#pragma unroll
    for (int u = 0; u < kPrepPer; ++u) {
      const int q = base - ((int)threadIdx.x * kPrepPer + u);
      if (q >= 0 && (q == 0 || rec_child(mg, q - 1) != rec_child(mg, q))) f = max(f, q);
    }
    prev = block_max(f, s_red[it & 3]);
    if (prev >= 0) break;
  }
  for (int base = p1; base < L; base += kPrepThreads * kPrepPer, ++it) {
    int f = -L;
#pragma unroll
    for (int u = 0; u < kPrepPer; ++u) {
      const int q = base + (int)threadIdx.x * kPrepPer + u;
      if (q < L && (q == L - 1 || rec_child(mg, q + 1) != rec_child(mg, q))) f = max(f, -q);
    }
    next = -block_max(f, s_red[it & 3]);
    if (next < L) break;
  }
  // my positions' run bounds (exclusive of my own starts / ends first)
  int lo = __shfl_up(cur, 1);
  int hi = __shfl_down(nxt, 1);
  {
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    if (lane == 0) {
      lo = -1;
      for (int k = 0; k < wave; ++k) lo = max(lo, s_tot[k]);
    }
    if (lane == 63) {
      hi = L;
      for (int k = wave + 1; k < kW; ++k) hi = min(hi, s_tot[kW + k]);
    }
  }
  if (lo < 0) lo = prev;
  if (hi >= L) hi = next;
  int lo_of[kPrepPer];
#pragma unroll
  for (int u = 0; u < kPrepPer; ++u) {
    const int pos = q0 + u;
    const int a = (int)(nr[u].aj >> 16);
    if (pos < p1 && ch[u] != a) lo = pos;
    lo_of[u] = lo;
  }
  int hi_of[kPrepPer];
#pragma unroll
  for (int u = kPrepPer - 1; u >= 0; --u) {
    const int pos = q0 + u;
    const int a = (int)(nr[u].aj >> 16);
    if (pos < p1 && ch[u + 2] != a) hi = pos;
    hi_of[u] = hi;
  }
#pragma unroll
  for (int u = 0; u < kPrepPer; ++u) {
    const int pos = q0 + u;
    if (pos >= p1) break;
    const int a = (int)(nr[u].aj >> 16);
    // truncating copy; the sweep reads it only when the bounds hold
    TriElemN n;
    n.v = (int32_t)nr[u].v;
    n.kc = ((uint32_t)a << 31) | (uint32_t)(own[u] & 0x7FFFFFFFull);
    n.mu = (int64_t)(uint64_t)nr[u].mu;
    n.vm = (int64_t)((uint64_t)nr[u].v * (uint64_t)nr[u].mu);
    n.run_lo = lo_of[u];
    n.run_hi = hi_of[u];
    outn[pos] = n;
  }
}

// ---------------------------------------------------------------------
// triangle apex sweep: grid (n_tri, d, ceil(w / kLaneThreads))
// ---------------------------------------------------------------------


// Two-child apex, all magnitudes below 2^30, messages in 64 bits.  Sweeping
// in descending kappa, a maximal run of one child's elements sees the other
// child's running sum fixed, so the run's terms collapse to
// (sum over the run of v * mu) * A_other: one 64 x 64 -> 128-bit product per
// run instead of one per element (counters of the apex take few distinct
// magnitudes, and ties go to the lower edge id, so runs are long).  The
// runs are found once by the merge (run_lo), so the sweep loops over runs
// and, inside one, over elements with no per-element branch.  Within a run
// the lane's conditioned message is mu = M if the element ranks below the
// cut element, else the constant C(J); with a lane mask m for "below", the
// run keeps sum(m & M), sum(m & v*M), sum(m & v) and count(m), next to the
// run's plain sum of v and length (wave-uniform, scalar), and rebuilds
//   sum of v * mu = sum(m & v*M) + C * (sum v - sum(m & v))
//   sum of mu     = sum(m & M)   + C * (length - count(m))
// at its end: per element one compare, and AND / add operations only.
struct FastRun {
  int64_t mb, xb;      // sums of M and of v*M over the elements below
  int32_t vb, nb;      // sum of v and count over the elements below
  int32_t vrun, nrun;  // sum of v and length (uniform)
};

__device__ __forceinline__ void fast_elem(FastRun &r, uint32_t kf, int32_t v,
                                          uint32_t kc, int64_t mu0,
                                          int64_t vm) {
  // all-ones iff key < kf (both below 2^31); opaque, so that the masking
  // stays AND instead of becoming per-lane selects of scalar operands
  int32_t m = (int32_t)((kc & 0x7FFFFFFFu) - kf) >> 31;
  __asm__("" : "+v"(m));
  const uint64_t m64 = ((uint64_t)(uint32_t)m << 32) | (uint32_t)m;
  r.mb += (int64_t)((uint64_t)mu0 & m64);
  r.xb += (int64_t)((uint64_t)vm & m64);
  r.vb += (int32_t)((uint32_t)v & (uint32_t)m);
  r.nb -= m;
  r.vrun += v;
  r.nrun += 1;
}



// ---------------------------------------------------------------------
// run ordering of two-child apexes: grid (n_tri, d, tiles), kOrderThreads
// ---------------------------------------------------------------------
// Within one same-child run the sweep needs, for the lane's threshold kf,
// the sums over the run's elements whose child key is below kf.  Every
// tile of kOrderTile positions of [z, L) (z = zero-prefix length) orders
// each run piece it holds by ascending key, keeping the pieces where they
// are, and takes tile-local exclusive prefix sums over the reordered
// elements: the elements below kf of a run piece inside one tile are then
// the positions [lo, p), with p found by binary search, and their sums are
// differences of prefix sums.  A run's elements may be reordered freely:
// within a run the other child's running sum is fixed, so only the run's
// totals matter.  Keys sort as
//   (piece start - tile start) << (31 + P) | key << P | position - tile start
// with P = log2(kOrderTile) bits per position.
// Lists with L - z > kOrderCap keep the element-wise sweep (its keys would
// not fit the sweep's LDS stage).
__device__ __forceinline__ size_t tpre_index(const EstBuffers &B,
                                             size_t slot_row, int tile, int q) {
  const int tiles = (B.Lprep + kOrderTile - 1) / kOrderTile;
  return (slot_row * tiles + tile) * (size_t)(kOrderTile + 1) + q;
}

// The segment bounds and piece table (tri_seg_block) need the run bounds
// only, not the ordering: their workgroups ride along as the last
// n_tri x d workgroups of this launch.
static_assert(kSegThreads == kOrderThreads, "one launch for both");
__device__ void tri_seg_block(const TriTask *tasks, const EstBuffers &B,
                              int task, int row, int32_t *s_ps,
                              uint32_t *s_wt);
__global__ __launch_bounds__(kOrderThreads) void tri_order_kernel(
    const TriTask *tasks, EstBuffers B, GridMap gm, int n_order) {
  extern __shared__ __align__(16) uint64_t odyn[];  // (kOrderCap + 1) words
  if ((int)blockIdx.x >= n_order) {
    __shared__ uint32_t s_wt[kSegThreads / 64];
    const int b = (int)blockIdx.x - n_order;
    tri_seg_block(tasks, B, b / B.d, b % B.d, reinterpret_cast<int32_t *>(odyn),
                  s_wt);
    return;
  }
  const GridPos gp = grid_pos(gm);
  if (!gp.ok) return;
  uint64_t *okey = odyn;  // kOrderTile keys
  __shared__ int64_t scm[kOrderThreads / 64], scx[kOrderThreads / 64];
  __shared__ uint32_t scv[kOrderThreads / 64];
  const TriTask &T = tasks[gp.task];
  if (T.guard.on != 1 + kTriFast) return;  // another rooting, or path
  const int row = gp.row;
  const size_t slot_row = (size_t)T.prep_slot * B.d + row;
  const int z = B.prep_z[slot_row];
  const int L = T.L;
  if (L - z > kOrderCap) return;
  const int tile = gp.c;
  const int t0 = z + tile * kOrderTile;
  if (t0 >= L) return;
  const int nt = min(kOrderTile, L - t0);
  const TriElemN *el = B.prepn + slot_row * (size_t)B.Lprep;
  constexpr int kPos = __builtin_ctz(kOrderTile);  // position bits
  constexpr int kR = kOrderTile / kOrderThreads;   // keys a lane sorts
  constexpr int kMinSort = 64 * kR;                // a wave's key block
  static_assert(kPos + 31 + kPos <= 64, "sort keys fit 64 bits");
  int n2 = 1;
  while (n2 < nt) n2 <<= 1;
  {
    // every lane's element loads in flight together (indexes clamped)
    constexpr int kU = kOrderTile / kOrderThreads;
    int32_t rlo[kU];
    uint32_t kcs[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const TriElemN &e = el[t0 + min((int)threadIdx.x + u * kOrderThreads, nt - 1)];
      rlo[u] = e.run_lo;
      kcs[u] = e.kc;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = (int)threadIdx.x + u * kOrderThreads;
      if (q >= (n2 < kMinSort ? kMinSort : n2)) continue;
      uint64_t k = ~0ull;
      if (q < nt) {
        const uint64_t rl = (uint64_t)(max(rlo[u], t0) - t0);
        k = (rl << (31 + kPos)) | ((uint64_t)(kcs[u] & 0x7FFFFFFFu) << kPos) |
            (uint64_t)q;
      }
      okey[q] = k;
    }
  }
  __syncthreads();
  // padding keys (all ones) sort last
  bitonic_sort_lds<kOrderThreads, kR>(
      reinterpret_cast<unsigned long long *>(okey), n2 < kMinSort ? kMinSort : n2);
  // each thread: a consecutive chunk of at most kOrderPer sorted slots;
  // all of its element loads are issued before the sums
  constexpr int kOrderPer = kOrderTile / kOrderThreads;
  uint32_t *tk = B.tkey + slot_row * (size_t)B.Lprep;
  const int q0 = min(nt, (int)threadIdx.x * kOrderPer);
  const int q1 = min(nt, q0 + kOrderPer);
  int64_t mu[kOrderPer], vm[kOrderPer];
  int32_t vv[kOrderPer];
#pragma unroll
  for (int u = 0; u < kOrderPer; ++u) {
    mu[u] = vm[u] = 0;
    vv[u] = 0;
    const int q = q0 + u;
    if (q < q1) {
      const uint64_t k = okey[q];
      const TriElemN &src = el[t0 + (int)(k & (kOrderTile - 1))];
      mu[u] = src.mu;
      vm[u] = src.vm;
      vv[u] = src.v;
      tk[t0 + q] = (uint32_t)((k >> kPos) & 0x7FFFFFFFull);
    }
  }
  uint64_t sm = 0, sx = 0;
  uint32_t sv = 0;
#pragma unroll
  for (int u = 0; u < kOrderPer; ++u) {
    sm += (uint64_t)mu[u];
    sx += (uint64_t)vm[u];
    sv += (uint32_t)vv[u];
  }
  // inclusive scans of the three thread sums: within each wave by
  // shuffles, then over the earlier waves' totals (wrapping)
  unsigned long long im = sm, ix = sx;
  uint32_t iv = sv;
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long a = __shfl_up(im, off);
    const unsigned long long c = __shfl_up(ix, off);
    const uint32_t e = (uint32_t)__shfl_up((int)iv, off);
    if (lane >= off) {
      im += a;
      ix += c;
      iv += e;
    }
  }
  if (lane == 63) {
    scm[wv] = (int64_t)im;
    scx[wv] = (int64_t)ix;
    scv[wv] = iv;
  }
  __syncthreads();
  for (int k = 0; k < wv; ++k) {
    im += (uint64_t)scm[k];
    ix += (uint64_t)scx[k];
    iv += scv[k];
  }
  // exclusive start of my chunk, then its running sums (wrapping)
  uint64_t em = (uint64_t)im - sm;
  uint64_t ex = (uint64_t)ix - sx;
  uint32_t ev = iv - sv;
  TriPre *E = B.tpre + tpre_index(B, slot_row, tile, 0);
#pragma unroll
  for (int u = 0; u < kOrderPer; ++u) {
    const int q = q0 + u;
    if (q < q1) {
      TriPre o;
      o.m = (int64_t)em;
      o.x = (int64_t)ex;
      o.v = (int32_t)ev;
      o.pad = 0;
      E[q] = o;
    }
    em += (uint64_t)mu[u];
    ex += (uint64_t)vm[u];
    ev += (uint32_t)vv[u];
  }
  if (threadIdx.x == kOrderThreads - 1) {
    TriPre o;
    o.m = (int64_t)im;
    o.x = (int64_t)ix;
    o.v = (int32_t)iv;
    o.pad = 0;
    E[nt] = o;
  }
}

// Segment bounds of the two-child sweep: the runs of [z, L) (a run
// straddling z counts from z) split into kFastSegs groups of equal run
// count, cut at run starts, so that the four sweep segments of a bucket
// do equal numbers of run pieces.  bounds[k] = first position of group k
// in ascending position order, bounds[kFastSegs] = L.
__device__ void tri_seg_block(const TriTask *tasks, const EstBuffers &B,
                              int task, int row, int32_t *s_ps,
                              uint32_t *s_wt) {
  // s_ps: piece starts (kOrderCap + 1); s_wt: kSegThreads / 64 words
  const TriTask &T = tasks[task];
  if (T.guard.on != 1 + kTriFast) return;  // another rooting, or path
  const size_t slot_row = (size_t)T.prep_slot * B.d + row;
  const int z = B.prep_z[slot_row];
  const int L = T.L;
  if (L - z > kOrderCap) {  // unordered lists: equal position ranges
    if (threadIdx.x <= kFastSegs)
      B.tseg[slot_row * (kFastSegs + 1) + threadIdx.x] =
          z + (int)((int64_t)(L - z) * threadIdx.x / kFastSegs);
    return;
  }
  const TriElemN *el = B.prepn + slot_row * (size_t)B.Lprep;
  int32_t *bounds = B.tseg + slot_row * (kFastSegs + 1);
  int32_t *pbounds = B.tsegp + slot_row * (kFastSegs + 1);
  // n <= kOrderCap positions: kSegPer consecutive ones per lane, loaded
  // together.  Run starts: z and every position that begins a same-child
  // run; piece starts: run starts and ordering tile starts.
  const int q0 = z + (int)threadIdx.x * kSegPer;
  uint32_t rs = 0, ps = 0;
  {
    int32_t rl[kSegPer];  // every load in flight together (clamped)
#pragma unroll
    for (int u = 0; u < kSegPer; ++u) rl[u] = el[min(q0 + u, L - 1)].run_lo;
#pragma unroll
    for (int u = 0; u < kSegPer; ++u) {
      const int p = q0 + u;
      if (p >= L) continue;
      const bool r = p == z || rl[u] == p;
      if (r) rs |= 1u << u;
      if (r || (p - z) % kOrderTile == 0) ps |= 1u << u;
    }
  }
  const int rc = __popc(rs), pc = __popc(ps);
  // inclusive scans of both counts at once (16-bit fields: at most
  // kOrderCap each), within the waves, then over the waves' totals
  const uint32_t mine = (uint32_t)rc | ((uint32_t)pc << 16);
  const uint32_t incl = wave_scan_incl(mine);
  const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
  if (lane == 63) s_wt[wave] = incl;
  __syncthreads();
  const uint32_t wsc = wave_scan_incl(lane < kSegThreads / 64 ? s_wt[lane] : 0u);
  const uint32_t before =
      wave > 0 ? (uint32_t)__builtin_amdgcn_readlane((int)wsc, wave - 1) : 0u;
  const uint32_t all =
      (uint32_t)__builtin_amdgcn_readlane((int)wsc, kSegThreads / 64 - 1);
  const uint32_t mine_incl = before + incl;
  const int R = (int)(all & 0xFFFFu);
  const int P = (int)(all >> 16);
  int g = (int)(mine_incl & 0xFFFFu) - rc;  // index of my first run start
  int h = (int)(mine_incl >> 16) - pc;      // index of my first piece start
  if (threadIdx.x == 0) {
    bounds[0] = z;
    bounds[kFastSegs] = L;
    pbounds[0] = 0;
    pbounds[kFastSegs] = P;
    for (int k = 1; k < kFastSegs; ++k)
      if ((int)(((int64_t)R * k) / kFastSegs) >= R) {
        bounds[k] = L;
        pbounds[k] = P;
      }
    s_ps[P] = L;
  }
  // groups of equal run count, cut at run starts (which are piece starts)
  for (uint32_t m = ps; m; m &= m - 1) {
    const int u = __builtin_ctz(m);
    const int p = q0 + u;
    s_ps[h] = p;
    if ((rs >> u) & 1u) {
      for (int k = 1; k < kFastSegs; ++k)
        if ((int)(((int64_t)R * k) / kFastSegs) == g) {
          bounds[k] = p;
          pbounds[k] = h;
        }
      ++g;
    }
    ++h;
  }
  __syncthreads();
  // the pieces: child, summed by search (runs of at least kSearchMin
  // elements in [z, L)), tile (the sweep reads the prefix sums at a
  // piece's ends from the ordering's tables, so this needs none of them)
  TriPiece *out = B.tpiece + slot_row * (size_t)B.Pcap;
  for (int i = threadIdx.x; i < P; i += kSegThreads) {
    const int lo = s_ps[i], hi = s_ps[i + 1] - 1;
    const TriElemN e = el[lo];
    const bool lng = e.run_hi - max(e.run_lo, z) + 1 >= kSearchMin;
    const int tile = (lo - z) / kOrderTile;
    TriPiece o;
    o.lo = lo;
    o.hi = hi;
    o.info = (int32_t)((e.kc >> 31) | (lng ? 2u : 0u) | ((uint32_t)tile << 2));
    o.pad = 0;
    out[i] = o;
  }
}

// Two-child apexes, by group: grid (groups, d, ceil(w / kLaneThreads)),
// kFastSegs slots of kLaneThreads lanes per workgroup.  The triangle tasks
// of a group share the apex's merged list, its runs and run pieces, the
// cut edge and its sides; they differ in the children's messages only.  A
// lane's binary search of a run piece (the first key at or above its
// threshold) is therefore the same for every member: it is done once, by
// one slot, and handed to the others through LDS.
//
// With nm members running (at most kTriGroupMax), slot s works for member
// s % nm on segment s / nm of S = kFastSegs / nm segments of the sweep (nm
// = 3 counts as 4: two slots only search); with K = kFastSegs run groups
// from tri_seg_block, segment g covers the groups [K - (g + 1) K / S,
// K - g K / S).  Many workgroups of few lanes (128 buckets J each) and
// more segments keep two workgroups on most CUs and shorten each slot's
// chain of rounds.  Cutting the descending sweep into
// segments is exact: a segment's runs see the other child's running sum
// of the earlier segments plus their own, so
//   G = sum_g [ G_g + A0(before g) * X1_g + A1(before g) * X0_g ]
// with X_c the segment's sum of the run terms of child c (v * mu summed).
// The slots of one segment go through its pieces in rounds of nm: in round
// r each searches one piece (writing its lanes' offsets into LDS), and
// after one barrier each closes all nm pieces for its member (prefix-sum
// reads of its own member at the searched positions).  The searches of
// round r + 1 are issued before the closes of round r (two LDS buffers).
// Short runs are summed element by element, lists too long to order
// element by element throughout.

struct SegOut {
  u128 G;
  int64_t A0, A1, X0, X1;
};
static_assert(sizeof(SegOut) * kFastSegs * kLaneThreads <= kFastStageBytes,
              "segment results reuse the key stage");
constexpr int kFastPbufBytes = 2 * kFastSegs * kLaneThreads * 2;
constexpr int kFastLds = kFastStageBytes + kFastPbufBytes;

// first index in [0, n) whose key is >= kf, n >= 1 (uniform trip count)
__device__ __forceinline__ int lds_lower_bound(const uint32_t *k, int n,
                                               uint32_t kf) {
  int base = 0;
  while (n > 1) {
    const int half = n >> 1;
    base = k[base + half] < kf ? base + half : base;
    n -= half;
  }
  return base + (k[base] < kf ? 1 : 0);
}

typedef const __attribute__((address_space(4))) TriPiece ConstPiece;

__global__ __launch_bounds__(kLaneThreads * kFastSegs, 8) void tri_fast_kernel(
    const TriTask *tasks, const TriGroup *groups, EstBuffers B, GridMap gm) {
  const GridPos gp = grid_pos(gm);
  if (!gp.ok) return;
  extern __shared__ __align__(16) uint32_t skey[];  // run-ordered keys of [z, L)
  // search offsets [buffer][slot][lane], addressed from my lane's column
  uint16_t *pcol = reinterpret_cast<uint16_t *>(
                       reinterpret_cast<char *>(skey) + kFastStageBytes) +
                   threadIdx.x % kLaneThreads;
  auto pbuf_at = [&](int buf, int sl) -> uint16_t & {
    return pcol[(buf * kFastSegs + sl) * kLaneThreads];
  };
  // the members that run (compacted with static indices, so that they stay
  // in scalar registers); slots past nm repeat the first
  const TriGroup &Gr = groups[gp.task];
  int mem[kTriGroupMax];
  int nm = 0;
#pragma unroll
  for (int q = 0; q < kTriGroupMax; ++q) {
    mem[q] = 0;
    if (q >= Gr.n) continue;
    const int t = Gr.member[q];
    if (tasks[t].guard.on != 1 + kTriFast) continue;  // another rooting, or path
#pragma unroll
    for (int g = 0; g <= q; ++g)
      if (g == nm) mem[g] = t;
    ++nm;
  }
  if (nm == 0) return;  // uniform
  const int S = kFastSegs / (nm == 3 ? 4 : nm);   // segments
  const int gs = kFastSegs / S;                    // run groups per segment
  const int row = gp.row;
  const int lane = threadIdx.x % kLaneThreads;
  // whole waves share a slot: make that visible to the compiler, so the
  // sweep's positions and element loads stay scalar
  const int slot = __builtin_amdgcn_readfirstlane(threadIdx.x / kLaneThreads);
  const bool working = slot < S * nm;  // nm = 3: one slot only searches
  const int mi = slot % nm;            // my member
  const int seg = slot / nm;           // my segment
  int my = mem[0];
#pragma unroll
  for (int g = 1; g < kTriGroupMax; ++g)
    if (g == mi) my = mem[g];
  ConstTask &T = *((ConstTask *)tasks + mem[0]);  // the shared structure
  ConstTask &M = *((ConstTask *)tasks + my);      // my member
  const int J = gp.c * kLaneThreads + lane;
  const bool active = J < B.w;
  const int Jc = active ? J : 0;
  const size_t slot_row = (size_t)T.prep_slot * B.d + row;
  const size_t my_row = (size_t)M.prep_slot * B.d + row;
  const int z = B.prep_z[slot_row];  // the sweep ends at the zero prefix
  const int len = T.L - z;
  const bool ordered = len <= kOrderCap;  // tri_order_kernel ran
  const uint32_t *tk = B.tkey + slot_row * (size_t)B.Lprep;
  if (ordered) {
    stage_lds<kLaneThreads * kFastSegs, 16>(skey, tk + z, len, StageCopy());
    __syncthreads();
  }

  // key < kf  <=>  kappa below the cut element's (ties in |v| go to the
  // lower edge id); the cut constants are my member's
  const int e0 = T.cut_child[0] == 0 ? 0 : 1;  // cut endpoint in slot 0
  uint32_t kf0, kf1;
  int64_t C0, C1;
  {
    uint32_t kf[2];
    int64_t cv[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      kf[e] = (uint32_t)abs_u64(counter_at(B, T.cut_side[e], row, Jc)) +
              (T.cut_peid[e] < T.cut_eid ? 1u : 0u);
      cv[e] = (int64_t)(uint64_t)child_msg_at(B, M.cut_cmsg[e], row, Jc);
    }
    kf0 = kf[e0];
    kf1 = kf[1 - e0];
    C0 = cv[e0];
    C1 = cv[1 - e0];
  }
  ConstElemN *el = (ConstElemN *)(B.prepn + my_row * (size_t)B.Lprep);
  u128 G = 0;
  // Runs close in alternating children (consecutive pieces of one child
  // are merged first, below), so the running sums are kept as "child of
  // the last close" (Ap, Xp) and "the other child" (Aq, Xq): a close
  // multiplies by Ap, adds its run to Aq and Xq, and the two swap roles.
  // No per-lane selects between the children's sums.
  int64_t Ap = 0, Aq = 0, Xp = 0, Xq = 0;
  uint32_t lastc = 0;  // child of the last close (before the first: any)
  auto close = [&](uint32_t c, const FastRun &r) {
    const int64_t cc = c ? C1 : C0;
    const int64_t x = r.xb + cc * (int64_t)(r.vrun - r.vb);
    const int64_t arun = r.mb + cc * (int64_t)(r.nrun - r.nb);
    G += mul_s64_s64(x, Ap);
    const int64_t an = Aq + arun, xn = Xq + x;
    Aq = Ap;
    Xq = Xp;
    Ap = an;
    Xp = xn;
    lastc = c;
  };
  // consecutive pieces of one child (a run cut at ordering tiles) close
  // as one: within a run the other child's running sum does not change,
  // and a piece's sums add
  FastRun pend;
  pend.mb = pend.xb = 0;
  pend.vb = pend.nb = pend.vrun = pend.nrun = 0;
  uint32_t pc = 2;  // child of the pending pieces (2: none)
  auto add_piece = [&](uint32_t c, const FastRun &r) {
    if (c == pc) {
      pend.mb += r.mb;
      pend.xb += r.xb;
      pend.vb += r.vb;
      pend.nb += r.nb;
      pend.vrun += r.vrun;
      pend.nrun += r.nrun;
    } else {
      if (pc < 2) close(pc, pend);
      pend = r;
      pc = c;
    }
  };
  // element by element over [lo, hi], descending (my member's elements)
  auto elements = [&](int lo, int hi, uint32_t c, FastRun &r) {
    constexpr int kGroup = 4;  // its loads stay in scalar registers
    const uint32_t kf = c ? kf1 : kf0;
    r.mb = r.xb = 0;
    r.vb = r.nb = 0;
    r.vrun = r.nrun = 0;
    int pos = hi;
    for (; pos - (kGroup - 1) >= lo; pos -= kGroup) {
      int32_t v[kGroup];
      uint32_t kc[kGroup];
      int64_t mu[kGroup], vm[kGroup];
#pragma unroll
      for (int q = 0; q < kGroup; ++q) {
        ConstElemN &e = el[pos - q];
        v[q] = e.v;
        kc[q] = e.kc;
        mu[q] = e.mu;
        vm[q] = e.vm;
      }
      // issue the whole group's scalar loads before the first use
#pragma unroll
      for (int q = 0; q < kGroup; ++q)
        __asm__ volatile("" ::"s"(v[q]), "s"(kc[q]), "s"(mu[q]), "s"(vm[q]));
#pragma unroll
      for (int q = 0; q < kGroup; ++q) fast_elem(r, kf, v[q], kc[q], mu[q], vm[q]);
    }
    for (; pos >= lo; --pos) {
      ConstElemN &e = el[pos];
      fast_elem(r, kf, e.v, e.kc, e.mu, e.vm);
    }
  };
  if (ordered) {
    // segment bounds in the piece table; rounds of nm pieces
    const int32_t *sp = B.tsegp + slot_row * (kFastSegs + 1);
    int rounds = 0;
    for (int g = 0; g < S; ++g) {  // uniform
      const int n = sp[kFastSegs - g * gs] - sp[kFastSegs - (g + 1) * gs];
      rounds = max(rounds, (n + nm - 1) / nm);
    }
    const int pb = __builtin_amdgcn_readfirstlane(sp[kFastSegs - (seg + 1) * gs]);
    const int pe = __builtin_amdgcn_readfirstlane(sp[kFastSegs - seg * gs]);
    ConstPiece *pcs = (ConstPiece *)B.tpiece + slot_row * (size_t)B.Pcap;
    const TriPre *mpre = B.tpre + tpre_index(B, my_row, 0, 0);
    // a piece's ends in the ordering's prefix tables (uniform reads): my
    // member's sums of M and v M at its start, the sums of v (the same for
    // every member) at both ends
    ConstPre *mpre_c = (ConstPre *)B.tpre + tpre_index(B, my_row, 0, 0);
    // my search of round r: piece pe - 1 - (nm r + mi), its lanes' offsets
    // into buffer r & 1
    auto search = [&](int r) {
      const int i = pe - 1 - (nm * r + mi);
      if (!working || i < pb) return;  // uniform
      const int info = pcs[i].info;
      if (!(info & 2)) return;
      const int lo = pcs[i].lo, hi = pcs[i].hi;
      const uint32_t kf = (info & 1) ? kf1 : kf0;
      const int p = lds_lower_bound(skey + (lo - z), hi - lo + 1, kf);
      pbuf_at(r & 1, slot) = (uint16_t)p;
    };
    search(0);
    for (int r = 0; r < rounds; ++r) {
      __syncthreads();  // round r's offsets are written
      // my member's prefixes at the searched positions of the round: the
      // first is loaded during the next round's search, each later one
      // during the close of the piece before it
      const int i0 = pe - 1 - nm * r;
      const int nq = working ? min(nm, i0 - pb + 1) : 0;  // my pieces left
      // (with them, the uniform prefixes at the piece's ends)
      struct Ends {
        int64_t m0, x0;
        int32_t v0, v1;
      };
      auto gather = [&](int q, TriPre &e, Ends &en) {
        e.m = e.x = 0;
        e.v = e.pad = 0;
        en.m0 = en.x0 = 0;
        en.v0 = en.v1 = 0;
        if (q >= nq) return;
        const int i = i0 - q;
        const int info = pcs[i].info;
        if (!(info & 2)) return;
        const int tile = info >> 2;
        const int lo = pcs[i].lo;
        const int p = lo + pbuf_at(r & 1, seg * nm + q);
        e = mpre[(size_t)tile * (kOrderTile + 1) + (p - z - tile * kOrderTile)];
        ConstPre *tp = mpre_c + (size_t)tile * (kOrderTile + 1) -
                       (z + tile * kOrderTile);
        en.m0 = tp[lo].m;
        en.x0 = tp[lo].x;
        en.v0 = tp[lo].v;
        en.v1 = tp[pcs[i].hi + 1].v;
      };
      TriPre ep;
      Ends en;
      gather(0, ep, en);
      if (r + 1 < rounds) search(r + 1);
#pragma unroll
      for (int q = 0; q < kTriGroupMax; ++q) {
        if (q >= nq) break;
        const int i = i0 - q;
        const int info = pcs[i].info;
        const int lo = pcs[i].lo, hi = pcs[i].hi;
        const uint32_t c = info & 1;
        FastRun rr;
        if (info & 2) {
          const TriPre &e = ep;
          const int p = lo + pbuf_at(r & 1, seg * nm + q);
          rr.mb = (int64_t)((uint64_t)e.m - (uint64_t)en.m0);
          rr.xb = (int64_t)((uint64_t)e.x - (uint64_t)en.x0);
          rr.vb = (int32_t)((uint32_t)e.v - (uint32_t)en.v0);
          rr.nb = p - lo;
          rr.vrun = (int32_t)((uint32_t)en.v1 - (uint32_t)en.v0);
          rr.nrun = hi - lo + 1;
        } else {
          elements(lo, hi, c, rr);
        }
        if (q + 1 < kTriGroupMax) gather(q + 1, ep, en);
        add_piece(c, rr);
      }
    }
  } else if (working) {
    // unordered list: runs element by element, segments by position
    const int32_t *sb = B.tseg + slot_row * (kFastSegs + 1);
    const int top = __builtin_amdgcn_readfirstlane(sb[kFastSegs - seg * gs]) - 1;
    const int bottom =
        __builtin_amdgcn_readfirstlane(sb[kFastSegs - (seg + 1) * gs]);
    int pos = top;
    while (pos >= bottom) {
      const uint32_t c = el[pos].kc >> 31;  // the run's child (uniform)
      const int lo = max(el[pos].run_lo, bottom);
      FastRun rr;
      elements(lo, pos, c, rr);
      add_piece(c, rr);
      pos = lo - 1;
    }
  }
  if (pc < 2) close(pc, pend);
  const int64_t A0 = lastc ? Aq : Ap, A1 = lastc ? Ap : Aq;
  const int64_t X0 = lastc ? Xq : Xp, X1 = lastc ? Xp : Xq;
  // segments combine exactly, per member (slot (mi, 0) sums its member's
  // S segments), then the member's lanes are summed
  __syncthreads();  // the key stage and the offset buffers are done with
  SegOut (*so)[kLaneThreads] = reinterpret_cast<SegOut (*)[kLaneThreads]>(skey);
  {
    SegOut &mine = so[slot][lane];
    mine.G = G;
    mine.A0 = A0;
    mine.A1 = A1;
    mine.X0 = X0;
    mine.X1 = X1;
  }
  __syncthreads();
  u128 tot = 0;
  if (working && seg == 0) {
    int64_t a0 = 0, a1 = 0;
    for (int g = 0; g < S; ++g) {
      const SegOut &o = so[g * nm + mi][lane];
      tot += o.G + mul_s64_s64(a0, o.X1) + mul_s64_s64(a1, o.X0);
      a0 += o.A0;
      a1 += o.A1;
    }
    if (!active) tot = 0;
  }
  // lanes: within each wave by shuffles, then the slot's waves
  __syncthreads();  // the segment results are read
  constexpr int kWps = kLaneThreads / 64;        // waves per slot
  u128 *red = reinterpret_cast<u128 *>(skey);  // [kFastSegs][kWps]
  {
    uint32_t w4[4] = {(uint32_t)tot, (uint32_t)(tot >> 32),
                      (uint32_t)(tot >> 64), (uint32_t)(tot >> 96)};
    // 128-bit sums: add 32-bit limbs with carries, one xor distance at a time
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      u128 o = 0;
#pragma unroll
      for (int k = 3; k >= 0; --k)
        o = (o << 32) | (uint32_t)__shfl_xor((int)w4[k], off);
      tot += o;
      w4[0] = (uint32_t)tot;
      w4[1] = (uint32_t)(tot >> 32);
      w4[2] = (uint32_t)(tot >> 64);
      w4[3] = (uint32_t)(tot >> 96);
    }
    if ((threadIdx.x & 63) == 0) red[slot * kWps + lane / 64] = tot;
  }
  __syncthreads();
  if (working && seg == 0 && lane == 0) {
    u128 sum = 0;
#pragma unroll
    for (int k = 0; k < kWps; ++k) sum += red[slot * kWps + k];
    B.partial[((size_t)M.partial_slot + gp.c) * B.d + row] = sum;
  }
}

// Other triangles (more apex children, or bounds beyond the compact
// sweep): grid (n_tri, d, ceil(w / kLaneThreads)); blocks of two-child
// tasks that tri_fast_kernel handles return at once.
__global__ __launch_bounds__(kLaneThreads) void tri_lane_kernel(
    const TriTask *tasks, EstBuffers B, GridMap gm) {
  const GridPos gp = grid_pos(gm);
  if (!gp.ok) return;
  __shared__ u128 red[kLaneThreads];
  // the task is the same for every lane: read it through the constant
  // address space so its fields live in scalar registers
  ConstTask &T = *((ConstTask *)tasks + gp.task);
  if (!T.guard.on) return;  // another rooting runs
  const int path = T.guard.on - 1;
  if (path == kTriFast) return;  // uniform: tri_fast_kernel's block
  const bool narrow = path == kTriNarrow;
  const int row = gp.row;
  const int J = gp.c * kLaneThreads + threadIdx.x;
  const bool active = J < B.w;
  const int Jc = active ? J : 0;
  const size_t slot_row = (size_t)T.prep_slot * B.d + row;
  const int z = B.prep_z[slot_row];  // the sweep ends at the zero prefix
  const int m = T.m;
  const int cu = T.cut_child[0], cv = T.cut_child[1];

  uint64_t qabs[2];
  u128 cval[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    qabs[e] = abs_u64(counter_at(B, T.cut_side[e], row, Jc));
    cval[e] = child_msg_at(B, T.cut_cmsg[e], row, Jc);
  }

  u128 G = 0;
  constexpr int kUnroll = 4;
  if (narrow) {
    typedef const __attribute__((address_space(4))) TriElem ConstElem;
    ConstElem *el = (ConstElem *)(B.prep + slot_row * (size_t)B.Lprep);
    uint64_t kf[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) kf[e] = (qabs[e] << 7) | (uint64_t)T.cut_eid;
    int64_t A[kMaxChild];
#pragma unroll
    for (int c = 0; c < kMaxChild; ++c) A[c] = 0;
    const int64_t c0 = (int64_t)(uint64_t)cval[0], c1 = (int64_t)(uint64_t)cval[1];
    int pos = T.L - 1;
    for (; pos >= z; pos -= kUnroll) {
      TriElem e[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        ConstElem &r = el[max(pos - u, 0)];
        e[u].v = r.v;
        e[u].key = r.key;
        e[u].mu = r.mu;
        e[u].child = r.child;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (pos - u < z) break;
        const int a = (int)e[u].child;
        int64_t mu = (int64_t)(uint64_t)e[u].mu;
        if (a == cu) mu = e[u].key < kf[0] ? mu : c0;
        if (a == cv) mu = e[u].key < kf[1] ? mu : c1;
        const int64_t vm = e[u].v * mu;
        u128 term = 0;
        bool first = true;
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c) {
          if (c < m && c != a) {
            term = first ? mul_s64_s64(vm, A[c]) : mul_u128_s64(term, A[c]);
            first = false;
          }
        }
        if (first) term = s64_to_u128(vm);
        G += term;
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c)
          if (c == a) A[c] += mu;
      }
    }
  } else {
    typedef const __attribute__((address_space(4))) TriElem ConstElem;
    ConstElem *el = (ConstElem *)(B.prep + slot_row * (size_t)B.Lprep);
    uint64_t kf[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) kf[e] = (qabs[e] << 7) | (uint64_t)T.cut_eid;
    u128 A[kMaxChild];
#pragma unroll
    for (int c = 0; c < kMaxChild; ++c) A[c] = 0;
    // descending kappa: A_c accumulates the elements already passed (larger
    // kappa), i.e. exactly the elements a term's bucket must rank below
    int pos = T.L - 1;
    for (; pos - (kUnroll - 1) >= z; pos -= kUnroll) {
      TriElem e[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        ConstElem &r = el[pos - u];
        e[u].v = r.v;
        e[u].key = r.key;
        e[u].mu = r.mu;
        e[u].child = r.child;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int a = (int)e[u].child;
        u128 mu = e[u].mu;
        if (a == cu) mu = e[u].key < kf[0] ? mu : cval[0];
        if (a == cv) mu = e[u].key < kf[1] ? mu : cval[1];
        u128 term = mul_s64_u128(e[u].v, mu);
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c)
          if (c < m && c != a) term = mul_u128(term, A[c]);
        G += term;
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c)
          if (c == a) A[c] += mu;
      }
    }
    for (; pos >= z; --pos) {
      TriElem e;
      e.v = el[pos].v;
      e.key = el[pos].key;
      e.mu = el[pos].mu;
      e.child = el[pos].child;
      const int a = (int)e.child;
      u128 mu = e.mu;
      if (a == cu) mu = e.key < kf[0] ? mu : cval[0];
      if (a == cv) mu = e.key < kf[1] ? mu : cval[1];
      u128 term = mul_s64_u128(e.v, mu);
#pragma unroll
      for (int c = 0; c < kMaxChild; ++c)
        if (c < m && c != a) term = mul_u128(term, A[c]);
      G += term;
#pragma unroll
      for (int c = 0; c < kMaxChild; ++c)
        if (c == a) A[c] += mu;
    }
  }
  red[threadIdx.x] = active ? G : (u128)0;
  __syncthreads();
  for (int off = kLaneThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    B.partial[((size_t)T.partial_slot + gp.c) * B.d + row] = red[0];
}

// ---------------------------------------------------------------------
// per sub-plan: rows, median, double, certificate
// ---------------------------------------------------------------------
__global__ void finish_kernel(const SubplanTask *sps, EstBuffers B,
                              const double *approx, uint64_t *row_est,
                              double *est, int32_t *flags, int32_t n_tables) {
  __shared__ u128 xs[64], ps[64];
  __shared__ double xd[64];
  const SubplanTask S = sps[blockIdx.x];
  const int d = B.d;
  const int i = threadIdx.x;
  // partial sums of the sweeps (one per block of cut buckets): every lane
  // takes one row and every per-th slot, its loads in flight together
  const bool parts = S.type == kSpTriangle || S.type == kSpGeneric;
  const int per = (int)blockDim.x / d;  // lanes per row (d <= 32: >= 2)
  if (parts) {
    u128 acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < per * d) {
      const int r = i % d, k = i / d;
      for (int z0 = k; z0 < S.n_partials; z0 += 8 * per) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int z = z0 + u * per;
          if (z < S.n_partials) acc[u] += B.partial[((size_t)S.x_slot + z) * d + r];
        }
      }
    }
    u128 a = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) a += acc[u];
    ps[i] = a;
    __syncthreads();
  }
  // the fp64 rows are read only when the 128-bit ones are not certified
  const bool cert = S.type == kSpSingle ||
                    (S.type != kSpUnsupported &&
                     subplan_certified(S, B.n_sel, n_tables, B.w));
  const bool use_approx = !cert && S.approx_slot >= 0;
  if (i < d) {
    u128 x = 0;
    if (S.type == kSpSingle) {
      x = s64_to_u128(B.n_sel[S.single_table]);
    } else if (S.type == kSpTree) {
      x = B.xout[(size_t)S.x_slot * d + i];
    } else if (parts) {
      for (int k = 0; k < per; ++k) x += ps[k * d + i];
    }
    xs[i] = x;
    if (use_approx) {
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int z = 0;
      for (; z + 8 <= S.n_approx; z += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          acc[u] += approx[((size_t)S.approx_slot + z + u) * d + i];
      }
      for (; z < S.n_approx; ++z)
        acc[0] += approx[((size_t)S.approx_slot + z) * d + i];
      double a = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) a += acc[u];
      xd[i] = a;
    }
    if (row_est) {
      row_est[((size_t)blockIdx.x * d + i) * 2 + 0] = (uint64_t)x;
      row_est[((size_t)blockIdx.x * d + i) * 2 + 1] = (uint64_t)(x >> 64);
    }
  }
  __syncthreads();
  if (i != 0) return;
  if (S.type == kSpUnsupported) {
    est[blockIdx.x] = __builtin_nan("");
    flags[blockIdx.x] = 2;
    return;
  }
  if (use_approx) {
    // the 128-bit values may have wrapped: the median of the fp64
    // evaluation, flagged approximate
    for (int a = 1; a < d; ++a) {
      const double v = xd[a];
      int b = a - 1;
      while (b >= 0 && xd[b] > v) {
        xd[b + 1] = xd[b];
        --b;
      }
      xd[b + 1] = v;
    }
    est[blockIdx.x] = (d & 1) ? xd[d / 2] : (xd[d / 2 - 1] + xd[d / 2]) * 0.5;
    flags[blockIdx.x] = 4;
    return;
  }
  // insertion sort as signed 128-bit values
  for (int a = 1; a < d; ++a) {
    const u128 v = xs[a];
    int b = a - 1;
    while (b >= 0 && (__int128)xs[b] > (__int128)v) {
      xs[b + 1] = xs[b];
      --b;
    }
    xs[b + 1] = v;
  }
  double e;
  if (d & 1)
    e = i128_to_double(xs[d / 2]);
  else
    e = i128_to_double(xs[d / 2 - 1] + xs[d / 2]) * 0.5;
  est[blockIdx.x] = e;
  flags[blockIdx.x] = cert ? 1 : 0;
}

// ---------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------
// The grid of n tasks x d rows x X chunks (see GridMap); 0 blocks when it
// would exceed a 1-D grid.
static GridMap grid_map(int X, int n, int d, int64_t *blocks) {
  GridMap m;
  m.X = X;
  m.Q = n * d;
  m.d = d;
  m.xcd = m.Q >= 8 ? 1 : 0;
  const int64_t b = m.xcd ? 8ll * X * ((m.Q + 7) / 8) : (int64_t)X * m.Q;
  *blocks = b < 0x7FFFFFFFll ? b : 0;
  return m;
}
#define COMPASS_GRID(X, n)                                \
  int64_t blocks_;                                        \
  const GridMap gm_ = grid_map((X), (n), B.d, &blocks_);  \
  if (blocks_ == 0) return hipErrorInvalidConfiguration;

hipError_t launch_sort_rows(const SortJob *jobs, int n_jobs,
                            ResolveArgs R, const EstBuffers &B,
                            hipStream_t st) {
  R.blocks = (R.n + R.n_tri + kSortThreads - 1) / kSortThreads;
  const int n_pairs = n_jobs * B.d;
  if (n_pairs + R.blocks == 0) return hipSuccess;
  const int kpt = (B.w + kSortThreads - 1) / kSortThreads;
  // keys (one pad entry per 16), 16 digit starts (16-bit) per thread, the
  // scan scratch and the waves' bases; rows of more than 8 keys a thread:
  // keys unpadded, the scratch and bases in the keys' space
  const bool pad = kpt <= 8;
  const size_t lds =
      (size_t)(kpt * kSortThreads + (pad ? kpt * kSortThreads / 16 : 0)) *
          sizeof(uint64_t) +
      (size_t)kSortThreads * 16 * sizeof(uint16_t) +
      (pad ? (size_t)2 * (kSortThreads / 64) * 8 * sizeof(uint32_t) : 0);
  if (kpt <= 8)
    hipLaunchKernelGGL(sort_rows_kernel<8>, dim3((uint32_t)(n_pairs + R.blocks)),
                       dim3(kSortThreads), lds, st, jobs, B, n_pairs, R);
  else
    hipLaunchKernelGGL(sort_rows_kernel<kSortKpt>,
                       dim3((uint32_t)(n_pairs + R.blocks)), dim3(kSortThreads),
                       lds, st, jobs, B, n_pairs, R);
  return hipGetLastError();
}

hipError_t launch_node_merge(const NodeTask *tasks, int n, int max_L,
                             const EstBuffers &B, int stage_bytes,
                             hipStream_t st) {
  COMPASS_GRID((max_L + kMergeChunk - 1) / kMergeChunk, n);
  hipLaunchKernelGGL(node_merge_kernel, dim3((uint32_t)blocks_),
                     dim3(kMergeThreads), (size_t)stage_bytes, st, tasks, B,
                     stage_bytes, gm_);
  return hipGetLastError();
}

hipError_t launch_node(const NodeTask *tasks, int n, const EstBuffers &B,
                       hipStream_t st) {
  hipLaunchKernelGGL(node_kernel, dim3(n, B.d), dim3(kNodeThreads), 0, st,
                     tasks, B);
  return hipGetLastError();
}

hipError_t launch_node1(const NodeTask *tasks, int n, const EstBuffers &B,
                        hipStream_t st) {
  const int nch = (B.w + kN1Chunk - 1) / kN1Chunk;
  {
    COMPASS_GRID(nch, n);
    hipLaunchKernelGGL(node1_prefix_kernel, dim3((uint32_t)blocks_),
                       dim3(kN1Threads), 0, st, tasks, B, gm_);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  COMPASS_GRID(2 * nch, n);
  hipLaunchKernelGGL(node1_emit_kernel, dim3((uint32_t)blocks_), dim3(kN1Threads),
                     B.counter_bits == 32 ? (size_t)B.w * 4 : 0, st, tasks, B,
                     gm_);
  return hipGetLastError();
}

hipError_t launch_apex_prep(const NodeTask *tasks, int n, int Lmax_apex,
                            const EstBuffers &B, hipStream_t st) {
  COMPASS_GRID((Lmax_apex + kPrepChunk - 1) / kPrepChunk, n);
  hipLaunchKernelGGL(apex_prep_kernel, dim3((uint32_t)blocks_),
                     dim3(kPrepThreads), 0, st, tasks, B, gm_);
  return hipGetLastError();
}

hipError_t launch_tri_order(const TriTask *tasks, int n, const EstBuffers &B,
                            hipStream_t st) {
  const int tiles = (std::min(B.Lprep, kOrderCap) + kOrderTile - 1) / kOrderTile;
  COMPASS_GRID(tiles, n);
  // the ordering's keys and the segment blocks' piece starts share the
  // dynamic LDS
  static_assert((kOrderCap + 1) * 4 >= kOrderTile * 8, "key stage fits");
  hipLaunchKernelGGL(tri_order_kernel,
                     dim3((uint32_t)(blocks_ + (int64_t)n * B.d)),
                     dim3(kOrderThreads), (size_t)(kOrderCap + 1) * sizeof(int32_t),
                     st, tasks, B, gm_, (int)blocks_);
  return hipGetLastError();
}

hipError_t launch_tri_lane(const TriTask *tasks, int n, const TriGroup *groups,
                           int n_groups, int zblocks, const EstBuffers &B,
                           hipStream_t st) {
  // each (task, row, chunk) block does its work in exactly one of the two
  if (n_groups > 0) {
    COMPASS_GRID(zblocks, n_groups);
    hipLaunchKernelGGL(tri_fast_kernel, dim3((uint32_t)blocks_),
                       dim3(kLaneThreads * kFastSegs), (size_t)kFastLds, st,
                       tasks, groups, B, gm_);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  COMPASS_GRID(zblocks, n);
  hipLaunchKernelGGL(tri_lane_kernel, dim3((uint32_t)blocks_),
                     dim3(kLaneThreads), 0, st, tasks, B, gm_);
  return hipGetLastError();
}

hipError_t launch_finish(const SubplanTask *sps, int n, const EstBuffers &B,
                         const double *approx, uint64_t *row_est, double *est,
                         int32_t *flags, int32_t n_tables, hipStream_t st) {
  hipLaunchKernelGGL(finish_kernel, dim3(n), dim3(64), 0, st, sps, B, approx,
                     row_est, est, flags, n_tables);
  return hipGetLastError();
}


}  // namespace compass
