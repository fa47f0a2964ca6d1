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

// Compact element of a two-child apex (both children are the cut edge's
// endpoints), used when every magnitude involved is below 2^30 and every
// message and product fits in 64 bits.  32 bytes: one scalar x8 load.
struct TriElemN {
  int32_t v;        // the apex's counter on the child's edge
  uint32_t kc;      // child slot << 31 | |child's own bucket on that edge|
  int64_t mu;       // the child's unconditioned message M
  int64_t vm;       // v * M
  int32_t run_lo;   // lowest position of the same-child run holding it
  int32_t run_hi;   // highest position of that run
};

// Exclusive prefix sums over one ordering tile of a two-child apex's
// merged list, after every run piece in the tile has been ordered by
// ascending child key: entry q holds the sums of M, v * M and v over the
// tile's first q reordered elements, wrapping modulo 2^64 / 2^32.
// Differences give the masked sums of any run piece inside the tile.
// 24 bytes.
struct TriPre {
  int64_t m;
  int64_t x;
  int32_t v;
  int32_t pad;
};

// One piece of the two-child sweep: a maximal same-child run of [z, L)
// cut at the ordering tiles' starts.  16 bytes.
struct TriPiece {
  int32_t lo, hi;   // positions [lo, hi]
  int32_t info;     // bit 0: child slot; bit 1: summed by search; bits 2..: tile
  int32_t pad;
};

// One element of a node's merged list, gathered once by the merge so that
// the node's sweeps read consecutive records (32 bytes).
struct NodeRec {
  u128 mu;        // the child's message at the bucket (child lists only)
  int64_t v;      // the node's counter at the bucket
  uint32_t aj;    // list << 16 | bucket
  uint32_t pad;
};

struct EstBuffers {
  const void *const *sides;   // [2 * n_edges] counter arrays (d x w)
  const int64_t *n_sel;       // [n_tables]
  const uint64_t *sorted;     // [side][row][w] keys (|v| << 16 | j)
  u128 *msg;                  // [slot][row][w]
  uint32_t *merged;           // [scratch slot][row][Lmax]
  NodeRec *nrec;              // [scratch slot][row][Lmax]
  u128 *n1tot;                // [scratch slot][row][2 * kN1MaxChunks]
  u128 *xout;                 // [slot][row]
  TriElem *prep;              // [prep slot][row][Lprep]
  TriElemN *prepn;            // [prep slot][row][Lprep] (two-child apexes)
  int32_t *prep_z;            // [prep slot][row] leading zero-counter run
  uint32_t *tkey;             // [prep slot][row][Lprep] run-ordered keys
  TriPre *tpre;               // [prep slot][row][tile][kOrderTile + 1]
  int32_t *tseg;              // [prep slot][row][kFastSegs + 1] sweep bounds
  TriPiece *tpiece;           // [prep slot][row][Pcap] run pieces
  int32_t *tsegp;             // [prep slot][row][kFastSegs + 1] piece bounds
  u128 *partial;              // [slot][row]
  int32_t counter_bits;
  int32_t d;
  int32_t w;
  int32_t Lmax;
  int32_t Lprep;
  int32_t Pcap;               // run pieces per (prep slot, row)
};

}  // namespace compass
