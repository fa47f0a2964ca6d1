// estimate_params.hpp -- device-side plan of a compass_estimate call.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace compass {

constexpr int kMaxChild = 6;
constexpr int kNodeThreads = 1024;
constexpr int kLaneThreads = 128;  // cut buckets J per triangle workgroup
constexpr int kMaxEstimateW = 16384;  // per-(sketch,row) sort held in LDS
constexpr int kSortThreads = 1024;    // one workgroup sorts a row's keys
constexpr int kSortKpt = kMaxEstimateW / kSortThreads;  // keys per thread
constexpr int kNodeStageBytes = 96 * 1024;  // node merge: staged magnitudes
constexpr size_t kNodeScratchBytes = (size_t)1 << 30;  // per level launch
constexpr int kMaxGridZ = 65535;  // tasks per launch (grid z)
constexpr int kMergeThreads = 512;  // node list merge
constexpr int kMergeChunk = 2048;  // merged elements per workgroup
constexpr int kN1Threads = 256;   // one-child nodes
constexpr int kN1Per = 4;
constexpr int kN1Chunk = kN1Threads * kN1Per;
constexpr int kN1MaxChunks = (kMaxEstimateW + kN1Chunk - 1) / kN1Chunk;
static_assert(kN1MaxChunks <= 64, "chunk offsets are scanned by one wave");
constexpr int kPrepThreads = 256;  // apex preparation
constexpr int kPrepPer = 4;
constexpr int kPrepChunk = kPrepThreads * kPrepPer;
constexpr int kOrderThreads = 1024;
constexpr int kSegThreads = 1024;
constexpr int kSegPer = 16;
constexpr int kFastSegs = 8;  // slots of a sweep workgroup (and run groups)
constexpr int kTriGroupMax = 4;  // triangle tasks swept together
constexpr int kSearchMin = 8;  // shortest run the sweep sums by search
constexpr int kOrderTile = 2048;  // positions ordered by one workgroup
constexpr int kOrderCap = 16384;  // longest two-child apex list run-ordered
constexpr int kFastStageBytes = kOrderCap * 4;  // its keys, staged in LDS
static_assert(kSegThreads * kSegPer >= kOrderCap, "one pass over the list");

enum { kModeMessage = 0, kModeTreeRoot = 1, kModeTriRootPrep = 2 };

// Several rootings of one sub-plan may be planned (the apex candidates of
// a triangle); each task carries the candidates' tables, and only the
// rooting whose table has the fewest selected rows (ties: the earlier
// candidate) does work.  n <= 1: always runs.  `on` is resolved on the
// device once per estimate, before the other launches (resolve_kernel):
// 0 = the task does nothing; a node task: 1, plus 2 for a two-child apex
// whose sweep is the compact one; a triangle task: 1 + its arithmetic path
// (kTriFast, kTriNarrow, kTriWide).
struct TaskGuard {
  int32_t n;
  int32_t self;
  int32_t tab[3];
  int32_t on;
};
enum { kSpSingle = 0, kSpTree = 1, kSpTriangle = 2, kSpUnsupported = 3,
       kSpGeneric = 4 };

// One node of one sub-plan's rooted spanning tree (blockIdx.y = sketch row).
// Lists: children 0..m-1 (weighted by their messages), then the parent
// bucket list (query points of the outgoing message) if parent_side >= 0,
// then the cut-edge bucket list (query points of the cut constants) if
// cut_side >= 0.
struct NodeTask {
  TaskGuard guard;
  int32_t mode;
  int32_t m;
  int32_t parent_side, parent_eid;
  int32_t cut_side, cut_eid;
  int32_t msg_slot;    // message out (mode 0)
  int32_t cmsg_slot;   // cut constants out (mode 0 with a cut edge)
  int32_t out_slot;    // tree-root X slot (mode 1) / root-prep slot (mode 2)
  int32_t scratch_slot;
  int32_t child_side[kMaxChild];
  int32_t child_eid[kMaxChild];
  int32_t child_msg[kMaxChild];
  int32_t child_cut[kMaxChild];   // mode 2: index (0/1) of the cut endpoint, or -1
  int32_t child_parent_eid[kMaxChild];  // mode 2: edge id of the child's parent edge
  int32_t tri;                    // mode 2: its triangle task
  int32_t pad;
};

// Triangle sub-plan: the root (apex) sweeps its merged child list once per
// cut-edge bucket J; the two cut endpoints' messages switch to their cut
// constant when their parent-edge element ranks above the cut element.
struct TriTask {
  TaskGuard guard;
  int32_t prep_slot;        // root merged-list arrays
  int32_t L;                // root merged-list length
  int32_t m;                // root children
  int32_t cut_eid;
  int32_t cut_side[2];      // sides (endpoint u, endpoint v) of the cut edge
  int32_t cut_cmsg[2];      // cut-constant slots of u and v
  int32_t cut_child[2];     // root child slots of u and v
  int32_t cut_peid[2];      // edge ids joining u and v to the apex
  int32_t partial_slot;     // first of gridDim.z partial sums
  int32_t root_table;
  uint64_t child_tables[kMaxChild];  // tables of each child's subtree
};

// Triangle tasks whose apex list, runs and cut edge are the same (the same
// apex table, child sides and cut edge; they differ in the messages of the
// subtrees below): the two-child sweep searches once for all of them.
struct TriGroup {
  int32_t n;
  int32_t member[kTriGroupMax];
  int32_t pad[3];
};

// One row sort: the sketch side and its counters (the pointer carried
// here saves the kernel a dependent load of the side table).
struct SortJob {
  const void *counters;
  int32_t side, pad;
};

// The tasks whose guards resolve_task sets (blocks: workgroups of
// kSortThreads lanes for them, one task a lane).
struct ResolveArgs {
  NodeTask *tasks;
  TriTask *tris;
  int32_t n, n_tri;
  int32_t blocks, pad;
};

struct SubplanTask {
  int32_t type;
  int32_t n_tables;
  int32_t n_edges;
  int32_t single_table;
  int32_t x_slot;           // tree: X slot; triangle, generic: first partial slot
  int32_t n_partials;
  uint64_t mask;
  int32_t approx_slot;      // first slot of the fp64 evaluation (-1: none)
  int32_t n_approx;         // its slots (summed per row)
};

}  // namespace compass
