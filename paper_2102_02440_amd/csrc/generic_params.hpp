// generic_params.hpp -- plans of the generic sub-plan contraction.
//
// Any connected sub-plan, by conditioning: the edges outside a spanning
// tree of the sub-plan are "conditioned" (their bucket fixed to J_e), the
// tree is contracted bottom-up for every assignment J, and the results are
// summed over the w^k assignments.  At a node, a conditioned edge is one
// more element (value = the node's counter at J_e) with weight 1.
#pragma once
#include <stdint.h>

#include "device_math.hpp"
#include "estimate_params.hpp"

namespace compass {

constexpr int kGenMaxGroups = 8;     // child groups (and separately fixed
                                     // groups) of one node
constexpr int kGenMaxCut = 6;        // conditioned edges of one sub-plan
constexpr int kGenThreads = 256;     // one tile of a node's list
constexpr uint32_t kGenQuery = 0xFFFFu;  // list code of the parent buckets

// One node of a sub-plan's rooted spanning tree; a plan's nodes are stored
// in post-order (children first, the root last).
struct GenNode {
  int32_t parent_side;   // this table's side on the parent edge (-1: root)
  int32_t parent_eid;
  int32_t n_child;
  int32_t n_fixed;
  int32_t list_off;      // merged list of the node within its plan's lists
  int32_t list_len;      // (n_child + (parent_side >= 0)) * w
  int32_t msg;           // its message index in the plan (-1: root)
  int32_t is_static;     // no conditioned edge at or below it
  int32_t c_side[kGenMaxGroups];  // child groups: this table's side on the edge
  int32_t c_eid[kGenMaxGroups];
  int32_t c_msg[kGenMaxGroups];   // the child's message index
  int32_t f_side[kGenMaxGroups];  // fixed groups: this table's side on the
  int32_t f_eid[kGenMaxGroups];   //   conditioned edge, its id and its digit
  int32_t f_cut[kGenMaxGroups];   //   in J
};

struct GenPlan {
  int32_t node0, n_nodes;
  int32_t n_msgs;        // non-root nodes
  int32_t n_cut;
  int64_t n_assign;      // w^n_cut
  int64_t lists_off;     // offset of block 0's merged lists
  int64_t msg_off;       // offset (values) of block 0's message scratch
  int32_t lists_len;     // merged list entries of one block (all nodes)
  int32_t pad;
  int32_t out_slot;      // first output slot (one per J block)
  int32_t n_blocks;      // J blocks per row
  int32_t sp;            // sub-plan index (for the certificate check)
  int32_t fp64;          // 1: evaluation in double for uncertified sub-plans
};

// A block of the contraction kernel: plan and J block (blockIdx.y = row).
struct GenBlock {
  int32_t plan, jb;
};

// Device views of one call's generic plans (kernel argument).
struct GenArgs {
  const GenNode *nodes;
  const GenPlan *plans;
  const GenBlock *blocks;
  uint32_t *lists;          // merged lists, one region per block
  char *msg;                // message scratch (16 bytes per value)
  u128 *partial;            // exact plans: [slot][row]
  double *approx;           // fp64 plans: [slot][row]
  const SubplanTask *sps;
  int32_t n_tables;
  int32_t pad;
};

}  // namespace compass
