// agms_params.hpp -- kernel arguments of the AGMS baseline (Section 4.1).
#pragma once
#include <stdint.h>

#include "build_params.hpp"

namespace compass {

constexpr int kAgmsMaxJoins = 4;
constexpr int kAgmsMaxCounters = 1024;  // r * b: at most one lane each

struct AgmsParams {
  int64_t n_rows;
  int64_t rows_per_chunk;
  int32_t n_preds;
  int32_t n_joins;
  int32_t K;                   // r * b basic sketches
  int32_t count_selected;
  int64_t *n_selected;
  int64_t *counters;           // K int64
  const RowSeeds *seeds;       // device, n_joins x K (b0, b1 unused)
  PredDev preds[kMaxPreds];
  KeyDev keys[kAgmsMaxJoins];
};

struct AgmsEstArgs {
  const int64_t *sk[16];       // per table: r x b counters
  const int64_t *n_sel[16];    // per table: selected rows (device)
  int32_t n_tables, r, b, pad;
};

}  // namespace compass
