// enumerate.hip -- join order enumeration over sketch estimates (host).
//
// Section 6, Algorithm 1: depth-first search over the join graph that
// builds left-deep orders without cross products.  Sources are visited in
// increasing f(v) = alpha card(v)/max card + beta deg(v)/max deg; from a
// partial order C the adjacent tables are tried in increasing order of the
// estimate of C extended by them; a branch is abandoned as soon as its
// running cost (sum of the estimates of every prefix) exceeds the best
// complete cost; at most max_plans complete plans are counted per source
// (max_plans <= 0: unlimited, i.e. exhaustive).  Estimates come from
// compass_estimate (copied to the host by the caller); this step runs on
// the host, as in the paper.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <unordered_map>
#include <vector>

#include "compass.h"

namespace compass {
void set_last_error(const std::string &s);
}

namespace {

struct Enum {
  int n;
  std::vector<uint64_t> adj;
  std::unordered_map<uint64_t, double> est;
  int max_plans;
  double best_cost = 1e308;
  std::vector<int> best_order;
  bool have_best = false;
  int64_t total = 0;
  int p = 0;
  bool abort = false;
  bool missing = false;
  uint64_t missing_mask = 0;

  double lookup(uint64_t m) {
    auto it = est.find(m);
    if (it == est.end()) {
      missing = true;
      missing_mask = m;
      return 0.0;
    }
    return it->second;
  }

  void dfs(std::vector<int> &order, uint64_t mask, double cost) {
    if (abort || missing) return;
    cost += lookup(mask);
    if (have_best && cost > best_cost) return;
    if ((int)order.size() == n) {
      if (!have_best || cost < best_cost) {
        best_cost = cost;
        best_order = order;
        have_best = true;
      }
      ++p;
      ++total;
      if (max_plans > 0 && p == max_plans) abort = true;
      return;
    }
    uint64_t cand = 0;
    for (int a : order) cand |= adj[a];
    cand &= ~mask;
    std::vector<std::pair<double, int>> ext;
    for (int v = 0; v < n; ++v)
      if (cand >> v & 1ull) ext.push_back({lookup(mask | (1ull << v)), v});
    std::sort(ext.begin(), ext.end());
    for (auto &e : ext) {
      order.push_back(e.second);
      dfs(order, mask | (1ull << e.second), cost);
      order.pop_back();
      if (abort || missing) return;
    }
  }
};

}  // namespace

extern "C" compass_status compass_enumerate(
    int32_t n_tables, int32_t n_edges, const int32_t *edge_u,
    const int32_t *edge_v, const uint64_t *masks, const double *est,
    int32_t n_masks, const double *card, int32_t max_plans, double alpha,
    double beta, int32_t *order_out, double *cost_out, int64_t *n_plans_out) {
  if (n_tables < 1 || n_tables > 64 || n_edges < 0 || !masks || !est ||
      !card || !order_out || !cost_out || (n_edges > 0 && (!edge_u || !edge_v))) {
    compass::set_last_error("bad enumeration arguments");
    return COMPASS_E_ARG;
  }
  Enum E;
  E.n = n_tables;
  E.max_plans = max_plans;
  E.adj.assign(n_tables, 0);
  std::vector<int> deg(n_tables, 0);
  for (int e = 0; e < n_edges; ++e) {
    const int u = edge_u[e], v = edge_v[e];
    if (u < 0 || u >= n_tables || v < 0 || v >= n_tables || u == v) {
      compass::set_last_error("edge with bad endpoints");
      return COMPASS_E_GRAPH;
    }
    E.adj[u] |= 1ull << v;
    E.adj[v] |= 1ull << u;
    deg[u] += 1;
    deg[v] += 1;
  }
  for (int i = 0; i < n_masks; ++i) E.est[masks[i]] = est[i];
  double mc = 0, md = 0;
  for (int v = 0; v < n_tables; ++v) {
    mc = std::max(mc, card[v]);
    md = std::max(md, (double)deg[v]);
  }
  if (mc <= 0) mc = 1;
  if (md <= 0) md = 1;
  std::vector<std::pair<double, int>> src;
  for (int v = 0; v < n_tables; ++v)
    src.push_back({alpha * card[v] / mc + beta * deg[v] / md, v});
  std::sort(src.begin(), src.end());
  for (auto &s : src) {
    E.p = 0;
    E.abort = false;
    std::vector<int> order{s.second};
    E.dfs(order, 1ull << s.second, 0.0);
    if (E.missing) {
      char buf[96];
      snprintf(buf, sizeof buf, "no estimate for sub-plan 0x%llx",
               (unsigned long long)E.missing_mask);
      compass::set_last_error(buf);
      return COMPASS_E_GRAPH;
    }
  }
  if (!E.have_best) {
    compass::set_last_error("no complete plan (graph not connected?)");
    return COMPASS_E_GRAPH;
  }
  for (int i = 0; i < n_tables; ++i) order_out[i] = E.best_order[i];
  *cost_out = E.best_cost;
  if (n_plans_out) *n_plans_out = E.total;
  return COMPASS_OK;
}

// The paper's default variant (Section 7.1; defined in Section 7.2.8):
// greedy left-deep search from ONE source, the smaller table (by card,
// ties to the lower id) of the two-table sub-plan with the smallest
// estimate (ties to the lower mask); from it the order grows by the
// adjacent table whose extended sub-plan has the smallest estimate, with
// no backtracking (Algorithm 1 with max_plans = 1 from that source alone).
extern "C" compass_status compass_enumerate_greedy(
    int32_t n_tables, int32_t n_edges, const int32_t *edge_u,
    const int32_t *edge_v, const uint64_t *masks, const double *est,
    int32_t n_masks, const double *card, int32_t *order_out, double *cost_out) {
  if (n_tables < 1 || n_tables > 64 || n_edges < 0 || !masks || !est ||
      !card || !order_out || !cost_out || (n_edges > 0 && (!edge_u || !edge_v))) {
    compass::set_last_error("bad enumeration arguments");
    return COMPASS_E_ARG;
  }
  Enum E;
  E.n = n_tables;
  E.max_plans = 1;
  E.adj.assign(n_tables, 0);
  for (int e = 0; e < n_edges; ++e) {
    const int u = edge_u[e], v = edge_v[e];
    if (u < 0 || u >= n_tables || v < 0 || v >= n_tables || u == v) {
      compass::set_last_error("edge with bad endpoints");
      return COMPASS_E_GRAPH;
    }
    E.adj[u] |= 1ull << v;
    E.adj[v] |= 1ull << u;
  }
  for (int i = 0; i < n_masks; ++i) E.est[masks[i]] = est[i];
  int source = 0;
  if (n_tables > 1) {
    bool found = false;
    double best = 0;
    uint64_t best_mask = 0;
    for (int u = 0; u < n_tables; ++u)
      for (int v = u + 1; v < n_tables; ++v) {
        if (!(E.adj[u] >> v & 1ull)) continue;
        const uint64_t m = (1ull << u) | (1ull << v);
        const double x = E.lookup(m);
        if (E.missing) break;
        if (!found || x < best || (x == best && m < best_mask)) {
          found = true;
          best = x;
          best_mask = m;
          source = card[v] < card[u] ? v : u;
        }
      }
    if (!found && !E.missing) {
      compass::set_last_error("no join edge");
      return COMPASS_E_GRAPH;
    }
  }
  std::vector<int> order{source};
  if (!E.missing) E.dfs(order, 1ull << source, 0.0);
  if (E.missing) {
    char buf[96];
    snprintf(buf, sizeof buf, "no estimate for sub-plan 0x%llx",
             (unsigned long long)E.missing_mask);
    compass::set_last_error(buf);
    return COMPASS_E_GRAPH;
  }
  if (!E.have_best) {
    compass::set_last_error("no complete plan (graph not connected?)");
    return COMPASS_E_GRAPH;
  }
  for (int i = 0; i < n_tables; ++i) order_out[i] = E.best_order[i];
  *cost_out = E.best_cost;
  return COMPASS_OK;
}
