#!/usr/bin/env python
"""Benchmark of the fused selection-scan + Fast-AGMS sketch build and the
merged-sketch sub-plan estimates on one MI355X.

One step = the whole hot path over the 6a-shaped five-table workload (ci
36M, mk 4.5M, t 2.5M, n 4.2M, k 134k rows; point / range / subset
selections; 10 attribute sketches, d=7, w=8192, int32 counters): one fused
scan per table building all of its sketches, then the estimates of all 19
connected sub-plans (4 of them contain the triangle).  Inputs are resident in
HBM before the timed region starts.

Prints one JSON line (see the fields at the bottom of main()).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=3_000_000,
                    help="cast_info rows in the oracle's timed sample")
    return ap.parse_args()


def algorithmic_work(q, n_sel):
    """Bytes every table scan must move at minimum, and hash updates.

    bytes = predicate columns x all rows + key columns x selected rows +
    counters written once; a column read by several predicates or sketches
    counts once.  updates = selected rows x sketches x d."""
    total_bytes = 0
    updates = 0
    for t, tb in enumerate(q.tables):
        inc = q.incident(t)
        pcols = {p.col for p in tb.preds}
        kcols = {c for (_, _, c) in inc}
        total_bytes += sum(tb.cols[c].dtype.itemsize * tb.n_rows for c in pcols)
        total_bytes += sum(tb.cols[c].dtype.itemsize * n_sel[t] for c in kcols)
        total_bytes += len(inc) * q.d * q.w * (q.counter_bits // 8)
        updates += n_sel[t] * len(inc) * q.d
    return total_bytes, updates


def cpu_baseline(q, sample_rows):
    """The oracle, as it stands, on a bounded sample of the same workload:
    every table but cast_info in full plus the first `sample_rows` rows of
    cast_info; rows scanned per second of oracle time."""
    from oracle import oracle as o
    o.build()
    rows = 0
    t0 = time.perf_counter()
    for t, tb in enumerate(q.tables):
        inc = q.incident(t)
        if tb.name == "ci":
            cols = {c: v[:sample_rows] for c, v in tb.cols.items()}
        else:
            cols = tb.cols
        mask = o.eval_predicates(cols, tb.preds)
        for (e, _, c) in inc:
            o.sketch(cols[c][mask], q.seeds[e], q.d, q.w)
        rows += len(next(iter(cols.values())))
    dt = time.perf_counter() - t0
    return {"value": rows / dt, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": "oracle sketch build (numpy predicates + single-threaded C "
                      "hash loop) of k, mk, t, n in full and the first %d rows of "
                      "ci: %d rows in %.1f s" % (sample_rows, rows, dt)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(sketches would shard by rows with one integer all-reduce; see "
              "the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2102_02440_amd import compass as C
    from paper_2102_02440_amd import workloads as W

    seed = W.DEFAULT_SEED if args.seed is None else args.seed
    t0 = time.time()
    q = W.job6a(seed=seed)
    print("[bench] generated 6a-shaped workload in %.1fs" % (time.time() - t0),
          file=sys.stderr, flush=True)
    dq = C.DeviceQuery(q, device="cuda")
    n_tab = len(q.tables)
    masks = []
    adj = {}
    for e in q.edges:
        adj.setdefault(e.u, set()).add(e.v)
        adj.setdefault(e.v, set()).add(e.u)
    for m in range(1, 1 << n_tab):
        tabs = [t for t in range(n_tab) if m >> t & 1]
        seen = {tabs[0]}
        stack = [tabs[0]]
        while stack:
            a = stack.pop()
            for b in adj.get(a, ()):
                if m >> b & 1 and b not in seen:
                    seen.add(b)
                    stack.append(b)
        if len(seen) == len(tabs):
            masks.append(m)
    masks.sort(key=lambda m: (bin(m).count("1"), m))
    torch.cuda.synchronize()

    def step():
        dq.build()
        return dq.estimate(masks)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_sel = dq.n_selected.cpu().tolist()

    C.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        row_est, est, flags = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    C.profile_enable(False)
    prof = {k: C.profile_take(k) for k in
            ["fill_zero", "scan_sketch", "sort_rows", "node", "tri_lane", "finish"]}

    ms_step = dt * 1e3 / args.steps
    rows_per_step = sum(tb.n_rows for tb in q.tables)
    value = rows_per_step * args.steps / dt
    alg_bytes, updates = algorithmic_work(q, n_sel)
    scan_n, scan_ms = prof["scan_sketch"]
    build_ms_step = (scan_ms + prof["fill_zero"][1]) / args.steps
    est_ms_step = sum(prof[k][1] for k in ["sort_rows", "node", "tri_lane",
                                           "finish"]) / args.steps
    # dominant kernel: the fused scan + sketch build
    scan_s_step = scan_ms / args.steps / 1e3
    achieved_gbs = alg_bytes / scan_s_step / 1e9
    upd_rate = updates / scan_s_step
    roofline = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
                "traffic": None, "kernel": "scan_sketch",
                "launches_per_step": scan_n / args.steps,
                "alg_bytes_per_step": alg_bytes,
                "hash_updates_per_step": updates,
                "hash_updates_per_s": upd_rate}
    # accuracy against stored exact truths (oracle hash aggregation)
    qerr = None
    tp = os.path.join(ROOT, "tests", "golden", "job6a_truth.json")
    if os.path.exists(tp):
        tr = json.load(open(tp))
        if tr.get("seed") == seed and tr.get("scale") == 1.0 and tr["masks"] == masks:
            e = np.maximum(est.cpu().numpy(), 1.0)
            t = np.maximum(np.asarray(tr["true"], dtype=np.float64), 1.0)
            qe = np.maximum(e / t, t / e)
            qerr = {"median": float(np.median(qe)), "p90": float(np.percentile(qe, 90)),
                    "max": float(qe.max())}
    out = {
        "metric": "filtered rows sketched/s (% HBM roofline); subplan estimates/s at q-error",
        "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "job6a-shaped five tables: ci 36M, mk 4.5M, t 2.5M, "
                               "n 4.2M, k 134k rows; 10 sketches d=7 w=8192 int32; "
                               "19 sub-plan estimates",
                   "rows_per_step": rows_per_step, "selected_rows": n_sel,
                   "seed": seed, "parallelism": "single-gpu"},
        "build_ms_per_step": build_ms_step,
        "estimate_ms_per_step": est_ms_step,
        "subplan_estimates_per_s": len(masks) / (est_ms_step / 1e3) if est_ms_step else None,
        "qerror": qerr,
        "kernel_ms_per_step": {k: v[1] / args.steps for k, v in prof.items()},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(q, args.cpu_sample_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
