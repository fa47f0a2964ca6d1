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
METRIC = "filtered rows sketched/s (% HBM roofline); subplan estimates/s at q-error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=1_000_000,
                    help="rows of mk and ci in the oracle's one-thread sample")
    ap.add_argument("--only-headline", action="store_true",
                    help="default workload: skip the large-scan and batched "
                         "sub-measurements")
    ap.add_argument("--config-steps", type=int, default=5,
                    help="timed launches of the large-scan and batched "
                         "sub-measurements")
    ap.add_argument("--workload", default="job6a",
                    choices=["job6a", "batch", "learned", "large", "partition",
                             "partition_kd", "agms", "select"],
                    help="job6a: the headline step (default); batch: 512 "
                         "queries in one graph-captured persistent launch vs "
                         "one launch per sketch; learned: train + evaluate "
                         "the correction network")
    ap.add_argument("--queries", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=30)
    return ap.parse_args()


def algorithmic_work(q, n_sel, with_preds=None):
    """Bytes every table scan must move at minimum, and hash updates.

    bytes = predicate columns x all rows + key columns x selected rows +
    counters written once; a column read by several predicates or sketches
    counts once.  updates = selected rows x sketches x d.  with_preds:
    None = every table; False = tables without predicates (the fused scan
    kernel builds them); True = tables with predicates (two-phase build)."""
    total_bytes = 0
    updates = 0
    for t, tb in enumerate(q.tables):
        if with_preds is not None and bool(tb.preds) != with_preds:
            continue
        inc = q.incident(t)
        pcols = {p.col for p in tb.preds}
        kcols = {c for (_, _, c) in inc}
        total_bytes += sum(tb.cols[c].dtype.itemsize * tb.n_rows for c in pcols)
        total_bytes += sum(tb.cols[c].dtype.itemsize * n_sel[t] for c in kcols)
        total_bytes += len(inc) * q.d * q.w * (q.counter_bits // 8)
        updates += n_sel[t] * len(inc) * q.d
    return total_bytes, updates


SCAN_SOURCES = ["scan_common.hpp", "build_kernels.hip", "build_params.hpp",
                "device_math.hpp"]

# Integer VALU peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# 32-bit operation per lane per clock (no packed 32-bit integer issue).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# fp32 vector peak of MI355X (FMA = 2 flops)
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Algorithmic 32-bit integer operations per unit of work:
#  hash update (key below 2^32): four Horner steps of a 61 x 32-bit
#    multiply-add mod 2^61-1 at 6 operations (two 32 x 32 -> 64
#    multiply-adds, one AND, one 64-bit shift, two 64-bit adds), two
#    canonical reductions at 3, sign 1, bucket 1, LDS add 1.
OPS_PER_HASH_UPDATE = 4 * 6 + 2 * 3 + 3


def source_hash(names):
    """sha256 over the given kernel sources (identifies the kernel build)."""
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2102_02440_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(profile, names):
    """HBM bytes per step of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy kernel),
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != source_hash(names):
        return None
    try:
        return float(vals["hbm_bytes_per_step"])
    except (KeyError, ValueError):
        return None


def timed_steps(C, torch, step, steps, dominant):
    """Runs `steps` steps between two device synchronisations; only the
    dominant kernel's launches carry timing events (the other kernels'
    events would add their own cost to the timed region).  Returns
    (seconds per step, (launches, total ms) of the dominant kernel)."""
    C.profile_take(dominant)
    C.profile_select([dominant])
    C.profile_enable(True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / steps
    C.profile_enable(False)
    C.profile_select(None)
    return dt, C.profile_take(dominant)


def profiled_steps(C, torch, step, steps, names):
    """Per-kernel (launches, total ms) over `steps` further steps with every
    kernel's events recorded (outside the timed region)."""
    for n in names:
        C.profile_take(n)
    C.profile_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    C.profile_enable(False)
    return {n: C.profile_take(n) for n in names}


def cpu_model():
    """CPU model name of this host (first 'model name' of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _median_time(fn, runs):
    ts = []
    for _ in range(runs):
        a = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - a)
    return float(sorted(ts)[len(ts) // 2])


def cpu_baseline(q, masks, n_sel_step, sample_rows=1_000_000, runs=3):
    """The oracle, as it stands, on the GPU machine's host cores, for the step
    the GPU line times: the selection + sketch build of all five tables and
    the 19 sub-plan estimates.  With every thread (OpenMP; sketches by
    threads with private counters, summed): the whole build (median of
    `runs`) and every estimate (one run).  With one thread: the build on a
    sample (k, t and n in full, the first `sample_rows` rows of mk and ci)
    and the estimates of the 15 tree sub-plans on all rows plus one row of
    the costliest triangle sub-plan, extrapolated to all 19 x d.  Value:
    selected rows per second of the all-thread step (build + estimates)."""
    import numpy as np
    from oracle import oracle as o
    o.build()
    nt = o.default_threads()

    def build(threads, sample=None):
        side = [None] * (2 * len(q.edges))
        ns = []
        for t, tb in enumerate(q.tables):
            cols = tb.cols
            if sample is not None and tb.name in ("mk", "ci"):
                cols = {c: v[:sample] for c, v in cols.items()}
            mask = o.eval_predicates(cols, tb.preds)
            ns.append(int(mask.sum()))
            for (e, sd, c) in q.incident(t):
                side[2 * e + sd] = o.sketch(cols[c][mask], q.seeds[e], q.d, q.w,
                                            threads=threads)
        return side, ns

    out = {}
    side, ns = build(nt)
    assert ns == list(n_sel_step)
    t_build = _median_time(lambda: build(nt), runs)
    o.set_threads(nt)
    a = time.perf_counter()
    o.estimate(len(q.tables), q.edge_u, q.edge_v, q.d, q.w, side, ns, masks)
    t_est = time.perf_counter() - a
    sel = sum(ns)
    # one thread
    _, ns1 = build(1, sample_rows)
    t_build1 = _median_time(lambda: build(1, sample_rows), 1)
    o.set_threads(1)
    tri = [m for m in masks if (m & 0b1110) == 0b1110]
    trees = [m for m in masks if m not in tri]
    a = time.perf_counter()
    o.estimate(len(q.tables), q.edge_u, q.edge_v, q.d, q.w, side, ns, trees)
    t_trees1 = time.perf_counter() - a
    worst = max(tri, key=lambda m: bin(m).count("1"))
    a = time.perf_counter()
    o.estimate(len(q.tables), q.edge_u, q.edge_v, 1, q.w, [x[:1] for x in side], ns,
               [worst])
    t_tri_row1 = time.perf_counter() - a
    o.set_threads(nt)
    t_est1 = t_trees1 + len(tri) * q.d * t_tri_row1
    out = {"value": sel / (t_build + t_est), "unit": "rows/s", "cores": nt,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": "%d threads: the whole step (all five tables' selections and "
                     "sketches, median of %d builds: %.2f s; the 19 sub-plan "
                     "estimates on all %d rows: %.2f s); rows/s = selected rows "
                     "(%d) per step second" % (nt, runs, t_build, q.d, t_est, sel),
           "build_selected_rows_per_s": sel / t_build,
           "subplan_estimates_per_s": len(masks) / t_est,
           "single_thread": {
               "build_selected_rows_per_s": sum(ns1) / t_build1,
               "subplan_estimates_per_s": len(masks) / t_est1,
               "value": sel / (sel / (sum(ns1) / t_build1) + t_est1),
               "sample": "build of k, t, n in full and the first %d rows of mk and "
                         "ci (%d selected rows, %.2f s); estimates: the %d tree "
                         "sub-plans on all rows (%.2f s) plus one row of the "
                         "five-table triangle sub-plan (%.2f s) taken for each of "
                         "the %d triangle sub-plans x %d rows" % (
                             sample_rows, sum(ns1), t_build1, len(trees), t_trees1,
                             t_tri_row1, len(tri), q.d)}}
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (sketches "
              "would shard by rows, then one integer sum all-reduce of the "
              "counters). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "learned":
        return run_learned(args)
    if args.workload == "large":
        return run_large(args)
    if args.workload == "partition":
        return run_partition(args)
    if args.workload == "partition_kd":
        return run_partition_kd(args)
    if args.workload == "agms":
        return run_agms(args)
    if args.workload == "select":
        return run_select(args)
    return run_job6a(args)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measure_batch(steps, warmup, seed, n_queries=512, cpu=True):
    """512 queries (2..17 tables over a pool of 48 tables of 10k..36M rows,
    ~4k attribute sketches, d in {5,7,11}, w in {1024..16384}): the batched
    persistent graph-captured build vs the plain path (one launch per
    sketch), same counters bit for bit."""
    import torch
    from paper_2102_02440_amd import compass as C
    from paper_2102_02440_amd import workloads as W
    t0 = time.time()
    pool = W.schema_pool(seed)
    qs = W.query_batch(pool, seed, n_queries=n_queries)
    log("[bench] batch: pool %d rows, %d queries in %.1fs" % (
        sum(p.n_rows for p in pool), len(qs), time.time() - t0))
    db = C.DeviceBatch(pool, qs)
    n_sketch = sum(len(j["keys"]) for j in db.jobs)
    rows = sum(j["n_rows"] for j in db.jobs)
    t0 = time.time()
    plan = db.plan()
    info = plan.info()
    log("[bench] batch: plan %s in %.1fs" % (info, time.time() - t0))

    def timed(fn, k):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / k

    t_batch = timed(plan.launch, steps)
    # work of one launch (the plan clears the counters and selected counts)
    updates, alg_bytes, sel = 0, 0, 0
    for j in db.jobs:
        ns = int(j["n_selected"].item())
        nk = len(j["keys"])
        sel += ns
        updates += ns * nk * j["d"]
        alg_bytes += sum(c.element_size() for c in j["pred_cols"]) * j["n_rows"]
        alg_bytes += sum(k.element_size() for k in set(j["keys"])) * ns
        alg_bytes += nk * j["d"] * j["w"] * (32 // 8)
    tops = updates * OPS_PER_HASH_UPDATE / t_batch / 1e12
    snap = [[x.clone() for x in sides] for sides in db.sides]
    t_plain = timed(db.build_per_sketch, max(1, steps // 2))
    same = all(torch.equal(a, b) for sa, sb in zip(snap, db.sides) for a, b in zip(sa, sb))
    t_table = timed(db.build_per_table, max(1, steps // 2))
    out = {"workload": "batched: %d queries, %d scan jobs, %d attribute sketches over a "
                       "48-table pool (10k..36M rows)" % (len(qs), len(db.jobs), n_sketch),
           "value": sel / t_batch, "unit": "rows/s", "ms_per_step": t_batch * 1e3,
           "steps": steps, "warmup": warmup, "dtype": "int32",
           "input_rows_per_s": rows / t_batch, "rows_per_step": rows,
           "selected_rows_per_step": sel,
           "sketches_per_s": n_sketch / t_batch,
           "plain_one_launch_per_sketch_ms": t_plain * 1e3,
           "one_launch_per_table_ms": t_table * 1e3,
           "speedup_vs_plain": t_plain / t_batch,
           "bit_exact_vs_plain": bool(same), "plan": info,
           # the whole plan is one graph launch (batch_scan, batch_compact,
           # batch_hash): its hash updates over the launch's host-clock time,
           # bound by integer ALU like the fused scan
           "roofline": {"bound": "alu", "achieved": tops, "peak": ALU_PEAK_TOPS,
                        "unit": "TOP/s", "frac": tops / ALU_PEAK_TOPS, "traffic": None,
                        "kernel": "batch plan (one graph launch)",
                        "hash_updates_per_step": updates,
                        "ops_per_hash_update": OPS_PER_HASH_UPDATE,
                        "hbm_view": {"alg_bytes_per_step": alg_bytes,
                                     "achieved_gbs": alg_bytes / t_batch / 1e9,
                                     "frac": alg_bytes / t_batch / 1e9 / HBM_PEAK_GBS}}}
    plan.close()
    if cpu:
        out["cpu_baseline"] = cpu_baseline_batch(pool, qs, seed)
    del db
    torch.cuda.empty_cache()
    return out


def cpu_baseline_batch(pool, qs, seed, rows_mt=300_000_000, rows_1=30_000_000):
    """The oracle builds the batch's sketches one job at a time (selection,
    then each sketch), on a seeded sample of the jobs: all threads on
    jobs totalling about `rows_mt` scanned rows, one thread on about
    `rows_1`."""
    import numpy as np
    from oracle import oracle as o
    o.build()
    nt = o.default_threads()
    jobs = []
    for pq in qs:
        for t, ptab in enumerate(pq.tables):
            inc = pq.incident(t)
            if inc:
                jobs.append((ptab, pq.preds[t], [(pq.seeds[e], c) for (e, _, c) in inc],
                             pq.d, pq.w))
    order = np.random.default_rng(seed + 77).permutation(len(jobs))

    def pick(budget):
        out, r = [], 0
        for j in order:
            if r >= budget:
                break
            out.append(jobs[j])
            r += pool[jobs[j][0]].n_rows
        return out, r

    def run(sample, threads):
        sel, nsk = 0, 0
        for (ptab, preds, sk, d, w) in sample:
            cols = pool[ptab].cols
            m = o.eval_predicates(cols, preds)
            sel += int(m.sum())
            for sd, c in sk:
                o.sketch(cols[c][m], sd, d, w, threads=threads)
                nsk += 1
        return sel, nsk

    s_mt, r_mt = pick(rows_mt)
    a = time.perf_counter()
    sel, nsk = run(s_mt, nt)
    t_mt = time.perf_counter() - a
    s_1, r_1 = pick(rows_1)
    a = time.perf_counter()
    sel1, nsk1 = run(s_1, 1)
    t_1 = time.perf_counter() - a
    return {"value": sel / t_mt, "unit": "rows/s", "cores": nt, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d of the %d scan jobs (seeded order), %d rows scanned, %d "
                      "qualifying, %d sketches, %d threads: %.2f s" % (
                          len(s_mt), len(jobs), r_mt, sel, nsk, nt, t_mt),
            "input_rows_per_s": r_mt / t_mt, "sketches_per_s": nsk / t_mt,
            "single_thread": {"value": sel1 / t_1, "input_rows_per_s": r_1 / t_1,
                              "sample": "%d jobs, %d rows, %.2f s" % (len(s_1), r_1, t_1)}}


def W_seed(args):
    from paper_2102_02440_amd import workloads as W
    return W.DEFAULT_SEED if args.seed is None else args.seed


def run_batch(args):
    m = measure_batch(args.steps, args.warmup, W_seed(args), n_queries=args.queries,
                      cpu=not args.no_cpu_baseline)
    out = {"metric": METRIC, "value": m["value"], "unit": "rows/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": m["workload"], "rows_per_step": m["rows_per_step"],
                      "parallelism": "single-gpu"}}
    out.update({k: v for k, v in m.items() if k not in out and k != "workload"})
    print(json.dumps(out), flush=True)


def measure_learned(epochs=30):
    """Trains the correction network with the library's kernels on ~213k
    sub-plans (exact truths stored by tests/golden/make_learned_truth.py),
    evaluates it against the raw median estimate on ~21k held-out sub-plans
    from disjoint seeds, and times the held-out workload end to end: the
    plain path (one build launch per sketch, raw estimates) against the
    batched + learned path (one graph launch, the same estimates, the
    network's correction)."""
    import numpy as np
    import torch
    from paper_2102_02440_amd import learned as Lrn
    from paper_2102_02440_amd import workloads as W
    tp = os.path.join(ROOT, "tests", "golden", "learned_truth.npz")
    tr = np.load(tp)
    n_tr, n_te = int(tr["n_train_queries"]), int(tr["n_test_queries"])
    t0 = time.time()
    pool_tr, q_tr = W.learned_workload(W.LEARNED_TRAIN_SEED, n_tr)
    pool_te, q_te = W.learned_workload(W.LEARNED_TEST_SEED, n_te)
    s_tr = W.learned_subplans(q_tr, W.LEARNED_TRAIN_SEED)
    s_te = W.learned_subplans(q_te, W.LEARNED_TEST_SEED)
    assert sum(map(len, s_tr)) == tr["train_true"].size
    assert sum(map(len, s_te)) == tr["test_true"].size
    log("[bench] learned workloads in %.1fs" % (time.time() - t0))
    t0 = time.time()
    x, b, e, f = Lrn.build_features(pool_tr, q_tr, s_tr, log=log)
    torch.cuda.synchronize()
    t_feat = time.time() - t0
    xt, bt, et, ft = Lrn.build_features(pool_te, q_te, s_te, log=log)
    tgt = torch.from_numpy(np.log1p(tr["train_true"]).astype(np.float32)).cuda()
    init = Lrn.init_params(0)
    torch.cuda.synchronize()
    t0 = time.time()
    mlp, hist = Lrn.train(x, b, tgt, init, epochs=epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    res = Lrn.evaluate(mlp, xt, bt, et, tr["test_true"])
    torch.cuda.synchronize()
    e2e = Lrn.compare_paths(pool_te, q_te, s_te, mlp, tr["test_true"],
                            tune=(262144, 131072, 1), log=log)
    a = time.perf_counter()
    for _ in range(10):
        mlp.forward(xt, bt)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - a) / 10
    n = x.shape[0]
    dims = [20, 64, 64, 64, 1]
    macs = sum(dims[i] * dims[i + 1] for i in range(len(dims) - 1))
    flops_per_sample = 2 * (3 * macs - dims[0] * dims[1])
    train_tflops = flops_per_sample * n * epochs / t_train / 1e12
    return {"workload": "learned correction: %d training and %d held-out sub-plans, "
                        "d=7 w=8192, MLP 20-64-64-64-1" % (n, xt.shape[0]),
            "value": xt.shape[0] / t_inf, "unit": "corrected estimates/s",
            "ms_per_step": t_train * 1e3 / max(1, epochs), "steps": epochs,
            "dtype": "bf16 weights / fp32 accumulate",
            "end_to_end_heldout": e2e,
            "train_samples_per_s": n * epochs / t_train,
            "feature_build_s": t_feat, "mse_first_last": [hist[0], hist[-1]],
            "qerror_heldout": res,
            # training kernels (forward, backward, gradient sum + Adam): fp32
            # FMA on the vector units; 2 flops per multiply-add of the three
            # products of each layer (forward, input gradient, weight
            # gradient; the first layer has no input gradient)
            "roofline": {"bound": "alu", "achieved": train_tflops,
                         "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": train_tflops / FP32_VECTOR_PEAK_TFLOPS,
                         "traffic": None,
                         "kernel": "mlp training step (fwd, bwd, reduce+Adam)",
                         "flops_per_sample": flops_per_sample,
                         "note": "512-sample batches of a 20-64-64-64-1 network: "
                                 "latency-bound, far from any roof"}}


def run_learned(args):
    m = measure_learned(args.epochs)
    out = {"metric": "subplan estimates/s at q-error (learned correction)",
           "value": m["value"], "unit": m["unit"], "n_gpus": 1, "steps": args.epochs,
           "warmup": 0, "ms_per_step": m["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": m["dtype"],
           "data": "synthetic",
           "config": {"workload": m["workload"], "parallelism": "single-gpu"}}
    out.update({k: v for k, v in m.items() if k not in out and k != "workload"})
    print(json.dumps(out), flush=True)


def measure_large(steps, warmup, seed, cpu=True, cpu_rows=50_000_000):
    """One 1B-row fact table: 4 range predicates (1% combined), 6 int64 key
    sketches, d=11, w=65536, int64 counters (two-phase build)."""
    import numpy as np
    import torch
    from paper_2102_02440_amd import compass as C
    from paper_2102_02440_amd import workloads as W
    n = int(os.environ.get("COMPASS_LARGE_ROWS", 1_000_000_000))
    t0 = time.time()
    cols, preds, seeds = W.large_scan_device(seed, n_rows=n)
    torch.cuda.synchronize()
    log("[bench] large: generated %d rows on the device in %.1fs" % (n, time.time() - t0))
    names = ["i0", "i1", "f0", "f1"]
    pd = [{"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
          for p in preds]
    keys = [cols["key%d" % k] for k in range(6)]
    d, w = 11, 65536
    cnt = [torch.zeros((d, w), dtype=torch.int64, device="cuda") for _ in keys]
    nsel = torch.zeros(1, dtype=torch.int64, device="cuda")

    def step():
        C.sketch_build(n, [cols[c] for c in names], pd, keys, list(seeds), cnt, nsel,
                       d, w, counter_bits=64)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    dt, (kn, kms) = timed_steps(C, torch, step, steps, "wide_compact")
    other = profiled_steps(C, torch, step, steps, ["wide_hash", "slab_reduce", "fill_zero"])
    hn, hms = other["wide_hash"]
    rn, rms = other["slab_reduce"]
    zn, zms = other["fill_zero"]
    sel = int(nsel.item())
    alg = 16 * n + sel * 6 * 8 + 6 * d * w * 8
    # dominant kernel: the predicate scan + compaction (phase A), which moves
    # the predicate columns and gathers the survivors' keys
    k_s = kms / steps / 1e3
    gbs = (alg - 6 * d * w * 8) / k_s / 1e9
    out = {"workload": "large scan: 1 table of %d rows, 4 range predicates "
                       "(1%% combined), 6 int64 key sketches d=11 w=65536 int64" % n,
           "value": sel / dt, "unit": "rows/s", "ms_per_step": dt * 1e3,
           "steps": steps, "warmup": warmup, "dtype": "int64",
           "input_rows_per_s": n / dt, "selected_rows": sel,
           "build_alg_gbs": alg / dt / 1e9,
           "build_hbm_frac": alg / dt / 1e9 / HBM_PEAK_GBS,
           "kernel_ms_per_step": {"wide_compact": kms / steps, "wide_hash": hms / steps,
                                  "slab_reduce": rms / steps, "fill_zero": zms / steps},
           "launches_per_step": {"wide_compact": kn / steps, "wide_hash": hn / steps,
                                 "slab_reduce": rn / steps},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                        "traffic": measured_traffic("wide_compact_traffic_large.md",
                                                    SCAN_SOURCES),
                        "kernel": "wide_compact", "alg_bytes_per_step": alg - 6 * d * w * 8,
                        "kernel_ms_per_step": k_s * 1e3,
                        "launches_per_step": kn / steps,
                        "hash_updates_per_step": sel * 6 * d}}
    if cpu:
        out["cpu_baseline"] = cpu_baseline_large(cols, names, preds, keys, seeds, d, w,
                                                 min(cpu_rows, n))
    del cols, keys, cnt
    torch.cuda.empty_cache()
    return out


def cpu_baseline_large(cols, names, preds, keys, seeds, d, w, rows, runs=3):
    """The oracle on the first `rows` rows of the 1B-row table (columns
    already on the host): predicates, then the six sketches of the
    qualifying rows' keys; all threads (median of `runs`) and one thread."""
    import torch
    from oracle import oracle as o
    o.build()
    nt = o.default_threads()
    host = {c: cols[c][:rows].cpu().numpy() for c in names}
    khost = [k[:rows].cpu().numpy() for k in keys]

    def run(threads):
        m = o.eval_predicates(host, preds)
        for k, sd in zip(khost, seeds):
            o.sketch(k[m], sd, d, w, threads=threads)
        return int(m.sum())

    sel = run(nt)
    t_mt = _median_time(lambda: run(nt), runs)
    t_1 = _median_time(lambda: run(1), 1)
    return {"value": sel / t_mt, "unit": "rows/s", "cores": nt, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "the first %d rows of the table (%d qualifying): predicates "
                      "(numpy) + six d=11 w=65536 sketches, %d threads, median of %d: "
                      "%.2f s" % (rows, sel, nt, runs, t_mt),
            "input_rows_per_s": rows / t_mt,
            "single_thread": {"value": sel / t_1, "input_rows_per_s": rows / t_1,
                              "seconds": t_1}}


def run_large(args):
    seed = W_seed(args)
    m = measure_large(args.steps, args.warmup, seed, cpu=not args.no_cpu_baseline)
    out = {"metric": METRIC, "value": m["value"], "unit": "rows/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int64", "data": "synthetic",
           "config": {"workload": m["workload"], "selected_rows": m["selected_rows"],
                      "parallelism": "single-gpu"}}
    out.update({k: v for k, v in m.items() if k not in out and k != "workload"})
    print(json.dumps(out), flush=True)


def run_partition(args):
    """Sketch partitioning (Section 5.1) on the 6a-shaped chain k - mk - t:
    one step = the one-dimensional sketches of k (on e0) and t (on e1), the
    two-dimensional sketch of mk (keyword x movie, 8192 x 8192 per row,
    d = 7), and the chain estimate; compared with the merged-sketch estimate
    of the same sub-plan and with the exact join size."""
    import numpy as np
    import torch
    from paper_2102_02440_amd import compass as C
    from paper_2102_02440_amd import workloads as W
    seed = W.DEFAULT_SEED if args.seed is None else args.seed
    q = W.job6a(seed=seed)
    k, mk, t = q.tables[0], q.tables[1], q.tables[2]
    d, w = q.d, q.w
    dev = "cuda"

    def prep(tb):
        cols = {c: torch.from_numpy(v).to(dev) for c, v in tb.cols.items()}
        names = list(cols)
        pr = []
        for p in tb.preds:
            e = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
            if p.kind == "subset":
                e["bitmap"] = torch.from_numpy(
                    np.asarray(p.bitmap, dtype=np.uint64).view(np.int64)).to(dev)
                e["domain"] = p.domain
            pr.append(e)
        return cols, list(cols.values()), pr

    kc, kcols, kp = prep(k)
    tc, tcols, tp = prep(t)
    mc, mcols, mp = prep(mk)
    A = torch.zeros((d, w), dtype=torch.int32, device=dev)
    B = torch.zeros((d, w), dtype=torch.int32, device=dev)
    P = torch.zeros((d, w, w), dtype=torch.int32, device=dev)
    na, npp, nb = (torch.zeros(1, dtype=torch.int64, device=dev) for _ in range(3))

    def step():
        C.sketch_build(k.n_rows, kcols, kp, [kc["id"]], [q.seeds[0]], [A], na, d, w)
        C.sketch_build(t.n_rows, tcols, tp, [tc["id"]], [q.seeds[1]], [B], nb, d, w)
        C.sketch_build_2d(mk.n_rows, mcols, mp, mc["keyword"], q.seeds[0],
                          mc["movie"], q.seeds[1], P, npp, d, w, w)
        return C.estimate_chain3(A, P, B, na, npp, nb)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    out_last = []

    def step_keep():
        out_last[:] = [step()]

    dt, scan2d_prof = timed_steps(C, torch, step_keep, args.steps, "scan2d")
    row_est, est, flags = out_last[0]
    prof = profiled_steps(C, torch, step, args.steps,
                          ["fill_zero", "scan_sketch", "slab_reduce", "chain3"])
    prof["scan2d"] = scan2d_prof
    kms = {kname: v[1] / args.steps for kname, v in prof.items()}
    # merged-sketch estimate of the same sub-plan (edges e0, e1) for contrast
    Amk0 = torch.zeros((d, w), dtype=torch.int32, device=dev)
    Amk1 = torch.zeros((d, w), dtype=torch.int32, device=dev)
    nmk = torch.zeros(1, dtype=torch.int64, device=dev)
    C.sketch_build(mk.n_rows, mcols, mp, [mc["keyword"], mc["movie"]],
                   [q.seeds[0], q.seeds[1]], [Amk0, Amk1], nmk, d, w)
    nsel3 = torch.cat([na, nmk, nb])
    _, est_m, _ = C.estimate(3, [0, 2], [1, 1], d, w, 32, nsel3,
                             [A, Amk0, B, Amk1], [0b111])
    torch.cuda.synchronize()
    true = None
    tp_ = os.path.join(ROOT, "tests", "golden", "job6a_truth.json")
    if os.path.exists(tp_):
        tr = json.load(open(tp_))
        if tr.get("seed") == seed and 0b111 in tr["masks"]:
            true = float(tr["true"][tr["masks"].index(0b111)])
    e_part = float(est.item())
    e_merge = float(est_m[0].item())

    def qe(e):
        if true is None:
            return None
        a_, b_ = max(e, 1.0), max(true, 1.0)
        return max(a_ / b_, b_ / a_)

    rows = k.n_rows + t.n_rows + mk.n_rows
    p_bytes = d * w * w * 4
    c_s = kms["chain3"] / 1e3
    s_s = kms["scan2d"] / 1e3
    if kms["chain3"] >= kms["scan2d"]:
        # the chain estimate streams the partitioned sketch once
        gbs = p_bytes / c_s / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "chain3",
                "alg_bytes_per_step": p_bytes}
    else:
        # the binned build (scan with records, counting sort by tile, one
        # workgroup per tile): its algorithmic bytes are the two key columns
        # of mk and the d x 8192 x 8192 matrix written once (1.9 GB)
        upd = int(npp.item()) * d
        b = mk.n_rows * 8 + p_bytes
        gbs = b / s_s / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                "kernel": "scan2d (binned: scan2d_bin, bin2d_offsets, bin2d_scan, "
                          "bin2d_scatter, bin2d_tile)",
                "alg_bytes_per_step": b, "updates_per_step": upd,
                "updates_per_s": upd / s_s}
    out = {"metric": METRIC,
           "value": rows / dt, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "sketch partitioning on the 6a-shaped chain k (134k) - "
                                  "mk (4.5M) - t (2.5M): 1-D sketches of k and t, "
                                  "2-D 8192 x 8192 sketch of mk, d=7; chain estimate",
                      "selected_rows": [int(na.item()), int(npp.item()), int(nb.item())],
                      "parallelism": "single-gpu"},
           "kernel_ms_per_step": kms, "roofline": roof,
           "estimate": {"partitioned": e_part, "merged": e_merge, "true": true,
                        "qerror_partitioned": qe(e_part), "qerror_merged": qe(e_merge),
                        "exact_flag": int(flags.item())}}
    print(json.dumps(out), flush=True)


def _pred_mask(tb, p):
    """Rows of table tb satisfying predicate p (numpy, for the exact size)."""
    import numpy as np
    col = tb.cols[p.col]
    if p.kind == "point":
        return col == p.lo
    if p.kind == "range":
        return (col >= p.lo) & (col <= p.hi)
    words = np.asarray(p.bitmap, dtype=np.uint64)
    c = col.astype(np.int64)
    ok = (c >= 0) & (c < p.domain)
    cc = np.where(ok, c, 0)
    bit = (words[cc >> 6] >> (cc & 63).astype(np.uint64)) & np.uint64(1)
    return ok & (bit == 1)


def run_partition_kd(args):
    """Partitioned sketches of a table with three joins (Section 5.1): the
    36M-row fact table of a star join gets a d x 128 x 128 x 128 tensor,
    its three dimension tables 1-D sketches (d = 5, w = 128); one step =
    the four builds and the tree estimate; compared with the merged-sketch
    estimate (d = 5, w = 8192) of the same join and with its exact size."""
    import numpy as np
    import torch
    from paper_2102_02440_amd import compass as C
    from paper_2102_02440_amd import workloads as W
    seed = W.DEFAULT_SEED if args.seed is None else args.seed
    t0 = time.time()
    q = W.star3(seed=seed)
    log("[bench] generated the star workload in %.1fs" % (time.time() - t0))
    d, w = q.d, q.w
    dev = "cuda"
    fact, dims = q.tables[0], q.tables[1:]

    def prep(tb):
        cols = {c: torch.from_numpy(v).to(dev) for c, v in tb.cols.items()}
        names = list(cols)
        pr = []
        for p in tb.preds:
            e = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
            if p.kind == "subset":
                e["bitmap"] = torch.from_numpy(
                    np.asarray(p.bitmap, dtype=np.uint64).view(np.int64)).to(dev)
                e["domain"] = p.domain
            pr.append(e)
        return cols, list(cols.values()), pr

    fc, fcols, fp = prep(fact)
    dp = [prep(tb) for tb in dims]
    fkeys = [fc["movie"], fc["person"], fc["company"]]
    T = torch.zeros((d, w, w, w), dtype=torch.int32, device=dev)
    S = [torch.zeros((d, w), dtype=torch.int32, device=dev) for _ in dims]
    ns = [torch.zeros(1, dtype=torch.int64, device=dev) for _ in range(4)]
    nsel = torch.zeros(4, dtype=torch.int64, device=dev)

    def step():
        for m, (tb, (cc, cl, pr)) in enumerate(zip(dims, dp)):
            C.sketch_build(tb.n_rows, cl, pr, [cc["id"]], [q.seeds[m]], [S[m]],
                           ns[m + 1], d, w)
        C.sketch_build_kd(fact.n_rows, fcols, fp, fkeys, list(q.seeds[:3]), T,
                          ns[0], d, [w, w, w])
        torch.cat(ns, out=nsel)
        return C.estimate_partitioned([0, 0, 0], [1, 2, 3], d, [w, w, w],
                                      [T] + S, nsel)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    out_last = []

    def step_keep():
        out_last[:] = [step()]

    dt, kd_prof = timed_steps(C, torch, step_keep, args.steps, "scan2d")
    row_est, est, flag = out_last[0]
    prof = profiled_steps(C, torch, step, args.steps,
                          ["fill_zero", "wide_compact", "wide_hash", "slab_reduce",
                           "tensor_tree"])
    prof["scan2d"] = kd_prof
    kms = {k: v[1] / args.steps for k, v in prof.items()}
    n_sel = [int(x.item()) for x in ns]
    # merged sketches (the default method) of the same join, w = 8192
    wm = 8192
    Fm = [torch.zeros((d, wm), dtype=torch.int32, device=dev) for _ in range(3)]
    Dm = [torch.zeros((d, wm), dtype=torch.int32, device=dev) for _ in range(3)]
    nf = torch.zeros(1, dtype=torch.int64, device=dev)
    C.sketch_build(fact.n_rows, fcols, fp, fkeys, list(q.seeds[:3]), Fm, nf, d, wm)
    for m, (tb, (cc, cl, pr)) in enumerate(zip(dims, dp)):
        C.sketch_build(tb.n_rows, cl, pr, [cc["id"]], [q.seeds[m]], [Dm[m]], ns[m + 1],
                       d, wm)
    sk = []
    for m in range(3):
        sk += [Fm[m], Dm[m]]
    _, est_m, _ = C.estimate(4, [0, 0, 0], [1, 2, 3], d, wm, 32,
                             torch.cat([nf] + ns[1:]), sk, [0b1111])
    torch.cuda.synchronize()
    # the exact size: fact rows whose three keys all hit selected rows
    sel = []
    for tb in dims:
        m = np.ones(tb.n_rows, dtype=bool)
        for p in tb.preds:
            m &= _pred_mask(tb, p)
        sel.append(m)
    true = float(np.count_nonzero(sel[0][fact.cols["movie"]] & sel[1][fact.cols["person"]]
                                  & sel[2][fact.cols["company"]]))

    def qe(e):
        a_, b_ = max(e, 1.0), max(true, 1.0)
        return max(a_ / b_, b_ / a_)

    e_part, e_merge = float(est.item()), float(est_m[0].item())
    rows = sum(tb.n_rows for tb in q.tables)
    # dominant kernel: the fact table's binned k-D build (scan with records,
    # counting sort by tile, one workgroup per tile); algorithmic bytes: its
    # three key columns and the d x 128^3 tensor written once
    t_bytes = d * w ** 3 * 4
    b = fact.n_rows * 12 + t_bytes
    s_s = kms["scan2d"] / 1e3
    gbs = b / s_s / 1e9
    out = {"metric": METRIC,
           "value": sum(n_sel) / dt, "unit": "rows/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": "partitioned sketches of a star join: fact 36M rows "
                                  "(3 joins, d=5 x 128^3 tensor), t 2.5M, n 4.2M, "
                                  "cn 200k (1-D, w=128); tree estimate",
                      "selected_rows": n_sel, "parallelism": "single-gpu"},
           "input_rows_per_s": rows / dt,
           "kernel_ms_per_step": kms,
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "scan2d (binned k-D build of the fact table)",
                        "alg_bytes_per_step": b,
                        "updates_per_step": n_sel[0] * d,
                        "updates_per_s": n_sel[0] * d / s_s},
           "estimate": {"partitioned": e_part, "merged_w8192": e_merge, "true": true,
                        "qerror_partitioned": qe(e_part), "qerror_merged": qe(e_merge),
                        "rel_error_partitioned": abs(e_part - true) / max(true, 1.0),
                        "rel_error_merged": abs(e_merge - true) / max(true, 1.0),
                        "exact_flag": int(flag.item())}}
    print(json.dumps(out), flush=True)


def run_agms(args):
    """The AGMS baseline (Section 4.1) on the 6a-shaped query: r x b = 7 x 16
    basic sketches per table, each composed over all of the table's joins;
    one step = the five table scans; compared with the Fast-AGMS build of
    the same tables (one launch per table, d = 7, w = 8192) and, for the
    whole five-table query, with the merged Fast-AGMS estimate and the exact
    size."""
    import numpy as np
    import torch
    from paper_2102_02440_amd import compass as C
    from paper_2102_02440_amd import workloads as W
    seed = W.DEFAULT_SEED if args.seed is None else args.seed
    q = W.job6a(seed=seed)
    r, b = 7, 16
    K = r * b
    seeds = W.draw_seeds(np.random.default_rng(seed + 1), len(q.edges), K)
    dev = "cuda"
    tabs = []
    for t, tb in enumerate(q.tables):
        cols = {c: torch.from_numpy(v).to(dev) for c, v in tb.cols.items()}
        names = list(cols)
        pr = []
        for p in tb.preds:
            e = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
            if p.kind == "subset":
                e["bitmap"] = torch.from_numpy(
                    np.asarray(p.bitmap, dtype=np.uint64).view(np.int64)).to(dev)
                e["domain"] = p.domain
            pr.append(e)
        inc = q.incident(t)
        tabs.append((tb, list(cols.values()), pr, [cols[c] for (_, _, c) in inc],
                     [seeds[e] for (e, _, _) in inc],
                     torch.zeros((r, b), dtype=torch.int64, device=dev),
                     torch.zeros(1, dtype=torch.int64, device=dev)))

    def step():
        for (tb, cl, pr, keys, sd, cnt, ns) in tabs:
            C.agms_build(tb.n_rows, cl, pr, keys, sd, cnt, ns, r, b)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dt, (kn, kms) = timed_steps(C, torch, step, args.steps, "agms_build")
    rows_g, est, flag = C.agms_estimate([x[5] for x in tabs], [x[6] for x in tabs])
    torch.cuda.synchronize()
    # Fast-AGMS on the same tables: build time and the merged estimate
    dq = C.DeviceQuery(q, device=dev)
    for _ in range(2):
        dq.build()
    torch.cuda.synchronize()
    a2 = time.perf_counter()
    for _ in range(args.steps):
        dq.build()
    torch.cuda.synchronize()
    fast_ms = (time.perf_counter() - a2) / args.steps * 1e3
    _, est_f, _ = dq.estimate([31])
    torch.cuda.synchronize()
    true = None
    tp_ = os.path.join(ROOT, "tests", "golden", "job6a_truth.json")
    if os.path.exists(tp_):
        tr = json.load(open(tp_))
        if tr.get("seed") == seed and 31 in tr["masks"]:
            true = float(tr["true"][tr["masks"].index(31)])

    def qe(e):
        if true is None:
            return None
        a_, b_ = max(e, 1.0), max(true, 1.0)
        return max(a_ / b_, b_ / a_)

    n_sel = [int(x[6].item()) for x in tabs]
    joins = [len(q.incident(t)) for t in range(len(q.tables))]
    # per (selected row, basic sketch): per join one sign = 3 Horner steps
    # of 6 operations + 3 for the residue's low bit + 1 multiply into the
    # product; then 1 add
    ops = sum(n * K * (22 * j + 1) for n, j in zip(n_sel, joins))
    k_s = kms / args.steps / 1e3
    tops = ops / k_s / 1e12
    rows = sum(tb.n_rows for tb in q.tables)
    e_a, e_f = float(est.item()), float(est_f[0].item())
    out = {"metric": METRIC,
           "value": rows / dt, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "AGMS baseline on the 6a-shaped query: 5 tables "
                                  "(47.1M rows), r x b = 7 x 16 composed sketches",
                      "selected_rows": n_sel, "parallelism": "single-gpu"},
           "roofline": {"bound": "alu", "achieved": tops, "peak": ALU_PEAK_TOPS,
                        "unit": "TOP/s", "frac": tops / ALU_PEAK_TOPS, "traffic": None,
                        "kernel": "agms_build", "launches_per_step": kn / args.steps,
                        "kernel_ms_per_step": k_s * 1e3},
           "fast_agms_build_ms": fast_ms,
           "agms_over_fast_agms_build_time": dt * 1e3 / fast_ms,
           "estimate": {"agms": e_a, "fast_agms_merged": e_f, "true": true,
                        "qerror_agms": qe(e_a), "qerror_fast_agms_merged": qe(e_f),
                        "exact_flag": int(flag.item())}}
    print(json.dumps(out), flush=True)


def run_select(args):
    """Selection output materialised next to the sketches (Section 3): the
    five 6a-shaped table scans of the headline step, each also writing its
    qualifying row indices (room for every row), against the same scans
    without the output."""
    import numpy as np
    import torch
    from paper_2102_02440_amd import compass as C
    from paper_2102_02440_amd import workloads as W
    seed = W.DEFAULT_SEED if args.seed is None else args.seed
    q = W.job6a(seed=seed)
    dev = "cuda"
    jobs = []
    for t, tb in enumerate(q.tables):
        cols = {c: torch.from_numpy(v).to(dev) for c, v in tb.cols.items()}
        names = list(cols)
        pr = []
        for p in tb.preds:
            e = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
            if p.kind == "subset":
                e["bitmap"] = torch.from_numpy(
                    np.asarray(p.bitmap, dtype=np.uint64).view(np.int64)).to(dev)
                e["domain"] = p.domain
            pr.append(e)
        inc = q.incident(t)
        keys = [cols[c] for (_, _, c) in inc]
        sd = [q.seeds[e] for (e, _, _) in inc]
        cnt = [torch.zeros((q.d, q.w), dtype=torch.int32, device=dev) for _ in inc]
        jobs.append((tb, list(cols.values()), pr, keys, sd, cnt,
                     torch.zeros(1, dtype=torch.int64, device=dev),
                     torch.empty(tb.n_rows, dtype=torch.int64, device=dev),
                     torch.zeros(1, dtype=torch.int64, device=dev)))

    def plain():
        for (tb, cl, pr, keys, sd, cnt, ns, rows, rc) in jobs:
            C.sketch_build(tb.n_rows, cl, pr, keys, sd, cnt, ns, q.d, q.w)

    def select():
        for (tb, cl, pr, keys, sd, cnt, ns, rows, rc) in jobs:
            C.sketch_build_select(tb.n_rows, cl, pr, keys, sd, cnt, ns, q.d, q.w, rows, rc)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / args.steps

    t_plain = timed(plain)
    C.profile_enable(True)
    t_sel = timed(select)
    C.profile_enable(False)
    sn, sms = C.profile_take("scan_sketch")
    for k in ["fill_zero", "slab_reduce"]:
        C.profile_take(k)
    written = [int(j[8].item()) for j in jobs]
    rows = sum(tb.n_rows for tb in q.tables)
    alg_out = sum(written) * 8
    k_s = sms / (args.steps + args.warmup) / 1e3
    out = {"metric": METRIC,
           "value": rows / t_sel, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t_sel * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "6a-shaped five table scans with the selection output "
                                  "materialised (room for every row)",
                      "rows_written": written, "parallelism": "single-gpu"},
           "plain_ms_per_step": t_plain * 1e3,
           "materialisation_overhead_ms": (t_sel - t_plain) * 1e3,
           "output_bytes_per_step": alg_out,
           "roofline": {"bound": "alu", "kernel": "scan_sketch",
                        "achieved": None, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                        "frac": None, "traffic": None,
                        "note": "same kernel as the headline step; see that line"}}
    print(json.dumps(out), flush=True)


def plan_quality(q, masks, est, n_sel, true):
    """Algorithm 1 on the step's GPU estimates in the four search spaces of
    Section 7.2.8; each chosen left-deep plan scored by its true cost (sum
    of the exact sizes of its prefixes) against the optimum of exhaustive
    search over the exact sizes."""
    from paper_2102_02440_amd import compass as C
    true_of = dict(zip(masks, true))
    card = [float(x) for x in n_sel]
    eu, ev = q.edge_u, q.edge_v
    n = len(q.tables)

    def true_cost(order):
        m, c = 0, 0.0
        for v in order:
            m |= 1 << v
            c += true_of[m]
        return c

    opt_order, opt_cost, _ = C.enumerate_plan(n, eu, ev, masks, true, card, max_plans=0)
    out = {"optimal": {"order": [q.tables[v].name for v in opt_order],
                       "true_cost": opt_cost}}
    for name, _ in C.ENUM_VARIANTS:
        a = time.perf_counter()
        order, cost = C.enumerate_variant(name, n, eu, ev, masks, list(est), card)
        us = (time.perf_counter() - a) * 1e6
        tc = true_cost(order)
        out[name] = {"order": [q.tables[v].name for v in order], "est_cost": cost,
                     "true_cost": tc, "true_cost_over_optimal": tc / opt_cost,
                     "host_us": us}
    return out


def run_job6a(args):
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

    out_last = []

    def step_keep():
        out_last[:] = [step()]

    dt1, scan_prof = timed_steps(C, torch, step_keep, args.steps, "scan_sketch")
    dt = dt1 * args.steps
    row_est, est, flags = out_last[0]
    # the other kernels' times: a second pass with every kernel's events
    prof = profiled_steps(C, torch, step, args.steps,
                          ["fill_zero", "scan_sketch", "slab_reduce", "wide_compact",
                           "wide_hash", "sort_rows", "node", "tri_order", "tri_lane",
                           "generic", "finish"])
    prof["scan_sketch"] = scan_prof
    # the 19 estimates alone, without any timing event: wall time per call
    torch.cuda.synchronize()
    a_ = time.perf_counter()
    for _ in range(args.steps):
        dq.estimate(masks)
    torch.cuda.synchronize()
    est_wall_ms = (time.perf_counter() - a_) * 1e3 / args.steps
    # the five builds alone, wall time per step (the tables with predicates
    # run on a second stream beside the fused scans, so the kernels' own
    # spans overlap and do not add up to it)
    torch.cuda.synchronize()
    a_ = time.perf_counter()
    for _ in range(args.steps):
        dq.build()
    torch.cuda.synchronize()
    build_wall_ms = (time.perf_counter() - a_) * 1e3 / args.steps

    ms_step = dt * 1e3 / args.steps
    rows_per_step = sum(tb.n_rows for tb in q.tables)
    # the metric counts filtered rows sketched: the rows that qualified
    value = sum(n_sel) * args.steps / dt
    # the fused scan kernel builds the tables without predicates; the
    # tables with predicates take the two-phase build
    alg_bytes, updates = algorithmic_work(q, n_sel, with_preds=False)
    sel_bytes, sel_updates = algorithmic_work(q, n_sel, with_preds=True)
    build_ms_step = sum(prof[k][1] for k in ["fill_zero", "scan_sketch", "slab_reduce",
                                             "wide_compact", "wide_hash"]) / args.steps
    est_ms_step = sum(prof[k][1] for k in ["sort_rows", "node", "tri_order",
                                           "tri_lane", "generic", "finish"]) / args.steps
    kernel_ms = {k: v[1] / args.steps for k, v in prof.items()}
    scan_s = kernel_ms["scan_sketch"] / 1e3
    scan_tops = updates * OPS_PER_HASH_UPDATE / scan_s / 1e12
    hbm_view = {"kernel": "scan_sketch", "alg_bytes_per_step": alg_bytes,
                "achieved_gbs": alg_bytes / scan_s / 1e9, "peak_gbs": HBM_PEAK_GBS,
                "frac": alg_bytes / scan_s / 1e9 / HBM_PEAK_GBS}
    # the scan is the dominant kernel of the step (the estimate kernels
    # together take a quarter of its time)
    roofline = {"bound": "alu", "achieved": scan_tops, "peak": ALU_PEAK_TOPS,
                "unit": "TOP/s", "frac": scan_tops / ALU_PEAK_TOPS,
                "traffic": measured_traffic("scan_sketch_traffic_job6a.md",
                                            SCAN_SOURCES),
                "kernel": "scan_sketch", "hash_updates_per_step": updates,
                "ops_per_hash_update": OPS_PER_HASH_UPDATE}
    roofline["launches_per_step"] = prof[roofline["kernel"]][0] / args.steps
    roofline["kernel_ms_per_step"] = kernel_ms[roofline["kernel"]]
    two_s = (kernel_ms["wide_compact"] + kernel_ms["wide_hash"]) / 1e3
    other = {"scan_sketch": {"alu_tops": scan_tops, "hash_updates_per_s": updates / scan_s},
             "scan_sketch_hbm": hbm_view,
             "two_phase": {"kernels": ["wide_compact", "wide_hash"],
                           "note": "second stream beside the fused scans: the "
                                   "kernels' event spans include time spent "
                                   "waiting for compute units",
                           "alg_bytes_per_step": sel_bytes,
                           "hash_updates_per_step": sel_updates,
                           "achieved_gbs": sel_bytes / two_s / 1e9 if two_s else None}}
    # accuracy against stored exact truths (oracle hash aggregation)
    qerr = None
    plans = None
    tp = os.path.join(ROOT, "tests", "golden", "job6a_truth.json")
    if os.path.exists(tp):
        tr = json.load(open(tp))
        if tr.get("seed") == seed and tr.get("scale") == 1.0 and tr["masks"] == masks:
            e = np.maximum(est.cpu().numpy(), 1.0)
            t = np.maximum(np.asarray(tr["true"], dtype=np.float64), 1.0)
            qe = np.maximum(e / t, t / e)
            qerr = {"median": float(np.median(qe)), "p90": float(np.percentile(qe, 90)),
                    "max": float(qe.max())}
            plans = plan_quality(q, masks, est.cpu().numpy().astype(np.float64),
                                 n_sel, tr["true"])
    out = {
        "metric": METRIC,
        "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "job6a-shaped five tables: ci 36M, mk 4.5M, t 2.5M, "
                               "n 4.2M, k 134k rows; 10 sketches d=7 w=8192 int32; "
                               "19 sub-plan estimates",
                   "rows_per_step": rows_per_step, "selected_rows": n_sel,
                   "seed": seed, "parallelism": "single-gpu"},
        "input_rows_per_s": rows_per_step * args.steps / dt,
        "build_ms_per_step": build_wall_ms,
        "build_kernel_span_ms_per_step": build_ms_step,
        "estimate_ms_per_step": est_ms_step,
        "estimate_wall_ms": est_wall_ms,
        "subplan_estimates_per_s": len(masks) / (est_wall_ms / 1e3),
        "qerror": qerr,
        "plan_enumeration": plans,
        "kernel_ms_per_step": kernel_ms,
        "roofline": roofline,
        "kernel_rooflines": other,
    }
    if not args.no_cpu_baseline:
        log("[bench] oracle baseline of the step")
        out["cpu_baseline"] = cpu_baseline(q, masks, n_sel, args.cpu_sample_rows)
    if not args.only_headline:
        del dq
        torch.cuda.empty_cache()
        cs, cw = args.config_steps, 2
        log("[bench] large scan")
        out["configs"] = {"large_scan": measure_large(cs, cw, seed,
                                                      cpu=not args.no_cpu_baseline)}
        log("[bench] batched build")
        out["configs"]["batched"] = measure_batch(cs, 1, seed,
                                                  cpu=not args.no_cpu_baseline)
        log("[bench] learned correction, end to end")
        out["configs"]["learned"] = measure_learned(args.epochs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
