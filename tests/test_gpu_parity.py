"""Parity of the HIP path against the CPU oracle (bit-exact integers).

Every case prints its name, seed and shape before touching the GPU.
"""
import os
import zlib

import numpy as np
import pytest

from paper_2102_02440_amd import workloads as W
from tests.shapes import expected_flag_est, supported_shape

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print("[case]", *a, flush=True)


def oracle_query(oracle, q):
    """Oracle sketches (per side) and selected counts of a workloads.Query."""
    side_sk = [None] * (2 * len(q.edges))
    n_sel = []
    for t, tb in enumerate(q.tables):
        inc = q.incident(t)
        ns, sks = oracle.build_table_sketches(
            tb, [c for (_, _, c) in inc], [q.seeds[e] for (e, _, _) in inc],
            q.d, q.w)
        n_sel.append(ns)
        for (e, side, _), s in zip(inc, sks):
            side_sk[2 * e + side] = s
    return side_sk, n_sel


def check_query(oracle, q, masks=None, name=""):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    _say(name, "tables", [tb.n_rows for tb in q.tables], "d", q.d, "w", q.w,
         "bits", q.counter_bits)
    dq = C.DeviceQuery(q)
    dq.build()
    torch.cuda.synchronize()
    side_sk, n_sel = oracle_query(oracle, q)
    assert dq.n_selected.cpu().tolist() == n_sel
    for s, (g, o) in enumerate(zip(dq.sketch_of_side, side_sk)):
        assert np.array_equal(g.cpu().numpy().astype(np.int64), o), "side %d" % s
    if masks is None:
        masks = oracle.connected_subplans(len(q.tables), q.edge_u, q.edge_v)
    row_est, est, flags = dq.estimate(masks)
    torch.cuda.synchronize()
    vals_o, est_o, flags_o = oracle.estimate(len(q.tables), q.edge_u, q.edge_v,
                                             q.d, q.w, side_sk, n_sel, masks)
    vals_g = C.row_values(row_est)
    fl = flags.cpu().numpy()
    for m in range(len(masks)):
        sup = supported_shape(q.edge_u, q.edge_v, masks[m], q.w, q.d)
        if sup is not None:
            assert bool(fl[m] & C.FLAG_UNSUPPORTED) == (not sup), "mask 0x%x" % masks[m]
        if fl[m] & C.FLAG_UNSUPPORTED:
            continue
        go = [v & ((1 << 128) - 1) for v in vals_o[m]]
        assert vals_g[m] == go, "mask 0x%x" % masks[m]
        f_x, e_x, tol = expected_flag_est(oracle, len(q.tables), q.edge_u, q.edge_v,
                                          q.d, q.w, side_sk, n_sel, masks[m],
                                          vals_o[m], flags_o[m], est_o[m])
        assert fl[m] == f_x, "mask 0x%x" % masks[m]
        assert abs(est.cpu().numpy()[m] - e_x) <= tol, "mask 0x%x" % masks[m]
    return dq, masks, fl


@gpu
def test_two_table_small(oracle):
    q = W.two_table(seed=5, n_r=50_000, n_s=5_000, domain=5_000, d=5, w=1024)
    check_query(oracle, q, name="two_table_small")


@gpu
def test_two_table_full(oracle):
    """R 1M (10% range), S 100k, Zipf(1.0) over 100k keys, d=5, w=1024."""
    q = W.two_table()
    check_query(oracle, q, name="two_table_full")


@gpu
@pytest.mark.parametrize("w", [1, 3, 1023, 1024, 4096])
@pytest.mark.parametrize("d", [1, 5, 11])
def test_two_table_shapes(oracle, d, w):
    q = W.two_table(seed=100 + d * 7 + w, n_r=30_000, n_s=9_001, domain=2_000,
                    d=d, w=w)
    check_query(oracle, q, name="two_table d=%d w=%d" % (d, w))


@gpu
def test_job6a_scaled(oracle):
    """6a-shaped five tables at 1% size: all 19 sub-plans, 4 with the triangle."""
    q = W.job6a(seed=7, scale=0.01, d=7, w=1024)
    _, masks, fl = check_query(oracle, q, name="job6a scale 0.01")
    assert len(masks) == 19
    assert not np.any(fl & 2)


@gpu
def test_build_overlap_matches_one_stream(oracle):
    """Tables with predicates built on a second stream (the default) give
    the oracle's counters and selected counts, as every table on one
    stream does; also on a caller's own stream, and with the counters
    dirtied between the builds (each build overwrites them)."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    q = W.job6a(seed=11, scale=0.01, d=7, w=1024)
    _say("build overlap", "tables", [tb.n_rows for tb in q.tables])
    assert any(tb.preds for tb in q.tables) and not all(tb.preds for tb in q.tables)
    side_sk, n_sel = oracle_query(oracle, q)
    dq = C.DeviceQuery(q)
    user = torch.cuda.Stream()
    for overlap, stream in [(False, None), (True, None), (True, user), (False, user)]:
        for c in dq.sketch_of_side:
            c.fill_(7)
        dq.n_selected.fill_(-1)
        torch.cuda.synchronize()
        if stream is None:
            dq.build(overlap=overlap)
        else:
            with torch.cuda.stream(stream):
                dq.build(stream=stream, overlap=overlap)
        torch.cuda.synchronize()
        assert dq.n_selected.cpu().tolist() == n_sel, (overlap, stream)
        for s, (g, o) in enumerate(zip(dq.sketch_of_side, side_sk)):
            assert np.array_equal(g.cpu().numpy().astype(np.int64), o), (overlap, s)


@gpu
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("cyclic", [False, True])
def test_random_queries(oracle, seed, cyclic):
    rng = np.random.default_rng(1000 + seed + 50 * cyclic)
    nt = int(rng.integers(2, 6))
    w = int(rng.choice([2, 5, 64, 257, 1024]))
    d = int(rng.choice([1, 3, 5]))
    q = W.small_random_query(rng, nt, int(rng.integers(1, 3000)),
                             int(rng.choice([3, 50, 100000])), d, w, cyclic=cyclic)
    check_query(oracle, q, name="random seed=%d cyclic=%d nt=%d" % (seed, cyclic, nt))


@gpu
def test_int64_keys_and_counters(oracle):
    rng = np.random.default_rng(77)
    q = W.small_random_query(rng, 3, 4000, 1000, 5, 512, cyclic=True)
    for tb in q.tables:
        # int64 keys incl. negatives and values above 2^32 and 2^61
        k = tb.cols["k0"].astype(np.int64)
        k = np.where(k % 3 == 0, k * 4_000_000_019, k)
        k = np.where(k % 7 == 1, -k - 5, k)
        k = np.where(k % 11 == 2, k + (1 << 62), k)
        tb.cols["k0"] = k
        tb.cols["k1"] = tb.cols["k1"].astype(np.int64) - 500
    q.counter_bits = 64
    check_query(oracle, q, name="int64 keys/counters")


@gpu
def test_negative_int32_keys(oracle):
    rng = np.random.default_rng(78)
    q = W.small_random_query(rng, 3, 3000, 100, 3, 256)
    for tb in q.tables:
        tb.cols["k0"] = (tb.cols["k0"] - 50).astype(np.int32)
        tb.cols["k1"] = (tb.cols["k1"] * -21474836).astype(np.int32)
    check_query(oracle, q, name="negative int32 keys")


@gpu
def test_edge_cases(oracle):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(5)
    d, w = 5, 1024
    seeds = W.draw_seeds(rng, 1, d)[0]
    dev = "cuda"
    for name, keys, vals, pred in [
        ("empty", np.zeros(0, np.int32), np.zeros(0, np.int32), None),
        ("all filtered", rng.integers(0, 100, 10_000).astype(np.int32),
         np.zeros(10_000, np.int32), {"col": 0, "kind": "point", "lo": 1}),
        ("all pass", rng.integers(0, 100, 10_000).astype(np.int32),
         np.zeros(10_000, np.int32), {"col": 0, "kind": "range", "lo": -5, "hi": 5}),
        ("hot key", np.full(200_003, 42, np.int32), np.arange(200_003).astype(np.int32), None),
        ("ragged", rng.integers(-10**9, 10**9, 4096 * 3 + 17).astype(np.int32),
         rng.integers(0, 10, 4096 * 3 + 17).astype(np.int32),
         {"col": 0, "kind": "range", "lo": 3, "hi": 6}),
    ]:
        _say("edge case", name, keys.size)
        kt = torch.from_numpy(keys).to(dev)
        vt = torch.from_numpy(vals).to(dev)
        cnt = torch.full((d, w), 7, dtype=torch.int32, device=dev)
        nsel = torch.full((1,), 3, dtype=torch.int64, device=dev)
        preds = [pred] if pred else []
        C.sketch_build(keys.size, [vt], preds, [kt], [seeds], [cnt], nsel, d, w)
        torch.cuda.synchronize()
        mask = np.ones(keys.size, bool) if not pred else (
            (vals == pred["lo"]) if pred["kind"] == "point"
            else (vals >= pred["lo"]) & (vals <= pred["hi"]))
        assert nsel.item() == int(mask.sum())
        assert np.array_equal(cnt.cpu().numpy().astype(np.int64),
                              oracle.sketch(keys[mask], seeds, d, w))


@gpu
def test_accumulate_is_linear(oracle):
    """Section 2: sketches of partitions add up to the sketch of the whole,
    across separate launches (accumulate=1) and different chunkings."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(9)
    d, w = 7, 2048
    seeds = W.draw_seeds(rng, 1, d)[0]
    keys = W.fk_column(rng, 600_000, 50_000, 1.1, rng.permutation(50_000))
    kt = torch.from_numpy(keys).to("cuda")
    whole = torch.zeros((d, w), dtype=torch.int32, device="cuda")
    parts = torch.zeros((d, w), dtype=torch.int32, device="cuda")
    n1 = torch.zeros(1, dtype=torch.int64, device="cuda")
    n2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    _say("linearity", keys.size)
    C.sketch_build(keys.size, [], [], [kt], [seeds], [whole], n1, d, w)
    cut = [0, 1, 4097, 250_000, keys.size]
    for a, b in zip(cut[:-1], cut[1:]):
        C.sketch_build(b - a, [], [], [kt[a:b]], [seeds], [parts], n2, d, w,
                       accumulate=True)
    torch.cuda.synchronize()
    assert torch.equal(whole, parts)
    assert n1.item() == n2.item() == keys.size
    assert np.array_equal(whole.cpu().numpy().astype(np.int64),
                          oracle.sketch(keys, seeds, d, w))


@gpu
def test_collision_free_exact_two_way(oracle):
    """b = (0, 1) makes h the identity on keys in [0, w): every row's
    estimate is the exact join size."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(12)
    q = W.two_table(seed=3, n_r=200_000, n_s=20_000, domain=16_384, d=5, w=16_384)
    q.seeds[:, :, 4] = 0
    q.seeds[:, :, 5] = 1
    dq = C.DeviceQuery(q)
    dq.build()
    row_est, est, flags = dq.estimate([3])
    mask = oracle.eval_predicates(q.tables[0].cols, q.tables[0].preds)
    r = q.tables[0].cols["key"][mask]
    s = q.tables[1].cols["key"]
    true = int((np.bincount(r, minlength=16384).astype(np.int64) *
                np.bincount(s, minlength=16384)).sum())
    assert C.row_values(row_est)[0] == [true] * 5
    assert est.item() == float(true)
    assert flags.item() == C.FLAG_EXACT


def _triangle_query(seed, extra_child):
    """Triangle 0-1-2 closed by edge (1, 2); table 0 is the apex.  With
    extra_child a fourth table hangs off the apex (three apex children)."""
    rng = np.random.default_rng(seed)
    n = [3000, 2500, 2000, 1500]
    tables = []
    for t in range(4 if extra_child else 3):
        cols = {"k0": rng.integers(0, 300, n[t]).astype(np.int32),
                "k1": rng.integers(0, 300, n[t]).astype(np.int32)}
        tables.append(W.Table("t%d" % t, cols, []))
    edges = [W.Edge(0, "k0", 1, "k0"), W.Edge(0, "k1", 2, "k0"),
             W.Edge(1, "k1", 2, "k1")]
    if extra_child:
        edges.append(W.Edge(0, "k0", 3, "k1"))
    return W.Query(tables, edges, 3, 512, W.draw_seeds(rng, len(edges), 3), 32)


@gpu
@pytest.mark.parametrize("extra_child", [False, True])
@pytest.mark.parametrize("inflate", ["none", "above_2^30", "above_2^62"])
def test_triangle_sweep_paths(oracle, extra_child, inflate):
    """The triangle sweep picks its arithmetic from the selected counts (they
    bound every counter and message): compact 64-bit for a two-child apex
    with all counts below 2^30, general 64-bit, or 128-bit.  Raising the
    counts keeps them valid bounds and forces each path on the same
    sketches; the oracle gets the same counts."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    q = _triangle_query(91 + extra_child, extra_child)
    _say("triangle paths", "extra_child", extra_child, "inflate", inflate)
    dq = C.DeviceQuery(q)
    dq.build()
    torch.cuda.synchronize()
    side_sk, n_sel = oracle_query(oracle, q)
    assert dq.n_selected.cpu().tolist() == n_sel
    add = {"none": 0, "above_2^30": 1 << 30, "above_2^62": 1 << 40}[inflate]
    n_sel = [x + add for x in n_sel]
    dq.n_selected.copy_(torch.tensor(n_sel, dtype=torch.int64))
    masks = oracle.connected_subplans(len(q.tables), q.edge_u, q.edge_v)
    row_est, est, flags = dq.estimate(masks)
    torch.cuda.synchronize()
    vals_o, est_o, flags_o = oracle.estimate(len(q.tables), q.edge_u, q.edge_v,
                                             q.d, q.w, side_sk, n_sel, masks)
    vals_g = C.row_values(row_est)
    fl = flags.cpu().numpy()
    n_tri = 0
    for m in range(len(masks)):
        assert not fl[m] & C.FLAG_UNSUPPORTED, "mask 0x%x" % masks[m]
        n_tri += (masks[m] & 7) == 7
        go = [v & ((1 << 128) - 1) for v in vals_o[m]]
        assert vals_g[m] == go, "mask 0x%x" % masks[m]
        f_x, e_x, tol = expected_flag_est(oracle, len(q.tables), q.edge_u, q.edge_v,
                                          q.d, q.w, side_sk, n_sel, masks[m],
                                          vals_o[m], flags_o[m], est_o[m])
        assert fl[m] == f_x, "mask 0x%x" % masks[m]
        assert abs(est.cpu().numpy()[m] - e_x) <= tol, "mask 0x%x" % masks[m]
    assert n_tri == (2 if extra_child else 1)


@gpu
@pytest.mark.parametrize("shape", ["long_runs", "zipf_apex", "above_order_cap"])
def test_triangle_run_order(oracle, shape):
    """Two-child triangle apexes whose merged list is ordered run by run and
    summed by binary search (runs of 8 or more elements), next to short
    runs summed element by element, and a list longer than the ordering
    holds (w = 16384: element-wise only)."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng({"long_runs": 5, "zipf_apex": 6,
                                 "above_order_cap": 7}[shape])
    w, d = {"long_runs": (4096, 2), "zipf_apex": (2048, 3),
            "above_order_cap": (16384, 1)}[shape]
    n = {"long_runs": [20000, 200000, 100000], "zipf_apex": [300000, 50000, 80000],
         "above_order_cap": [40000, 30000, 20000]}[shape]
    tables = []
    for t in range(3):
        if shape == "zipf_apex" and t == 0:
            k0 = (rng.zipf(1.3, n[t]) % 5000).astype(np.int32)
            k1 = (rng.zipf(1.1, n[t]) % 5000).astype(np.int32)
        else:
            k0 = rng.integers(0, 50000, n[t]).astype(np.int32)
            k1 = rng.integers(0, 50000, n[t]).astype(np.int32)
        tables.append(W.Table("t%d" % t, {"k0": k0, "k1": k1}, []))
    edges = [W.Edge(0, "k0", 1, "k0"), W.Edge(0, "k1", 2, "k0"),
             W.Edge(1, "k1", 2, "k1")]
    q = W.Query(tables, edges, d, w, W.draw_seeds(rng, 3, d), 32)
    masks = [0b111, 0b011, 0b110]
    check_query(oracle, q, masks=masks, name="triangle run order " + shape)


def _triangle_group_query(seed, w, d):
    """Triangle 0-1-2 (table 0 the smallest, so the apex of every rooting
    that runs) with table 3 hanging off table 1 and table 4 off table 2: the
    sub-plans {0,1,2}, {0,1,2,3}, {0,1,2,4}, {0,1,2,3,4} share the apex's
    list, runs and cut edge and differ in the cut endpoints' messages."""
    rng = np.random.default_rng(seed)
    n = [1500, 6000, 5000, 4000, 3000]
    tables = []
    for t in range(5):
        cols = {"k0": rng.integers(0, 400, n[t]).astype(np.int32),
                "k1": rng.integers(0, 400, n[t]).astype(np.int32)}
        tables.append(W.Table("t%d" % t, cols, []))
    edges = [W.Edge(0, "k0", 1, "k0"), W.Edge(0, "k1", 2, "k0"),
             W.Edge(1, "k1", 2, "k1"), W.Edge(1, "k0", 3, "k0"),
             W.Edge(2, "k1", 4, "k1")]
    return W.Query(tables, edges, d, w, W.draw_seeds(rng, len(edges), d), 32)


_GROUP_CASES = ([(m, 512, 3, x) for m in (1, 2, 3, 4) for x in (False, True)] +
                [(2, 16384, 1, False), (3, 16384, 1, True)])


@gpu
@pytest.mark.parametrize("members,w,d,mixed", _GROUP_CASES)
def test_triangle_groups(oracle, members, w, d, mixed):
    """Triangle sub-plans that share one two-child apex are swept together
    (the binary searches once for all of them): groups of 1 to 4 running
    members, ordered lists and lists beyond the ordering (w = 16384), and
    groups where the sub-plans holding table 3 take the general sweep
    instead (its selected count raised above 2^30, a valid bound)."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    q = _triangle_group_query(300 + members + w, w, d)
    _say("triangle groups", "members", members, "w", w, "d", d, "mixed", mixed)
    dq = C.DeviceQuery(q)
    dq.build()
    torch.cuda.synchronize()
    side_sk, n_sel = oracle_query(oracle, q)
    assert dq.n_selected.cpu().tolist() == n_sel
    if mixed:
        n_sel[3] += 1 << 30
        dq.n_selected.copy_(torch.tensor(n_sel, dtype=torch.int64))
    tri = [0b00111, 0b01111, 0b10111, 0b11111][:members]
    masks = tri + [0b00011, 0b01010, 0b10100]
    row_est, est, flags = dq.estimate(masks)
    torch.cuda.synchronize()
    vals_o, est_o, flags_o = oracle.estimate(len(q.tables), q.edge_u, q.edge_v,
                                             q.d, q.w, side_sk, n_sel, masks)
    vals_g = C.row_values(row_est)
    fl = flags.cpu().numpy()
    for m in range(len(masks)):
        assert not fl[m] & C.FLAG_UNSUPPORTED, "mask 0x%x" % masks[m]
        go = [v & ((1 << 128) - 1) for v in vals_o[m]]
        assert vals_g[m] == go, "mask 0x%x" % masks[m]
        f_x, e_x, tol = expected_flag_est(oracle, len(q.tables), q.edge_u, q.edge_v,
                                          q.d, q.w, side_sk, n_sel, masks[m],
                                          vals_o[m], flags_o[m], est_o[m])
        assert fl[m] == f_x, "mask 0x%x" % masks[m]
        assert abs(est.cpu().numpy()[m] - e_x) <= tol, "mask 0x%x" % masks[m]


@gpu
def test_job6a_full_size(oracle):
    """Full-size 6a-shaped workload (ci 36M, mk 4.5M, t 2.5M, n 4.2M, k 134k;
    d=7, w=8192) in the launch configuration the benchmark times: every
    sketch of every table (ci's 756M hash updates included) element by
    element against the oracle's (multi-threaded, private counters summed),
    the selected counts, and all 19 sub-plans on all 7 rows (the four with
    the triangle too), their medians and flags.  Also linearity across
    launches with a different chunking of ci."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    q = W.job6a()
    _say("job6a full size", [tb.n_rows for tb in q.tables])
    dq = C.DeviceQuery(q)
    dq.build()
    torch.cuda.synchronize()
    side_sk, n_sel = oracle_query(oracle, q)
    assert dq.n_selected.cpu().tolist() == n_sel
    for k, (g, o) in enumerate(zip(dq.sketch_of_side, side_sk)):
        assert np.array_equal(g.cpu().numpy().astype(np.int64), o), "side %d" % k
    # linearity across launches: ci in three slices accumulated into new
    # counters equals the one-call build
    ci = 3
    tb = q.tables[ci]
    inc = q.incident(ci)
    keys = [dq.tables[ci]["keys"][k] for k in range(len(inc))]
    acc = [torch.zeros_like(dq.tables[ci]["counters"][k]) for k in range(len(inc))]
    nacc = torch.zeros(1, dtype=torch.int64, device="cuda")
    cuts = [0, 1_000_000, 20_000_003, tb.n_rows]
    for a, b in zip(cuts[:-1], cuts[1:]):
        C.sketch_build(b - a, [], [], [k[a:b] for k in keys],
                       [q.seeds[e] for (e, _, _) in inc], acc, nacc, q.d, q.w,
                       accumulate=True)
    torch.cuda.synchronize()
    for k in range(len(inc)):
        assert torch.equal(acc[k], dq.tables[ci]["counters"][k])
    assert nacc.item() == tb.n_rows
    # estimates: all sub-plans, all rows
    masks = oracle.connected_subplans(5, q.edge_u, q.edge_v)
    assert len(masks) == 19
    row_est, est, flags = dq.estimate(masks)
    torch.cuda.synchronize()
    got = C.row_values(row_est)
    fl = flags.cpu().numpy()
    assert not np.any(fl & C.FLAG_UNSUPPORTED)
    vals, e_o, f_o = oracle.estimate(5, q.edge_u, q.edge_v, q.d, q.w, side_sk,
                                     n_sel, masks)
    e_g = est.cpu().numpy()
    for m in range(len(masks)):
        assert got[m] == [x & ((1 << 128) - 1) for x in vals[m]], hex(masks[m])
        assert e_g[m] == e_o[m], hex(masks[m])
        assert fl[m] == f_o[m], hex(masks[m])


@gpu
@pytest.mark.parametrize("w,bits", [(65536, 64), (40000, 32), (1 << 20, 64)])
def test_wide_sketches_direct_path(oracle, w, bits):
    """Rows too wide for LDS partials (w * 4 > 128 KiB) take the two-phase
    path (survivor compaction, bucket-range LDS hashing, slab reduction):
    same counters as the oracle, int32 and int64, pre-filled counters
    overwritten."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(w)
    n = 300_001
    d = 11
    keys = [rng.integers(-2**40, 2**40, n).astype(np.int64),
            W.fk_column(rng, n, 50_000, 1.1, rng.permutation(50_000)).astype(np.int64)]
    a = rng.integers(0, 1_000_000, n).astype(np.int32)
    f = rng.random(n).astype(np.float32)
    seeds = [W.draw_seeds(rng, 1, d)[0] for _ in keys]
    preds = [{"col": 0, "kind": "range", "lo": 0, "hi": 316_227},
             {"col": 1, "kind": "range", "lo": 0.0, "hi": 0.316227}]
    cdt = torch.int64 if bits == 64 else torch.int32
    cnt = [torch.full((d, w), 5, dtype=cdt, device="cuda") for _ in keys]
    nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("[case] wide", w, bits, flush=True)
    C.sketch_build(n, [torch.from_numpy(a).cuda(), torch.from_numpy(f).cuda()], preds,
                   [torch.from_numpy(k).cuda() for k in keys], seeds, cnt, nsel, d, w,
                   counter_bits=bits)
    torch.cuda.synchronize()
    mask = (a <= 316_227) & (f >= np.float32(0.0)) & (f <= np.float32(0.316227))
    assert nsel.item() == int(mask.sum())
    for k, c in zip(keys, range(2)):
        o = oracle.sketch(k[mask], seeds[c], d, w)
        assert np.array_equal(cnt[c].cpu().numpy().astype(np.int64), o)


@gpu
def test_large_scan_full_size(oracle):
    """1B-row fact table (6 int64 Zipf(1.1) keys over 50M, 4 range
    predicates, 1% combined; d=11, w=65536, int64 counters) in the launch
    configuration the benchmark times (batches of rows compacted into the
    survivor buffer, one hashing pass).  The oracle evaluates the predicates
    on the host over the whole table (columns copied back in chunks), the
    qualifying rows' keys are copied back by index, and all six sketches
    are compared element by element with the oracle's; plus linearity
    across three launches with accumulate."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    n = 1_000_000_000
    _say("large scan", n)
    cols, preds, seeds = W.large_scan_device(n_rows=n)
    names = ["i0", "i1", "f0", "f1"]
    pd = [{"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
          for p in preds]
    keys = [cols["key%d" % k] for k in range(6)]
    d, w = 11, 65536
    cnt = [torch.zeros((d, w), dtype=torch.int64, device="cuda") for _ in keys]
    nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
    pc = [cols[c] for c in names]
    C.sketch_build(n, pc, pd, keys, list(seeds), cnt, nsel, d, w, counter_bits=64)
    torch.cuda.synchronize()
    # the oracle's selection over the whole table, chunk by chunk
    idx = []
    step = 1 << 26
    for a in range(0, n, step):
        b = min(n, a + step)
        host = {c: cols[c][a:b].cpu().numpy() for c in names}
        idx.append(np.flatnonzero(oracle.eval_predicates(host, preds)) + a)
    idx = np.concatenate(idx)
    _say("large scan: oracle selected", idx.size)
    assert nsel.item() == idx.size
    it = torch.from_numpy(idx).cuda()
    for k in range(6):
        kh = keys[k].index_select(0, it).cpu().numpy()
        o = oracle.sketch(kh, seeds[k], d, w)
        assert np.array_equal(cnt[k].cpu().numpy(), o), k
    del it
    # linearity across launches
    acc = [torch.zeros_like(c) for c in cnt]
    n2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    cuts = [0, 333_333_331, 700_000_000, n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        C.sketch_build(b - a, [x[a:b] for x in pc], pd, [k[a:b] for k in keys],
                       list(seeds), acc, n2, d, w, counter_bits=64, accumulate=True)
    torch.cuda.synchronize()
    assert n2.item() == idx.size
    for a_, c in zip(acc, cnt):
        assert torch.equal(a_, c)
    del cols, keys, pc
    torch.cuda.empty_cache()


def _with_env(name, value, fn):
    old = os.environ.get(name)
    os.environ[name] = str(value)
    try:
        return fn()
    finally:
        if old is None:
            del os.environ[name]
        else:
            os.environ[name] = old


@gpu
@pytest.mark.parametrize("preds_on,w", [(False, 4096), (True, 65536), (True, 1000)])
def test_serial_mode_matches_default(preds_on, w):
    """Serial mode (COMPASS_SERIAL=1: one chunk per slice group, one
    compaction workgroup, no two workgroups combining partial counters)
    gives the default launch's counters and selected count bit for bit: a
    difference would be a lost or doubled update.  Fused scan (no
    predicates) and two-phase build (with predicates)."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(w + preds_on)
    n = 2_000_003
    d = 3
    keys = [W.fk_column(rng, n, 300_000, 1.1, rng.permutation(300_000)).astype(np.int32)]
    a = rng.integers(0, 100, n).astype(np.int32)
    preds = [{"col": 0, "kind": "range", "lo": 10, "hi": 69}] if preds_on else []
    seeds = [W.draw_seeds(rng, 1, d)[0] for _ in keys]
    _say("serial mode", preds_on, w)

    def run():
        cnt = [torch.zeros((d, w), dtype=torch.int32, device="cuda") for _ in keys]
        nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
        C.sketch_build(n, [torch.from_numpy(a).cuda()] if preds_on else [], preds,
                       [torch.from_numpy(k).cuda() for k in keys], seeds, cnt, nsel, d, w)
        torch.cuda.synchronize()
        return [c.cpu().numpy() for c in cnt], int(nsel.item())

    par = run()
    ser = _with_env("COMPASS_SERIAL", 1, run)
    assert ser[1] == par[1]
    for x, y in zip(ser[0], par[0]):
        assert np.array_equal(x, y)
    assert par[1] == (int(((a >= 10) & (a <= 69)).sum()) if preds_on else n)


@gpu
@pytest.mark.parametrize("w,bits,pattern", [
    (65536, 64, "uniform"), (65536, 32, "bursts"), (1024, 32, "bursts"),
    (40000, 64, "uniform"), (8192, 32, "all_then_none")])
def test_two_phase_many_batches(oracle, w, bits, pattern):
    """The two-phase build with its survivor buffer capped at 98,304 rows
    (batches of 49,152 rows): many compaction batches, and flushes
    (hashing + reduction) whenever the next batch might not fit, at points
    that depend on how many rows qualified so far: uniform 40%
    selectivity, bursts (whole batches qualifying, then almost none), and
    every row qualifying in the first half, none in the second.  Counters
    and selected count element by element against the oracle."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(w + bits + len(pattern))
    n = 1_500_007
    d = 5
    keys = [W.fk_column(rng, n, 200_000, 1.1, rng.permutation(200_000)).astype(np.int64),
            rng.integers(-2**40, 2**40, n).astype(np.int64)]
    if pattern == "uniform":
        a = rng.integers(0, 100, n).astype(np.int32)
    elif pattern == "bursts":
        a = np.where((np.arange(n) // 150_000) % 2 == 0,
                     rng.integers(0, 40, n), rng.integers(39, 100, n)).astype(np.int32)
    else:
        a = np.where(np.arange(n) < n // 2, 0, 99).astype(np.int32)
    preds = [{"col": 0, "kind": "range", "lo": 0, "hi": 39}]
    seeds = [W.draw_seeds(rng, 1, d)[0] for _ in keys]
    cdt = torch.int64 if bits == 64 else torch.int32
    cnt = [torch.full((d, w), 3, dtype=cdt, device="cuda") for _ in keys]
    nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
    _say("two-phase batches", w, bits, pattern)

    def run():
        C.sketch_build(n, [torch.from_numpy(a).cuda()], preds,
                       [torch.from_numpy(k).cuda() for k in keys], seeds, cnt, nsel,
                       d, w, counter_bits=bits)
        torch.cuda.synchronize()

    _with_env("COMPASS_SURVIVOR_CAP_ROWS", 100_000, run)
    mask = (a >= 0) & (a <= 39)
    assert nsel.item() == int(mask.sum())
    for i, (k, c) in enumerate(zip(keys, cnt)):
        o = oracle.sketch(k[mask], seeds[i], d, w)
        assert np.array_equal(c.cpu().numpy().astype(np.int64), o), i


@gpu
def test_predicate_semantics(oracle):
    """Every predicate kind and column type at its edges against the oracle's
    reading: inclusive int32 ranges with negative values, float32 point
    (-0 equals +0) and ranges (NaN and infinities), subsets with codes below
    0, at and beyond the domain, an empty domain; and a conjunction of
    three.  Selected count and sketch rows must match exactly."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(404)
    n = 40_000 + 123
    a = rng.integers(-50, 200, n).astype(np.int32)
    f = rng.normal(size=n).astype(np.float32)
    special = np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, 1.0, -1.0], np.float32)
    pick = rng.random(n) < 0.2
    f[pick] = special[rng.integers(0, special.size, int(pick.sum()))]
    c = rng.integers(-5, 1100, n).astype(np.int32)
    bits = rng.random(1024) < 0.3
    bitmap = np.zeros(16, np.uint64)
    for j in range(1000):
        if bits[j]:
            bitmap[j >> 6] |= np.uint64(1) << np.uint64(j & 63)
    keys = W.fk_column(rng, n, 30_000, 1.0, rng.permutation(30_000)).astype(np.int32)
    d, w = 5, 2048
    seeds = W.draw_seeds(rng, 1, d)[0]
    cols = {"a": a, "f": f, "c": c}
    names = list(cols)
    dev = {k: torch.from_numpy(v).cuda() for k, v in cols.items()}
    bm_dev = torch.from_numpy(bitmap.view(np.int64)).cuda()
    kt = torch.from_numpy(keys).cuda()
    cases = [
        [W.Predicate("a", "point", 7)],
        [W.Predicate("a", "range", -10, 10)],
        [W.Predicate("f", "point", 0.0)],
        [W.Predicate("f", "range", -1.0, 1.0)],
        [W.Predicate("f", "range", -np.inf, 0.5)],
        [W.Predicate("c", "subset", bitmap=bitmap, domain=1000)],
        [W.Predicate("c", "subset", bitmap=bitmap, domain=0)],
        [W.Predicate("a", "range", 0, 150), W.Predicate("f", "range", -2.0, 2.0),
         W.Predicate("c", "subset", bitmap=bitmap, domain=1000)],
    ]
    for preds in cases:
        _say("predicates", [(p.col, p.kind, p.lo, p.hi, p.domain) for p in preds])
        pd = []
        for p in preds:
            e = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
            if p.kind == "subset":
                e["bitmap"] = bm_dev
                e["domain"] = p.domain
            pd.append(e)
        cnt = torch.full((d, w), 9, dtype=torch.int32, device="cuda")
        nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
        C.sketch_build(n, [dev[k] for k in names], pd, [kt], [seeds], [cnt], nsel, d, w)
        torch.cuda.synchronize()
        mask = oracle.eval_predicates(cols, preds)
        assert nsel.item() == int(mask.sum())
        assert np.array_equal(cnt.cpu().numpy().astype(np.int64),
                              oracle.sketch(keys[mask], seeds, d, w))


@gpu
def test_key_width_classes(oracle):
    """The fused scan picks the Horner step per wave from its keys' widths:
    all below 2^31, all below 2^32, or wider (61-bit).  int64 keys at the
    class edges (2^31 - 1, 2^31, 2^32 - 1, 2^32, p - 1, negative), in runs
    that give every wave one class and in a mixed run, against the oracle."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(31)
    n_run = 8192 * 3
    small = rng.integers(0, 2**31, n_run)
    mid = rng.integers(2**31, 2**32, n_run)
    wide = rng.integers(2**32, 2**61 - 1, n_run)
    edges = np.array([2**31 - 1, 2**31, 2**32 - 1, 2**32, 2**61 - 2, -1, 0, 1],
                     np.int64)
    mixed = np.concatenate([edges, rng.choice(np.concatenate([small, mid, wide]), 20_000)])
    keys = np.concatenate([small, mid, wide, mixed, edges]).astype(np.int64)
    d, w = 7, 4096
    seeds = W.draw_seeds(rng, 1, d)[0]
    kt = torch.from_numpy(keys).cuda()
    cnt = torch.zeros((d, w), dtype=torch.int32, device="cuda")
    nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
    _say("key width classes", keys.size)
    C.sketch_build(keys.size, [], [], [kt], [seeds], [cnt], nsel, d, w)
    torch.cuda.synchronize()
    assert nsel.item() == keys.size
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64),
                          oracle.sketch(keys, seeds, d, w))


@gpu
@pytest.mark.parametrize("bits", [32, 64])
def test_counters_not_16_byte_aligned(oracle, bits):
    """Counter arrays that start 4 or 8 bytes past a 16-byte boundary take
    the reduction's scalar path; same counters as the oracle, for the fused
    scan and the two-phase build."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(55 + bits)
    d, n = 5, 200_003
    keys = torch.from_numpy(W.fk_column(rng, n, 20_000, 1.0,
                                        rng.permutation(20_000))).cuda()
    a = torch.from_numpy(rng.integers(0, 10, n).astype(np.int32)).cuda()
    seeds = W.draw_seeds(rng, 1, d)[0]
    cdt = torch.int32 if bits == 32 else torch.int64
    for w, preds in [(2048, []), (65536, [{"col": 0, "kind": "range", "lo": 0, "hi": 6}])]:
        _say("unaligned counters", bits, w, len(preds))
        big = torch.full((d * w + 1,), 7, dtype=cdt, device="cuda")
        cnt = big[1:].view(d, w)
        assert cnt.data_ptr() % 16 != 0
        nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
        C.sketch_build(n, [a], preds, [keys], [seeds], [cnt], nsel, d, w, bits)
        torch.cuda.synchronize()
        mask = np.ones(n, bool) if not preds else (a.cpu().numpy() <= 6)
        assert nsel.item() == int(mask.sum())
        assert big[0].item() == 7
        assert np.array_equal(cnt.cpu().numpy().astype(np.int64),
                              oracle.sketch(keys.cpu().numpy()[mask], seeds, d, w))


def _graph_query(rng, n, eu, ev, rows, domain, d, w, bits=32):
    """Tables with one key column per incident edge (k<edge id>)."""
    tables = []
    for t in range(n):
        cols = {}
        for e, (u, v) in enumerate(zip(eu, ev)):
            if t in (u, v):
                cols["k%d" % e] = rng.integers(0, domain, rows[t]).astype(np.int32)
        cols["a"] = rng.integers(0, 100, rows[t]).astype(np.int32)
        preds = [W.Predicate("a", "range", 0, int(rng.integers(40, 100)))]
        tables.append(W.Table("t%d" % t, cols, preds))
    edges = [W.Edge(u, "k%d" % e, v, "k%d" % e) for e, (u, v) in enumerate(zip(eu, ev))]
    return W.Query(tables, edges, d, w, W.draw_seeds(rng, len(edges), d), bits)


GENERAL_SHAPES = {
    # name: (n_tables, edge_u, edge_v)
    "4-cycle": (4, [0, 1, 2, 3], [1, 2, 3, 0]),
    "5-cycle+tail": (6, [0, 1, 2, 3, 4, 2], [1, 2, 3, 4, 0, 5]),
    "two triangles": (4, [0, 1, 2, 1, 3], [1, 2, 0, 3, 2]),
    "K4": (4, [0, 0, 0, 1, 1, 2], [1, 2, 3, 2, 3, 3]),
    "parallel edges": (3, [0, 0, 1], [1, 1, 2]),
    "star of 9": (9, [0] * 8, [1, 2, 3, 4, 5, 6, 7, 8]),
    "triangle + 4-cycle": (6, [0, 1, 2, 2, 3, 4, 5], [1, 2, 0, 3, 4, 5, 2]),
}


@gpu
@pytest.mark.parametrize("shape", sorted(GENERAL_SHAPES))
@pytest.mark.parametrize("w,d", [(4, 3), (32, 1), (128, 2)])
def test_general_cycles(oracle, shape, w, d):
    """Shapes beyond trees plus one triangle (longer cycles, several cycles,
    K4, two edges between one pair, a table with 8 children) through the
    generic conditioned contraction: every connected sub-plan, rows modulo
    2^128, medians and flags against the oracle's exact evaluation."""
    n, eu, ev = GENERAL_SHAPES[shape]
    rng = np.random.default_rng(zlib.crc32(("%s %d %d" % (shape, w, d)).encode()))
    rows = [int(rng.integers(200, 3000)) for _ in range(n)]
    q = _graph_query(rng, n, eu, ev, rows, 3 * w, d, w)
    masks = oracle.connected_subplans(n, eu, ev)
    if len(masks) > 200:
        masks = [masks[i] for i in sorted(rng.choice(len(masks), 200, replace=False))]
    _, _, fl = check_query(oracle, q, masks=masks, name="general " + shape)
    assert not np.any(fl & 2)


@gpu
@pytest.mark.parametrize("shape", ["chain4", "triangle", "4-cycle"])
def test_approx_when_uncertified_small_values(oracle, shape):
    """Selected counts raised far above the sketches' sums (still valid
    bounds) make the certificate fail while every row value stays small:
    the estimate is then the median of the fp64 evaluation, flagged APPROX
    and not EXACT, equal to the exact median (small integers are exact in
    fp64); the 128-bit rows are unchanged."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    n, eu, ev = {"chain4": (4, [0, 1, 2], [1, 2, 3]),
                 "triangle": (3, [0, 1, 2], [1, 2, 0]),
                 "4-cycle": GENERAL_SHAPES["4-cycle"]}[shape]
    rng = np.random.default_rng(zlib.crc32(shape.encode()))
    q = _graph_query(rng, n, eu, ev, [3000] * n, 200, 5, 64)
    _say("approx", shape)
    dq = C.DeviceQuery(q)
    dq.build()
    torch.cuda.synchronize()
    side_sk, n_sel = oracle_query(oracle, q)
    big = [x + (1 << 45) for x in n_sel]   # product of 3+ tables > 2^127
    dq.n_selected.copy_(torch.tensor(big, dtype=torch.int64))
    masks = [m for m in oracle.connected_subplans(n, eu, ev) if bin(m).count("1") >= 3]
    row_est, est, flags = dq.estimate(masks)
    torch.cuda.synchronize()
    vals_o, est_o, flags_o = oracle.estimate(n, eu, ev, q.d, q.w, side_sk, big, masks)
    got = C.row_values(row_est)
    fl = flags.cpu().numpy()
    e = est.cpu().numpy()
    for k, m in enumerate(masks):
        assert flags_o[k] == 0, hex(m)            # the oracle cannot certify
        assert fl[k] == C.FLAG_APPROX, (hex(m), fl[k])
        assert got[k] == [v & ((1 << 128) - 1) for v in vals_o[k]], hex(m)
        exact = sorted(oracle.row_values_exact(n, eu, ev, q.d, q.w, side_sk, m))
        assert e[k] == float(exact[q.d // 2]), hex(m)


@gpu
@pytest.mark.parametrize("w", [1, 7, 1024, 1025, 8192, 9000, 16384])
def test_row_sort_extremes(oracle, w):
    """The per-row radix sort of the estimate path: rows of zeros (no pass),
    rows with one counter near 2^46 among small ones (12 passes), rows of
    many equal magnitudes of both signs (ties keep bucket order), ragged
    row lengths and the largest rows (16 keys a lane).  Sketches are given
    directly (int64 counters); chain and star sub-plans, plus a triangle at
    small w, against the oracle."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(4000 + w)
    n, eu, ev = 4, [0, 1, 2, 0], [1, 2, 0, 3]
    d = 4
    sk = []
    for s in range(2 * len(eu)):
        x = np.zeros((d, w), dtype=np.int64)
        x[1] = rng.integers(-50, 51, w)
        x[1, rng.integers(0, w)] = (1 << 46) - 3
        x[2] = rng.choice([-3, 3, -2, 2, 0], w)
        x[3] = rng.integers(-(1 << 20), 1 << 20, w)
        if s % 3 == 0:
            x[0] = rng.integers(-5, 6, w)  # one side keeps a live row 0
        sk.append(x)
    n_sel = [int(max(np.abs(sk[2 * e + t]).sum(axis=1).max()
                     for e in range(len(eu)) for t in (0, 1)))] * n
    dev = [torch.from_numpy(x).cuda() for x in sk]
    ns = torch.tensor(n_sel, dtype=torch.int64, device="cuda")
    masks = [0b0011, 0b0110, 0b1001, 0b1011, 0b1101]
    if w <= 1025:
        masks += [0b0111, 0b1111]
    _say("row sort extremes", "w", w, "masks", len(masks))
    row_est, est, flags = C.estimate(n, eu, ev, d, w, 64, ns, dev, masks)
    torch.cuda.synchronize()
    vals_o, est_o, flags_o = oracle.estimate(n, eu, ev, d, w, sk, n_sel, masks)
    got = C.row_values(row_est)
    fl = flags.cpu().numpy()
    for k, m in enumerate(masks):
        assert not fl[k] & C.FLAG_UNSUPPORTED, hex(m)
        assert got[k] == [v & ((1 << 128) - 1) for v in vals_o[k]], hex(m)


@gpu
def test_approx_when_values_exceed_128_bits(oracle):
    """Counters of about 2^40 in a four-table chain: row values near 2^160
    wrap modulo 2^128.  The fp64 evaluation's median agrees with the exact
    (unbounded integer) median to 1e-12 of the same contraction over
    absolute values."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(99)
    n, eu, ev = 4, [0, 1, 2], [1, 2, 3]
    d, w = 5, 16
    sk = [rng.integers(-2**40, 2**40, (d, w)).astype(np.int64) for _ in range(2 * len(eu))]
    n_sel = [int(max(np.abs(sk[2 * e + s]).sum(axis=1).max()
                     for e in range(len(eu)) for s in (0, 1)))] * n
    dev = [torch.from_numpy(x).cuda() for x in sk]
    ns = torch.tensor(n_sel, dtype=torch.int64, device="cuda")
    masks = [0b1111, 0b0111, 0b1110]
    _say("approx beyond 128 bits")
    row_est, est, flags = C.estimate(n, eu, ev, d, w, 64, ns, dev, masks)
    torch.cuda.synchronize()
    e = est.cpu().numpy()
    fl = flags.cpu().numpy()
    got = C.row_values(row_est)
    for k, m in enumerate(masks):
        exact = oracle.row_values_exact(n, eu, ev, d, w, sk, m)
        absb = oracle.row_values_exact(n, eu, ev, d, w, [np.abs(x) for x in sk], m)
        assert fl[k] == C.FLAG_APPROX, hex(m)
        assert got[k] == [v & ((1 << 128) - 1) for v in exact], hex(m)
        med = sorted(exact)[d // 2]
        assert abs(e[k] - med) <= 1e-12 * max(absb), (hex(m), e[k], med)
