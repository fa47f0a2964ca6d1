"""Parity of the partitioned-sketch path (Section 5.1) with the oracle:
two-dimensional sketch counters bit for bit, chain estimates (128-bit rows,
median, flag) exactly."""
import numpy as np
import pytest

from paper_2102_02440_amd import workloads as W

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print("[case]", *a, flush=True)


def _tables(rng, n_a, n_p, n_b, dom1, dom2, key_dtype=np.int32):
    ka = rng.integers(0, dom1, n_a).astype(key_dtype)
    kb = rng.integers(0, dom2, n_b).astype(key_dtype)
    kp1 = rng.integers(0, dom1, n_p).astype(key_dtype)
    kp2 = rng.integers(0, dom2, n_p).astype(key_dtype)
    attr = rng.integers(0, 1000, n_p).astype(np.int32)
    return ka, kb, kp1, kp2, attr


def _run(oracle, ka, kb, kp1, kp2, attr, d, w1, w2, bits, preds, name,
         nb_override=None, np_override=None):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    _say(name, "n_p", kp1.size, "d", d, "w1", w1, "w2", w2, "bits", bits)
    rng = np.random.default_rng(kp1.size + w1 * 7 + w2)
    s1, s2 = W.draw_seeds(rng, 2, d)
    dev = "cuda"
    ct = torch.int32 if bits == 32 else torch.int64
    A = torch.zeros((d, w1), dtype=ct, device=dev)
    B = torch.zeros((d, w2), dtype=ct, device=dev)
    P = torch.zeros((d, w1, w2), dtype=ct, device=dev)
    na = torch.zeros(1, dtype=torch.int64, device=dev)
    nb = torch.zeros(1, dtype=torch.int64, device=dev)
    npp = torch.zeros(1, dtype=torch.int64, device=dev)
    ta, tb = torch.from_numpy(ka).to(dev), torch.from_numpy(kb).to(dev)
    tp1, tp2 = torch.from_numpy(kp1).to(dev), torch.from_numpy(kp2).to(dev)
    tattr = torch.from_numpy(attr).to(dev)
    C.sketch_build(ka.size, [], [], [ta], [s1], [A], na, d, w1, counter_bits=bits)
    C.sketch_build(kb.size, [], [], [tb], [s2], [B], nb, d, w2, counter_bits=bits)
    C.sketch_build_2d(kp1.size, [tattr], preds, tp1, s1, tp2, s2, P, npp, d, w1,
                      w2, counter_bits=bits)
    n_b = kb.size
    if nb_override is not None:  # a larger selected count: wider inner sums
        n_b = nb_override
        nb.fill_(n_b)
    torch.cuda.synchronize()
    n_p_built = int(npp.item())
    n_p = n_p_built
    if np_override is not None:  # with nb_override: beyond the certificate
        n_p = np_override
        npp.fill_(n_p)
    row_est, est, flags = C.estimate_chain3(A, P, B, na, npp, nb, counter_bits=bits)
    torch.cuda.synchronize()
    mask = np.ones(kp1.size, bool)
    for p in preds:
        if p["kind"] == "range":
            mask &= (attr >= p["lo"]) & (attr <= p["hi"])
        elif p["kind"] == "point":
            mask &= attr == p["lo"]
    assert n_p_built == int(mask.sum())
    Po = oracle.sketch2d(kp1[mask], kp2[mask], s1, s2, d, w1, w2)
    assert np.array_equal(P.cpu().numpy().astype(np.int64), Po)
    Ao = oracle.sketch(ka, s1, d, w1)
    Bo = oracle.sketch(kb, s2, d, w2)
    vals, est_o, flag_o = oracle.chain3(Ao, Po, Bo, [ka.size, n_p, n_b])
    vals_g = C.row_values(row_est.reshape(1, d, 2))[0]
    assert vals_g == [v & ((1 << 128) - 1) for v in vals]
    assert est.item() == est_o
    assert flags.item() == flag_o


@gpu
@pytest.mark.parametrize("bits", [32, 64])
def test_chain3_small(oracle, bits):
    rng = np.random.default_rng(3)
    t = _tables(rng, 3000, 20000, 2500, 500, 300)
    _run(oracle, *t, 5, 64, 32, bits, [{"col": 0, "kind": "range", "lo": 100, "hi": 700}],
         "chain3 small")


@gpu
def test_chain3_odd_widths_int64_keys(oracle):
    """Non-power-of-two widths, int64 keys (negative and above 2^32), a point
    predicate, ragged row count."""
    rng = np.random.default_rng(4)
    ka, kb, kp1, kp2, attr = _tables(rng, 2000, 4096 * 3 + 77, 1500, 400, 200,
                                     key_dtype=np.int64)
    big = np.int64(1) << 40
    kp1 = np.where(kp1 % 3 == 0, kp1 * 977 - big, kp1)
    ka = np.where(ka % 3 == 0, ka * 977 - big, ka)
    attr = (attr % 4).astype(np.int32)
    _run(oracle, ka, kb, kp1, kp2, attr, 3, 100, 37, 64,
         [{"col": 0, "kind": "point", "lo": 2}], "chain3 odd widths")


@gpu
@pytest.mark.parametrize("w1,w2,nb_override", [
    (64, 30, None),          # w2 not a multiple of 4: one column per load
    (9, 12, None),           # one quad per lane, most lanes past the end
    (40, 4100, None),        # ragged: lanes past the row's end in the last quad
    (33, 16384, None),       # widest rows: eight quads per lane
    (40, 4096, 1 << 62),     # 128-bit inner sums (selected counts too large)
    (64, 30, 1 << 62),
    (40, 4096, -1),          # selected counts beyond the certificate: flag 0
])
def test_chain3_row_layouts(oracle, w1, w2, nb_override):
    """int32 chain estimates across the row layouts of the estimate kernel
    (16-byte loads of 1, 2, 4 or 8 quads per lane; column-wise loads when
    w2 is not a multiple of 4) and both inner-sum widths."""
    rng = np.random.default_rng(w1 * 31 + w2)
    t = _tables(rng, 1500, 6000, 1200, 300, 700)
    np_override = None
    if nb_override == -1:
        nb_override = np_override = 1 << 62
    _run(oracle, *t, 3, w1, w2, 32, [{"col": 0, "kind": "range", "lo": 0, "hi": 899}],
         "chain3 layout", nb_override=nb_override, np_override=np_override)


@gpu
@pytest.mark.parametrize("bits", [32, 64])
def test_sketch2d_batches_accumulate_and_atomic_path(oracle, bits):
    """The binned two-dimensional build in several row batches (a small
    record budget), accumulating over two calls, against the oracle; and a
    width beyond one LDS tile (w2 = 40000), which takes the scan with one
    device-scope atomic per update."""
    import os
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(11 + bits)
    n = 50_000
    kp1 = rng.integers(0, 3000, n).astype(np.int32)
    kp2 = rng.integers(0, 5000, n).astype(np.int32)
    attr = rng.integers(0, 1000, n).astype(np.int32)
    d = 3
    s1, s2 = W.draw_seeds(rng, 2, d)
    ct = torch.int32 if bits == 32 else torch.int64
    t1, t2, ta = (torch.from_numpy(v).cuda() for v in (kp1, kp2, attr))
    pr = [{"col": 0, "kind": "range", "lo": 0, "hi": 599}]
    mask = attr <= 599
    for w1, w2, budget in [(200, 96, 4096 * 3 * 4 * 3 + 8), (4, 40000, None)]:
        _say("sketch2d batches", w1, w2, budget, bits)
        old = os.environ.get("COMPASS_2D_RECORD_BYTES")
        if budget is not None:
            os.environ["COMPASS_2D_RECORD_BYTES"] = str(budget)
        try:
            P = torch.full((d, w1, w2), 7, dtype=ct, device="cuda")
            nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
            half = 23_457
            C.sketch_build_2d(half, [ta[:half]], pr, t1[:half], s1, t2[:half], s2,
                              P, nsel, d, w1, w2, counter_bits=bits)
            C.sketch_build_2d(n - half, [ta[half:]], pr, t1[half:], s1, t2[half:], s2,
                              P, nsel, d, w1, w2, counter_bits=bits, accumulate=True)
            torch.cuda.synchronize()
        finally:
            if budget is not None:
                if old is None:
                    del os.environ["COMPASS_2D_RECORD_BYTES"]
                else:
                    os.environ["COMPASS_2D_RECORD_BYTES"] = old
        assert nsel.item() == int(mask.sum())
        Po = oracle.sketch2d(kp1[mask], kp2[mask], s1, s2, d, w1, w2)
        assert np.array_equal(P.cpu().numpy().astype(np.int64), Po)


@gpu
def test_chain3_empty_selection(oracle):
    rng = np.random.default_rng(5)
    t = _tables(rng, 100, 500, 100, 50, 50)
    _run(oracle, *t, 3, 16, 16, 32, [{"col": 0, "kind": "range", "lo": 2000, "hi": 3000}],
         "chain3 empty selection")


@gpu
def test_chain3_6a_shape_full_width(oracle):
    """The 6a-shaped chain k - mk - t at its full size and width
    (mk 4.5M rows, w1 = w2 = 8192, d = 7): every row of the partitioned
    sketch against the oracle's sketch of that row (seeds of one row,
    d = 1), every chain row value, and the median and flag."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    q = W.job6a(seed=W.DEFAULT_SEED, scale=1.0)
    k, mk, t = q.tables[0], q.tables[1], q.tables[2]
    d, w = q.d, q.w
    s_e0, s_e1 = q.seeds[0], q.seeds[1]
    _say("6a chain full width", mk.n_rows, d, w)
    dev = "cuda"
    A = torch.zeros((d, w), dtype=torch.int32, device=dev)
    B = torch.zeros((d, w), dtype=torch.int32, device=dev)
    P = torch.zeros((d, w, w), dtype=torch.int32, device=dev)
    na, npp, nb = (torch.zeros(1, dtype=torch.int64, device=dev) for _ in range(3))

    def dcols(tb):
        return {c: torch.from_numpy(v).to(dev) for c, v in tb.cols.items()}

    def dpreds(tb, cols):
        names = list(cols)
        out = []
        for p in tb.preds:
            e = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
            if p.kind == "subset":
                e["bitmap"] = torch.from_numpy(p.bitmap.view(np.int64)).to(dev)
                e["domain"] = p.domain
            out.append(e)
        return out

    kc, tc, mc = dcols(k), dcols(t), dcols(mk)
    C.sketch_build(k.n_rows, list(kc.values()), dpreds(k, kc), [kc["id"]], [s_e0],
                   [A], na, d, w)
    C.sketch_build(t.n_rows, list(tc.values()), dpreds(t, tc), [tc["id"]], [s_e1],
                   [B], nb, d, w)
    C.sketch_build_2d(mk.n_rows, list(mc.values()), dpreds(mk, mc), mc["keyword"],
                      s_e0, mc["movie"], s_e1, P, npp, d, w, w)
    row_est, est, flags = C.estimate_chain3(A, P, B, na, npp, nb)
    torch.cuda.synchronize()
    vals_g = C.row_values(row_est.reshape(1, d, 2))[0]
    mk_mask = oracle.eval_predicates(mk.cols, mk.preds)
    k_keys = k.cols["id"][oracle.eval_predicates(k.cols, k.preds)]
    t_keys = t.cols["id"][oracle.eval_predicates(t.cols, t.preds)]
    assert npp.item() == int(mk_mask.sum())
    vals_o = []
    for i in range(d):
        Po = oracle.sketch2d(mk.cols["keyword"][mk_mask], mk.cols["movie"][mk_mask],
                             s_e0[i:i + 1], s_e1[i:i + 1], 1, w, w)
        assert np.array_equal(P[i].cpu().numpy().astype(np.int64), Po[0]), i
        Ao = oracle.sketch(k_keys, s_e0[i:i + 1], 1, w)
        Bo = oracle.sketch(t_keys, s_e1[i:i + 1], 1, w)
        v, _, _ = oracle.chain3(Ao, Po, Bo, [k_keys.size, int(mk_mask.sum()), t_keys.size])
        assert vals_g[i] == v[0] & ((1 << 128) - 1), i
        vals_o.append(v[0])
        del Po
    # median (odd d: the middle row value) and certificate
    mid = sorted(vals_o)[d // 2]
    assert est.item() == oracle.i128_to_double(mid)
    ns = [k_keys.size, int(mk_mask.sum()), t_keys.size]
    assert flags.item() == (1 if ns[0] * ns[1] * ns[2] < 2**127 else 0)


# ---------------------------------------------------------------------------
# partitioned sketches of tables with 3 and 4 joins, and tree estimates
# ---------------------------------------------------------------------------
@gpu
@pytest.mark.parametrize("k,widths,bits,preds_on,n", [
    (3, [16, 8, 4], 32, False, 300_001),         # binned, flattened 32
    (3, [64, 64, 32], 32, True, 1_000_003),      # binned, flattened 2048
    (4, [8, 8, 8, 8], 64, True, 500_000),        # binned, flattened 512
    (3, [4, 256, 256], 32, False, 200_000),      # flattened 65536: atomics
    (4, [3, 5, 7, 9], 32, True, 123_457),        # widths not powers of two
])
def test_build_kd_matches_oracle(oracle, k, widths, bits, preds_on, n):
    """compass_sketch_build_kd against the oracle's k-D sketch, every
    counter, with and without predicates, binned and atomic paths."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    _say("build_kd", k, widths, bits, preds_on, n)
    rng = np.random.default_rng(k * 1000 + sum(widths) + n)
    d = 3
    keys = [W.fk_column(rng, n, 50_000, 1.05, rng.permutation(50_000)).astype(np.int64)
            if m % 2 == 0 else rng.integers(-2**40, 2**40, n).astype(np.int64)
            for m in range(k)]
    attr = rng.integers(0, 100, n).astype(np.int32)
    preds = [{"col": 0, "kind": "range", "lo": 5, "hi": 64}] if preds_on else []
    seeds = list(W.draw_seeds(rng, k, d))
    ct = torch.int32 if bits == 32 else torch.int64
    T = torch.full((d,) + tuple(widths), 7, dtype=ct, device="cuda")
    nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
    C.sketch_build_kd(n, [torch.from_numpy(attr).cuda()] if preds_on else [], preds,
                      [torch.from_numpy(x).cuda() for x in keys], seeds, T, nsel, d,
                      widths, counter_bits=bits)
    torch.cuda.synchronize()
    mask = (attr >= 5) & (attr <= 64) if preds_on else np.ones(n, bool)
    assert nsel.item() == int(mask.sum())
    o = oracle.sketch_kd([x[mask] for x in keys], seeds, d, widths)
    assert np.array_equal(T.cpu().numpy().astype(np.int64), o)


def _tree_case(rng, kind):
    """(n_tables, edge_u, edge_v, widths, per-table key columns by edge)."""
    if kind == "star":        # center 0 with three leaves
        return 4, [0, 0, 0], [1, 2, 3], [16, 8, 12]
    if kind == "chain4":      # 0 - 1 - 2 - 3: two 2-D tables in the middle
        return 4, [0, 1, 2], [1, 2, 3], [8, 16, 8]
    if kind == "snowflake":   # 0 - 1 (3 joins) - {2, 3}, 3 - 4
        return 5, [0, 1, 1, 3], [1, 2, 3, 4], [8, 8, 4, 16]
    if kind == "pair":        # two tables
        return 2, [0], [1], [64]
    raise ValueError(kind)


@gpu
@pytest.mark.parametrize("kind,bits", [("star", 32), ("chain4", 64), ("snowflake", 32),
                                       ("pair", 32)])
def test_estimate_partitioned_matches_oracle(oracle, kind, bits):
    """compass_estimate_partitioned against the oracle's literal sum over
    every bucket assignment: 128-bit rows, median and flag.  Every table's
    sketch is built on the GPU (1-D for tables with one join, k-D
    otherwise) and checked against the oracle's too."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    _say("partitioned", kind, bits)
    rng = np.random.default_rng(len(kind) * 31 + bits)
    nt, eu, ev, widths = _tree_case(rng, kind)
    d = 5
    seeds = list(W.draw_seeds(rng, len(eu), d))
    ct = torch.int32 if bits == 32 else torch.int64
    tensors, o_tensors, n_sel = [], [], []
    for t in range(nt):
        inc = [e for e in range(len(eu)) if t in (eu[e], ev[e])]
        n = int(rng.integers(2_000, 40_000))
        cols = [rng.integers(0, 3_000, n).astype(np.int32) for _ in inc]
        attr = rng.integers(0, 10, n).astype(np.int32)
        preds = [{"col": 0, "kind": "range", "lo": 0, "hi": 6}]
        mask = attr <= 6
        ns = torch.zeros(1, dtype=torch.int64, device="cuda")
        wt = [widths[e] for e in inc]
        T = torch.zeros((d,) + tuple(wt), dtype=ct, device="cuda")
        if len(inc) == 1:
            C.sketch_build(n, [torch.from_numpy(attr).cuda()], preds,
                           [torch.from_numpy(cols[0]).cuda()], [seeds[inc[0]]], [T], ns,
                           d, wt[0], counter_bits=bits)
            o = oracle.sketch(cols[0][mask], seeds[inc[0]], d, wt[0])
        else:
            C.sketch_build_kd(n, [torch.from_numpy(attr).cuda()], preds,
                              [torch.from_numpy(c).cuda() for c in cols],
                              [seeds[e] for e in inc], T, ns, d, wt, counter_bits=bits)
            o = oracle.sketch_kd([c[mask] for c in cols], [seeds[e] for e in inc], d, wt)
        torch.cuda.synchronize()
        assert np.array_equal(T.cpu().numpy().astype(np.int64), o), t
        tensors.append(T)
        o_tensors.append(o)
        n_sel.append(int(ns.item()))
    nst = torch.tensor(n_sel, dtype=torch.int64, device="cuda")
    rows, est, flag = C.estimate_partitioned(eu, ev, d, widths, tensors, nst,
                                             counter_bits=bits)
    torch.cuda.synchronize()
    vals, e_o, f_o = oracle.tensor_join(nt, eu, ev, d, widths, o_tensors, n_sel)
    r = rows.cpu().numpy().astype(np.int64)
    got = [(int(r[i, 0]) & (2**64 - 1)) | ((int(r[i, 1]) & (2**64 - 1)) << 64)
           for i in range(d)]
    assert got == vals
    assert float(est.item()) == e_o
    assert int(flag.item()) == f_o
