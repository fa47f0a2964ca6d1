"""Parity of the AGMS baseline (Section 4.1) with the oracle: counters bit
for bit, estimates (exact row sums, median of averages, flag) exactly."""
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


def _agms_seeds(q, r, b):
    """One independent family per join and basic sketch: (n_edges, r*b, 6)."""
    rng = np.random.default_rng(4242 + len(q.edges))
    return W.draw_seeds(rng, len(q.edges), r * b)


def _device_preds(tb, cols, dev):
    import torch
    names = list(cols)
    out = []
    for p in tb.preds:
        e = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
        if p.kind == "subset":
            e["bitmap"] = torch.from_numpy(np.asarray(p.bitmap, np.uint64).view(np.int64)).to(dev)
            e["domain"] = p.domain
        out.append(e)
    return out


def _check_query(oracle, q, r, b, name):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    _say(name, [tb.n_rows for tb in q.tables], "r", r, "b", b)
    dev = "cuda"
    seeds = _agms_seeds(q, r, b)
    sks, ns, sks_o, ns_o = [], [], [], []
    for t, tb in enumerate(q.tables):
        inc = q.incident(t)
        cols = {c: torch.from_numpy(v).to(dev) for c, v in tb.cols.items()}
        cnt = torch.zeros((r, b), dtype=torch.int64, device=dev)
        nsel = torch.zeros(1, dtype=torch.int64, device=dev)
        C.agms_build(tb.n_rows, list(cols.values()), _device_preds(tb, cols, dev),
                     [cols[c] for (_, _, c) in inc], [seeds[e] for (e, _, _) in inc],
                     cnt, nsel, r, b)
        mask = oracle.eval_predicates(tb.cols, tb.preds)
        co = oracle.agms_sketch([tb.cols[c][mask] for (_, _, c) in inc],
                                [seeds[e] for (e, _, _) in inc], r, b)
        torch.cuda.synchronize()
        assert nsel.item() == int(mask.sum()), tb.name
        assert np.array_equal(cnt.cpu().numpy(), co), tb.name
        sks.append(cnt)
        ns.append(nsel)
        sks_o.append(co)
        ns_o.append(int(mask.sum()))
    rows, est, flag = C.agms_estimate(sks, ns)
    torch.cuda.synchronize()
    rows_o, est_o, flag_o = oracle.agms_estimate(sks_o, ns_o)
    rg = C.row_values(rows.reshape(1, r, 2))[0]
    assert rg == [v & ((1 << 128) - 1) for v in rows_o]
    assert est.item() == est_o
    assert flag.item() == flag_o


@gpu
@pytest.mark.parametrize("seed", range(3))
def test_agms_random_queries(oracle, seed):
    rng = np.random.default_rng(600 + seed)
    q = W.small_random_query(rng, int(rng.integers(2, 5)), int(rng.integers(100, 5000)),
                             int(rng.choice([10, 1000, 10**6])), 1, 8,
                             cyclic=bool(seed % 2))
    _check_query(oracle, q, int(rng.choice([1, 3, 4])), int(rng.choice([1, 7, 64])),
                 "agms random seed=%d" % seed)


@gpu
def test_agms_6a_scaled(oracle):
    q = W.job6a(seed=9, scale=0.01)
    _check_query(oracle, q, 7, 16, "agms 6a scale 0.01")


@gpu
def test_agms_int64_keys_four_joins(oracle):
    """A table with four joins, int64 keys incl. negatives and values above
    2^32, r * b = 1024 (one lane per basic sketch), a ragged row count."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(77)
    n = 4096 * 2 + 123
    keys = [rng.integers(-2**40, 2**40, n).astype(np.int64) for _ in range(4)]
    keys[1] = (keys[1] % 1000).astype(np.int64)
    r, b = 16, 64
    seeds = W.draw_seeds(rng, 4, r * b)
    _say("agms four joins", n, r, b)
    dk = [torch.from_numpy(k).to("cuda") for k in keys]
    cnt = torch.zeros((r, b), dtype=torch.int64, device="cuda")
    nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
    C.agms_build(n, [], [], dk, list(seeds), cnt, nsel, r, b)
    co = oracle.agms_sketch(keys, list(seeds), r, b)
    torch.cuda.synchronize()
    assert np.array_equal(cnt.cpu().numpy(), co)
    assert nsel.item() == n


@gpu
def test_agms_full_size_cast_info_sampled(oracle):
    """cast_info of the 6a shape at full size (36M rows, three joins) in the
    configuration the benchmark times (r = 7, b = 16): two sampled basic
    sketches computed by the oracle one at a time."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    q = W.job6a(seed=W.DEFAULT_SEED)
    t = 3
    tb = q.tables[t]
    inc = q.incident(t)
    r, b = 7, 16
    seeds = _agms_seeds(q, r, b)
    _say("agms cast_info full size", tb.n_rows)
    cols = {c: torch.from_numpy(v).to("cuda") for c, v in tb.cols.items()}
    cnt = torch.zeros((r, b), dtype=torch.int64, device="cuda")
    nsel = torch.zeros(1, dtype=torch.int64, device="cuda")
    C.agms_build(tb.n_rows, [], [], [cols[c] for (_, _, c) in inc],
                 [seeds[e] for (e, _, _) in inc], cnt, nsel, r, b)
    got = cnt.cpu().numpy().reshape(-1)
    assert nsel.item() == tb.n_rows
    for c in (5, r * b - 1):
        one = oracle.agms_sketch([tb.cols[col] for (_, _, col) in inc],
                                 [seeds[e][c:c + 1] for (e, _, _) in inc], 1, 1)
        assert got[c] == one[0, 0], c
