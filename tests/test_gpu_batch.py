"""The batched persistent graph-captured build gives the same counters and
selected counts as one build call per table (bit-exact), for every tuning
candidate and on repeated graph replays; spot checks against the oracle."""
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


def snapshot(db):
    return ([[s.clone() for s in sides] for sides in db.sides],
            [n.clone() for n in db.n_selected])


@gpu
@pytest.mark.parametrize("tune", [None, (65536, 65536, 2), (4096, 131072, 1),
                                  (1 << 20, 65536, 1)])
def test_batch_equals_per_table(oracle, tune, tmp_path, monkeypatch):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    monkeypatch.setenv("COMPASS_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    pool = W.schema_pool(seed=3, n_tables=12, scale=0.004)
    qs = W.query_batch(pool, seed=4, n_queries=24, w_choices=(64, 1000, 1024, 4096))
    print("[case] batch tune", tune, "jobs", sum(len(q.tables) for q in qs), flush=True)
    db = C.DeviceBatch(pool, qs)
    db.build_per_table()
    torch.cuda.synchronize()
    ref_sides, ref_n = snapshot(db)
    for sides in db.sides:
        for s in sides:
            s.fill_(12345)
    plan = db.plan(tune=tune)
    print("[case] plan", plan.info(), flush=True)
    for rep in range(3):
        plan.launch()
        torch.cuda.synchronize()
        for qi in range(len(qs)):
            assert torch.equal(db.n_selected[qi], ref_n[qi]), (rep, qi)
            for a, b in zip(db.sides[qi], ref_sides[qi]):
                assert torch.equal(a, b), (rep, qi)
        # eager work between replays
        torch.cuda.synchronize()
    # oracle spot check of three queries
    for qi in range(0, len(qs), 9):
        q = W.pool_query_as_query(pool, qs[qi])
        for t, tb in enumerate(q.tables):
            mask = oracle.eval_predicates(tb.cols, tb.preds)
            assert db.n_selected[qi][t].item() == int(mask.sum())
            for (e, side, c) in q.incident(t):
                o = oracle.sketch(tb.cols[c][mask], q.seeds[e], q.d, q.w)
                assert np.array_equal(db.sides[qi][2 * e + side].cpu().numpy().astype(np.int64), o)
    plan.close()


@gpu
@pytest.mark.parametrize("w_choices", [(512, 1000, 2048), (1024, 20000, 32768)])
def test_batch_two_phase_rounds(oracle, tmp_path, monkeypatch, w_choices):
    """Jobs with predicates cut into many segments and rounds (a 1 MiB
    survivor arena instead of 8 GiB): still bit-exact against one build
    call per table, on repeated graph replays.  Rows of at most 16384
    buckets hash into int32 LDS counters, wider ones into 16-bit pairs; the
    second case mixes both in the same rounds."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    monkeypatch.setenv("COMPASS_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    monkeypatch.setenv("COMPASS_BATCH_ARENA_BYTES", str(1 << 20))
    pool = W.schema_pool(seed=5, n_tables=10, scale=0.004)
    qs = W.query_batch(pool, seed=6, n_queries=16, w_choices=w_choices)
    print("[case] batch rounds jobs", sum(len(q.tables) for q in qs), w_choices,
          flush=True)
    db = C.DeviceBatch(pool, qs)
    db.build_per_table()
    torch.cuda.synchronize()
    ref_sides, ref_n = snapshot(db)
    for sides in db.sides:
        for s in sides:
            s.fill_(-7)
    plan = db.plan(tune=(65536, 65536, 1))
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for qi in range(len(qs)):
            assert torch.equal(db.n_selected[qi], ref_n[qi]), (rep, qi)
            for a, b in zip(db.sides[qi], ref_sides[qi]):
                assert torch.equal(a, b), (rep, qi)
    plan.close()


@gpu
def test_batch_estimates_match_oracle(oracle):
    """Estimates over batch-built sketches (trees and triangles) vs oracle."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    pool = W.schema_pool(seed=8, n_tables=10, scale=0.002)
    qs = W.query_batch(pool, seed=9, n_queries=12, w_choices=(256, 512), tri_prob=0.5)
    db = C.DeviceBatch(pool, qs)
    plan = db.plan(tune=(65536, 65536, 1))
    plan.launch()
    torch.cuda.synchronize()
    for qi, pq in enumerate(qs):
        eu = [e.u for e in pq.edges]
        ev = [e.v for e in pq.edges]
        masks = oracle.connected_subplans(len(pq.tables), eu, ev, max_tables=4)[:40]
        print("[case] batch estimates query", qi, len(pq.tables), len(masks), flush=True)
        row_est, est, flags = db.estimate(qi, masks)
        torch.cuda.synchronize()
        sides = [s.cpu().numpy().astype(np.int64) for s in db.sides[qi]]
        n_sel = db.n_selected[qi].cpu().tolist()
        vals, e_o, f_o = oracle.estimate(len(pq.tables), eu, ev, pq.d, pq.w, sides,
                                         n_sel, masks)
        got = C.row_values(row_est)
        fl = flags.cpu().numpy()
        for m in range(len(masks)):
            sup = supported_shape(eu, ev, masks[m], pq.w, pq.d)
            if sup is not None:
                assert bool(fl[m] & C.FLAG_UNSUPPORTED) == (not sup), hex(masks[m])
            if fl[m] & C.FLAG_UNSUPPORTED:
                continue
            assert got[m] == [v & ((1 << 128) - 1) for v in vals[m]]
            f_x, e_x, tol = expected_flag_est(oracle, len(pq.tables), eu, ev, pq.d,
                                              pq.w, sides, n_sel, masks[m], vals[m],
                                              f_o[m], e_o[m])
            assert abs(est.cpu().numpy()[m] - e_x) <= tol
            assert fl[m] == f_x
