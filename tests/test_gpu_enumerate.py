"""Plan enumeration (Algorithm 1, Section 6) fed with the GPU's estimates,
in the four search spaces of Section 7.2.8 (greedy, full-greedy, limit-10,
exhaustive).  The library's choice on the GPU estimates equals the
oracle's enumeration on the same estimates, and every chosen plan is scored
by its true cost (sum of the exact sizes of its prefixes, oracle hash
aggregation) against the optimum that exhaustive search finds with the
exact sizes."""
import numpy as np
import pytest

from paper_2102_02440_amd import workloads as W
from tests.shapes import supported_shape

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def score_plans(oracle, C, n, eu, ev, masks, est, card, true_of):
    """Per variant: (order, estimated cost, true cost); and the optimum."""
    est_of = dict(zip(masks, est))
    out = {}
    for name, mp in C.ENUM_VARIANTS:
        order, cost = C.enumerate_variant(name, n, eu, ev, masks, est, card)
        if mp is None:
            o_order, o_cost = oracle.plan_greedy(n, eu, ev, est_of, card)
        else:
            o_order, o_cost, _ = oracle.plan_enumeration(n, eu, ev, est_of, card, mp)
        assert (order, cost) == (o_order, o_cost), name
        out[name] = (order, cost, oracle.plan_cost(order, true_of))
    opt_order, opt_cost, _ = oracle.plan_enumeration(n, eu, ev, true_of, card, 0)
    assert opt_cost == oracle.plan_cost(opt_order, true_of)
    for name in out:
        assert out[name][2] >= opt_cost * (1 - 1e-12), name
    return out, opt_cost


@gpu
def test_enumeration_on_gpu_estimates_job6a(oracle):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    q = W.job6a(seed=7, scale=0.01, d=7, w=1024)
    print("[case] enumeration 6a scale 0.01", flush=True)
    dq = C.DeviceQuery(q)
    dq.build()
    masks = oracle.connected_subplans(5, q.edge_u, q.edge_v)
    _, est, flags = dq.estimate(masks)
    torch.cuda.synchronize()
    est = est.cpu().numpy().astype(np.float64).tolist()
    card = [float(x) for x in dq.n_selected.cpu().tolist()]
    filt = []
    for tb in q.tables:
        m = oracle.eval_predicates(tb.cols, tb.preds)
        filt.append({c: v[m] for c, v in tb.cols.items()})
    edges = [(e.u, e.ucol, e.v, e.vcol) for e in q.edges]
    true_of = {m: oracle.true_cardinality(filt, edges, m) for m in masks}
    res, opt = score_plans(oracle, C, 5, q.edge_u, q.edge_v, masks, est, card, true_of)
    print("[case] 6a plans", {k: (v[0], v[2] / opt) for k, v in res.items()}, flush=True)
    # exhaustive on the estimates is optimal for the estimates
    assert res["exhaustive"][1] <= min(v[1] for v in res.values())


@gpu
def test_enumeration_on_gpu_estimates_batch_queries(oracle):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    pool = W.schema_pool(seed=8, n_tables=12, scale=0.002)
    qs = W.query_batch(pool, seed=19, n_queries=16, max_tables=6,
                       w_choices=(512, 1024), tri_prob=0.3)
    db = C.DeviceBatch(pool, qs)
    plan = db.plan(tune=(65536, 65536, 1))
    plan.launch()
    torch.cuda.synchronize()
    scored = 0
    for qi, pq in enumerate(qs):
        n = len(pq.tables)
        if n < 3:
            continue
        eu = [e.u for e in pq.edges]
        ev = [e.v for e in pq.edges]
        masks = oracle.connected_subplans(n, eu, ev)
        if not all(supported_shape(eu, ev, m) for m in masks):
            continue
        print("[case] enumeration batch query", qi, n, len(masks), flush=True)
        _, est, flags = db.estimate(qi, masks)
        torch.cuda.synchronize()
        est = est.cpu().numpy().astype(np.float64).tolist()
        card = [float(x) for x in db.n_selected[qi].cpu().tolist()]
        q = W.pool_query_as_query(pool, pq)
        filt = []
        for tb in q.tables:
            m = oracle.eval_predicates(tb.cols, tb.preds)
            filt.append({c: v[m] for c, v in tb.cols.items()})
        edges = [(e.u, e.ucol, e.v, e.vcol) for e in q.edges]
        true_of = {m: oracle.true_cardinality(filt, edges, m) for m in masks}
        res, opt = score_plans(oracle, C, n, eu, ev, masks, est, card, true_of)
        print("[case] plans", {k: (v[0], v[2] / max(opt, 1.0)) for k, v in res.items()},
              flush=True)
        scored += 1
    plan.close()
    assert scored >= 4
