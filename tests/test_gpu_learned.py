"""End to end: sketches and estimates from the HIP path, features from the
feature kernel, the network trained by the library's kernels on exact
oracle join sizes; on held-out sub-plans (disjoint seeds) the corrected
estimate beats the raw median estimate in median q-error."""
import numpy as np
import pytest

from paper_2102_02440_amd import workloads as W

gpu = pytest.mark.gpu


def _truths(oracle, pool, queries, subs):
    out = []
    for pq, masks in zip(queries, subs):
        q = W.pool_query_as_query(pool, pq)
        filt = []
        for tb in q.tables:
            m = oracle.eval_predicates(tb.cols, tb.preds)
            filt.append({c: v[m] for c, v in tb.cols.items()})
        edges = [(e.u, e.ucol, e.v, e.vcol) for e in q.edges]
        dom = [pool[t].n_rows for t in pq.tables]
        out += [oracle.true_cardinality_fk_tree(filt, edges, m, dom) for m in masks]
    return np.asarray(out)


@gpu
def test_learned_beats_raw_on_held_out(oracle):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_02440_amd import learned as Lrn
    kw = dict(pool_tables=16, size_range=(10_000, 200_000), d=7, w=1024)
    pool_tr, q_tr = W.learned_workload(31, 900, **kw)
    pool_te, q_te = W.learned_workload(32, 250, **kw)
    s_tr = W.learned_subplans(q_tr, 31, max_per_query=12)
    s_te = W.learned_subplans(q_te, 32, max_per_query=12)
    print("[case] learned small: train", sum(map(len, s_tr)), "test",
          sum(map(len, s_te)), flush=True)
    t_tr = _truths(oracle, pool_tr, q_tr, s_tr)
    t_te = _truths(oracle, pool_te, q_te, s_te)
    x, b, e, f = Lrn.build_features(pool_tr, q_tr, s_tr, tune=(65536, 65536, 1))
    xt, bt, et, ft = Lrn.build_features(pool_te, q_te, s_te, tune=(65536, 65536, 1))
    tgt = torch.from_numpy(np.log1p(t_tr).astype(np.float32)).cuda()
    mlp, hist = Lrn.train(x, b, tgt, oracle.mlp_init(1).astype(np.float32),
                          epochs=25, lr=2e-3)
    res = Lrn.evaluate(mlp, xt, bt, et, t_te)
    print("[case] learned vs raw", res, flush=True)
    assert hist[-1] < hist[0]
    assert res["learned"]["median"] <= res["raw"]["median"]
