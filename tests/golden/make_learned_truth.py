"""Writes learned_truth.npz: exact join sizes (oracle, foreign-key tree
message passing) of the sampled sub-plans of the learned-correction
workload, for the training and the held-out seeds.  Calls only the seeded
generators and the oracle.

usage: python tests/golden/make_learned_truth.py [n_train_queries n_test_queries]
"""
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as o  # noqa: E402
from paper_2102_02440_amd import workloads as W  # noqa: E402

_STATE = {}


def _init(seed, n_queries):
    pool, qs = W.learned_workload(seed, n_queries)
    _STATE["pool"], _STATE["qs"] = pool, qs
    _STATE["subs"] = W.learned_subplans(qs, seed)


def _work(qi):
    pool, pq, masks = _STATE["pool"], _STATE["qs"][qi], _STATE["subs"][qi]
    q = W.pool_query_as_query(pool, pq)
    filt = []
    for tb in q.tables:
        m = o.eval_predicates(tb.cols, tb.preds)
        filt.append({c: tb.cols[c][m] for c in set(
            [e.ucol for e in q.edges if q.tables[e.u] is tb] +
            [e.vcol for e in q.edges if q.tables[e.v] is tb] + ["id"])})
    edges = [(e.u, e.ucol, e.v, e.vcol) for e in q.edges]
    dom = [pool[t].n_rows for t in pq.tables]
    return [(qi, m, o.true_cardinality_fk_tree(filt, edges, m, dom)) for m in masks]


def compute(seed, n_queries, procs=8):
    with Pool(procs, initializer=_init, initargs=(seed, n_queries)) as p:
        res = p.map(_work, range(n_queries), chunksize=8)
    flat = [r for part in res for r in part]
    return (np.array([r[0] for r in flat], dtype=np.int32),
            np.array([r[1] for r in flat], dtype=np.uint64),
            np.array([r[2] for r in flat], dtype=np.float64))


def main(n_train=12000, n_test=1200):
    t0 = time.time()
    qi_tr, m_tr, t_tr = compute(W.LEARNED_TRAIN_SEED, n_train)
    print("train", len(t_tr), "sub-plans in %.0fs" % (time.time() - t0), flush=True)
    qi_te, m_te, t_te = compute(W.LEARNED_TEST_SEED, n_test)
    print("test", len(t_te), "sub-plans in %.0fs" % (time.time() - t0), flush=True)
    path = os.path.join(HERE, "learned_truth.npz")
    np.savez_compressed(path, train_query=qi_tr, train_mask=m_tr, train_true=t_tr,
                        test_query=qi_te, test_mask=m_te, test_true=t_te,
                        n_train_queries=n_train, n_test_queries=n_test)
    print("wrote", path)


if __name__ == "__main__":
    a = [int(x) for x in sys.argv[1:3]]
    main(*a)
