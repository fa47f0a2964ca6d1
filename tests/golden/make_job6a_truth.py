"""Writes job6a_truth.json: exact join sizes (oracle hash aggregation) of all
19 connected sub-plans of the 6a-shaped five-table workload at full size,
default seed.  Calls only the seeded generators and the oracle."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as o  # noqa: E402
from paper_2102_02440_amd import workloads as W  # noqa: E402


def main(seed=W.DEFAULT_SEED, scale=1.0):
    q = W.job6a(seed=seed, scale=scale)
    filt = []
    for tb in q.tables:
        m = o.eval_predicates(tb.cols, tb.preds)
        filt.append({c: v[m] for c, v in tb.cols.items()})
    edges = [(e.u, e.ucol, e.v, e.vcol) for e in q.edges]
    masks = o.connected_subplans(len(q.tables), q.edge_u, q.edge_v)
    true = [o.true_cardinality(filt, edges, m) for m in masks]
    out = {"generator": "workloads.job6a", "seed": seed, "scale": scale,
           "masks": masks, "true": true,
           "n_selected": [len(next(iter(f.values()))) for f in filt]}
    path = os.path.join(HERE, "job6a_truth.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
