"""Learned correction of merged-sketch estimates, end to end on the GPU.

Dataset: every query of a workload is sketched with the batched persistent
build, its sampled sub-plans are estimated with compass_estimate, and the 20
features per sub-plan are computed by the library's feature kernel.  The
network (compass_mlp_*) is trained by the library's forward / backward /
Adam kernels on ln(1 + true) targets supplied by the caller (exact join
sizes from an independent counter), and evaluated against the raw median
estimate on held-out sub-plans by q-error.  The raw estimate stays the
fallback: the network predicts a correction on top of it.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import compass as C


def init_params(seed: int, n_in=20, hidden=64, layers=3) -> np.ndarray:
    """He-uniform hidden weights, zero biases, zero output layer (the
    untrained network returns the raw estimate)."""
    rng = np.random.default_rng(seed)
    dims = [n_in] + [hidden] * layers + [1]
    flat = []
    for i in range(len(dims) - 1):
        lim = np.sqrt(6.0 / dims[i])
        W = rng.uniform(-lim, lim, size=(dims[i + 1], dims[i]))
        if i == len(dims) - 2:
            W[:] = 0.0
        flat += [W.reshape(-1), np.zeros(dims[i + 1])]
    return np.concatenate(flat).astype(np.float32)


def build_features(pool, queries, subplans, device="cuda", group=1500,
                   tune=(262144, 131072, 1), log=None):
    """(x [N,20], base [N], est [N] float64, flags [N]) device tensors for the
    sub-plans `subplans[q]` of every query q, in query order."""
    pool_cols = C.upload_pool(pool, device)
    xs, bases, ests, flags = [], [], [], []
    t0 = time.time()
    for g0 in range(0, len(queries), group):
        qs = queries[g0:g0 + group]
        db = C.DeviceBatch(pool, qs, device=device, pool_cols=pool_cols)
        plan = db.plan(tune=tune)
        plan.launch()
        for k, pq in enumerate(qs):
            masks = subplans[g0 + k]
            if not masks:
                continue
            eu = [e.u for e in pq.edges]
            ev = [e.v for e in pq.edges]
            row_est, est, fl = db.estimate(k, masks)
            md = torch.from_numpy(np.asarray(masks, dtype=np.uint64).view(np.int64)).to(device)
            x, base = C.features(row_est, est, md, db.n_selected[k], len(pq.tables), eu, ev)
            xs.append(x)
            bases.append(base)
            ests.append(est)
            flags.append(fl)
        torch.cuda.synchronize()
        plan.close()
        del db
        if log:
            log("[learned] features of queries %d..%d in %.1fs" %
                (g0, g0 + len(qs), time.time() - t0))
    return torch.cat(xs), torch.cat(bases), torch.cat(ests), torch.cat(flags)


def train(x, base, target, init, epochs=30, batch=512, lr=1e-3, seed=0,
          log=None):
    """Adam on mean squared error of ln(1 + card); returns (mlp, losses)."""
    mlp = C.MLP(init)
    n = x.shape[0]
    g = torch.Generator(device=x.device)
    g.manual_seed(seed)
    hist = []
    for ep in range(epochs):
        # one library call per epoch: the batches gather their rows through
        # the permutation inside the kernels
        perm = torch.randperm(n, device=x.device, generator=g).to(torch.int32)
        losses = mlp.train_epoch(x, base, target, perm, batch, lr)
        hist.append(float(losses.double().mean().item()) if losses.numel() else 0.0)
        if log:
            log("[learned] epoch %d mse %.4f" % (ep, hist[-1]))
    return mlp, hist


def qerror(est, true):
    e = np.maximum(np.asarray(est, dtype=np.float64), 1.0)
    t = np.maximum(np.asarray(true, dtype=np.float64), 1.0)
    return np.maximum(e / t, t / e)


def summarize(q):
    return {"median": float(np.median(q)), "p90": float(np.percentile(q, 90)),
            "p99": float(np.percentile(q, 99)), "max": float(np.max(q))}


def evaluate(mlp, x, base, est, true):
    """q-error of the raw median estimate and of the corrected estimate."""
    y = mlp.forward(x, base)
    learned = np.expm1(y.double().cpu().numpy())
    raw = est.cpu().numpy()
    return {"raw": summarize(qerror(raw, true)),
            "learned": summarize(qerror(learned, true)),
            "n": int(len(true))}


def compare_paths(pool, queries, subplans, mlp, true, device="cuda", tune=None,
                  log=None, reps=2):
    """End to end on one workload, same GPU: the plain path (one
    compass_sketch_build launch per sketch, then the raw median estimates)
    against the batched + learned path (one graph launch for every sketch,
    the same estimates, the feature kernel and the network's forward pass).
    Returns wall times (host clock, after a warm-up of each path) and the
    q-error of each path's estimates against `true`."""
    pool_cols = C.upload_pool(pool, device)
    db = C.DeviceBatch(pool, queries, device=device, pool_cols=pool_cols)
    plan = db.plan(tune=tune)
    todo = [(k, subplans[k]) for k in range(len(queries)) if subplans[k]]
    masks_dev = {k: torch.from_numpy(np.asarray(m, dtype=np.uint64).view(np.int64)).to(device)
                 for k, m in todo}

    def estimates():
        return [(k,) + tuple(db.estimate(k, m)) for k, m in todo]

    def plain():
        db.build_per_sketch()
        outs = estimates()
        return torch.cat([o[2] for o in outs])

    def batched_learned():
        plan.launch()
        outs = estimates()
        xs, bs = [], []
        for (k, row_est, est, fl) in outs:
            pq = queries[k]
            x, b = C.features(row_est, est, masks_dev[k], db.n_selected[k],
                              len(pq.tables), [e.u for e in pq.edges],
                              [e.v for e in pq.edges])
            xs.append(x)
            bs.append(b)
        return mlp.forward(torch.cat(xs), torch.cat(bs))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            a = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - a
            best = dt if best is None else min(best, dt)
        return best, out

    t_plain, raw = timed(plain)
    t_bl, y = timed(batched_learned)
    raw = raw.cpu().numpy()
    learned = np.expm1(y.double().cpu().numpy())
    plan.close()
    n_sk = sum(len(j["keys"]) for j in db.jobs)
    res = {"queries": len(queries), "sub_plans": int(len(true)), "sketches": n_sk,
           "plain_s": t_plain, "batched_learned_s": t_bl,
           "speedup": t_plain / t_bl,
           "qerror_plain_raw": summarize(qerror(raw, true)),
           "qerror_batched_learned": summarize(qerror(learned, true))}
    if log:
        log("[learned] end to end: plain %.3f s, batched + learned %.3f s" % (t_plain, t_bl))
    return res
