"""CPU oracle for the online sketch-based query optimisation hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product (the HIP library
and its Python binding) never imports this module, and this module never
imports the product.  Inputs come from the seeded generators, which hold
none of the method's arithmetic.

What each function follows (paper: Izenov et al., "Online Sketch-based
Query Optimization", arXiv 2102.02440):

* ``eval_predicates``  -- Section 1 (query 6a: point, subset and range
  selections) and Section 3 "Partitioned query execution" (conjunctive
  selections pushed down; only qualifying tuples reach the sketch).
* ``sketch``           -- Section 4.2, Fast-AGMS counter definition, with the
  hash families of ``compass_oracle.c`` (Carter-Wegman polynomials mod
  2^61-1; the paper names no family).
* ``estimate``         -- Section 4.2.1 (two-way inner product, median over
  rows), Section 5.1 (3-way contraction), Section 5.2 (min-abs sketch
  merging, applied iteratively to any number of joins).
* ``true_cardinality`` -- exact join size by hash aggregation over attribute
  equivalence classes (the ground truth the estimates are judged by).
* ``qerror`` / ``ratio`` / ``l1_permutation_distance`` -- Section 5.2 accuracy
  measures (estimate/true ratio, normalised L1 permutation distance) and the
  q-error used to summarise them.
* ``mlp_*``            -- learned correction network (not in the paper),
  forward/backward in float64 NumPy on bfloat16-rounded parameters.

Each reading of a silent or ambiguous passage is stated next to the code
that applies it.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "compass_oracle.c")

P61 = (1 << 61) - 1
FLAG_EXACT = 1


def build(force: bool = False) -> str:
    """Compiles the C part of the oracle next to its source."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH)):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC_PATH])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_hash.argtypes = [u64p, ctypes.c_int64, ctypes.c_int64,
                                    i64p, i32p]
        lib.oracle_hash.restype = None
        lib.oracle_sketch.argtypes = [i64p, ctypes.c_int64, u64p,
                                      ctypes.c_int32, ctypes.c_int64, i64p]
        lib.oracle_sketch_mt.argtypes = [i64p, ctypes.c_int64, u64p,
                                         ctypes.c_int32, ctypes.c_int64, i64p,
                                         ctypes.c_int32]
        lib.oracle_sketch.restype = None
        lib.oracle_estimate.argtypes = [
            ctypes.c_int32, ctypes.c_int32, i32p, i32p, ctypes.c_int32,
            ctypes.c_int64, ctypes.POINTER(i64p), i64p, u64p, ctypes.c_int32,
            ctypes.c_int32, u64p, ctypes.POINTER(ctypes.c_double), i32p]
        lib.oracle_estimate.restype = ctypes.c_int32
        lib.oracle_sketch2d.argtypes = [i64p, i64p, ctypes.c_int64, u64p, u64p,
                                        ctypes.c_int32, ctypes.c_int64,
                                        ctypes.c_int64, i64p]
        lib.oracle_sketch2d.restype = None
        lib.oracle_sketch_kd.argtypes = [ctypes.POINTER(i64p), ctypes.c_int32,
                                         ctypes.c_int64, ctypes.POINTER(u64p),
                                         ctypes.c_int32, i64p, i64p]
        lib.oracle_sketch_kd.restype = None
        lib.oracle_tensor_join.argtypes = [
            ctypes.c_int32, ctypes.c_int32, i32p, i32p, ctypes.c_int32, i64p,
            ctypes.POINTER(i64p), i64p, u64p, ctypes.POINTER(ctypes.c_double), i32p]
        lib.oracle_tensor_join.restype = None
        lib.oracle_chain3.argtypes = [i64p, i64p, i64p, ctypes.c_int32,
                                      ctypes.c_int64, ctypes.c_int64, i64p, u64p,
                                      ctypes.POINTER(ctypes.c_double), i32p]
        lib.oracle_chain3.restype = None
        lib.oracle_agms_sketch.argtypes = [ctypes.POINTER(i64p), ctypes.c_int64,
                                           u64p, ctypes.c_int32, ctypes.c_int32,
                                           i64p]
        lib.oracle_agms_sketch.restype = None
        lib.oracle_agms_estimate.argtypes = [ctypes.POINTER(i64p), ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, i64p,
                                             u64p, ctypes.POINTER(ctypes.c_double),
                                             i32p]
        lib.oracle_agms_estimate.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int32]
        lib.oracle_i128_to_double.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_i128_to_double.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# --------------------------------------------------------------------------
# Hash (one key, one row)
# --------------------------------------------------------------------------
def hash_key(seeds6, key: int, w: int):
    """(bucket, sign) of ``key`` under one row's seeds {a0,a1,a2,a3,b0,b1}."""
    lib = _load()
    s = np.ascontiguousarray(np.asarray(seeds6, dtype=np.uint64))
    b = ctypes.c_int64()
    sg = ctypes.c_int32()
    lib.oracle_hash(_ptr(s, ctypes.c_uint64), int(key), int(w),
                    ctypes.byref(b), ctypes.byref(sg))
    return b.value, sg.value


# --------------------------------------------------------------------------
# Selections (conjunctive push-down predicates)
# --------------------------------------------------------------------------
def eval_predicates(columns: dict, preds) -> np.ndarray:
    """Boolean mask of rows that satisfy every predicate.

    Reading (the paper is silent on these details): RANGE bounds are
    inclusive; float columns use IEEE comparisons (NaN fails every
    comparison, -0 equals +0); SUBSET tests bit ``code`` of a bitmap over
    the code domain [0, domain) and fails outside the domain; no NULLs.
    With no predicates every row qualifies.
    """
    n = None
    for c in columns.values():
        n = len(c)
        break
    mask = np.ones(n if n is not None else 0, dtype=bool)
    for p in preds:
        v = columns[p.col]
        if p.kind == "point":
            mask &= (v == v.dtype.type(p.lo))
        elif p.kind == "range":
            mask &= (v >= v.dtype.type(p.lo)) & (v <= v.dtype.type(p.hi))
        elif p.kind == "subset":
            code = v.astype(np.int64)
            inside = (code >= 0) & (code < p.domain)
            safe = np.where(inside, code, 0)
            words = np.asarray(p.bitmap, dtype=np.uint64)[safe >> 6]
            bit = (words >> (safe & 63).astype(np.uint64)) & np.uint64(1)
            mask &= inside & (bit == 1)
        else:
            raise ValueError(p.kind)
    return mask


# --------------------------------------------------------------------------
# Sketch build
# --------------------------------------------------------------------------
def default_threads() -> int:
    """Threads the oracle's parallel loops use: OMP_NUM_THREADS when set,
    else the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.strip().isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def sketch(keys: np.ndarray, seeds: np.ndarray, d: int, w: int,
           threads: int | None = None) -> np.ndarray:
    """Fast-AGMS counters (d x w, int64) of the given (already filtered) keys.

    ``threads``: 1 runs the literal loop; more split the keys into
    contiguous parts with private counters that are summed at the end
    (default: ``default_threads()``)."""
    lib = _load()
    k = np.ascontiguousarray(np.asarray(keys).astype(np.int64))
    s = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(d, 6))
    out = np.zeros((d, w), dtype=np.int64)
    nt = default_threads() if threads is None else int(threads)
    lib.oracle_sketch_mt(_ptr(k, ctypes.c_int64), int(k.size),
                         _ptr(s, ctypes.c_uint64), int(d), int(w),
                         _ptr(out, ctypes.c_int64), nt)
    return out


def sketch2d(keys1, keys2, seeds1, seeds2, d: int, w1: int, w2: int) -> np.ndarray:
    """Partitioned sketch (Section 5.1) of the (already filtered) key pairs:
    d x w1 x w2 int64 counters."""
    lib = _load()
    k1 = np.ascontiguousarray(np.asarray(keys1).astype(np.int64))
    k2 = np.ascontiguousarray(np.asarray(keys2).astype(np.int64))
    assert k1.size == k2.size
    s1 = np.ascontiguousarray(np.asarray(seeds1, dtype=np.uint64).reshape(d, 6))
    s2 = np.ascontiguousarray(np.asarray(seeds2, dtype=np.uint64).reshape(d, 6))
    out = np.zeros((d, w1, w2), dtype=np.int64)
    lib.oracle_sketch2d(_ptr(k1, ctypes.c_int64), _ptr(k2, ctypes.c_int64),
                        int(k1.size), _ptr(s1, ctypes.c_uint64),
                        _ptr(s2, ctypes.c_uint64), int(d), int(w1), int(w2),
                        _ptr(out, ctypes.c_int64))
    return out


def chain3(A, P, B, n_sel3):
    """Three-table chain estimate of Section 5.1 from the sketches A (d x w1),
    P (d x w1 x w2) and B (d x w2): (row values as python ints, median,
    exactness flag)."""
    lib = _load()
    P = np.ascontiguousarray(np.asarray(P, dtype=np.int64))
    d, w1, w2 = P.shape
    A = np.ascontiguousarray(np.asarray(A, dtype=np.int64).reshape(d, w1))
    B = np.ascontiguousarray(np.asarray(B, dtype=np.int64).reshape(d, w2))
    ns = np.ascontiguousarray(np.asarray(n_sel3, dtype=np.int64).reshape(3))
    rows = np.zeros((d, 2), dtype=np.uint64)
    est = ctypes.c_double()
    flag = ctypes.c_int32()
    lib.oracle_chain3(_ptr(A, ctypes.c_int64), _ptr(P, ctypes.c_int64),
                      _ptr(B, ctypes.c_int64), int(d), int(w1), int(w2),
                      _ptr(ns, ctypes.c_int64), _ptr(rows, ctypes.c_uint64),
                      ctypes.byref(est), ctypes.byref(flag))
    vals = [i128_to_int(rows[i, 0], rows[i, 1]) for i in range(d)]
    return vals, est.value, flag.value


def sketch_kd(keys_per_join, seeds_per_join, d: int, widths) -> np.ndarray:
    """Partitioned sketch (Section 5.1) of a table with k joins: one (already
    filtered) key array and one (d, 6) seed table per join; returns the
    d x w_1 x .. x w_k int64 tensor."""
    lib = _load()
    k = len(keys_per_join)
    ks = [np.ascontiguousarray(np.asarray(x).astype(np.int64)) for x in keys_per_join]
    n = ks[0].size
    assert all(x.size == n for x in ks) and len(seeds_per_join) == k == len(widths)
    ss = [np.ascontiguousarray(np.asarray(x, dtype=np.uint64).reshape(d, 6))
          for x in seeds_per_join]
    w = np.ascontiguousarray(np.asarray(widths, dtype=np.int64))
    out = np.zeros((d,) + tuple(int(x) for x in widths), dtype=np.int64)
    kp = (ctypes.POINTER(ctypes.c_int64) * k)(*[_ptr(x, ctypes.c_int64) for x in ks])
    sp = (ctypes.POINTER(ctypes.c_uint64) * k)(*[_ptr(x, ctypes.c_uint64) for x in ss])
    lib.oracle_sketch_kd(kp, k, int(n), sp, int(d), _ptr(w, ctypes.c_int64),
                         _ptr(out, ctypes.c_int64))
    return out


def tensor_join(n_tables, edge_u, edge_v, d, widths, tensors, n_sel):
    """Estimate of a join graph from partitioned sketches (Section 5.1):
    tensors[t] is table t's d x (widths of its edges, in increasing edge
    id) sketch; the literal sum over every bucket assignment of the edges.
    Returns (row values as python ints mod 2^128, median, exactness flag)."""
    lib = _load()
    ne = len(edge_u)
    eu = np.ascontiguousarray(np.asarray(edge_u, dtype=np.int32))
    ev = np.ascontiguousarray(np.asarray(edge_v, dtype=np.int32))
    w = np.ascontiguousarray(np.asarray(widths, dtype=np.int64))
    ts = [np.ascontiguousarray(np.asarray(x, dtype=np.int64)) for x in tensors]
    tp = (ctypes.POINTER(ctypes.c_int64) * n_tables)(*[_ptr(x, ctypes.c_int64) for x in ts])
    ns = np.ascontiguousarray(np.asarray(n_sel, dtype=np.int64))
    rows = np.zeros((d, 2), dtype=np.uint64)
    est = ctypes.c_double()
    flag = ctypes.c_int32()
    lib.oracle_tensor_join(int(n_tables), int(ne), _ptr(eu, ctypes.c_int32),
                           _ptr(ev, ctypes.c_int32), int(d), _ptr(w, ctypes.c_int64),
                           tp, _ptr(ns, ctypes.c_int64), _ptr(rows, ctypes.c_uint64),
                           ctypes.byref(est), ctypes.byref(flag))
    vals = [int(rows[i, 0]) | (int(rows[i, 1]) << 64) for i in range(d)]
    return vals, est.value, flag.value


def agms_sketch(keys_per_join, seeds_per_join, r: int, b: int) -> np.ndarray:
    """AGMS sketch (Section 4.1) of one table's (already filtered) tuples:
    ``keys_per_join`` one key array per join of the table, ``seeds_per_join``
    one (r * b, 6) seed array per join; returns r x b int64 counters."""
    lib = _load()
    K = r * b
    ks = [np.ascontiguousarray(np.asarray(k).astype(np.int64)) for k in keys_per_join]
    n = ks[0].size
    assert all(k.size == n for k in ks)
    arr = (ctypes.POINTER(ctypes.c_int64) * len(ks))(*[_ptr(k, ctypes.c_int64) for k in ks])
    sd = np.ascontiguousarray(np.stack([np.asarray(s, dtype=np.uint64).reshape(K, 6)
                                        for s in seeds_per_join]))
    out = np.zeros(K, dtype=np.int64)
    lib.oracle_agms_sketch(arr, int(n), _ptr(sd, ctypes.c_uint64), len(ks), K,
                           _ptr(out, ctypes.c_int64))
    return out.reshape(r, b)


def agms_estimate(sketches, n_sel):
    """AGMS estimate from the tables' (r, b) sketches: (row sums as python
    ints, estimate, exactness flag)."""
    lib = _load()
    sks = [np.ascontiguousarray(np.asarray(s, dtype=np.int64)) for s in sketches]
    r, b = sks[0].shape
    arr = (ctypes.POINTER(ctypes.c_int64) * len(sks))(*[_ptr(s, ctypes.c_int64) for s in sks])
    ns = np.ascontiguousarray(np.asarray(n_sel, dtype=np.int64))
    rows = np.zeros((r, 2), dtype=np.uint64)
    est = ctypes.c_double()
    flag = ctypes.c_int32()
    lib.oracle_agms_estimate(arr, len(sks), int(r), int(b), _ptr(ns, ctypes.c_int64),
                             _ptr(rows, ctypes.c_uint64), ctypes.byref(est),
                             ctypes.byref(flag))
    return [i128_to_int(rows[i, 0], rows[i, 1]) for i in range(r)], est.value, flag.value


def build_table_sketches(table, edge_cols, seeds_per_edge, d, w):
    """Selection push-down + one sketch per incident join attribute.

    ``edge_cols``: list of key-column names, one per incident edge;
    ``seeds_per_edge``: matching list of (d, 6) seed arrays.
    Returns (n_selected, [counters...]).
    """
    mask = eval_predicates(table.cols, table.preds)
    sk = [sketch(table.cols[c][mask], s, d, w)
          for c, s in zip(edge_cols, seeds_per_edge)]
    return int(mask.sum()), sk


# --------------------------------------------------------------------------
# Estimates
# --------------------------------------------------------------------------
def i128_to_int(lo: int, hi: int) -> int:
    v = (int(hi) << 64) | int(lo)
    return v - (1 << 128) if v >> 127 else v


def set_threads(n: int | None = None) -> None:
    """Threads of the oracle's OpenMP loops (None: ``default_threads()``)."""
    _load().oracle_set_threads(default_threads() if n is None else int(n))


def estimate(n_tables, edge_u, edge_v, d, w, sketches, n_sel, masks,
             method: str = "fast"):
    """Row estimates (python ints), medians (float) and flags per sub-plan.

    ``sketches[2*e + side]`` is the (d, w) counter array of edge e on the
    side of edge_u[e] (side 0) or edge_v[e] (side 1).
    """
    lib = _load()
    ne = len(edge_u)
    eu = np.ascontiguousarray(np.asarray(edge_u, dtype=np.int32))
    ev = np.ascontiguousarray(np.asarray(edge_v, dtype=np.int32))
    sks = [np.ascontiguousarray(np.asarray(s, dtype=np.int64).reshape(d, w))
           for s in sketches]
    arr = (ctypes.POINTER(ctypes.c_int64) * max(1, 2 * ne))(
        *[_ptr(s, ctypes.c_int64) for s in sks])
    ns = np.ascontiguousarray(np.asarray(n_sel, dtype=np.int64))
    ms = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    nm = ms.size
    rows = np.zeros((nm, d, 2), dtype=np.uint64)
    est = np.zeros(nm, dtype=np.float64)
    flags = np.zeros(nm, dtype=np.int32)
    rc = lib.oracle_estimate(int(n_tables), int(ne), _ptr(eu, ctypes.c_int32),
                             _ptr(ev, ctypes.c_int32), int(d), int(w), arr,
                             _ptr(ns, ctypes.c_int64), _ptr(ms, ctypes.c_uint64),
                             int(nm), 0 if method == "literal" else 1,
                             _ptr(rows, ctypes.c_uint64),
                             _ptr(est, ctypes.c_double),
                             _ptr(flags, ctypes.c_int32))
    if rc != 0:
        raise ValueError("sub-plan empty or not connected")
    vals = [[i128_to_int(rows[m, i, 0], rows[m, i, 1]) for i in range(d)]
            for m in range(nm)]
    return vals, est, flags


def row_values_exact(n_tables, edge_u, edge_v, d, w, sketches, mask):
    """The sub-plan's row values X_0..X_{d-1} as unbounded Python integers
    (no wrap modulo 2^128): the same definition as ``estimate`` (Section 5.1
    contraction with the Section 5.2 min-abs merge), evaluated by
    conditioning on the buckets of the edges outside a spanning tree and
    passing messages up the tree.  For one node, with its elements (parent
    buckets as queries, child buckets weighted by the children's messages,
    conditioned buckets weighted 1) ordered by kappa = (|value|, edge id,
    bucket), the message for a query q is
        value(q) * prod_groups W_g(above q) + sum over weighted elements z
        below q of value(z) * weight(z) * prod_{g != group(z)} W_g(above z),
    W_g(above k) = total weight of group g's elements ordered after k.
    For sizes where the exact value exceeds 128 bits (uncertified
    sub-plans).  ``sketches[2e + side]``: (d, w) integer arrays."""
    tabs = [t for t in range(n_tables) if mask >> t & 1]
    edges = [e for e in range(len(edge_u))
             if mask >> edge_u[e] & 1 and mask >> edge_v[e] & 1]
    if len(tabs) == 1:
        raise ValueError("single table: the selected count, not a contraction")

    def side(t, e):
        return 2 * e + (0 if edge_u[e] == t else 1)

    # spanning tree by breadth-first search from the lowest table
    parent = {tabs[0]: None}
    order = [tabs[0]]
    tree = set()
    for a in order:
        for e in edges:
            if a in (edge_u[e], edge_v[e]):
                b = edge_v[e] if edge_u[e] == a else edge_u[e]
                if b not in parent:
                    parent[b] = (a, e)
                    tree.add(e)
                    order.append(b)
    if len(order) != len(tabs):
        raise ValueError("not connected")
    cut = [e for e in edges if e not in tree]
    children = {t: [] for t in tabs}
    for b in order[1:]:
        children[parent[b][0]].append((b, parent[b][1]))
    out = []
    for i in range(d):
        sk = [np.asarray(sketches[k])[i].astype(object) if sketches[k] is not None
              else None for k in range(len(sketches))]
        total = 0
        for J in itertools.product(range(w), repeat=len(cut)):
            fixed = dict(zip(cut, J))
            msg = {}
            root_val = 0
            for t in reversed(order):
                elems = []   # (kappa, group, weight or None for queries, value, bucket)
                groups = []
                for (b, e) in children[t]:
                    g = len(groups)
                    groups.append(sum(msg[b]))
                    for j in range(w):
                        v = int(sk[side(t, e)][j])
                        elems.append(((abs(v), e, j), g, msg[b][j], v, j))
                for e, j in fixed.items():
                    if t in (edge_u[e], edge_v[e]):
                        g = len(groups)
                        groups.append(1)
                        v = int(sk[side(t, e)][j])
                        elems.append(((abs(v), e, j), g, 1, v, j))
                if parent[t] is not None:
                    pe = parent[t][1]
                    for j in range(w):
                        v = int(sk[side(t, pe)][j])
                        elems.append(((abs(v), pe, j), -1, None, v, j))
                elems.sort(key=lambda z: z[0])
                above = list(groups)   # W_g(above the current element)
                below = 0              # sum over weighted elements passed
                m = [0] * w
                for (_, g, wt, v, j) in elems:
                    if g < 0:
                        p = v
                        for x in above:
                            p *= x
                        m[j] = p + below
                    else:
                        above[g] -= wt
                        p = v * wt
                        for k, x in enumerate(above):
                            if k != g:
                                p *= x
                        below += p
                if parent[t] is None:
                    root_val = below
                else:
                    msg[t] = m
            total += root_val
        out.append(total)
    return out


def i128_to_double(v: int) -> float:
    """Round-to-nearest-even conversion of a signed 128-bit value (C libgcc)."""
    u = v & ((1 << 128) - 1)
    return _load().oracle_i128_to_double(u & ((1 << 64) - 1), u >> 64)


# --------------------------------------------------------------------------
# Sub-plan enumeration helpers
# --------------------------------------------------------------------------
def connected_subplans(n_tables, edge_u, edge_v, max_tables=None):
    """All connected table subsets (bitmasks), by size then value."""
    adj = [0] * n_tables
    for u, v in zip(edge_u, edge_v):
        adj[u] |= 1 << v
        adj[v] |= 1 << u
    out = []
    for m in range(1, 1 << n_tables):
        k = bin(m).count("1")
        if max_tables is not None and k > max_tables:
            continue
        low = m & -m
        seen = low
        while True:
            grow = seen
            t = 0
            s = seen
            while s:
                if s & 1:
                    grow |= adj[t] & m
                s >>= 1
                t += 1
            if grow == seen:
                break
            seen = grow
        if seen == m:
            out.append(m)
    out.sort(key=lambda m: (bin(m).count("1"), m))
    return out


# --------------------------------------------------------------------------
# Ground truth: exact join sizes
# --------------------------------------------------------------------------
def true_cardinality(filtered_cols, edges, mask) -> float:
    """Exact |join of the selected rows| for the tables in ``mask``.

    ``filtered_cols[t]`` maps column name -> array of the rows of table t
    that satisfy its selections; ``edges`` is a list of (u, ucol, v, vcol).
    Join attributes linked by the sub-plan's equality edges form classes
    (union-find); each table becomes a count table over its class values
    and classes are summed out one at a time (hash aggregation).  Counts
    are float64: exact up to 2^53, relative rounding 1e-16 beyond.
    """
    import pandas as pd

    tabs = [t for t in range(len(filtered_cols)) if mask >> t & 1]
    sub_edges = [e for e in edges if (mask >> e[0] & 1) and (mask >> e[2] & 1)]
    parent = {}

    def find(a):
        while parent.setdefault(a, a) != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for (u, uc, v, vc) in sub_edges:
        ra, rb = find((u, uc)), find((v, vc))
        if ra != rb:
            parent[ra] = rb
    classes = {}
    factors = []
    for t in tabs:
        attrs = sorted({a for a in parent if a[0] == t}, key=lambda a: a[1])
        cols = filtered_cols[t]
        n = len(next(iter(cols.values()))) if cols else 0
        if not attrs:
            factors.append(pd.DataFrame({"__c": [float(n)]}))
            continue
        by_class = {}
        for a in attrs:
            by_class.setdefault(find(a), []).append(a)
        keep = np.ones(n, dtype=bool)
        data = {}
        for cls, al in by_class.items():
            name = classes.setdefault(cls, "v%d" % len(classes))
            base = np.asarray(cols[al[0][1]]).astype(np.int64)
            for a in al[1:]:
                keep &= base == np.asarray(cols[a[1]]).astype(np.int64)
            data[name] = base
        df = pd.DataFrame({k: v[keep] for k, v in data.items()})
        f = df.groupby(list(df.columns), sort=False).size().astype(np.float64)
        f = f.rename("__c").reset_index()
        factors.append(f)
    # sum out class variables one at a time (fewest factors first)
    while True:
        vars_left = sorted({c for f in factors for c in f.columns if c != "__c"})
        if not vars_left:
            break
        var = min(vars_left, key=lambda x: (sum(x in f.columns for f in factors),
                                            x))
        inv = [f for f in factors if var in f.columns]
        rest = [f for f in factors if var not in f.columns]
        acc = inv[0]
        for f in inv[1:]:
            on = [c for c in acc.columns if c in f.columns and c != "__c"]
            acc = acc.merge(f, on=on, suffixes=("", "_r"))
            acc["__c"] = acc["__c"] * acc["__c_r"]
            acc = acc.drop(columns=["__c_r"])
        keep_vars = [c for c in acc.columns if c not in ("__c", var)]
        if keep_vars:
            acc = acc.groupby(keep_vars, sort=False)["__c"].sum().reset_index()
        else:
            acc = pd.DataFrame({"__c": [float(acc["__c"].sum())]})
        factors = rest + [acc]
    total = 1.0
    for f in factors:
        total *= float(f["__c"].sum())
    return total


# --------------------------------------------------------------------------
# Accuracy measures
# --------------------------------------------------------------------------
def qerror(est, true) -> np.ndarray:
    """max(e/t, t/e) with both clamped below at 1 (estimates can be <= 0)."""
    e = np.maximum(np.asarray(est, dtype=np.float64), 1.0)
    t = np.maximum(np.asarray(true, dtype=np.float64), 1.0)
    return np.maximum(e / t, t / e)


def ratio(est, true) -> np.ndarray:
    """estimate / true, the accuracy ratio of Section 5.2."""
    return np.asarray(est, dtype=np.float64) / np.maximum(
        np.asarray(true, dtype=np.float64), 1.0)


def l1_permutation_distance(est, true) -> int:
    """Section 5.2: sum over sub-plans of |position by estimate - position by
    true cardinality|, both orders ascending (ties by input order)."""
    est = list(est)
    true = list(true)
    by_true = sorted(range(len(true)), key=lambda i: (true[i], i))
    by_est = sorted(range(len(est)), key=lambda i: (est[i], i))
    pos_t = {s: p for p, s in enumerate(by_true)}
    pos_e = {s: p for p, s in enumerate(by_est)}
    return sum(abs(pos_e[s] - pos_t[s]) for s in range(len(est)))


# --------------------------------------------------------------------------
# Learned correction network (not in the paper; spec addition).
# Layers in -> 64 -> 64 -> 64 -> 1 with ReLU.  Every layer's input
# activations and weights are rounded to bfloat16 (round to nearest even)
# as a bfloat16 matrix product would see them; products and sums are exact
# here (float64).  Output = base + network(x), base = ln(1 + max(raw, 0)),
# so a zero network returns the raw sketch estimate.  Loss = mean squared
# error against ln(1 + true).  Gradients treat the roundings as identity
# (straight-through).  Parameter layout, per layer: W (out x in, row-major)
# then b (out).
# --------------------------------------------------------------------------
MLP_DIMS = (20, 64, 64, 64, 1)


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_unpack(params, dims=MLP_DIMS):
    p = np.asarray(params, dtype=np.float64)
    out, k = [], 0
    for i in range(len(dims) - 1):
        n_in, n_out = dims[i], dims[i + 1]
        W = p[k:k + n_in * n_out].reshape(n_out, n_in)
        k += n_in * n_out
        b = p[k:k + n_out]
        k += n_out
        out.append((W, b))
    assert k == p.size
    return out


def mlp_n_params(dims=MLP_DIMS) -> int:
    return sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1))


def mlp_forward(params, x, base, dims=MLP_DIMS, rounding=True):
    """Returns (prediction, cache for the backward pass)."""
    rnd = bf16_round if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    layers = mlp_unpack(params, dims)
    a = np.asarray(x, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        ar = rnd(a)
        Wr = rnd(W)
        z = ar @ Wr.T + b
        cache.append((ar, Wr, z))
        a = np.maximum(z, 0.0) if li < len(layers) - 1 else z
    y = np.asarray(base, dtype=np.float64) + a[:, 0]
    return y, cache


def mlp_loss_grad(params, x, base, target, dims=MLP_DIMS, rounding=True):
    """(loss, gradient w.r.t. params) of mean((y - target)^2)."""
    y, cache = mlp_forward(params, x, base, dims, rounding)
    t = np.asarray(target, dtype=np.float64)
    n = y.size
    loss = float(np.mean((y - t) ** 2))
    dz = (2.0 * (y - t) / n)[:, None]
    grads = []
    for li in range(len(cache) - 1, -1, -1):
        ar, Wr, z = cache[li]
        if li < len(cache) - 1:
            dz = dz * (z > 0)
        dW = dz.T @ ar
        db = dz.sum(axis=0)
        grads.append((dW, db))
        dz = dz @ Wr
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.reshape(-1))
        flat.append(db)
    return loss, np.concatenate(flat)


def adam_step(params, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected; returns new p, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def mlp_init(seed: int, dims=MLP_DIMS) -> np.ndarray:
    """He-uniform weights, zero biases, and a zero output layer (so the
    untrained network returns the raw estimate)."""
    rng = np.random.default_rng(seed)
    flat = []
    for i in range(len(dims) - 1):
        n_in, n_out = dims[i], dims[i + 1]
        lim = np.sqrt(6.0 / n_in)
        W = rng.uniform(-lim, lim, size=(n_out, n_in))
        if i == len(dims) - 2:
            W[:] = 0.0
        flat.append(W.reshape(-1))
        flat.append(np.zeros(n_out))
    return np.concatenate(flat)


def plan_greedy(n_tables, edge_u, edge_v, est_of, card):
    """The greedy search of Section 7.2.8 (the default of Section 7.1):
    start from the smaller table (by card; ties to the lower id) of the
    two-way join with the smallest estimate (ties to the lower mask), then
    repeatedly append the not-yet-joined table adjacent to the order whose
    extended sub-plan has the smallest estimate (ties to the lower id).
    Returns (order, cost) with cost = sum of the estimates of every prefix."""
    adj = [set() for _ in range(n_tables)]
    for u, v in zip(edge_u, edge_v):
        adj[u].add(v)
        adj[v].add(u)
    if n_tables == 1:
        return [0], est_of[1]
    pairs = sorted({(min(u, v), max(u, v)) for u, v in zip(edge_u, edge_v)})
    best = min(pairs, key=lambda p: (est_of[(1 << p[0]) | (1 << p[1])],
                                     (1 << p[0]) | (1 << p[1])))
    u, v = best
    order = [v] if card[v] < card[u] else [u]
    mask = 1 << order[0]
    cost = est_of[mask]
    while len(order) < n_tables:
        cand = sorted({b for a in order for b in adj[a]} - set(order))
        nxt = min(cand, key=lambda x: (est_of[mask | (1 << x)], x))
        order.append(nxt)
        mask |= 1 << nxt
        cost += est_of[mask]
    return order, cost


def plan_cost(order, value_of):
    """Cost of a left-deep order under any cardinality map: the sum over
    its prefixes (one table, two, ..., all) of value_of[prefix mask].  With
    exact join sizes this is the plan's true cost (the sum of its
    intermediate result sizes, Section 2)."""
    m, c = 0, 0.0
    for v in order:
        m |= 1 << v
        c += float(value_of[m])
    return c


def true_cardinality_fk_tree(filtered_cols, edges, mask, domain_of):
    """Exact join size of a tree-shaped sub-plan whose every edge joins a
    foreign-key column to a dense primary key "id" in [0, domain) (the
    batched/learned workloads).  Message passing toward the lowest table:
    a child's message is the per-key count of its joining tuples, each
    weighted by the product of the messages into it (numpy bincount).
    Counts are float64 (exact to 2^53).  ``domain_of[t]`` = size of table
    t's id domain.  Pinned against the hash-aggregation oracle."""
    tabs = [t for t in range(len(filtered_cols)) if mask >> t & 1]
    sub = [e for e in edges if (mask >> e[0] & 1) and (mask >> e[2] & 1)]
    if len(sub) != len(tabs) - 1:
        raise ValueError("not a tree")
    adj = {t: [] for t in tabs}
    for e in sub:
        adj[e[0]].append(e)
        adj[e[2]].append(e)
    root = tabs[0]
    order, parent_edge = [root], {root: None}
    for a in order:
        for e in adj[a]:
            b = e[2] if e[0] == a else e[0]
            if b not in parent_edge:
                parent_edge[b] = e
                order.append(b)
    weight = {t: np.ones(len(filtered_cols[t]["id"]), dtype=np.float64)
              for t in tabs}
    for b in reversed(order[1:]):
        e = parent_edge[b]
        a = e[2] if e[0] == b else e[0]
        bcol = e[1] if e[0] == b else e[3]
        acol = e[3] if e[0] == b else e[1]
        # b's tuples grouped by their join key, weighted; looked up by a
        bkey = np.asarray(filtered_cols[b][bcol], dtype=np.int64)
        akey = np.asarray(filtered_cols[a][acol], dtype=np.int64)
        dom = int(max(domain_of[b] if bcol == "id" else 0,
                      domain_of[a] if acol == "id" else 0,
                      (bkey.max() + 1) if bkey.size else 0,
                      (akey.max() + 1) if akey.size else 0))
        msg = np.bincount(bkey, weights=weight[b], minlength=dom)
        weight[a] = weight[a] * msg[akey]
    return float(weight[root].sum())


def shape_stats(n_tables, edge_u, edge_v, masks):
    """Shape of each sub-plan over the query's join graph, the learned
    model's last 5 features: number of tables, number of join edges between
    them, diameter (largest over table pairs of the fewest edges on a path
    inside the sub-plan), largest number of edges at one table, and
    independent cycles (edges - tables + 1 for a connected sub-plan).
    Returns an n x 5 float64 array."""
    out = np.zeros((len(masks), 5))
    for k, m in enumerate(masks):
        m = int(m)
        tabs = [t for t in range(n_tables) if m >> t & 1]
        es = [(u, v) for u, v in zip(edge_u, edge_v) if m >> u & 1 and m >> v & 1]
        # all-pairs fewest edges (Floyd-Warshall over the sub-plan)
        inf = float("inf")
        dist = {(a, b): (0 if a == b else inf) for a in tabs for b in tabs}
        for u, v in es:
            dist[(u, v)] = dist[(v, u)] = 1
        for c in tabs:
            for a in tabs:
                for b in tabs:
                    if dist[(a, c)] + dist[(c, b)] < dist[(a, b)]:
                        dist[(a, b)] = dist[(a, c)] + dist[(c, b)]
        deg = [sum((u == t) + (v == t) for u, v in es) for t in tabs]
        out[k] = (len(tabs), len(es), max(dist.values()), max(deg), len(es) - len(tabs) + 1)
    return out


def mlp_features(rows, est, n_sel_sub, shape):
    """Reference of the learned model's 20 features of one sub-plan (same
    definition as compass_mlp_features): 7 order statistics (positions
    round(k (d-1) / 6)) of sign(X) ln(1 + |X|) over the sorted exact row
    values; log2(1 + n_sel) of the sub-plan's tables, descending, first 8,
    zero padded; 5 shape statistics; base = ln(1 + max(est, 0))."""
    d = len(rows)
    v = sorted(i128_to_double(r) for r in rows)
    x = []
    for k in range(7):
        r = v[(k * (d - 1) + 3) // 6]
        x.append(-np.log1p(-r) if r < 0 else np.log1p(r))
    ls = sorted((np.log2(1.0 + n) for n in n_sel_sub), reverse=True)[:8]
    x += ls + [0.0] * (8 - len(ls))
    x += list(shape)
    return np.array(x, dtype=np.float64), float(np.log1p(max(est, 0.0)))


# --------------------------------------------------------------------------
# Plan enumeration (Section 6, Algorithm 1): DFS over the join graph that
# builds left-deep orders without cross products, sources ordered by
# f(v) = alpha card(v)/max card + beta deg(v)/max deg, children visited in
# increasing order of the estimate of the extended sub-plan, pruning when
# the running cost exceeds the best complete cost, at most max_plans
# complete plans per source.  cost = sum of the estimates of every prefix
# (the single table, each intermediate join and the full join).
# --------------------------------------------------------------------------
def plan_enumeration(n_tables, edge_u, edge_v, est_of, card, max_plans,
                     alpha=0.5, beta=0.5):
    """Returns (best order, best cost, complete plans reached)."""
    deg = [0] * n_tables
    adj = [set() for _ in range(n_tables)]
    for u, v in zip(edge_u, edge_v):
        deg[u] += 1
        deg[v] += 1
        adj[u].add(v)
        adj[v].add(u)
    mc = max(card) if max(card) > 0 else 1
    md = max(deg) if max(deg) > 0 else 1
    f = [alpha * card[v] / mc + beta * deg[v] / md for v in range(n_tables)]
    sources = sorted(range(n_tables), key=lambda v: (f[v], v))
    best = {"cost": float("inf"), "order": None}
    total = [0]

    class Abort(Exception):
        pass

    def dfs(order, mask, cost, p):
        cost = cost + est_of[mask]
        if cost > best["cost"]:
            return
        if len(order) == n_tables:
            if cost < best["cost"]:
                best["cost"] = cost
                best["order"] = list(order)
            p[0] += 1
            total[0] += 1
            if p[0] == max_plans:
                raise Abort()
            return
        cand = sorted({b for a in order for b in adj[a]} - set(order))
        ext = sorted(cand, key=lambda v: (est_of[mask | (1 << v)], v))
        for v in ext:
            dfs(order + [v], mask | (1 << v), cost, p)

    for s in sources:
        try:
            dfs([s], 1 << s, 0.0, [0])
        except Abort:
            pass
    return best["order"], best["cost"], total[0]
