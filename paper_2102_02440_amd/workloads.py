"""Seeded synthetic workloads shaped like the paper's queries.

This module only draws inputs: table columns, selection predicates, join
graphs and the random hash seeds the sketches consume.  It holds none of the
sketch or estimate arithmetic, so both the HIP path and the independent
oracle take their inputs from here.

Shapes follow the paper's running example, query 6a of the JOB benchmark
(Section 1: five tables, point / subset / range selections, five join
predicates with a triangle among title, movie_keyword and cast_info), with
synthetic data standing in for the IMDB tables: primary keys are dense ids,
foreign keys are Zipf-distributed ranks mapped through a seeded permutation
of the referenced key domain (so heavy hitters line up across tables that
reference the same domain, as foreign keys do).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

P61 = (1 << 61) - 1  # seeds are drawn uniformly from [0, 2^61 - 1)

DEFAULT_SEED = 20210202


@dataclass
class Predicate:
    col: str
    kind: str          # "point" | "range" | "subset"
    lo: float = 0      # point constant or range low bound (inclusive)
    hi: float = 0      # range high bound (inclusive)
    bitmap: np.ndarray | None = None   # subset: uint64 words over [0, domain)
    domain: int = 0


@dataclass
class Table:
    name: str
    cols: dict
    preds: list = field(default_factory=list)

    @property
    def n_rows(self) -> int:
        return len(next(iter(self.cols.values())))


@dataclass
class Edge:
    u: int
    ucol: str
    v: int
    vcol: str


@dataclass
class Query:
    tables: list
    edges: list
    d: int
    w: int
    seeds: np.ndarray        # (n_edges, d, 6) uint64: a0 a1 a2 a3 b0 b1
    counter_bits: int = 32

    @property
    def edge_u(self):
        return [e.u for e in self.edges]

    @property
    def edge_v(self):
        return [e.v for e in self.edges]

    def incident(self, t):
        """[(edge id, side, key column)] of table t in edge-id order."""
        out = []
        for i, e in enumerate(self.edges):
            if e.u == t:
                out.append((i, 0, e.ucol))
            elif e.v == t:
                out.append((i, 1, e.vcol))
        return out


def rng_of(seed: int, *stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [int(seed)] + [int(s) for s in stream])))


def draw_seeds(rng: np.random.Generator, n_edges: int, d: int) -> np.ndarray:
    """Independent hash seeds per (edge, row): six values in [0, 2^61-1)."""
    return rng.integers(0, P61, size=(n_edges, d, 6), dtype=np.uint64)


class Zipf:
    """Zipf(s) ranks over [0, n): P(rank k) proportional to (k+1)^-s.

    A sample of ``size`` draws is taken as multinomial counts per rank,
    expanded and shuffled (the same distribution as ``size`` independent
    draws, at a fraction of the cost of inverse-CDF search)."""

    def __init__(self, n: int, s: float):
        w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
        self.p = w / w.sum()
        self.n = n

    def sample(self, rng: np.random.Generator, size: int) -> np.ndarray:
        counts = rng.multinomial(size, self.p)
        ranks = np.repeat(np.arange(self.n, dtype=np.int64), counts)
        rng.shuffle(ranks)
        return ranks


def fk_column(rng, size, domain, s, perm, dtype=np.int32):
    ranks = Zipf(domain, s).sample(rng, size)
    return perm[ranks].astype(dtype)


def subset_bitmap(codes: np.ndarray, domain: int) -> np.ndarray:
    words = np.zeros((domain + 63) // 64, dtype=np.uint64)
    codes = np.asarray(codes, dtype=np.int64)
    np.bitwise_or.at(words, codes >> 6,
                     np.left_shift(np.uint64(1), (codes & 63).astype(np.uint64)))
    return words


# --------------------------------------------------------------------------
# Star join for partitioned sketches (Section 5.1): a fact table of 36M rows
# with three foreign keys (Zipf 1.0 over 2.5M movies, 0.8 over 4.2M people,
# 1.1 over 200k companies) and three dimension tables keyed by id, each with
# one predicate (year range ~10%, subset 20%, country range 30%).  Edges: fact-t
# (0), fact-n (1), fact-cn (2); table order [fact, t, n, cn].
# --------------------------------------------------------------------------
def star3(seed: int = DEFAULT_SEED, scale: float = 1.0, d: int = 5,
          w: int = 128) -> Query:
    rng = rng_of(seed, 30)

    def sz(n):
        return max(8, int(round(n * scale)))

    n_f, n_t, n_n, n_c = sz(36_000_000), sz(2_500_000), sz(4_200_000), sz(200_000)
    perm_t = rng.permutation(n_t).astype(np.int64)
    perm_n = rng.permutation(n_n).astype(np.int64)
    perm_c = rng.permutation(n_c).astype(np.int64)
    fact = Table("f", {"movie": fk_column(rng, n_f, n_t, 1.0, perm_t),
                       "person": fk_column(rng, n_f, n_n, 0.8, perm_n),
                       "company": fk_column(rng, n_f, n_c, 1.1, perm_c)})
    t = Table("t", {"id": np.arange(n_t, dtype=np.int32),
                    "year": rng.integers(1900, 2020, size=n_t,
                                         dtype=np.int64).astype(np.int32)},
              [Predicate("year", "range", 2008, 2019)])
    chosen = rng.choice(n_n, size=max(1, n_n // 5), replace=False)
    n = Table("n", {"id": np.arange(n_n, dtype=np.int32),
                    "name_code": np.arange(n_n, dtype=np.int32)},
              [Predicate("name_code", "subset", bitmap=subset_bitmap(chosen, n_n),
                         domain=n_n)])
    cn = Table("cn", {"id": np.arange(n_c, dtype=np.int32),
                      "country": rng.integers(0, 100, size=n_c,
                                              dtype=np.int64).astype(np.int32)},
               [Predicate("country", "range", 0, 29)])
    edges = [Edge(0, "movie", 1, "id"), Edge(0, "person", 2, "id"),
             Edge(0, "company", 3, "id")]
    seeds = draw_seeds(rng_of(seed, 31), len(edges), d)
    return Query([fact, t, n, cn], edges, d, w, seeds, 32)


# --------------------------------------------------------------------------
# Plain two-table equi-join: R 1M rows (range predicate, 10%), S 100k rows,
# Zipf(1.0) keys over a 100k domain; d=5, w=1024, int32 counters.
# --------------------------------------------------------------------------
def two_table(seed: int = DEFAULT_SEED, n_r: int = 1_000_000,
              n_s: int = 100_000, domain: int = 100_000, zipf_s: float = 1.0,
              d: int = 5, w: int = 1024, counter_bits: int = 32) -> Query:
    rng = rng_of(seed, 1)
    perm = rng.permutation(domain).astype(np.int64)
    r_key = fk_column(rng, n_r, domain, zipf_s, perm)
    r_a = rng.integers(0, 1_000_000, size=n_r, dtype=np.int64).astype(np.int32)
    s_key = fk_column(rng, n_s, domain, zipf_s, perm)
    # selectivity 10%: a in [0, 99999] of a uniform [0, 1e6)
    R = Table("R", {"key": r_key, "a": r_a},
              [Predicate("a", "range", 0, 99_999)])
    S = Table("S", {"key": s_key})
    seeds = draw_seeds(rng_of(seed, 2), 1, d)
    return Query([R, S], [Edge(0, "key", 1, "key")], d, w, seeds, counter_bits)


# --------------------------------------------------------------------------
# Five tables shaped like JOB 6a (Section 1): k, mk, t, ci, n.
#   e0 k.id = mk.keyword   e1 t.id = mk.movie   e2 t.id = ci.movie
#   e3 ci.movie = mk.movie e4 n.id = ci.person
# Point predicate on k (1%), range on t (10%), subset on n (0.5%).
# Full size: ci 36M, mk 4.5M, t 2.5M, n 4.2M, k 134k rows; d=7, w=8192.
# ``scale`` shrinks every table (and key domain) for oracle-sized tests.
# --------------------------------------------------------------------------
JOB6A_TABLES = ["k", "mk", "t", "ci", "n"]


def job6a(seed: int = DEFAULT_SEED, scale: float = 1.0, d: int = 7,
          w: int = 8192, counter_bits: int = 32) -> Query:
    rng = rng_of(seed, 10)

    def sz(n):
        return max(8, int(round(n * scale)))

    n_k, n_mk, n_t, n_ci, n_n = (sz(134_000), sz(4_500_000), sz(2_500_000),
                                 sz(36_000_000), sz(4_200_000))
    perm_t = rng.permutation(n_t).astype(np.int64)
    perm_n = rng.permutation(n_n).astype(np.int64)
    perm_k = rng.permutation(n_k).astype(np.int64)
    k = Table("k", {"id": np.arange(n_k, dtype=np.int32),
                    "kw_code": rng.integers(0, 100, size=n_k,
                                            dtype=np.int64).astype(np.int32)},
              [Predicate("kw_code", "point", 7)])
    mk = Table("mk", {"keyword": fk_column(rng, n_mk, n_k, 1.2, perm_k),
                      "movie": fk_column(rng, n_mk, n_t, 1.0, perm_t)})
    t = Table("t", {"id": np.arange(n_t, dtype=np.int32),
                    "year": rng.integers(1900, 2020, size=n_t,
                                         dtype=np.int64).astype(np.int32)},
              [Predicate("year", "range", 2008, 2019)])
    ci = Table("ci", {"movie": fk_column(rng, n_ci, n_t, 1.0, perm_t),
                      "person": fk_column(rng, n_ci, n_n, 0.8, perm_n)})
    name_code = rng.permutation(n_n).astype(np.int32)
    chosen = rng.choice(n_n, size=max(1, n_n // 200), replace=False)
    n = Table("n", {"id": np.arange(n_n, dtype=np.int32), "name_code": name_code},
              [Predicate("name_code", "subset", bitmap=subset_bitmap(chosen, n_n),
                         domain=n_n)])
    edges = [Edge(0, "id", 1, "keyword"), Edge(2, "id", 1, "movie"),
             Edge(2, "id", 3, "movie"), Edge(3, "movie", 1, "movie"),
             Edge(4, "id", 3, "person")]
    seeds = draw_seeds(rng_of(seed, 11), len(edges), d)
    return Query([k, mk, t, ci, n], edges, d, w, seeds, counter_bits)


def small_random_query(rng: np.random.Generator, n_tables: int, n_rows: int,
                       domain: int, d: int, w: int, cyclic: bool = False,
                       pred_prob: float = 0.6) -> Query:
    """A small random connected join graph for parity tests: a random tree
    over ``n_tables`` tables plus, optionally, one extra edge closing a
    triangle.  Every table gets one or two int32 key columns, an int32 and
    a float32 attribute, and random predicates of all three kinds."""
    tables = []
    for t in range(n_tables):
        cols = {
            "k0": rng.integers(0, domain, size=n_rows).astype(np.int32),
            "k1": rng.integers(0, domain, size=n_rows).astype(np.int32),
            "a": rng.integers(0, 1000, size=n_rows).astype(np.int32),
            "f": rng.random(n_rows).astype(np.float32),
        }
        preds = []
        if rng.random() < pred_prob:
            kind = ["point", "range", "subset", "frange"][rng.integers(0, 4)]
            if kind == "point":
                preds.append(Predicate("a", "point", int(rng.integers(0, 10))))
                cols["a"] = (cols["a"] % 10).astype(np.int32)
            elif kind == "range":
                lo = int(rng.integers(0, 500))
                preds.append(Predicate("a", "range", lo, lo + int(rng.integers(0, 500))))
            elif kind == "subset":
                chosen = rng.choice(1000, size=int(rng.integers(1, 400)), replace=False)
                preds.append(Predicate("a", "subset", bitmap=subset_bitmap(chosen, 1000),
                                       domain=1000))
            else:
                lo = float(rng.random() * 0.5)
                preds.append(Predicate("f", "range", lo, lo + 0.4))
        tables.append(Table("t%d" % t, cols, preds))
    edges = []
    for t in range(1, n_tables):
        p = int(rng.integers(0, t))
        edges.append(Edge(p, "k%d" % int(rng.integers(0, 2)), t,
                          "k%d" % int(rng.integers(0, 2))))
    if cyclic and n_tables >= 3:
        # close a triangle: pick a node with a parent and grandparent or
        # a node with two tree neighbours
        adj = {t: set() for t in range(n_tables)}
        for e in edges:
            adj[e.u].add(e.v)
            adj[e.v].add(e.u)
        for mid in range(n_tables):
            nb = sorted(adj[mid])
            if len(nb) >= 2:
                a, b = nb[0], nb[1]
                edges.append(Edge(a, "k%d" % int(rng.integers(0, 2)), b,
                                  "k%d" % int(rng.integers(0, 2))))
                break
    seeds = draw_seeds(rng, len(edges), d)
    return Query(tables, edges, d, w, seeds, 32)


# --------------------------------------------------------------------------
# Batched workload: a pool of tables with primary keys and Zipf foreign keys,
# and many queries over it, each with its own selections, sketch shape
# (d, w) and hash seeds.  Shapes follow the 6a recipe above; table sizes are
# log-uniform, so filtered sizes are very uneven across the batch.
# --------------------------------------------------------------------------
@dataclass
class PoolTable:
    name: str
    cols: dict
    fks: list          # [(column, referenced pool table)]

    @property
    def n_rows(self) -> int:
        return len(self.cols["id"])


def schema_pool(seed: int = DEFAULT_SEED, n_tables: int = 48,
                size_range=(10_000, 36_000_000), scale: float = 1.0,
                fk_range=(2, 3)):
    rng = rng_of(seed, 30)
    lo, hi = np.log(size_range[0]), np.log(size_range[1])
    sizes = [max(64, int(np.exp(rng.uniform(lo, hi)) * scale))
             for _ in range(n_tables)]
    perms = [None] * n_tables
    pool = []
    for t in range(n_tables):
        n = sizes[t]
        cols = {"id": np.arange(n, dtype=np.int32),
                "a_uni": rng.integers(0, 1_000_000, size=n, dtype=np.int64).astype(np.int32),
                "a_cat": rng.integers(0, 1000, size=n, dtype=np.int64).astype(np.int32),
                "a_f": rng.random(n, dtype=np.float32)}
        fks = []
        for k in range(int(rng.integers(fk_range[0], fk_range[1] + 1))):
            ref = int(rng.integers(0, n_tables - 1))
            ref = ref if ref < t else ref + 1
            if perms[ref] is None:
                perms[ref] = rng_of(seed, 31, ref).permutation(sizes[ref]).astype(np.int64)
            s = float(rng.uniform(0.8, 1.2))
            cols["fk%d" % k] = fk_column(rng, n, sizes[ref], s, perms[ref])
            fks.append(("fk%d" % k, ref))
        pool.append(PoolTable("p%d" % t, cols, fks))
    return pool


@dataclass
class PoolQuery:
    tables: list       # pool table indices (query-local order)
    edges: list        # Edge over query-local indices
    preds: list        # per query-local table: list of Predicate
    d: int
    w: int
    seeds: np.ndarray  # (n_edges, d, 6)

    def incident(self, t):
        out = []
        for i, e in enumerate(self.edges):
            if e.u == t:
                out.append((i, 0, e.ucol))
            elif e.v == t:
                out.append((i, 1, e.vcol))
        return out


def random_predicates(rng, pred_prob=0.7):
    """None, or one selection of selectivity log-uniform in [0.1%, 20%]."""
    if rng.random() >= pred_prob:
        return []
    sel = float(np.exp(rng.uniform(np.log(0.001), np.log(0.2))))
    kind = ["range", "subset", "point", "frange"][int(rng.integers(0, 4))]
    if kind == "range":
        width = max(1, int(sel * 1_000_000))
        lo = int(rng.integers(0, 1_000_000 - width + 1))
        return [Predicate("a_uni", "range", lo, lo + width - 1)]
    if kind == "subset":
        k = max(1, int(round(sel * 1000)))
        codes = rng.choice(1000, size=k, replace=False)
        return [Predicate("a_cat", "subset", bitmap=subset_bitmap(codes, 1000),
                          domain=1000)]
    if kind == "point":
        return [Predicate("a_cat", "point", int(rng.integers(0, 1000)))]
    lo = float(rng.random() * (1.0 - sel))
    return [Predicate("a_f", "range", lo, lo + sel)]


def query_batch(pool, seed: int = DEFAULT_SEED, n_queries: int = 512,
                max_tables: int = 17, mean_tables: float = 4.5,
                d_choices=(5, 7, 11), w_choices=(1024, 2048, 4096, 8192, 16384),
                tri_prob: float = 0.15, pred_prob: float = 0.7):
    """Connected queries over the pool's foreign-key graph.  Each join edge
    is a foreign key = primary key predicate; with probability tri_prob a
    query also gets the transitive equality of two foreign keys that
    reference the same table of the query (a triangle, as in 6a)."""
    rng = rng_of(seed, 40)
    links = []  # (a, acol, b): a.acol references b.id
    for a, pt in enumerate(pool):
        for (c, b) in pt.fks:
            links.append((a, c, b))
    out = []
    for _ in range(n_queries):
        target = int(min(max_tables, max(2, 1 + rng.geometric(1.0 / (mean_tables - 1)))))
        start = int(rng.integers(0, len(pool)))
        tabs = [start]
        edges = []
        while len(tabs) < target:
            cand = [(a, c, b) for (a, c, b) in links
                    if (a in tabs) != (b in tabs)]
            if not cand:
                break
            a, c, b = cand[int(rng.integers(0, len(cand)))]
            new = b if a in tabs else a
            tabs.append(new)
            edges.append(Edge(tabs.index(a), c, tabs.index(b), "id"))
        if rng.random() < tri_prob:
            # two foreign keys of the query referencing the same query table
            by_ref = {}
            for e in edges:
                if e.vcol == "id":
                    by_ref.setdefault(e.v, []).append(e)
            for v, es in by_ref.items():
                if len(es) >= 2:
                    e1, e2 = es[0], es[1]
                    edges.append(Edge(e1.u, e1.ucol, e2.u, e2.ucol))
                    break
        preds = [random_predicates(rng, pred_prob) for _ in tabs]
        d = int(rng.choice(d_choices))
        w = int(rng.choice(w_choices))
        seeds = draw_seeds(rng, len(edges), d)
        out.append(PoolQuery(tabs, edges, preds, d, w, seeds))
    return out


def pool_query_as_query(pool, pq: PoolQuery) -> Query:
    """A standalone Query (tables with their columns and selections)."""
    tables = [Table(pool[t].name, pool[t].cols, pq.preds[i])
              for i, t in enumerate(pq.tables)]
    return Query(tables, pq.edges, pq.d, pq.w, pq.seeds, 32)


# --------------------------------------------------------------------------
# Learned-correction workload: pools of tables of 10k..2M rows (so exact
# join sizes stay affordable for the oracle), tree-shaped queries of up to 8
# tables, d=7, w=8192; training and held-out sets come from disjoint seeds.
# --------------------------------------------------------------------------
LEARNED_TRAIN_SEED = 1001
LEARNED_TEST_SEED = 2002


def learned_workload(seed: int, n_queries: int, pool_tables: int = 48,
                     size_range=(10_000, 2_000_000), max_tables: int = 8,
                     d: int = 7, w: int = 8192, scale: float = 1.0):
    pool = schema_pool(seed, n_tables=pool_tables, size_range=size_range,
                       scale=scale)
    queries = query_batch(pool, seed + 1, n_queries, max_tables=max_tables,
                          d_choices=(d,), w_choices=(w,), tri_prob=0.0)
    return pool, queries


def connected_masks(n_tables, edge_u, edge_v, min_tables=1, max_tables=64):
    adj = [0] * n_tables
    for u, v in zip(edge_u, edge_v):
        adj[u] |= 1 << v
        adj[v] |= 1 << u
    out = []
    for m in range(1, 1 << n_tables):
        k = bin(m).count("1")
        if k < min_tables or k > max_tables:
            continue
        seen = m & -m
        while True:
            grow = seen
            s, t = seen, 0
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
    return out


def learned_subplans(queries, seed: int, max_per_query: int = 24):
    """Per query: its connected sub-plans of >= 2 tables, a seeded sample of
    at most max_per_query of them."""
    rng = rng_of(seed, 50)
    out = []
    for pq in queries:
        ms = connected_masks(len(pq.tables), [e.u for e in pq.edges],
                             [e.v for e in pq.edges], min_tables=2)
        if len(ms) > max_per_query:
            idx = rng.choice(len(ms), size=max_per_query, replace=False)
            ms = [ms[i] for i in sorted(idx)]
        out.append(ms)
    return out


# --------------------------------------------------------------------------
# Large scan: one fact table of 1B rows generated directly in device memory
# (64 GB of columns; host generation would take minutes): six int64 join
# keys Zipf(1.1) over a 50M-key domain (a seeded permutation per column),
# two int32 columns uniform in [0, 1e6) and two float32 columns uniform in
# [0, 1), four range predicates of ~31.6% each (1% combined), d=11,
# w=65536, int64 counters.
# --------------------------------------------------------------------------
def large_scan_device(seed: int = DEFAULT_SEED, n_rows: int = 1_000_000_000,
                      domain: int = 50_000_000, zipf_s: float = 1.1,
                      n_keys: int = 6, d: int = 11, w: int = 65536,
                      device="cuda", chunk: int = 1 << 26):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 7919 + 5)
    ranks = torch.arange(1, domain + 1, dtype=torch.float64, device=device)
    cdf = torch.cumsum(ranks.pow_(-float(zipf_s)), 0)
    cdf /= cdf[-1].clone()
    del ranks
    cols = {}
    for k in range(n_keys):
        perm = torch.randperm(domain, generator=g, device=device)
        out = torch.empty(n_rows, dtype=torch.int64, device=device)
        for a in range(0, n_rows, chunk):
            b = min(n_rows, a + chunk)
            u = torch.rand(b - a, generator=g, device=device, dtype=torch.float64)
            r = torch.searchsorted(cdf, u).clamp_(max=domain - 1)
            out[a:b] = perm[r]
        cols["key%d" % k] = out
        del perm
    for k in range(2):
        cols["i%d" % k] = torch.randint(0, 1_000_000, (n_rows,), generator=g,
                                        device=device, dtype=torch.int32)
    for k in range(2):
        cols["f%d" % k] = torch.rand(n_rows, generator=g, device=device,
                                     dtype=torch.float32)
    del cdf
    preds = [Predicate("i0", "range", 0, 316_227), Predicate("i1", "range", 0, 316_227),
             Predicate("f0", "range", 0.0, 0.316227), Predicate("f1", "range", 0.0, 0.316227)]
    seeds = draw_seeds(rng_of(seed, 60), n_keys, d)
    return cols, preds, seeds
