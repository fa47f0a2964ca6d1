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
