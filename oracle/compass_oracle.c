/*
 * compass_oracle.c -- plain, slow, obviously correct CPU oracle for the
 * online sketch-based query optimisation hot path (Izenov, Datta, Rusu,
 * Shin, "Online Sketch-based Query Optimization", arXiv 2102.02440).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant with
 * the HIP library: every definition below is written out again from the
 * paper and from the readings listed at the top of each function.
 *
 * Arithmetic is exact: hash polynomials use unsigned __int128 products
 * reduced with the % operator, counters are int64, and multi-way estimates
 * are accumulated in 128-bit two's complement that wraps modulo 2^128
 * (unsigned __int128, so wrap-around is defined behaviour in C).
 *
 * Build: gcc -O2 -fPIC -shared -fopenmp -o liboracle.so compass_oracle.c
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

/* The prime field of the hash families: p = 2^61 - 1. */
static const uint64_t ORACLE_P = 2305843009213693951ULL;

/* ------------------------------------------------------------------ */
/* Hash families (Section 4.1: xi is a 4-wise independent +-1 family;  */
/* Section 4.2: each Fast-AGMS row has one bucket hash h and one xi).  */
/* The paper names no concrete family.  Reading used here: Carter-    */
/* Wegman polynomials over GF(p), p = 2^61-1.                          */
/*   x  = ((uint64)(int64)key) mod p                                   */
/*   v  = a0 + a1 x + a2 x^2 + a3 x^3  (mod p)   -> xi = +1 if v even  */
/*   g  = b0 + b1 x                   (mod p)   -> h  = g mod w        */
/* seeds = {a0, a1, a2, a3, b0, b1}, each in [0, p).                   */
/* ------------------------------------------------------------------ */

static uint64_t field_of_key(int64_t key)
{
    return ((uint64_t)key) % ORACLE_P;
}

static uint64_t mulmod(uint64_t a, uint64_t b)
{
    return (uint64_t)(((u128)a * (u128)b) % ORACLE_P);
}

static uint64_t addmod(uint64_t a, uint64_t b)
{
    return (uint64_t)(((u128)a + (u128)b) % ORACLE_P);
}

/* Evaluates the two polynomials term by term (no Horner, no lazy
 * reduction) so that the code reads like the definition. */
void oracle_hash(const uint64_t *seeds, int64_t key, int64_t w,
                 int64_t *bucket, int32_t *sign)
{
    uint64_t x = field_of_key(key);
    uint64_t x2 = mulmod(x, x);
    uint64_t x3 = mulmod(x2, x);
    uint64_t v = seeds[0] % ORACLE_P;
    v = addmod(v, mulmod(seeds[1], x));
    v = addmod(v, mulmod(seeds[2], x2));
    v = addmod(v, mulmod(seeds[3], x3));
    uint64_t g = addmod(seeds[4] % ORACLE_P, mulmod(seeds[5], x));
    *sign = (v & 1ULL) ? -1 : +1;
    *bucket = (int64_t)(g % (uint64_t)w);
}

/* ------------------------------------------------------------------ */
/* Fast-AGMS sketch of a multiset of keys (Section 4.2 counter          */
/* definition: counter j of a row sums xi over the tuples whose key     */
/* hashes to j).  The caller passes only the keys of tuples that        */
/* satisfy the table's selection predicates (Section 3, push-down).     */
/* counters: d rows x w buckets, row-major, int64, ADDED to.            */
/* ------------------------------------------------------------------ */
void oracle_sketch(const int64_t *keys, int64_t n, const uint64_t *seeds,
                   int32_t d, int64_t w, int64_t *counters)
{
    for (int64_t r = 0; r < n; ++r) {
        for (int32_t i = 0; i < d; ++i) {
            int64_t b;
            int32_t s;
            oracle_hash(seeds + 6 * i, keys[r], w, &b, &s);
            counters[(int64_t)i * w + b] += s;
        }
    }
}

/* The same counters computed by n_threads OpenMP threads: thread k sums
 * the tuples of its contiguous share of the keys into counters of its own
 * (the literal loop above, on a part of the input), and the parts' counters
 * are then added.  Integer addition is exact and order-free, so the result
 * equals the single-threaded one (Section 2: the sketch of a union is the
 * sum of the parts' sketches).  counters: d x w int64, ADDED to. */
void oracle_sketch_mt(const int64_t *keys, int64_t n, const uint64_t *seeds,
                      int32_t d, int64_t w, int64_t *counters,
                      int32_t n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if ((int64_t)n_threads > n / 4096 + 1) n_threads = (int32_t)(n / 4096 + 1);
    const int64_t cells = (int64_t)d * w;
    if (n_threads == 1) {
        oracle_sketch(keys, n, seeds, d, w, counters);
        return;
    }
    int64_t *part = (int64_t *)calloc((size_t)n_threads * (size_t)cells,
                                      sizeof(int64_t));
    if (!part) {  /* not enough memory for private counters: one thread */
        oracle_sketch(keys, n, seeds, d, w, counters);
        return;
    }
#pragma omp parallel for num_threads(n_threads) schedule(static, 1)
    for (int32_t k = 0; k < n_threads; ++k) {
        const int64_t r0 = n * k / n_threads, r1 = n * (k + 1) / n_threads;
        oracle_sketch(keys + r0, r1 - r0, seeds, d, w, part + (int64_t)k * cells);
    }
#pragma omp parallel for num_threads(n_threads) schedule(static)
    for (int64_t c = 0; c < cells; ++c) {
        int64_t s = 0;
        for (int32_t k = 0; k < n_threads; ++k) s += part[(int64_t)k * cells + c];
        counters[c] += s;
    }
    free(part);
}

/* ------------------------------------------------------------------ */
/* Join graph and sub-plans.                                           */
/*   edge e joins table eu[e] and table ev[e]; edge id = index e.       */
/*   sk[2e+0] = sketch row-set of table eu[e] on edge e (d x w int64)   */
/*   sk[2e+1] = sketch row-set of table ev[e] on edge e                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n_tables, n_edges, d;
    int64_t w;
    const int32_t *eu, *ev;
    const int64_t *const *sk;
} graph_t;

static const int64_t *sketch_row(const graph_t *g, int32_t e, int32_t t,
                                 int32_t row)
{
    int side = (g->eu[e] == t) ? 0 : 1;
    return g->sk[2 * e + side] + (int64_t)row * g->w;
}

static int64_t abs64(int64_t v) { return v < 0 ? -v : v; }

/* Sketch merging (Section 5.2): among the buckets a table's sketches
 * pick for the current assignment, the one with the smallest absolute
 * value wins; on equal magnitude the first sketch wins (the "<=" of the
 * merge rule), and "first" is read as the lowest edge id when more than
 * two sketches are merged.  Returns the winning counter value. */
static int64_t merged_value(const graph_t *g, int32_t t, const int32_t *inc,
                            int32_t n_inc, const int64_t *assign, int32_t row)
{
    /* inc[] is in increasing edge-id order */
    int64_t best = sketch_row(g, inc[0], t, row)[assign[inc[0]]];
    for (int32_t k = 1; k < n_inc; ++k) {
        int64_t v = sketch_row(g, inc[k], t, row)[assign[inc[k]]];
        if (abs64(v) < abs64(best)) best = v;
    }
    return best;
}

/* Collects the tables and induced edges of sub-plan `mask`. */
static int collect(const graph_t *g, uint64_t mask, int32_t *tabs,
                   int32_t *nt, int32_t *edges, int32_t *ne)
{
    *nt = 0;
    *ne = 0;
    for (int32_t t = 0; t < g->n_tables; ++t)
        if (mask >> t & 1ULL) tabs[(*nt)++] = t;
    for (int32_t e = 0; e < g->n_edges; ++e)
        if ((mask >> g->eu[e] & 1ULL) && (mask >> g->ev[e] & 1ULL))
            edges[(*ne)++] = e;
    return 0;
}

/* Connectivity of the sub-plan over its induced edges (cross products
 * are excluded from enumeration, Section 3 "Plan enumeration"). */
static int connected(const graph_t *g, uint64_t mask)
{
    uint64_t seen = mask & (~mask + 1ULL); /* lowest table */
    for (;;) {
        uint64_t grow = seen;
        for (int32_t e = 0; e < g->n_edges; ++e) {
            uint64_t bu = 1ULL << g->eu[e], bv = 1ULL << g->ev[e];
            if (!(mask & bu) || !(mask & bv)) continue;
            if (seen & (bu | bv)) grow |= bu | bv;
        }
        if (grow == seen) break;
        seen = grow;
    }
    return seen == mask;
}

/* ------------------------------------------------------------------ */
/* Estimate, literal definition.  Row i of a sub-plan with tables C and */
/* induced edges E_C:                                                   */
/*   X_i = sum over all bucket assignments iota in [0,w)^{E_C} of       */
/*         prod over t in C of merged_t(iota)                           */
/* which is the contraction of Section 5.1 (3-table case written out    */
/* there) with each table's merged sketch (Section 5.2) substituted,    */
/* applied iteratively to any number of joins.  A single table's        */
/* estimate is its exact filtered cardinality (Section 3).              */
/* Cost w^{|E_C|}: tiny w only.                                         */
/* ------------------------------------------------------------------ */
static u128 row_estimate_literal(const graph_t *g, const int32_t *tabs,
                                 int32_t nt, const int32_t *edges, int32_t ne,
                                 int32_t row)
{
    int64_t assign[64];
    int32_t inc[64][64];
    int32_t n_inc[64];
    for (int32_t a = 0; a < nt; ++a) {
        n_inc[a] = 0;
        for (int32_t k = 0; k < ne; ++k) {
            int32_t e = edges[k];
            if (g->eu[e] == tabs[a] || g->ev[e] == tabs[a])
                inc[a][n_inc[a]++] = e;
        }
    }
    for (int32_t k = 0; k < ne; ++k) assign[edges[k]] = 0;
    u128 total = 0;
    for (;;) {
        u128 prod = 1;
        for (int32_t a = 0; a < nt; ++a)
            prod *= (u128)(i128)merged_value(g, tabs[a], inc[a], n_inc[a],
                                             assign, row);
        total += prod;
        int32_t k = 0;
        while (k < ne) {
            if (++assign[edges[k]] < g->w) break;
            assign[edges[k]] = 0;
            ++k;
        }
        if (k == ne) break;
    }
    return total;
}

/* ------------------------------------------------------------------ */
/* Estimate, exact fast evaluation (our re-association of the literal   */
/* sum; pinned against it by brute force in the tests).                 */
/*                                                                      */
/* Spanning tree by BFS from the lowest table, edges scanned in id      */
/* order; the remaining induced edges form the cut set K.  For every    */
/* assignment J of the cut edges the tree is contracted bottom-up, and  */
/* the results are summed over J (w^{|K|} assignments).                 */
/*                                                                      */
/* A node t sees elements: its parent-edge buckets (query points), its  */
/* child-edge buckets (each weighted by the child's message mu_c), and  */
/* one fixed element per cut edge at t (value s_{t,f}[J_f]).  Elements  */
/* are ordered by kappa = (|value|, edge id).  The merged value of t is */
/* the element of smallest kappa, so with A_c(k) = sum of mu_c over     */
/* child-c elements of kappa > k (fixed elements: 1 if kappa > k else   */
/* 0), the message for parent bucket j is                               */
/*   M(j) = x_j * prod_c A_c(kappa_j) + G(kappa_j),                     */
/*   G(k) = sum over child/fixed elements z with kappa_z < k of         */
/*          value_z * mu_z * prod_{c != c(z)} A_c(kappa_z),             */
/* and the root's contribution is G(+inf).                              */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t absv;   /* |value| */
    int32_t edge;   /* edge id */
    int32_t kind;   /* 0 parent, 1 child, 2 fixed */
    int32_t slot;   /* child slot or fixed slot */
    int64_t j;      /* bucket index */
    int64_t value;
} elem_t;

static int elem_cmp(const void *pa, const void *pb)
{
    const elem_t *a = (const elem_t *)pa, *b = (const elem_t *)pb;
    if (a->absv != b->absv) return a->absv < b->absv ? -1 : 1;
    if (a->edge != b->edge) return a->edge < b->edge ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}

typedef struct {
    int32_t table;
    int32_t parent_edge;     /* -1 at the root */
    int32_t parent_node;
    int32_t n_child;
    int32_t child_edge[64];
    int32_t child_node[64];
    int32_t n_fixed;
    int32_t fixed_edge[64];
    /* elements that do not depend on the cut assignment, sorted */
    elem_t *base;
    int64_t n_base;
    u128 *msg;               /* message to the parent, length w */
} tnode_t;

static u128 contract_tree(const graph_t *g, tnode_t *nodes, int32_t nn,
                          const int32_t *order, const int64_t *cut_assign,
                          int32_t row)
{
    u128 root_value = 0;
    for (int32_t oi = nn - 1; oi >= 0; --oi) {
        tnode_t *nd = &nodes[order[oi]];
        int32_t t = nd->table;
        /* fixed elements for this assignment, sorted by kappa */
        elem_t fx[64];
        for (int32_t f = 0; f < nd->n_fixed; ++f) {
            int32_t e = nd->fixed_edge[f];
            int64_t v = sketch_row(g, e, t, row)[cut_assign[e]];
            fx[f].absv = abs64(v);
            fx[f].edge = e;
            fx[f].kind = 2;
            fx[f].slot = f;
            fx[f].j = cut_assign[e];
            fx[f].value = v;
        }
        qsort(fx, (size_t)nd->n_fixed, sizeof(elem_t), elem_cmp);
        /* A values start at the full sums */
        u128 A[128];
        for (int32_t c = 0; c < nd->n_child; ++c) {
            u128 s = 0;
            const u128 *mu = nodes[nd->child_node[c]].msg;
            for (int64_t j = 0; j < g->w; ++j) s += mu[j];
            A[c] = s;
        }
        for (int32_t f = 0; f < nd->n_fixed; ++f) A[nd->n_child + f] = 1;
        int32_t nA = nd->n_child + nd->n_fixed;
        u128 G = 0;
        int64_t bi = 0;
        int32_t fi = 0;
        while (bi < nd->n_base || fi < nd->n_fixed) {
            const elem_t *z;
            if (fi < nd->n_fixed &&
                (bi >= nd->n_base || elem_cmp(&fx[fi], &nd->base[bi]) < 0))
                z = &fx[fi++];
            else
                z = &nd->base[bi++];
            u128 val = (u128)(i128)z->value;
            if (z->kind == 0) {
                u128 p = val;
                for (int32_t a = 0; a < nA; ++a) p *= A[a];
                nd->msg[z->j] = p + G;
            } else {
                int32_t own = (z->kind == 1) ? z->slot : nd->n_child + z->slot;
                u128 mu = (z->kind == 1) ? nodes[nd->child_node[z->slot]].msg[z->j]
                                         : (u128)1;
                u128 term = val * mu;
                for (int32_t a = 0; a < nA; ++a)
                    if (a != own) term *= A[a];
                G += term;
                A[own] -= mu;
            }
        }
        if (nd->parent_edge < 0) root_value = G;
    }
    return root_value;
}

static u128 row_estimate_fast(const graph_t *g, const int32_t *tabs,
                              int32_t nt, const int32_t *edges, int32_t ne,
                              int32_t row)
{
    tnode_t *nodes = (tnode_t *)calloc((size_t)nt, sizeof(tnode_t));
    int32_t node_of[64];
    for (int32_t t = 0; t < 64; ++t) node_of[t] = -1;
    int32_t order[64];
    int32_t n_order = 0;
    int32_t is_tree_edge[64];
    int32_t cut[64];
    int32_t n_cut = 0;
    memset(is_tree_edge, 0, sizeof(is_tree_edge));
    /* BFS spanning tree */
    nodes[0].table = tabs[0];
    nodes[0].parent_edge = -1;
    nodes[0].parent_node = -1;
    node_of[tabs[0]] = 0;
    order[n_order++] = 0;
    int32_t n_nodes = 1;
    for (int32_t head = 0; head < n_order; ++head) {
        int32_t cur = order[head];
        int32_t t = nodes[cur].table;
        for (int32_t k = 0; k < ne; ++k) {
            int32_t e = edges[k];
            int32_t other;
            if (g->eu[e] == t) other = g->ev[e];
            else if (g->ev[e] == t) other = g->eu[e];
            else continue;
            if (node_of[other] >= 0) continue;
            int32_t nn = n_nodes++;
            nodes[nn].table = other;
            nodes[nn].parent_edge = e;
            nodes[nn].parent_node = cur;
            node_of[other] = nn;
            is_tree_edge[k] = 1;
            nodes[cur].child_edge[nodes[cur].n_child] = e;
            nodes[cur].child_node[nodes[cur].n_child++] = nn;
            order[n_order++] = nn;
        }
    }
    for (int32_t k = 0; k < ne; ++k) {
        if (is_tree_edge[k]) continue;
        int32_t e = edges[k];
        cut[n_cut++] = e;
        tnode_t *a = &nodes[node_of[g->eu[e]]];
        tnode_t *b = &nodes[node_of[g->ev[e]]];
        a->fixed_edge[a->n_fixed++] = e;
        b->fixed_edge[b->n_fixed++] = e;
    }
    /* assignment-independent elements, sorted once */
    for (int32_t a = 0; a < n_nodes; ++a) {
        tnode_t *nd = &nodes[a];
        int32_t groups = nd->n_child + (nd->parent_edge >= 0 ? 1 : 0);
        nd->base = (elem_t *)malloc(sizeof(elem_t) * (size_t)(groups * g->w + 1));
        nd->msg = (u128 *)calloc((size_t)g->w, sizeof(u128));
        nd->n_base = 0;
        for (int32_t gi = 0; gi < groups; ++gi) {
            int32_t is_parent = (nd->parent_edge >= 0 && gi == nd->n_child);
            int32_t e = is_parent ? nd->parent_edge : nd->child_edge[gi];
            const int64_t *s = sketch_row(g, e, nd->table, row);
            for (int64_t j = 0; j < g->w; ++j) {
                elem_t *z = &nd->base[nd->n_base++];
                z->absv = abs64(s[j]);
                z->edge = e;
                z->kind = is_parent ? 0 : 1;
                z->slot = is_parent ? 0 : gi;
                z->j = j;
                z->value = s[j];
            }
        }
        qsort(nd->base, (size_t)nd->n_base, sizeof(elem_t), elem_cmp);
    }
    int64_t cut_assign[64];
    for (int32_t e = 0; e < 64; ++e) cut_assign[e] = 0;
    u128 total = 0;
    for (;;) {
        total += contract_tree(g, nodes, n_nodes, order, cut_assign, row);
        int32_t k = 0;
        while (k < n_cut) {
            if (++cut_assign[cut[k]] < g->w) break;
            cut_assign[cut[k]] = 0;
            ++k;
        }
        if (k == n_cut) break;
    }
    for (int32_t a = 0; a < n_nodes; ++a) {
        free(nodes[a].base);
        free(nodes[a].msg);
    }
    free(nodes);
    return total;
}

/* ------------------------------------------------------------------ */
/* Median over the d rows (Section 4.1 and 4.2: the final estimate is  */
/* the median of the independent basic estimates).  Odd d: the middle  */
/* value.  Even d (never used by the configured workloads; the paper is */
/* silent): the mean of the two middle values.  The double is rounded  */
/* to nearest-even from the exact integer by the C conversion.          */
/* ------------------------------------------------------------------ */
static int i128_cmp(const void *pa, const void *pb)
{
    i128 a = *(const i128 *)pa, b = *(const i128 *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static double median_of(const u128 *rows, int32_t d)
{
    i128 *v = (i128 *)malloc(sizeof(i128) * (size_t)d);
    for (int32_t i = 0; i < d; ++i) v[i] = (i128)rows[i];
    qsort(v, (size_t)d, sizeof(i128), i128_cmp);
    double out;
    if (d & 1) {
        out = (double)v[d / 2];
    } else {
        i128 s = (i128)((u128)v[d / 2 - 1] + (u128)v[d / 2]);
        out = (double)s * 0.5;
    }
    free(v);
    return out;
}

/* Certificate that the 128-bit row values are the true integers:
 * every row value is bounded in magnitude by prod_t n_sel(t) times
 * w^(|E_C| - |C|) when the sub-plan has more edges than tables (each
 * bucket row sums to at most n_sel in absolute value, and a one-to-one
 * assignment of tables to incident edges factorises the bound).  The
 * flag is set when that bound is below 2^127. */
static int certified(const graph_t *g, const int64_t *n_sel,
                     const int32_t *tabs, int32_t nt, int32_t ne)
{
    /* exact product with saturation at 2^127 */
    const u128 LIM = (u128)1 << 127;
    u128 b = 1;
    for (int32_t a = 0; a < nt; ++a) {
        u128 f = (u128)(n_sel[tabs[a]] < 0 ? 0 : n_sel[tabs[a]]);
        if (f == 0) return 1;
        if (b > LIM / f) return 0;
        b *= f;
    }
    for (int32_t k = 0; k < ne - nt; ++k) {
        if (b > LIM / (u128)g->w) return 0;
        b *= (u128)g->w;
    }
    return b < LIM;
}

/* Flag bits of one estimate */
#define ORACLE_FLAG_EXACT 1

/* Estimates every sub-plan in `masks`.
 * sk: array of 2*n_edges pointers to d x w int64 counters.
 * method: 0 literal definition, 1 fast exact evaluation.
 * out_rows: n_masks x d x 2 uint64 (lo, hi of the 128-bit row values).
 * Returns 0, or -1 when a mask is empty or not connected. */
int oracle_estimate(int32_t n_tables, int32_t n_edges, const int32_t *eu,
                    const int32_t *ev, int32_t d, int64_t w,
                    const int64_t *const *sk, const int64_t *n_sel,
                    const uint64_t *masks, int32_t n_masks, int32_t method,
                    uint64_t *out_rows, double *out_est, int32_t *out_flags)
{
    graph_t g = {n_tables, n_edges, d, w, eu, ev, sk};
    for (int32_t m = 0; m < n_masks; ++m)
        if (masks[m] == 0 || !connected(&g, masks[m])) return -1;
    int32_t bad = 0;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int32_t m = 0; m < n_masks; ++m) {
        for (int32_t i = 0; i < d; ++i) {
            int32_t tabs[64], edges[64], nt, ne;
            collect(&g, masks[m], tabs, &nt, edges, &ne);
            u128 x;
            if (nt == 1)
                x = (u128)(i128)n_sel[tabs[0]];
            else if (method == 0)
                x = row_estimate_literal(&g, tabs, nt, edges, ne, i);
            else
                x = row_estimate_fast(&g, tabs, nt, edges, ne, i);
            out_rows[((int64_t)m * d + i) * 2 + 0] = (uint64_t)x;
            out_rows[((int64_t)m * d + i) * 2 + 1] = (uint64_t)(x >> 64);
        }
    }
    for (int32_t m = 0; m < n_masks; ++m) {
        int32_t tabs[64], edges[64], nt, ne;
        collect(&g, masks[m], tabs, &nt, edges, &ne);
        u128 *rows = (u128 *)malloc(sizeof(u128) * (size_t)d);
        for (int32_t i = 0; i < d; ++i)
            rows[i] = (u128)out_rows[((int64_t)m * d + i) * 2 + 0] |
                      ((u128)out_rows[((int64_t)m * d + i) * 2 + 1] << 64);
        out_est[m] = median_of(rows, d);
        out_flags[m] = certified(&g, n_sel, tabs, nt, ne) ? ORACLE_FLAG_EXACT : 0;
        free(rows);
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* Sketch partitioning (Section 5.1).  For a table taking part in two   */
/* joins, the counters of one sketch row are arranged as a w1 x w2      */
/* matrix: a tuple with join keys (a, b) adds xi1(a) * xi2(b) to the    */
/* entry [h1(a)][h2(b)], where (h1, xi1) are the row's functions of the */
/* first join (the same seeds as the neighbour's one-dimensional sketch */
/* on that join) and (h2, xi2) those of the second.                     */
/* counters: d x w1 x w2 int64, row-major, ADDED to.                    */
/* ------------------------------------------------------------------ */
void oracle_sketch2d(const int64_t *keys1, const int64_t *keys2, int64_t n,
                     const uint64_t *seeds1, const uint64_t *seeds2,
                     int32_t d, int64_t w1, int64_t w2, int64_t *counters)
{
    for (int64_t r = 0; r < n; ++r) {
        for (int32_t i = 0; i < d; ++i) {
            int64_t b1, b2;
            int32_t s1, s2;
            oracle_hash(seeds1 + 6 * i, keys1[r], w1, &b1, &s1);
            oracle_hash(seeds2 + 6 * i, keys2[r], w2, &b2, &s2);
            counters[((int64_t)i * w1 + b1) * w2 + b2] += (int64_t)(s1 * s2);
        }
    }
}

/* Partitioned sketch of a table with k joins (Section 5.1: the sketch of a
 * table with k joins is a k-dimensional tensor): for every row r and
 * sketch row i, adds the product over joins m of xi_{m,i}(keys[m][r]) to
 * entry [h_{1,i}(keys[0][r])] .. [h_{k,i}(keys[k-1][r])] of row i's tensor
 * (row-major, widths w[0] .. w[k-1]).  seeds[m] is join m's d x 6 seed
 * table. */
void oracle_sketch_kd(const int64_t *const *keys, int32_t k, int64_t n,
                      const uint64_t *const *seeds, int32_t d, const int64_t *w,
                      int64_t *counters)
{
    int64_t size = 1;
    for (int32_t m = 0; m < k; ++m) size *= w[m];
    for (int64_t r = 0; r < n; ++r) {
        for (int32_t i = 0; i < d; ++i) {
            int64_t idx = 0;
            int32_t sign = 1;
            for (int32_t m = 0; m < k; ++m) {
                int64_t b;
                int32_t g;
                oracle_hash(seeds[m] + 6 * i, keys[m][r], w[m], &b, &g);
                idx = idx * w[m] + b;
                sign *= g;
            }
            counters[(int64_t)i * size + idx] += (int64_t)sign;
        }
    }
}

/* Estimate of a join graph from partitioned sketches (Section 5.1): table
 * t's sketch row i is a tensor with one dimension per incident edge (edges
 * in increasing id, widths w[e]); the row value is the sum over every
 * assignment of a bucket j_e to each edge e of the product over tables of
 * their entries at those buckets, exact in 128-bit two's complement, taken
 * literally: one term per assignment.  The estimate is the median over rows
 * and the flag certifies the rows when the product of the tables' selected
 * rows is below 2^127.
 *   tensors[t]: d x prod of w over t's edges (int64); out_rows: d x 2 */
void oracle_tensor_join(int32_t n_tables, int32_t n_edges, const int32_t *eu,
                        const int32_t *ev, int32_t d, const int64_t *w,
                        const int64_t *const *tensors, const int64_t *n_sel,
                        uint64_t *out_rows, double *out_est, int32_t *out_flag)
{
    int32_t *j = (int32_t *)calloc((size_t)(n_edges > 0 ? n_edges : 1), sizeof(int32_t));
    int64_t *size = (int64_t *)calloc((size_t)n_tables, sizeof(int64_t));
    for (int32_t t = 0; t < n_tables; ++t) {
        size[t] = 1;
        for (int32_t e = 0; e < n_edges; ++e)
            if (eu[e] == t || ev[e] == t) size[t] *= w[e];
    }
    u128 *rows = (u128 *)malloc(sizeof(u128) * (size_t)d);
    for (int32_t i = 0; i < d; ++i) {
        u128 x = 0;
        for (int32_t e = 0; e < n_edges; ++e) j[e] = 0;
        for (;;) {
            u128 term = 1;
            for (int32_t t = 0; t < n_tables; ++t) {
                int64_t idx = 0;  /* the table's entry: its edges in id order */
                for (int32_t e = 0; e < n_edges; ++e)
                    if (eu[e] == t || ev[e] == t) idx = idx * w[e] + j[e];
                term *= (u128)(i128)tensors[t][(int64_t)i * size[t] + idx];
            }
            x += term;
            int32_t e = n_edges - 1;  /* next assignment */
            while (e >= 0 && ++j[e] == w[e]) j[e--] = 0;
            if (e < 0) break;
        }
        rows[i] = x;
        out_rows[2 * i + 0] = (uint64_t)x;
        out_rows[2 * i + 1] = (uint64_t)(x >> 64);
    }
    *out_est = median_of(rows, d);
    /* |X_i| <= product of n_sel (the entries of a table's sketch row sum to
     * at most its selected rows in absolute value) */
    const u128 lim = (u128)1 << 127;
    u128 b = 1;
    int ok = 1;
    for (int32_t t = 0; t < n_tables && ok; ++t) {
        const u128 f = (u128)(n_sel[t] < 0 ? 0 : n_sel[t]);
        if (f == 0) { b = 0; break; }
        if (b > lim / f) ok = 0;
        else b *= f;
    }
    *out_flag = ok && b < lim ? 1 : 0;
    free(rows);
    free(size);
    free(j);
}

/* The three-table chain estimate of Section 5.1: for row i, the sum over
 * all entries (j1, j2) of A[j1] * P[j1][j2] * B[j2] (the matrix scaled by
 * the first sketch along its rows and by the second along its columns,
 * then summed), exact in 128-bit two's complement; the estimate is the
 * median over rows.  The flag certifies the row values when
 * n_A * n_P * n_B < 2^127: every |A[j1]| <= n_A, every |B[j2]| <= n_B and
 * the |P| entries sum to at most n_P.
 *   A: d x w1, P: d x w1 x w2, B: d x w2 (int64); n_sel3 = {n_A, n_P, n_B}
 *   out_rows: d x 2 uint64 (lo, hi) */
void oracle_chain3(const int64_t *A, const int64_t *P, const int64_t *B,
                   int32_t d, int64_t w1, int64_t w2, const int64_t *n_sel3,
                   uint64_t *out_rows, double *out_est, int32_t *out_flag)
{
    u128 *rows = (u128 *)malloc(sizeof(u128) * (size_t)d);
    for (int32_t i = 0; i < d; ++i) {
        u128 x = 0;
        for (int64_t j1 = 0; j1 < w1; ++j1) {
            for (int64_t j2 = 0; j2 < w2; ++j2) {
                i128 t = (i128)A[(int64_t)i * w1 + j1] *
                         (i128)P[((int64_t)i * w1 + j1) * w2 + j2];
                x += (u128)t * (u128)(i128)B[(int64_t)i * w2 + j2];
            }
        }
        rows[i] = x;
        out_rows[2 * i + 0] = (uint64_t)x;
        out_rows[2 * i + 1] = (uint64_t)(x >> 64);
    }
    *out_est = median_of(rows, d);
    const u128 LIM = (u128)1 << 127;
    u128 b = 1;
    int ok = 1;
    for (int k = 0; k < 3 && ok; ++k) {
        u128 f = (u128)(n_sel3[k] < 0 ? 0 : n_sel3[k]);
        if (f == 0) { b = 0; break; }
        if (b > LIM / f) ok = 0; else b *= f;
    }
    *out_flag = (ok && b < LIM) ? ORACLE_FLAG_EXACT : 0;
    free(rows);
}

/* ------------------------------------------------------------------ */
/* AGMS sketches (Section 4.1), the baseline Fast-AGMS improves on.     */
/* A table's sketch for one query is r x b independent basic sketches, */
/* each a single counter: the sum over the table's qualifying tuples   */
/* of the product, over the joins the table takes part in, of that     */
/* join's +-1 variable of the tuple's key (one independent family per  */
/* join and basic sketch; the composed sketch of Section 4.1.2).       */
/* keys: n_joins arrays of n keys; seeds: n_joins x K x 6 (only a0..a3  */
/* are used), K = r * b; counters: K int64, ADDED to.                   */
/* ------------------------------------------------------------------ */
void oracle_agms_sketch(const int64_t *const *keys, int64_t n,
                        const uint64_t *seeds, int32_t n_joins, int32_t K,
                        int64_t *counters)
{
    /* basic sketches are independent: threads split the counters, or
     * the rows when there are few counters */
#pragma omp parallel for schedule(dynamic, 1) if (K >= 8)
    for (int32_t c = 0; c < K; ++c) {
        int64_t sum = 0;
#pragma omp parallel for reduction(+ : sum) if (K < 8)
        for (int64_t t = 0; t < n; ++t) {
            int32_t prod = 1;
            for (int32_t e = 0; e < n_joins; ++e) {
                int64_t bucket;
                int32_t sign;
                oracle_hash(seeds + ((int64_t)e * K + c) * 6, keys[e][t], 1,
                            &bucket, &sign);
                prod *= sign;
            }
            sum += prod;
        }
        counters[c] += sum;
    }
}

/* AGMS estimate of the query whose tables' sketches are given: basic
 * estimate (i, j) = product of the tables' counters (i, j); the b basic
 * estimates of row i are averaged and the median is taken over the r
 * averages (Section 4.1.1).  Row sums are exact in 128 bits; an average is
 * the round-to-nearest-even double of the sum divided by b in IEEE
 * arithmetic; even r takes the mean of the two middle averages.
 * sk: n_tables pointers to K = r * b int64 counters (row-major r x b).
 * out_rows: r x 2 uint64 (lo, hi of the row sums); flag EXACT when the
 * product of the tables' selected counts is below 2^127. */
void oracle_agms_estimate(const int64_t *const *sk, int32_t n_tables,
                          int32_t r, int32_t b, const int64_t *n_sel,
                          uint64_t *out_rows, double *out_est,
                          int32_t *out_flag)
{
    double *avg = (double *)malloc(sizeof(double) * (size_t)r);
    for (int32_t i = 0; i < r; ++i) {
        u128 sum = 0;
        for (int32_t j = 0; j < b; ++j) {
            u128 x = 1;
            for (int32_t t = 0; t < n_tables; ++t)
                x *= (u128)(i128)sk[t][(int64_t)i * b + j];
            sum += x;
        }
        out_rows[2 * i + 0] = (uint64_t)sum;
        out_rows[2 * i + 1] = (uint64_t)(sum >> 64);
        avg[i] = (double)(i128)sum / (double)b;
    }
    for (int32_t i = 1; i < r; ++i) {  /* insertion sort */
        double v = avg[i];
        int32_t k = i - 1;
        while (k >= 0 && avg[k] > v) { avg[k + 1] = avg[k]; --k; }
        avg[k + 1] = v;
    }
    *out_est = (r & 1) ? avg[r / 2] : (avg[r / 2 - 1] + avg[r / 2]) * 0.5;
    const u128 LIM = (u128)1 << 127;
    u128 p = 1;
    int ok = 1;
    for (int32_t t = 0; t < n_tables && ok; ++t) {
        u128 f = (u128)(n_sel[t] < 0 ? 0 : n_sel[t]);
        if (f == 0) { p = 0; break; }
        if (p > LIM / f) ok = 0; else p *= f;
    }
    *out_flag = (ok && p < LIM) ? ORACLE_FLAG_EXACT : 0;
    free(avg);
}

/* Exact conversion of one 128-bit value to double (round to nearest
 * even), exported so tests can pin the median conversion. */
double oracle_i128_to_double(uint64_t lo, uint64_t hi)
{
    u128 u = (u128)lo | ((u128)hi << 64);
    return (double)(i128)u;
}

/* Number of threads the OpenMP loops of the estimate use from now on
 * (the CPU baseline times the oracle with one thread and with all). */
void oracle_set_threads(int32_t n)
{
    omp_set_num_threads(n < 1 ? 1 : n);
}
