/*
 * compass.h -- C ABI of the MI355X (gfx950) hot path of online sketch-based
 * query optimisation (Izenov, Datta, Rusu, Shin, "Online Sketch-based Query
 * Optimization", arXiv 2102.02440).
 *
 * Two operations, as the paper splits them:
 *   1. compass_sketch_build  -- push-down selection fused with Fast-AGMS
 *      sketch building over the qualifying tuples (Section 3, "Workflow" and
 *      "Partitioned query execution"; Section 4.2 counter definition).
 *   2. compass_estimate      -- join-size estimates of sub-plans from the
 *      two-way sketches only: inner product + median for two tables
 *      (Section 4.2.1), min-abs sketch merging composed over the join graph
 *      for more (Section 5.2 with the contraction of Section 5.1).
 * Plus a batched build of many tables' sketches in one graph-captured
 * persistent launch, and a small learned correction network.
 *
 * Conventions shared by every entry point
 *   - Every function returns a compass_status and never throws.  On failure
 *     compass_last_error() returns a message (thread-local, valid until the
 *     next call on the same thread).
 *   - Device pointers: column data, predicate bitmaps, counters, outputs.
 *     Host pointers: seeds, graph arrays, sub-plan masks; they are copied
 *     before the call returns.  The caller owns every buffer; the library
 *     never frees caller memory.
 *   - All GPU work is enqueued on `stream` (0 = the null stream) and is
 *     asynchronous: outputs are valid once the stream has synchronised.
 *   - Scratch memory is cached by the library per (device, stream) and
 *     released by compass_release().  Calls on different streams never
 *     share scratch, so they may be in flight at the same time (reentrant
 *     across streams); calls on one stream run in stream order.  Host entry
 *     is serialised by one library-wide lock.
 *
 * Hash families (the paper requires a 4-wise independent +-1 family xi and
 * one bucket hash h per sketch row, Sections 4.1 and 4.2, and names no
 * concrete family).  With p = 2^61 - 1 and seeds {a0,a1,a2,a3,b0,b1} in
 * [0, p) for one row:
 *     x  = ((uint64_t)(int64_t)key) mod p      (int32 keys sign-extended)
 *     xi = +1 if (a0 + a1 x + a2 x^2 + a3 x^3 mod p) is even, else -1
 *     h  = ((b0 + b1 x) mod p) mod w
 * Both sketches of one join edge must use the same seeds (Section 4.1.1).
 */
#ifndef COMPASS_H
#define COMPASS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    COMPASS_OK = 0,
    COMPASS_E_ARG = 1,          /* null pointer, bad size / kind / dtype, seed >= p */
    COMPASS_E_RANGE = 2,        /* a size exceeds what the exact arithmetic allows */
    COMPASS_E_GRAPH = 3,        /* sub-plan empty / not connected / bad edge */
    COMPASS_E_HIP = 4,          /* HIP runtime failure */
    COMPASS_E_UNSUPPORTED = 5   /* valid request outside what this library runs */
} compass_status;

enum { COMPASS_I32 = 0, COMPASS_F32 = 1, COMPASS_I64 = 2 };
enum { COMPASS_PRED_POINT = 0, COMPASS_PRED_RANGE = 1, COMPASS_PRED_SUBSET = 2 };

/* One selection predicate on one column (Section 1: point, subset (LIKE over
 * a dictionary) and range selections; Section 3: conjunctive, pushed down).
 *   POINT : value == lo
 *   RANGE : lo <= value <= hi           (inclusive; IEEE compares for F32,
 *                                         so NaN fails, -0 == +0)
 *   SUBSET: 0 <= value < domain and bit `value` of `bitmap` is set
 *           (dtype must be I32; bitmap = device array of (domain+63)/64
 *           uint64 words, bit k of word k/64 is code k) */
typedef union {
    int32_t i;
    float f;
} compass_scalar;

typedef struct {
    int32_t col;                 /* index into pred_cols */
    int32_t kind;                /* COMPASS_PRED_* */
    int32_t dtype;               /* COMPASS_I32 or COMPASS_F32 */
    int32_t reserved;
    compass_scalar lo, hi;
    const uint64_t *bitmap;      /* SUBSET only, device */
    int64_t domain;              /* SUBSET only */
} compass_pred;

/* One attribute sketch to build during the scan.  One table has as many
 * sketches as joins it takes part in, even when two joins use the same
 * column (Section 3, "Workflow"). */
typedef struct {
    const void *key_col;         /* device, n_rows keys */
    int32_t key_dtype;           /* COMPASS_I32 or COMPASS_I64 */
    int32_t reserved;
    const uint64_t *seeds;       /* host, d x 6: a0 a1 a2 a3 b0 b1 per row */
    void *counters;              /* device, d x w row-major, int32 or int64 */
} compass_sketch_spec;

/* compass_sketch_build -- one scan of one table: evaluates the conjunction
 * of `preds` on every row and, for the rows that satisfy it, adds xi_i(key)
 * to counter h_i(key) of row i of every sketch (Section 4.2 counter
 * definition), and adds the number of qualifying rows to *n_selected (the
 * exact selected cardinality of Section 3).
 *   n_rows        rows of the table (0 allowed; < 2^47)
 *   pred_cols     host array of n_pred_cols device column pointers
 *   preds         host array of n_preds predicates (n_preds may be 0)
 *   sketches      host array of n_sketches specs (1 <= n_sketches <= 16)
 *   d, w          rows and buckets of every sketch (1 <= d <= 32, 1 <= w <= 2^20)
 *   counter_bits  32 or 64 (int32 counters need n_rows < 2^31)
 *   accumulate    0: counters and *n_selected are overwritten; 1: added to
 *                 (sketches are mergeable by addition, Section 2)
 *   n_selected    device int64
 * Tables with predicates, and rows wider than 32768 buckets, are built in
 * two phases: batches of rows have their qualifying rows' key field
 * elements compacted into a survivor buffer (8 bytes per sketch per row),
 * which is hashed into the counters only when the next batch might not fit
 * it and after the last batch (so a selective scan hashes once).  The
 * buffer takes at most 8.5 GiB of scratch (environment: COMPASS_TWO_PHASE_
 * BYTES sets that budget, COMPASS_SURVIVOR_CAP_ROWS caps the buffer's rows;
 * both exist to force many batches in tests).  E_RANGE if one batch of
 * 4096 rows cannot fit the budget.  COMPASS_SERIAL=1 (a debugging mode,
 * read at each call) builds with one chunk per group of sketch rows and a
 * single compaction workgroup, so that no two workgroups combine partial
 * counters: its results equal the default launch's bit for bit. */
compass_status compass_sketch_build(int64_t n_rows,
                                    const void *const *pred_cols,
                                    int32_t n_pred_cols,
                                    const compass_pred *preds, int32_t n_preds,
                                    const compass_sketch_spec *sketches,
                                    int32_t n_sketches, int32_t d, int32_t w,
                                    int32_t counter_bits, int32_t accumulate,
                                    int64_t *n_selected, hipStream_t stream);

/* compass_sketch_build_noalloc -- compass_sketch_build for callers that
 * cannot allocate memory during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): same arguments,
 * same kernels, same results, but no hipMalloc, hipFree, host or pinned
 * allocation and no timing events.  Its scratch (slab of partial
 * counters, survivor buffer, seeds) is one fixed 256 MiB region of device
 * memory per GPU, held until the process ends, with the work cut to fit
 * it (fewer chunks, smaller survivor batches).  E_RANGE, before any GPU
 * work, when the build cannot fit: one chunk of partial counters
 * (n_sketches x d x w x 4 bytes) above 256 MiB in the fused scan, or in
 * the two-phase build a slab of n_sketches x d x w x 4 bytes plus one
 * survivor batch of 4096 rows x n_sketches x 8 bytes above it.  Every call
 * on one GPU uses that GPU's region (the previous call's contents are
 * overwritten; what must start at zero is cleared by the call), so calls
 * that overlap on one GPU, on any streams, race: the caller serialises
 * them. */
compass_status compass_sketch_build_noalloc(int64_t n_rows,
                                            const void *const *pred_cols,
                                            int32_t n_pred_cols,
                                            const compass_pred *preds,
                                            int32_t n_preds,
                                            const compass_sketch_spec *sketches,
                                            int32_t n_sketches, int32_t d,
                                            int32_t w, int32_t counter_bits,
                                            int32_t accumulate,
                                            int64_t *n_selected,
                                            hipStream_t stream);

/* compass_sketch_build_select -- compass_sketch_build that also
 * materialises the selection output (Section 3, "Partitioned query
 * execution": the selection output is kept when it is small): the indices
 * of the qualifying rows, plus row_base, are written to rows_out[k] for the
 * k-th qualifying row seen (in no particular order) while k < rows_cap, and
 * *rows_count counts every qualifying row (zeroed first unless
 * accumulate).  The output is complete, without duplicates, iff the final
 * *rows_count <= rows_cap; beyond that the caller drops it (the sketches
 * and *n_selected are unaffected).
 *   rows_out    device int64, rows_cap entries (may be NULL if rows_cap = 0)
 *   rows_count  device int64
 *   row_base    0 <= row_base < 2^47 (e.g. the first row of this partition) */
compass_status compass_sketch_build_select(
    int64_t n_rows, const void *const *pred_cols, int32_t n_pred_cols,
    const compass_pred *preds, int32_t n_preds,
    const compass_sketch_spec *sketches, int32_t n_sketches, int32_t d,
    int32_t w, int32_t counter_bits, int32_t accumulate, int64_t *n_selected,
    int64_t *rows_out, int64_t rows_cap, int64_t *rows_count, int64_t row_base,
    hipStream_t stream);

/* A query join graph with its attribute sketches (Section 3, "Plan
 * enumeration": estimates take only the two-way sketches as input).
 * Edge e joins tables edge_u[e] and edge_v[e]; its id is e, and a lower id
 * is "first" in the merge tie rule of Section 5.2.
 * sketch[2e+0] = counters of table edge_u[e] on edge e, sketch[2e+1] = of
 * table edge_v[e]; both built with the same seeds.  n_selected[t] = exact
 * selected cardinality of table t (device).  It must also bound the sum of
 * absolute values of every row of t's sketches (always true of sketches
 * built from those selected rows): the estimate picks 64-bit arithmetic
 * where these bounds prove it exact, and 128-bit arithmetic otherwise. */
typedef struct {
    int32_t n_tables;            /* 1..64 */
    int32_t n_edges;             /* 0..64 */
    int32_t d, w;                /* sketch shape (w <= 65536) */
    int32_t counter_bits;        /* 32 or 64 */
    int32_t reserved;
    const int32_t *edge_u;       /* host, n_edges */
    const int32_t *edge_v;       /* host, n_edges */
    const int64_t *n_selected;   /* device, n_tables */
    const void *const *sketch;   /* host array of 2*n_edges device pointers */
} compass_join_graph;

typedef struct {
    uint64_t lo;
    int64_t hi;
} compass_i128;

/* Flag bits of one sub-plan estimate. */
enum {
    /* the row values are certified to be the true integers (no wrap):
     * prod over the sub-plan's tables of n_selected, times w^(#edges -
     * #tables) when positive, is below 2^127 */
    COMPASS_FLAG_EXACT = 1,
    /* the sub-plan's shape is outside what this library evaluates (more
     * than 6 independent cycles, a table with more than 8 join edges inside
     * the sub-plan, or more than 2^36 element steps of the conditioned
     * contraction, w^cycles x list length x d); its outputs are zero / NaN */
    COMPASS_FLAG_UNSUPPORTED = 2,
    /* the row values could not be certified (EXACT is clear) and est is the
     * median of an fp64 evaluation of the same contraction (relative
     * rounding of about 1e-15 times the same sum over absolute values);
     * row_est still holds the 128-bit values modulo 2^128 */
    COMPASS_FLAG_APPROX = 4
};

/* compass_estimate -- for each sub-plan C (bitmask of tables, connected over
 * the graph's edges between its tables) and each sketch row i:
 *   |C| = 1 : X_i = n_selected of the table (Section 3)
 *   |C| >= 2: X_i = sum over bucket assignments of C's induced edges of the
 *             product over C's tables of the table's merged sketch, where
 *             the merged value is the incident sketch bucket of smallest
 *             absolute value, ties to the lower edge id (Section 5.2 merge
 *             rule, generalised iteratively; Section 5.1 contraction;
 *             Section 4.2.1 inner product for two tables).
 * X_i is exact in 128-bit two's complement (wrapping mod 2^128), and the
 * estimate is the median over rows (Section 4.2.1; even d: mean of the two
 * middle values), converted to double with round-to-nearest-even.
 *   masks      host, n_subplans bitmasks
 *   row_est    device, n_subplans x d (may be NULL)
 *   est        device, n_subplans doubles
 *   flags      device, n_subplans int32 (COMPASS_FLAG_*)
 * Shapes: trees and trees plus one triangle take the specialised path
 * (message passing; the triangle by conditioning on one edge's bucket with
 * run-ordered sweeps).  Every other connected shape (longer cycles, several
 * cycles, two edges between one pair of tables, tables with more than 6
 * children) takes the generic contraction: the edges outside a spanning
 * tree are conditioned on their buckets (w^k assignments, each contracted
 * bottom-up), exact in the same 128-bit arithmetic, slower by about w per
 * conditioned edge.  Shapes beyond its bounds get COMPASS_FLAG_UNSUPPORTED
 * and do not fail the call.  When a sub-plan's values are not certified,
 * its estimate comes from an fp64 evaluation (COMPASS_FLAG_APPROX); that
 * evaluation runs on the device only for those sub-plans. */
compass_status compass_estimate(const compass_join_graph *g,
                                const uint64_t *masks, int32_t n_subplans,
                                compass_i128 *row_est, double *est,
                                int32_t *flags, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Sketch partitioning (Section 5.1): for a table that takes part in two
 * joins, the counters of each sketch row form a w1 x w2 matrix; the
 * estimate of the three-table chain through it combines the matrix with
 * the neighbours' one-dimensional sketches of the two joins.
 * --------------------------------------------------------------------- */

/* compass_sketch_build_2d -- one scan of the middle table: for every row
 * that satisfies the conjunction of `preds`, with join keys a (first) and
 * b (second), and for every sketch row i, adds xi1_i(a) * xi2_i(b) to
 * entry [h1_i(a)][h2_i(b)] of row i's matrix, where (h1_i, xi1_i) are the
 * functions of `first->seeds` row i and (h2_i, xi2_i) those of
 * `second->seeds` row i (the seeds of the two joins, shared with the
 * neighbours' sketches).  Adds the number of qualifying rows to
 * *n_selected.
 *   first, second  key column, key dtype and seeds (host, d x 6) of the two
 *                  joins; their `counters` fields are ignored
 *   d              1 .. 24
 *   w1, w2         1 .. 2^20 each, w1 * w2 <= 2^28
 *   counters       device, d x w1 x w2 row-major, int32 or int64
 *   other arguments as for compass_sketch_build.
 * The matrices exceed LDS at useful sizes: the updates are written as
 * records, counting-sorted by tile (2^r rows of one sketch row's matrix,
 * at most 32768 counters) and summed per tile in LDS, each tile written
 * once (rows of at most 1 GiB of records per pass).  Widths without such a
 * tiling (w2 > 32768, or more than 32768 tiles) take one device-scope
 * integer atomic per update.  Both are exact and order-independent. */
compass_status compass_sketch_build_2d(int64_t n_rows,
                                       const void *const *pred_cols,
                                       int32_t n_pred_cols,
                                       const compass_pred *preds,
                                       int32_t n_preds,
                                       const compass_sketch_spec *first,
                                       const compass_sketch_spec *second,
                                       int32_t d, int32_t w1, int32_t w2,
                                       int32_t counter_bits, int32_t accumulate,
                                       void *counters, int64_t *n_selected,
                                       hipStream_t stream);

/* compass_sketch_build_kd -- the partitioned sketch of a table that takes
 * part in k = 2 .. 4 joins (Section 5.1: a table with k joins has a k-D
 * tensor as its sketch): for every row that satisfies the conjunction of
 * `preds`, with join keys a_1 .. a_k, and every sketch row i, adds
 * prod_m xi_{m,i}(a_m) to entry [h_{1,i}(a_1)] .. [h_{k,i}(a_k)] of row i's
 * w_1 x .. x w_k tensor (row-major), (h_{m,i}, xi_{m,i}) being row i's
 * functions of joins[m].seeds.  k = 2 is compass_sketch_build_2d.
 *   joins     host array of k specs (key column, dtype, seeds d x 6; the
 *             counters fields are ignored)
 *   d         1 .. 48 / k
 *   w         host array of k widths, each 1 .. 2^20, product <= 2^28
 *   counters  device, d x w_1 x .. x w_k, int32 or int64
 * Joins 2 .. k form the second dimension of the binned build (their
 * indices flattened); other arguments, errors and exactness as for
 * compass_sketch_build_2d. */
compass_status compass_sketch_build_kd(int64_t n_rows,
                                       const void *const *pred_cols,
                                       int32_t n_pred_cols,
                                       const compass_pred *preds,
                                       int32_t n_preds,
                                       const compass_sketch_spec *joins,
                                       int32_t k, int32_t d, const int32_t *w,
                                       int32_t counter_bits, int32_t accumulate,
                                       void *counters, int64_t *n_selected,
                                       hipStream_t stream);

/* A tree of tables with partitioned sketches (Section 5.1): table t's
 * sketch has one dimension per incident edge, in increasing edge id, of
 * that edge's width; a table with one join has a d x w sketch, one with k
 * joins a d x w_e1 x .. x w_ek tensor (compass_sketch_build_kd, keys in
 * the same edge order; both sides of an edge share its seeds). */
typedef struct {
  int32_t n_tables;        /* 2 .. 64 */
  int32_t n_edges;         /* n_tables - 1 (a tree) */
  int32_t d;               /* 1 .. 32 */
  int32_t counter_bits;    /* 32 or 64, all tables */
  const int32_t *edge_u;   /* host, n_edges */
  const int32_t *edge_v;   /* host, n_edges */
  const int32_t *width;    /* host, n_edges: buckets of each join */
  const void *const *tensor;  /* host array of n_tables device pointers */
  const int64_t *n_selected;  /* device, n_tables: selected rows */
} compass_tensor_graph;

/* compass_estimate_partitioned -- the join size estimate of the whole tree
 * from partitioned sketches (Section 5.1): for each sketch row i,
 *   X_i = sum over a bucket j_e of every edge e of
 *         prod over tables t of T_t[i][j_e for the edges e at t],
 * exact in 128-bit two's complement (message passing from the leaves to
 * table 0); est = median over rows (even d: mean of the two middle
 * values), round-to-nearest-even; flags = COMPASS_FLAG_EXACT when the
 * product of the tables' selected rows is below 2^127 (it bounds |X_i|).
 *   row_est  device, d values (may be NULL); est, flags device, 1 each
 * E_GRAPH if the edges do not form a tree over the tables; E_UNSUPPORTED
 * for a table with more than 4 joins; E_ARG for a tensor above 2^28
 * entries per row. */
compass_status compass_estimate_partitioned(const compass_tensor_graph *g,
                                            compass_i128 *row_est, double *est,
                                            int32_t *flags, hipStream_t stream);

/* compass_estimate_chain3 -- the chain A join P join B (P joins A on its
 * first key and B on its second): for each sketch row i,
 *   X_i = sum over j1 < w1, j2 < w2 of A[i][j1] * P[i][j1][j2] * B[i][j2]
 * exact in 128-bit two's complement; est = median over rows (even d: mean
 * of the two middle values), round-to-nearest-even; flags =
 * COMPASS_FLAG_EXACT when n_A * n_P * n_B < 2^127 (|X_i| is below that
 * product).
 *   a  device, d x w1 (the first neighbour's sketch on the first join)
 *   p  device, d x w1 x w2 (compass_sketch_build_2d)
 *   b  device, d x w2 (the second neighbour's sketch on the second join)
 *   counter_bits  32 or 64, the same for all three
 *   d 1 .. 32; w1 1 .. 2^20; w2 1 .. 16384; w1 * w2 <= 2^28
 *   n_a, n_p, n_b device int64 selected rows of the three tables (each must
 *                 also bound its sketch rows' sums of absolute values)
 *   row_est  device, d values (may be NULL); est, flags device, 1 each */
compass_status compass_estimate_chain3(const void *a, const void *p,
                                       const void *b, int32_t counter_bits,
                                       int32_t d, int32_t w1, int32_t w2,
                                       const int64_t *n_a, const int64_t *n_p,
                                       const int64_t *n_b, compass_i128 *row_est,
                                       double *est, int32_t *flags,
                                       hipStream_t stream);

/* ------------------------------------------------------------------------
 * AGMS baseline (Section 4.1): r x b independent basic sketches per table,
 * each one counter; composed over every join the table takes part in.
 * --------------------------------------------------------------------- */

/* compass_agms_build -- one scan of one table for one query: for every row
 * that satisfies the conjunction of `preds`, basic sketch c = i * b + j
 * adds the product over the table's joins e of xi^e_c(key_e), where xi^e_c
 * is the +-1 variable of `joins[e].seeds` row c (a0..a3 of the degree-3
 * polynomial above; b0, b1 are not used).  Every basic sketch sees every
 * row: K = r * b sign evaluations per join per row.
 *   joins     host array of n_joins (1 .. 4) specs: key column, key dtype,
 *             seeds (host, r*b x 6); `counters` ignored.  Tables joined by
 *             a join must use that join's seeds.
 *   r, b      1 <= r <= 64, r * b <= 1024
 *   counters  device, r x b int64; overwritten (accumulate 0) or added to
 *   n_selected device int64, as for compass_sketch_build */
compass_status compass_agms_build(int64_t n_rows, const void *const *pred_cols,
                                  int32_t n_pred_cols, const compass_pred *preds,
                                  int32_t n_preds,
                                  const compass_sketch_spec *joins,
                                  int32_t n_joins, int32_t r, int32_t b,
                                  int32_t accumulate, int64_t *counters,
                                  int64_t *n_selected, hipStream_t stream);

/* compass_agms_estimate -- the query's estimate from its tables' AGMS
 * sketches: basic estimate (i, j) = product over the tables of counter
 * (i, j); row i's average = (exact 128-bit sum over j) / b, converted to
 * double with round-to-nearest-even then divided in IEEE arithmetic; est =
 * median of the r averages (even r: mean of the two middle ones); flag =
 * COMPASS_FLAG_EXACT when the product of the tables' selected counts is
 * below 2^127.
 *   sketches, n_selected  host arrays of n_tables (1 .. 16) device pointers
 *   row_sums  device, r values (may be NULL); est, flag device, 1 each */
compass_status compass_agms_estimate(const int64_t *const *sketches,
                                     const int64_t *const *n_selected,
                                     int32_t n_tables, int32_t r, int32_t b,
                                     compass_i128 *row_sums, double *est,
                                     int32_t *flag, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched build: the sketch builds of many tables (for instance every table
 * of hundreds of queries) as ONE persistent launch captured in a HIP graph.
 * Each job is exactly one compass_sketch_build call (same fields, same
 * result, bit for bit); a launch overwrites every job's counters and
 * n_selected (accumulate = 0).  Pointers in the jobs must stay valid for the
 * life of the plan; seeds and predicates are copied at creation.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_rows;
    const void *const *pred_cols;        /* host array of device columns */
    int32_t n_pred_cols;
    int32_t n_preds;
    const compass_pred *preds;           /* host */
    const compass_sketch_spec *sketches; /* host */
    int32_t n_sketches;
    int32_t d, w;
    int32_t reserved;
    int64_t *n_selected;                 /* device */
} compass_build_job;

/* Tile parameters of the persistent kernel.  Zero fields = autotune: every
 * candidate is timed on the batch itself (the plan's jobs run several times
 * during creation) and the winner is cached per (gfx arch, shape class) in
 * $COMPASS_AUTOTUNE_CACHE (default ~/.cache/compass_autotune.txt). */
typedef struct {
    int64_t rows_per_item;   /* table rows per work item */
    int32_t lds_budget;      /* bytes of partial counters per workgroup */
    int32_t blocks_per_cu;   /* persistent workgroups per compute unit */
} compass_tune;

typedef struct compass_batch_plan_s *compass_batch_plan;

/* Validates the jobs (as compass_sketch_build), builds the work-item list,
 * tunes, and captures "zero outputs + persistent kernel" into a graph.
 * Synchronous; runs on `stream` when autotuning.  Every kernel's LDS
 * (static + dynamic) is checked against what one workgroup may allocate on
 * the device (or a smaller COMPASS_LDS_LIMIT_BYTES) before anything runs:
 * E_UNSUPPORTED if one does not fit.  When the autotune winner cannot be
 * written to the cache file the call still succeeds and
 * compass_last_error() says why. */
compass_status compass_batch_plan_create(const compass_build_job *jobs,
                                         int32_t n_jobs, int32_t counter_bits,
                                         const compass_tune *tune,
                                         hipStream_t stream,
                                         compass_batch_plan *plan);
/* One hipGraphLaunch of the captured batch on `stream` (asynchronous). */
compass_status compass_batch_plan_launch(compass_batch_plan plan,
                                         hipStream_t stream);
/* The tile parameters in use, the number of work items and the grid size. */
compass_status compass_batch_plan_info(compass_batch_plan plan,
                                       compass_tune *tune, int32_t *n_items,
                                       int32_t *grid);
compass_status compass_batch_plan_destroy(compass_batch_plan plan);

/* ------------------------------------------------------------------------
 * Learned correction (a small MLP; not in the paper).  Maps sub-plan
 * features to y = ln(1 + max(raw, 0)) + net(x), raw = the median sketch
 * estimate, so the zero network returns the raw estimate (the fallback).
 * Layers n_in -> hidden (x n_hidden_layers, ReLU) -> 1; weights in fp32
 * (master + Adam state) and bfloat16 (read by the products); each layer
 * rounds its input activations to bfloat16 and accumulates in fp32.
 * Flat parameter layout, per layer: W (out x in, row-major) then b (out).
 * Training: loss = mean (y - target)^2, Adam (beta 0.9 / 0.999, eps 1e-8).
 * ------------------------------------------------------------------------ */
typedef struct compass_mlp_s *compass_mlp;

/* init: host array of compass_mlp_n_params() floats.  1 <= n_in, hidden
 * <= 64, 1 <= n_hidden_layers <= 7.  Synchronous. */
compass_status compass_mlp_create(int32_t n_in, int32_t hidden,
                                  int32_t n_hidden_layers, const float *init,
                                  compass_mlp *out);
int64_t compass_mlp_n_params(compass_mlp m);
/* Adam steps taken so far (the bias-correction count); with
 * compass_mlp_read (parameters, first and second moments) it is all a
 * checkpoint needs, and compass_mlp_write restores it. */
int64_t compass_mlp_adam_steps(compass_mlp m);
/* y[i] = base[i] + net(x[i]); x: device n x n_in fp32, base/y: device n. */
compass_status compass_mlp_forward(compass_mlp m, const float *x,
                                   const float *base, int32_t n, float *y,
                                   hipStream_t stream);
/* One Adam step on the mini-batch (x, base, target); *loss (device float)
 * receives the batch's mean squared error before the update.  lr = 0
 * computes loss and gradients without updating (and without advancing the
 * Adam step count). */
compass_status compass_mlp_train_step(compass_mlp m, const float *x,
                                      const float *base, const float *target,
                                      int32_t n, float lr, float *loss,
                                      hipStream_t stream);
/* An epoch of Adam steps without a host round trip per step: step k
 * trains on samples idx[k * batch .. (k + 1) * batch) (device int32 row
 * indices into x, base and target, e.g. a permutation) and writes its
 * batch's mean squared error before the update to losses[k] (device,
 * n_batches floats).  The same arithmetic as n_batches calls of
 * compass_mlp_train_step on the gathered rows.  lr > 0.  The indices are
 * not checked: each must be a row of x, base and target. */
compass_status compass_mlp_train_epoch(compass_mlp m, const float *x,
                                       const float *base, const float *target,
                                       const int32_t *idx, int32_t n_batches,
                                       int32_t batch, float lr, float *losses,
                                       hipStream_t stream);
/* Copies to host (synchronous): what = 0 parameters, 1 last gradients,
 * 2 Adam first moments, 3 Adam second moments. */
compass_status compass_mlp_read(compass_mlp m, int32_t what, float *host_out);
/* Replaces parameters (and optionally Adam state and step count). */
compass_status compass_mlp_write(compass_mlp m, const float *params,
                                 const float *adam_m, const float *adam_v,
                                 int64_t step);
compass_status compass_mlp_destroy(compass_mlp m);
/* Features of n sub-plans of one query (device in, device out): x = n x 20
 * floats: 7 order statistics (positions round(k (d-1) / 6), k = 0..6) of
 * sign(X) ln(1 + |X|) over the sorted row estimates; log2(1 + n_sel) of the
 * sub-plan's tables, descending, first 8, zero padded; 5 shape statistics
 * of the sub-plan over the query's join graph (edge_u/edge_v: host arrays
 * of n_edges <= 64 edges): number of tables, number of edges between them,
 * diameter (in edges), largest degree, independent cycles (edges - tables
 * + 1).  base = ln(1 + max(est, 0)). */
compass_status compass_mlp_features(const compass_i128 *row_est, int32_t d,
                                    const double *est, const uint64_t *masks,
                                    const int64_t *n_selected,
                                    int32_t n_tables, int32_t n_edges,
                                    const int32_t *edge_u, const int32_t *edge_v,
                                    int32_t n, float *x, float *base,
                                    hipStream_t stream);

/* Join order enumeration (Section 6, Algorithm 1), on the host: DFS over
 * the join graph building left-deep orders without cross products; sources
 * in increasing f(v) = alpha card(v)/max card + beta deg(v)/max deg;
 * extensions in increasing estimate of the extended sub-plan; a branch is
 * pruned when its running cost (sum of the estimates of all its prefixes)
 * exceeds the best complete cost; at most max_plans complete plans per
 * source (max_plans <= 0: exhaustive).  masks/est: host arrays of the
 * estimates of (at least) every connected sub-plan the search visits, e.g.
 * compass_estimate's output copied back; card: host, per table (the
 * single-table estimates).  Outputs: the best order (n_tables ids), its
 * cost and the number of complete plans reached. */
compass_status compass_enumerate(int32_t n_tables, int32_t n_edges,
                                 const int32_t *edge_u, const int32_t *edge_v,
                                 const uint64_t *masks, const double *est,
                                 int32_t n_masks, const double *card,
                                 int32_t max_plans, double alpha, double beta,
                                 int32_t *order_out, double *cost_out,
                                 int64_t *n_plans_out);

/* compass_enumerate_greedy -- the greedy variant, the paper's default
 * (Section 7.1, defined in Section 7.2.8): one source only, the smaller
 * table (by card; ties to the lower id) of the two-table sub-plan with the
 * smallest estimate (ties to the lower mask), then the left-deep order
 * grows by the adjacent table whose extended sub-plan has the smallest
 * estimate (ties to the lower id), without backtracking.  Same inputs and
 * outputs as compass_enumerate; *cost_out = sum of the estimates of every
 * prefix.  (full-greedy, limit-10 and exhaustive are compass_enumerate with
 * max_plans 1, 10 and 0.) */
compass_status compass_enumerate_greedy(int32_t n_tables, int32_t n_edges,
                                        const int32_t *edge_u,
                                        const int32_t *edge_v,
                                        const uint64_t *masks, const double *est,
                                        int32_t n_masks, const double *card,
                                        int32_t *order_out, double *cost_out);

/* Kernel timing for measurement: while enabled, the library records a pair
 * of HIP events on the launch stream around each kernel launch it makes.
 * compass_profile_take(name) waits for the recorded events of kernel `name`
 * ("scan_sketch", "slab_reduce", "wide_compact", "wide_hash", "fill_zero",
 * "sort_rows", "node", "tri_order", "tri_lane", "finish", "scan2d",
 * "chain3", "agms_build", "agms_estimate", "generic"),
 * returns their count and summed elapsed milliseconds, and forgets them.
 * compass_profile_select(names) restricts the recording to the kernels in
 * the comma-separated list `names` (NULL or "": every kernel), so that a
 * timed region pays for the events of the kernels it measures only. */
compass_status compass_profile_enable(int32_t on);
compass_status compass_profile_select(const char *names);
compass_status compass_profile_take(const char *name, int64_t *count,
                                    double *total_ms);

/* Frees the library's cached scratch memory on the current device. */
compass_status compass_release(void);

/* Message of the last failure on this thread ("" if none). */
const char *compass_last_error(void);

/* Library version string. */
const char *compass_version(void);

#ifdef __cplusplus
}
#endif
#endif /* COMPASS_H */
