/*
 * lmfao.h — C ABI of the MI355X (gfx950) aggregate-batch engine.
 *
 * The engine evaluates a batch of group-by aggregate queries over the natural
 * join of an acyclic database (paper, Section 1.1 problem statement and
 * Section 2, equation (1)):
 *
 *     Q(F_1..F_f; alpha_1..alpha_l) += R_1(w_1), ..., R_m(w_m)
 *
 * where each alpha_i = sum_j c_j * prod_k X_jk is a sum of products of
 * identity functions of continuous attributes (the empty product is the
 * constant 1), a query may carry a conjunction of Kronecker-delta factors
 * 1[X op t] (Section 1.1) that restricts which join tuples it sums, and every
 * group-by attribute is categorical (cell = code) or continuous with sorted
 * thresholds t_0 < ... < t_{T-1} (cell = #{k : t_k < x}, the buckets of the
 * CART splits X <= t of Section 2).  COUNT is reported for every cell.
 *
 * Evaluation follows Section 3: queries are decomposed into directional views
 * along the join tree towards the root (Section 3.2), identical and
 * same-group-by views are merged (Section 3.4), views leaving the same
 * relation form a view group evaluated by one multi-output scan over that
 * relation (Section 3.5), and independent groups of one tree level run
 * together (Section 1.2, parallelization).
 *
 * Supported join trees: every edge joins its two relations on exactly one
 * shared int32 attribute, which is a unique key of the child relation (the
 * star and snowflake schemas of the paper's datasets), or, declared
 * LMFAO_KEY_MANY in the child, a join attribute whose values may repeat (a
 * many-to-many join, where the join is larger than its relations: Section 4,
 * Yelp).  Keys lie in [0, domain) of the key column.  A fact row whose key
 * has no matching child row does not join (natural-join semantics).
 *
 * Many-to-many children are evaluated by count-weighted views (Section 3.2:
 * a view of a child subtree carries, per key, the aggregates of that subtree
 * the batch needs): per key the child's view holds its row count, the mean
 * of each of its continuous attributes, and the within-key scatter of every
 * pair of them; the root scan weights each of its rows by the product of its
 * children's counts, and the covariance entries of two attributes of one
 * such child are completed from that child's scatter weighted by how often
 * the root reaches each key.  A query that groups by, filters on, or (when
 * grouped or filtered, or in a product of three or four factors) multiplies
 * attributes of such a child is evaluated at that child as its root (see
 * lmfao_plan_opts.root_policy): a view from the tree root keyed by the join
 * key, each fact row weighted by the counts of the other children, joined
 * with the child's rows.  Supported: many-to-many children that are leaves
 * of the root; a query touching two of them that way, a grouped sum of a
 * product of two attributes of one of them in a query evaluated elsewhere,
 * and a BF16 covariance block with one, are UNSUPPORTED (the covariance
 * block runs in FP32).
 *
 * Conventions
 *  - Every function returns lmfao_status: LMFAO_OK (0) or a negative error;
 *    lmfao_last_error() then describes it.  No C++ exception crosses the ABI.
 *  - Column data and result/workspace buffers are DEVICE pointers owned by
 *    the caller, who keeps them alive until lmfao_sync() returns.  The
 *    library never allocates device memory itself.
 *  - Column-major relations: each column is a contiguous array of n_rows
 *    elements (int32 or float32).
 *  - Call order: create -> add_relation* -> set_join_tree -> add_query* ->
 *    plan -> workspace_size/result_size -> bind -> (execute -> sync)* ->
 *    destroy.  Calls out of order fail with LMFAO_ERR_STATE.
 *  - One context per host thread; a context is not thread-safe.
 */
#ifndef LMFAO_H
#define LMFAO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lmfao_status;

enum {
    LMFAO_OK = 0,
    LMFAO_ERR_INVALID_ARG = -1,  /* null pointer, bad enum, size out of range */
    LMFAO_ERR_NOT_ACYCLIC = -2,  /* edges do not form a tree, or running intersection fails */
    LMFAO_ERR_UNKNOWN_ATTR = -3, /* query names an attribute no relation holds */
    LMFAO_ERR_TYPE = -4,         /* attribute kind/type does not fit its use */
    LMFAO_ERR_DOMAIN = -5,       /* categorical code or key outside its domain (device check) */
    LMFAO_ERR_TOO_LARGE = -6,    /* more features/filters/cells than the engine supports */
    LMFAO_ERR_WORKSPACE = -7,    /* bound buffer smaller than required */
    LMFAO_ERR_STATE = -8,        /* call out of order */
    LMFAO_ERR_HIP = -9,          /* a HIP runtime call failed */
    LMFAO_ERR_UNSUPPORTED = -10  /* join shape outside the supported class (e.g. duplicate child key) */
};

/* ---- context ------------------------------------------------------------ */

typedef struct lmfao_ctx lmfao_ctx;

/* Create a context bound to HIP device `hip_device`.  *out receives the
 * context (NULL on failure). */
lmfao_status lmfao_create(lmfao_ctx **out, int32_t hip_device);

/* Release host-side state.  Device memory belongs to the caller. */
void lmfao_destroy(lmfao_ctx *ctx);

/* Human-readable description of the last error of this context ("" if none).
 * The string is owned by the context and valid until the next call. */
const char *lmfao_last_error(const lmfao_ctx *ctx);

/* ---- relations (Section 2, query language: relations R_1..R_m) --------- */

enum { LMFAO_I32 = 0, LMFAO_F32 = 1 };                 /* dtype */
enum { LMFAO_KEY = 0, LMFAO_CONT = 1, LMFAO_CAT = 2, LMFAO_KEY_MANY = 3 };  /* kind  */

typedef struct {
    const char *attr;   /* attribute name; equal names join (natural join) */
    int32_t dtype;      /* LMFAO_I32 for KEY/CAT, LMFAO_F32 for CONT */
    int32_t kind;       /* LMFAO_KEY, LMFAO_CONT, LMFAO_CAT, or LMFAO_KEY_MANY: the join attribute
                           of a child relation whose values may repeat (a many-to-many join) */
    int32_t domain;     /* KEY: values in [0, domain); CAT: codes in [0, domain); CONT: ignored */
    const void *data;   /* device pointer to n_rows elements (borrowed) */
} lmfao_col;

/* Register relation `name` with `n_cols` columns of `n_rows` rows each.
 * *rel_id receives its index (0, 1, ... in call order).  Column pointers are
 * borrowed; names are copied. */
lmfao_status lmfao_add_relation(lmfao_ctx *ctx, const char *name, int64_t n_rows, int32_t n_cols,
                                const lmfao_col *cols, int32_t *rel_id);

/* Join tree (Section 3.1): `edges` holds n_edges pairs {parent, child} of
 * relation ids; n_edges must be (number of relations - 1) and the edges must
 * form a tree.  Each edge joins on the single attribute the two relations
 * share, which must be a KEY of the child.  Returns LMFAO_ERR_NOT_ACYCLIC if
 * the edges do not form a tree or an attribute's holders are not connected
 * in it (running intersection). */
lmfao_status lmfao_set_join_tree(lmfao_ctx *ctx, int32_t n_edges, const int32_t *edges);

/* ---- queries (Section 2, equation (1)) ---------------------------------- */

enum { LMFAO_LE = 0, LMFAO_LT = 1, LMFAO_GE = 2, LMFAO_GT = 3, LMFAO_EQ = 4, LMFAO_NE = 5 };

typedef struct {
    const char *attr;          /* CAT attribute, or CONT attribute with thresholds */
    int32_t n_thresholds;      /* 0 for CAT; else number of sorted fp32 thresholds */
    const float *thresholds;   /* host pointer, strictly increasing; copied */
} lmfao_groupby;

typedef struct {
    const char *attr;          /* factor 1[attr op value] */
    int32_t op;                /* LMFAO_LE .. LMFAO_NE */
    double value;              /* CONT: compared in fp32 with the constant rounded to fp32.
                                  KEY/CAT: compared exactly with the real constant, which need
                                  not be an integer (c >= 2.5 holds for c >= 3; c = 2.5 never).
                                  NaN is INVALID_ARG. */
} lmfao_pred;

typedef struct {
    double coeff;              /* c_j */
    int32_t n_factors;         /* 0 to 4 identity factors (degree-2 polynomial regression needs
                                  products of up to four attributes, Section 2) */
    const char *factors[4];    /* CONT attribute names */
} lmfao_term;

typedef struct {
    int32_t n_terms;           /* alpha = sum of terms */
    const lmfao_term *terms;
} lmfao_agg;

typedef struct {
    int32_t n_groupby;
    const lmfao_groupby *groupby;
    int32_t n_preds;           /* WHERE: conjunction of all predicates */
    const lmfao_pred *preds;
    int32_t n_aggs;
    const lmfao_agg *aggs;
} lmfao_query;

/* Add one query; *qid receives its index.  All descriptor memory is copied.
 * Errors: UNKNOWN_ATTR, TYPE (e.g. a factor that is not CONT), TOO_LARGE
 * (more than 2^31 cells, or a term of more than four factors).  A term of
 * three or four factors is evaluated as the product of two staged values,
 * one of them (or both) the product of two attributes formed per row by the
 * root scan: f1 * (f2 f3) and (f1 f2) * (f3 f4), factors in staged order; at
 * most 63 attributes and such products together. */
lmfao_status lmfao_add_query(lmfao_ctx *ctx, const lmfao_query *q, int32_t *qid);

/* ---- planning ------------------------------------------------------------ */

enum { LMFAO_FP32 = 0, LMFAO_BF16X3 = 1, LMFAO_BF16X4 = 2, LMFAO_BF16X6 = 3 }; /* covariance-block arithmetic */
enum { LMFAO_PLAIN = 0, LMFAO_BATCHED = 1 };                        /* schedule */
enum { LMFAO_HEURISTIC = 0, LMFAO_AUTOTUNE = 1, LMFAO_LEARNED = 2 }; /* tile/grouping choice */
enum { LMFAO_ROOT_TREE = 0, LMFAO_ROOT_FIND = 1 };                  /* root of each query */

typedef struct {
    int32_t precision;     /* FP32: fp32 FMAs; BF16X3: bf16 hi+lo split on MFMA (hi*hi+hi*lo+lo*hi),
                              fp32 accumulate; BF16X4 adds lo*lo; BF16X6: three bf16 pieces
                              x = hi+mid+lo (hi*hi+hi*mid+mid*hi+mid*mid+hi*lo+lo*hi), which keeps every
                              term down to 2^-16 of a product (about 1e-7 per product; BF16X3 and
                              BF16X4 drop up to 3 and 2 times 2^-16, which a sum dominated by one
                              repeated value keeps).  Cross-block merge is fp64 in all. */
    int32_t schedule;      /* PLAIN: one launch per view; BATCHED: one fused launch per tree level,
                              captured in a hipGraph and replayed */
    int32_t planner;       /* HEURISTIC: fixed rules; AUTOTUNE: time every candidate tile config
                              on the device during lmfao_plan_tune; LEARNED: cost-model prediction
                              (falls back to HEURISTIC without a model) */
    int32_t block_rows;    /* reserved, must be 0: rows per workgroup follow from grid_blocks */
    int32_t grid_blocks;   /* override: workgroups of the fact scan (0 = planner's choice) */
    int32_t gram_block;    /* override: FP32 register block edge 2/4/6/8 (0 = planner's choice);
                              other values are INVALID_ARG */
    const char *cost_model;/* LEARNED: path of the weights file written by lmfao_train_cost_model */
    int32_t scan_every_table; /* 0: a grouped table whose key is another table's key (same WHERE
                              filter) with one component left out is not updated by the fact
                              scan but summed from that table's cells afterwards (its sums are
                              added to the finer table's); chains of such tables are summed
                              longest key first.  1: the fact scan updates every table.  Other
                              values are INVALID_ARG.  Results agree up to the order of fp64
                              additions; counts are identical. */
    int32_t no_row_codes;  /* 0: filtered tables over several LDS partitions are updated from per-row
                              codes when they qualify (see lmfao_stats.code_scan); 1: the root scan
                              updates them itself, once per partition.  Other values are INVALID_ARG. */
    int32_t no_hist;       /* 0: unfiltered COUNT-only tables that the root scan cannot keep in one LDS
                              partition are counted by the count-table scan (see lmfao_stats.hist_scan);
                              1: the root scan updates them.  Other values are INVALID_ARG. */
    int32_t root_policy;   /* Where each query is evaluated (Section 3.3: each aggregate to its own
                              root).  ROOT_TREE: at the join tree's root.  ROOT_FIND: the paper's
                              root assignment: every grouped or filtered query gives each relation
                              the fraction of its group-by attributes that relation holds (1/m to
                              every relation when it has none); relations are taken by decreasing
                              total weight, ties to the larger relation, and each becomes the root
                              of every query not yet assigned that holds a group-by attribute in it
                              (or has none).  Readings for the device: the ungrouped, unfiltered
                              sums (the covariance block) stay at the tree root, where one fused scan
                              computes them, and take no part in the weights; a relation below a
                              child of the tree root passes its queries to that child; a query whose
                              view towards its root would exceed 2^24 cells, or group by more than
                              three attributes outside the root's subtree, stays at the tree root.
                              A query at root R != tree root is evaluated by a view flowing from the
                              tree root towards R (Section 3.2, directional views): a grouped table
                              of the root scan keyed by the join key of R and the query's group-by
                              attributes outside R's subtree, then a scan of R's keys (or, for a
                              many-to-many R, of R's rows) that joins it with R's side of the query.
                              Under both policies, a query that groups by, filters on or multiplies
                              two attributes of one many-to-many child is evaluated at that child.
                              Other values are INVALID_ARG. */
} lmfao_plan_opts;

/* Build the evaluation plan for all queries added so far. */
lmfao_status lmfao_plan(lmfao_ctx *ctx, const lmfao_plan_opts *opts);

/* Plan statistics, the analogue of the paper's Table 2. */
typedef struct {
    int32_t app_aggregates;      /* A: aggregates the queries ask for (incl. one COUNT per query) */
    int32_t inter_aggregates;    /* I: additional per-key aggregates carried by child views */
    int32_t views;               /* V: views after merging */
    int32_t groups;              /* G: view groups */
    int32_t levels;              /* dependency levels of view groups */
    int32_t features;            /* continuous features in the covariance block (incl. constant 1) */
    int32_t filters;             /* distinct WHERE conjunctions */
    int32_t tables;              /* grouped result tables */
    int64_t table_cells;         /* cells over all grouped tables */
    int32_t launches;            /* kernel launches per execution */
    int32_t block_rows;          /* fact rows per workgroup of the root scan (a multiple of 64 * waves) */
    int32_t grid_blocks;         /* workgroups of the root scan */
    int32_t gram_block;          /* FP32: register block edge; BF16: padded feature count */
    int32_t lds_tables;          /* grouped tables: 0 global atomics, 1 greedy LDS, 2 partitioned LDS (the root
                                    scan rescans per partition), 3 partitioned LDS with per-row codes and the
                                    count-table scan where they apply (the heuristic choice) */
    int32_t waves;               /* waves per workgroup of the root scan */
    int32_t nbuf;                /* staging buffers per wave (2: next tile copied during this one) */
    int32_t lds_bytes;           /* dynamic LDS of the root scan workgroup */
    int32_t dedicated_scan;      /* 1: the covariance-only root scan runs on the dedicated BF16 kernel */
    int32_t derived_tables;      /* grouped tables summed from a finer table after the scan */
    int32_t strided_families;    /* filtered table families whose LDS tables are addressed from the
                                    filter's rank instead of per-table descriptors */
    int32_t code_scan;           /* 1: filtered tables (at most 4 sums each) over several LDS partitions;
                                    the root scan writes each row's filter mask, key cells and summed
                                    feature values once (4 bytes per column and row of workspace, at
                                    most 16 GiB) and a code scan per partition updates the tables */
    int32_t hist_scan;           /* 1: unfiltered COUNT-only tables (pairwise counts, Section 2, equation
                                    (7)) beyond the root scan's LDS are counted apart: the root scan writes
                                    each row's group-by component values once as 16-bit codes (2 bytes per
                                    component and row of workspace, at most 16 GiB), and the count-table
                                    scan counts them into LDS slices of the tables, one partition of
                                    slices per grid row, adding its cells to the global u64 counts */
    int32_t hist_parts;          /* LDS partitions of the count-table scan */
    int32_t target_queries;      /* queries evaluated at a root other than the join tree's root (see
                                    lmfao_plan_opts.root_policy) */
} lmfao_stats;

lmfao_status lmfao_plan_stats(const lmfao_ctx *ctx, lmfao_stats *stats);

/* Relation at which query `qid` is evaluated (its root, Section 3.3), after
 * lmfao_plan.  Errors: STATE before planning, INVALID_ARG for a bad qid. */
lmfao_status lmfao_query_root(const lmfao_ctx *ctx, int32_t qid, int32_t *rel);

/* Root assignment chosen by measurement (Section 3.3): plans the batch with
 * every query at the join tree's root and with the paper's root assignment
 * (LMFAO_ROOT_TREE, LMFAO_ROOT_FIND of lmfao_plan_opts.root_policy), each with
 * the heuristic tile configuration, times `reps` whole executions of each on
 * `hip_stream` (a plan that needs more workspace or result memory than is
 * bound, or that puts no query elsewhere, is not timed), keeps the faster,
 * executes it once and stores its policy in *policy.  When the kept plan
 * needs more memory than is bound, the context is left planned and unbound:
 * query the sizes and bind again.  Errors: INVALID_ARG for reps below 1;
 * STATE before lmfao_bind. */
lmfao_status lmfao_choose_root(lmfao_ctx *ctx, void *hip_stream, int32_t reps, int32_t *policy);

/* ---- memory -------------------------------------------------------------- */

/* Device scratch the plan needs (views, partials, tables, descriptors). */
lmfao_status lmfao_workspace_size(const lmfao_ctx *ctx, size_t *bytes);

/* Size of the result arena and the layout of query `qid` inside it:
 * counts at byte offset *counts_off (uint64[n_cells]); sums at byte offset
 * *sums_off (double[n_cells * n_sums], sums[cell * n_sums + i] = alpha_i).
 * Cells are dense over the product of the group-by domains, first group-by
 * most significant. */
lmfao_status lmfao_result_size(const lmfao_ctx *ctx, size_t *bytes);
lmfao_status lmfao_result_layout(const lmfao_ctx *ctx, int32_t qid, int64_t *n_cells, int32_t *n_sums,
                                 size_t *counts_off, size_t *sums_off);

/* Bind caller-allocated device buffers (256-byte aligned) of at least the
 * reported sizes.  Errors: WORKSPACE (too small or misaligned). */
lmfao_status lmfao_bind(lmfao_ctx *ctx, void *workspace, size_t ws_bytes, void *results, size_t res_bytes);

/* Bind without allocating: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The workspace is the library's own scratch array, a static
 * device array of 64 MiB that every GPU the library runs on holds until the
 * process ends; `results` (device memory of at least lmfao_result_size()
 * bytes, 8-byte aligned) is still the caller's.  Nothing is allocated: the
 * descriptors are copied into the array and every execution clears what must
 * start at zero.  Errors: WORKSPACE when the plan needs more than 64 MiB of
 * workspace (lmfao_workspace_size tells) or `results` is too small, HIP when
 * the array cannot be looked up on the context's device.  All contexts on one
 * GPU share its array: binding another context to it (here, or through
 * lmfao_select_candidate / lmfao_autotune re-binding) overwrites this
 * context's descriptors, after which lmfao_execute, lmfao_time_root_group,
 * lmfao_autotune and the learned choices return STATE until this context is
 * bound again; executions of two contexts that overlap in time on one GPU
 * race on the array.  Results equal those of lmfao_bind with a caller's
 * workspace (the same plan and kernels). */
lmfao_status lmfao_bind_scratch(lmfao_ctx *ctx, void *results, size_t res_bytes);

/* ---- execution ----------------------------------------------------------- */

/* Enqueue one evaluation of the whole batch on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  Asynchronous: results are valid after
 * lmfao_sync().  With LMFAO_BATCHED the launches are captured in a hipGraph
 * on the first call and replayed afterwards. */
lmfao_status lmfao_execute(lmfao_ctx *ctx, void *hip_stream);

/* Wait for the last execution and surface device-side errors: DOMAIN for a
 * categorical code or key outside its domain, UNSUPPORTED for a duplicate
 * child key, HIP for runtime failures. */
lmfao_status lmfao_sync(lmfao_ctx *ctx);

/* Time the fact-scan view group alone: runs it `reps` times after `warmup`
 * runs on `hip_stream` and stores the mean milliseconds per run in *ms
 * (hipEvents on that stream).  The views of lower levels must be current
 * (call after one lmfao_execute). */
lmfao_status lmfao_time_root_group(lmfao_ctx *ctx, void *hip_stream, int32_t warmup, int32_t reps, double *ms);

/* ---- tile choice: exhaustive autotuner and learned cost model ------------ */

/* Number of candidate tile configurations of the current plan, and the
 * candidate `i` as {waves per workgroup, staging buffers per wave, workgroups,
 * fp32 register block edge (0 for bf16), table placement policy (as
 * lmfao_stats.lds_tables)}.  Candidates vary the tile configuration and the
 * grouping of tables: all global, greedy LDS, LDS partitions rescanned by the
 * root scan, or LDS partitions fed by per-row codes or the count-table scan. */
lmfao_status lmfao_candidates(const lmfao_ctx *ctx, int32_t *n);
lmfao_status lmfao_candidate(const lmfao_ctx *ctx, int32_t i, int32_t cfg[5]);

/* Feature vector of the root view group under candidate `i` (input of the
 * cost model): LMFAO_N_FEATURES floats.  Feature 2 is the number of rounds
 * of workgroups the root scan takes under the candidate (its workgroups over
 * the workgroups the chip holds at once), found by planning the candidate on
 * the side; the context is left as it was. */
#define LMFAO_N_FEATURES 16
lmfao_status lmfao_candidate_features(const lmfao_ctx *ctx, int32_t i, float *features);

/* Re-plan with candidate `i` as the tile configuration (must be bound again). */
lmfao_status lmfao_select_candidate(lmfao_ctx *ctx, int32_t i);

/* Exhaustive autotuner: time every candidate (needs bound buffers), append
 * one line per candidate to the timing file `timing_db` (16 features, the 5
 * configuration values of lmfao_candidate, milliseconds; may be NULL),
 * select the fastest and execute it once on `hip_stream` (so that
 * lmfao_time_root_group can follow).  *best receives its index. */
lmfao_status lmfao_autotune(lmfao_ctx *ctx, void *hip_stream, const char *timing_db, int32_t reps, int32_t *best);

/* Learned choice: score every candidate with the cost model in `weights`
 * (inference runs on the device in the workspace), select the lowest
 * predicted time, execute it once on `hip_stream`, and store its index in
 * *best.  Keeps the heuristic configuration (and returns LMFAO_OK with
 * *best = -1) if the model is missing or predicts a non-finite time.  When
 * the chosen configuration needs more workspace or result memory than is
 * bound, it is selected but not executed and the context is left unbound:
 * query the sizes and bind again before executing. */
lmfao_status lmfao_choose_learned(lmfao_ctx *ctx, const char *weights, void *hip_stream, int32_t *best);

/* Learned choice judged by measurement: rank every candidate with the cost
 * model as lmfao_choose_learned does, then time the configuration in place
 * and the `top_k` best-ranked candidates on `hip_stream` as lmfao_autotune
 * does (`reps` timed runs each), select the fastest, execute it once and
 * store its candidate index in *best (-1 when the configuration in place
 * stays).  A candidate replaces the configuration in place only when it is
 * more than 2% faster (the run-to-run spread of such timings).  The model
 * prunes the search; the timing decides, so the result is never slower than
 * the configuration in place beyond timing noise.  Same
 * fallback as lmfao_choose_learned (configuration kept, *best = -1, LMFAO_OK)
 * when the model is missing or predicts a non-finite time; INVALID_ARG for
 * top_k or reps below 1; STATE before lmfao_bind. */
lmfao_status lmfao_choose_learned_verified(lmfao_ctx *ctx, const char *weights, void *hip_stream, int32_t top_k,
                                           int32_t reps, int32_t *best);

/* ---- unit throughput probes (roofline peaks) ----------------------------- */

enum {
    LMFAO_PEAK_READ = 0,          /* streaming read of the buffer, 16 bytes per lane per load */
    LMFAO_PEAK_LDS_U32 = 1,       /* LDS u32 atomic adds at random addresses of a 32K-word table */
    LMFAO_PEAK_LDS_U32_SPREAD = 2,/* LDS u32 atomic adds, the 64 lanes of a wave on distinct banks */
    LMFAO_PEAK_LDS_F64 = 3,       /* LDS fp64 atomic adds at random addresses of a 16K-cell table */
    LMFAO_PEAK_GLOBAL_U64 = 4     /* device-scope u64 atomic adds at random cells of the buffer */
};

/* Time one probe launch (4 workgroups of 1024 threads per CU; for READ,
 * `iters` passes over the buffer) on `hip_stream` of the current device with
 * HIP events: *ms receives the milliseconds and *units the bytes read (READ)
 * or atomic adds issued (the others), so *units / *ms is the unit's rate.
 * Each thread issues `iters` atomics.  `buf` is caller-owned device memory:
 * the data to read, the u64 counters to add to (GLOBAL_U64; its contents are
 * changed), or room for one 4-byte result per workgroup (LDS probes; READ
 * also writes those results at its start and reads the rest).  Errors:
 * INVALID_ARG for a bad kind, iters < 1 or null outputs; WORKSPACE when the
 * buffer is too small; HIP on a runtime failure.  A measurement aid: the
 * engine's entry points do not use it. */
lmfao_status lmfao_measure_peak(int32_t kind, void *buf, size_t buf_bytes, int32_t iters, void *hip_stream,
                                double *ms, double *units);

/* ---- application loops on the device (Section 2) ------------------------ */

/* Ridge linear regression by batch gradient descent over the non-centred
 * covariance matrix (Section 2, linear regression): `cov` is a device array of
 * n x n doubles, row-major and symmetric, over the vector [1, X_1, ...]
 * (cov[0] = |D|, the count), `label` (1..n-1) the index of the response,
 * whose coefficient is fixed at -1.  Minimises
 *     J = 1/(2|D|) sum (theta . X)^2 + lambda/2 |theta_free|^2
 * with Barzilai-Borwein step sizes (the first 1/(trace/|D| + lambda)) until the
 * gradient norm is at most tol times its first value or max_iters steps ran,
 * all in one launch on `hip_stream`.  Writes theta[n] (device; -1 at the label)
 * and info[3] (device: J, steps taken, final gradient norm).  n <= 64, else
 * INVALID_ARG, as for a label outside 1..n-1, lambda < 0 or tol < 0. */
lmfao_status lmfao_ridge_bgd(const double *cov, int32_t n, int32_t label, double lambda, int32_t max_iters,
                             double tol, double *theta, double *info, void *hip_stream);

/* Mutual information of attribute pairs (Section 2, equation (7)) from their
 * pairwise COUNT GROUP BY tables: tables[p] (a device array of device pointers)
 * points at dom_a x dom_b u64 counts, row-major, with doms[2p], doms[2p+1]
 * (device int32); mi[p] (device) receives sum over nonzero cells of
 * delta/alpha * log(alpha * delta / (beta * gamma)), alpha the total and
 * beta, gamma the row and column sums (natural log; 0 for an empty table).
 * max_dom bounds every domain (at most 2048, else TOO_LARGE). */
lmfao_status lmfao_mutual_information(const unsigned long long *const *tables, const int32_t *doms, int32_t n_pairs,
                                      int32_t max_dom, double *mi, void *hip_stream);

/* Chow-Liu tree over n attributes (2..64, else INVALID_ARG / TOO_LARGE):
 * `mi` is a device n x n symmetric array of mutual informations; pairs
 * (i < j) are taken by decreasing value (equal values: lower pair index i, j
 * in row-major order first) when they join two components.  Writes
 * edges[2 * (n - 1)] (device int32 pairs i, j in the order taken) and
 * total[1] (device: the sum of their mutual informations). */
lmfao_status lmfao_chow_liu(const double *mi, int32_t n, int32_t *edges, double *total, void *hip_stream);

enum { LMFAO_SPLIT_VARIANCE = 0, LMFAO_SPLIT_GINI = 1 };

typedef struct {
    const uint64_t *counts;   /* device: VARIANCE [n_cells]; GINI [n_labels][n_cells] */
    const double *sums;       /* device, VARIANCE only: cell c's SUM(y) at sums[c * sum_stride],
                                 SUM(y^2) at sums[c * sum_stride + 1] */
    int32_t sum_stride;
    int32_t n_cells;          /* buckets (thresholds + 1) or categories of the split attribute */
    int32_t categorical;      /* 0: split X <= t_c puts buckets 0..c left; 1: split X = c puts cell c left */
    int32_t node;             /* tree node (0..n_nodes-1) these histograms belong to */
} lmfao_split_input;

typedef struct {
    double cost;              /* lowest cost of the node's splits */
    int32_t input;            /* its input (index into the inputs array), -1 if the node has none */
    int32_t cell;             /* its threshold index (continuous) or category (categorical) */
    int32_t pad;
    int32_t pad2;
} lmfao_split_result;

/* Best split of every node of a decision-tree level (Section 2, decision
 * trees) from per-(node, attribute) histograms, one workgroup per node:
 * VARIANCE (regression trees): cost = sum y^2 - (sum y)^2 / n of both sides;
 * GINI (classification trees, n_labels <= 16): cost = n (1 - sum_k p_k^2) of
 * both sides.  Splits with an empty side are skipped; the lowest (cost,
 * input, cell) wins.  `inputs` and `out[n_nodes]` are device arrays. */
lmfao_status lmfao_best_splits(const lmfao_split_input *inputs, int32_t n_inputs, int32_t n_nodes, int32_t criterion,
                               int32_t n_labels, lmfao_split_result *out, void *hip_stream);

/* ---- training the cost model --------------------------------------------- */

typedef struct {
    int32_t hidden;     /* hidden units per layer (1..1024; see lmfao_mlp_param_count) */
    int32_t epochs;     /* full-batch Adam steps (1..16384) */
    float lr;           /* Adam step size */
    int32_t pad;
    uint64_t seed;      /* seed of the He-style initialisation */
} lmfao_train_opts;

/* Device workspace (bytes) lmfao_train_cost_model needs for the timing file
 * `timing_db` (the lines lmfao_autotune appends) and `hidden` units, with room
 * for up to 16384 epochs' losses.  INVALID_ARG for an unreadable or malformed
 * file. */
lmfao_status lmfao_train_workspace_size(const char *timing_db, int32_t hidden, size_t *bytes);

/* Train the cost model of lmfao_choose_learned on the timings in `timing_db`
 * and write its weights file `weights_out`.  Lines whose workload features
 * (features 0, 1, 3-8, 12, 13: those that do not describe the tile candidate)
 * agree form one workload; each line's target is min(log(ms / best ms of its
 * workload), log 4).  Features and targets are standardised, the parameters
 * drawn from `opts->seed`, and `opts->epochs` full-batch Adam steps run on the
 * device (lmfao_mlp_train) on `hip_stream` inside the caller's 256-byte
 * aligned `workspace` (lmfao_train_workspace_size bytes; the library
 * allocates nothing).  *final_loss (may be NULL) receives the last step's
 * mean squared error on the standardised targets.  Weights file: "LMFAOMLP",
 * int32 hidden, float32 feature means[16] and scales[16], target mean and
 * scale, then the parameters in the layout of lmfao_mlp_forward.  Errors:
 * INVALID_ARG (bad options, unreadable or malformed timing file, unwritable
 * output), WORKSPACE, HIP. */
lmfao_status lmfao_train_cost_model(const char *timing_db, const char *weights_out, const lmfao_train_opts *opts,
                                    void *workspace, size_t ws_bytes, void *hip_stream, float *final_loss);

/* ---- cost-model network (hand-written device kernels) -------------------- */

/* A fully connected network  in(16) -> H -> H -> 1  with ReLU, predicting
 * log(milliseconds).  Parameters live in one fp32 device array laid out as
 * W1[H][16], b1[H], W2[H][H], b2[H], W3[1][H], b3[1]. */
int32_t lmfao_mlp_param_count(int32_t hidden);

/* y[n] = f(x[n][16]) for device arrays x, y, params. */
lmfao_status lmfao_mlp_forward(int32_t hidden, const float *params, const float *x, int32_t n, float *y,
                               void *hip_stream);

/* Mean-squared-error loss over n samples and its gradient w.r.t. all
 * parameters (device arrays; grad has lmfao_mlp_param_count() floats,
 * loss is one float).  `scratch` needs lmfao_mlp_scratch_floats(hidden, n). */
int64_t lmfao_mlp_scratch_floats(int32_t hidden, int32_t n);
lmfao_status lmfao_mlp_loss_grad(int32_t hidden, const float *params, const float *x, const float *target,
                                 int32_t n, float *loss, float *grad, float *scratch, void *hip_stream);

/* One Adam step (Kingma & Ba 2015) on device arrays: m, v are the moment
 * estimates, `step` the 1-based step count. */
lmfao_status lmfao_adam_step(int32_t n_params, float *params, const float *grad, float *m, float *v,
                             int32_t step, float lr, float beta1, float beta2, float eps, void *hip_stream);

/* Full-batch training loop on the device: `epochs` steps of
 * lmfao_mlp_loss_grad followed by lmfao_adam_step (beta1 0.9, beta2 0.999,
 * eps 1e-8), storing each step's loss in the device array losses[epochs].
 * `grad` holds lmfao_mlp_param_count() floats, m and v start at zero. */
lmfao_status lmfao_mlp_train(int32_t hidden, float *params, float *m, float *v, const float *x, const float *target,
                             int32_t n, int32_t epochs, float lr, float *grad, float *scratch, float *losses,
                             void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LMFAO_H */
