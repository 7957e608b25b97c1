/*
 * CPU oracle for batches of group-by aggregates over a natural join.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark.
 * It shares no source with the GPU engine.
 *
 * What it computes is the plain definition of the query batch (paper,
 * Section 1.1 problem statement; Section 2, equation (1)):
 *
 *   for every query Q(F; alpha_1..alpha_l) and every cell f of the product of
 *   the group-by domains,
 *     COUNT(f)   = |{ t in J : where(t) and t[F] = f }|
 *     SUM_i(f)   = sum over those t of alpha_i(t)
 *   where J = R_1 join ... join R_m is the natural join under bag semantics.
 *
 * It does NOT use views, pushdown, merging, grouping or any plan (Sections
 * 3.1-3.5 are an exact rewriting of this definition by distributivity and
 * are what the engine under test implements).  The join is enumerated by
 * walking the join tree: for every row of the root relation, each other
 * relation contributes every row whose shared attributes equal those of the
 * already chosen row of its tree parent.  With the running-intersection
 * property of a join tree (Section 3.1) this enumerates exactly the natural
 * join; a pure-Python cross-product check pins that on tiny inputs.
 *
 * Arithmetic: counts are uint64.  Every term coeff * prod(x) is evaluated in
 * double (a product of two fp32 values is exact in double) and summed with
 * Neumaier's compensated summation; the sum of |term| is kept alongside for
 * the conditioning of each result.  Threads own private accumulators over
 * contiguous ranges of root rows; partials are merged in thread order with
 * the same compensated addition.
 *
 * Predicates 1[X op t] compare fp32 attribute values with the constant
 * rounded to fp32, and integer attributes with the real constant exactly
 * (1[c >= 2.5] holds for c >= 3).  A bucket
 * group-by over sorted thresholds t_0 < ... < t_{T-1} maps x to
 * #{k : t_k < x}, i.e. x <= t_k  <=>  bucket <= k (the split X <= t of
 * Section 2, decision trees).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_I32 = 0, OR_F32 = 1 };
enum { OP_LE = 0, OP_LT = 1, OP_GE = 2, OP_GT = 3, OP_EQ = 4, OP_NE = 5 };
enum { OR_OK = 0, OR_ERR_ARG = -1, OR_ERR_DOMAIN = -2, OR_ERR_NOMEM = -3 };

typedef struct {
    int64_t n_rows;
    int32_t n_cols;
    const int32_t *col_attr;      /* global attribute id of each column */
    const int32_t *col_type;      /* OR_I32 or OR_F32 */
    const void *const *col_data;  /* column-major arrays of n_rows */
} or_relation;

typedef struct {
    int32_t parent, child;        /* relation indices */
    int32_t n_shared;             /* shared attributes (natural join) */
    const int32_t *parent_col;    /* column index in parent, per shared attr */
    const int32_t *child_col;     /* column index in child */
} or_edge;

typedef struct {
    int32_t n_groupby;
    const int32_t *gb_attr;       /* attribute ids */
    const int32_t *gb_nthr;       /* 0: categorical code; >0: bucket over thresholds */
    const float *const *gb_thr;   /* sorted thresholds per group-by (or NULL) */
    const int32_t *gb_dom;        /* domain size per group-by */
    int32_t n_preds;
    const int32_t *pred_attr;
    const int32_t *pred_op;
    const double *pred_val;
    int32_t n_aggs;
    const int32_t *agg_nterms;    /* terms per aggregate */
    const double *term_coeff;     /* all terms, aggregate by aggregate */
    const int32_t *term_nfac;     /* factors per term */
    const int32_t *fac_attr;      /* all factors, term by term */
    /* outputs, dense over cells (first group-by most significant) */
    uint64_t *counts;             /* [n_cells] */
    double *sums;                 /* [n_cells * n_aggs] */
    double *abs_sums;             /* [n_cells * n_aggs] */
} or_query;

/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t rel;                  /* relation holding the attribute */
    int32_t col;
} attr_loc;

typedef struct {
    const or_relation *rels;
    int32_t n_rels;
    const or_edge *edges;
    int32_t n_edges;
    int32_t root;
    int32_t *order;               /* non-root relations, parents first */
    int32_t *edge_of;             /* edge whose child is relation r (-1 for root) */
    int64_t **index;              /* per relation: row ids sorted by shared-attr tuple with parent */
    attr_loc *attrs;
    int32_t n_attr_ids;
} ctx_t;

static int64_t ival(const or_relation *r, int32_t col, int64_t row) {
    if (r->col_type[col] == OR_I32) return ((const int32_t *)r->col_data[col])[row];
    return (int64_t)((const float *)r->col_data[col])[row];
}

static float fval(const or_relation *r, int32_t col, int64_t row) {
    if (r->col_type[col] == OR_F32) return ((const float *)r->col_data[col])[row];
    return (float)((const int32_t *)r->col_data[col])[row];
}

/* Comparison of child rows by their shared-attribute tuple (for sorting). */
static const ctx_t *g_sort_ctx;
static int32_t g_sort_edge;

static int cmp_child_rows(const void *pa, const void *pb) {
    const or_edge *e = &g_sort_ctx->edges[g_sort_edge];
    const or_relation *c = &g_sort_ctx->rels[e->child];
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    for (int k = 0; k < e->n_shared; ++k) {
        int64_t va = ival(c, e->child_col[k], a), vb = ival(c, e->child_col[k], b);
        if (va != vb) return va < vb ? -1 : 1;
    }
    return a < b ? -1 : (a > b);
}

/* compare child row `cr` against the parent's shared tuple of row `pr` */
static int cmp_child_parent(const ctx_t *cx, const or_edge *e, int64_t cr, int64_t pr) {
    const or_relation *c = &cx->rels[e->child], *p = &cx->rels[e->parent];
    for (int k = 0; k < e->n_shared; ++k) {
        int64_t vc = ival(c, e->child_col[k], cr), vp = ival(p, e->parent_col[k], pr);
        if (vc != vp) return vc < vp ? -1 : 1;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */

typedef struct {
    uint64_t *counts;
    double *sum, *comp, *abs;
} qacc;

static void neumaier_add(double *s, double *c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

static int pred_holds(const ctx_t *cx, const int64_t *row, int32_t attr, int32_t op, double v) {
    const attr_loc *L = &cx->attrs[attr];
    const or_relation *r = &cx->rels[L->rel];
    if (r->col_type[L->col] == OR_F32) {
        float x = fval(r, L->col, row[L->rel]);
        float t = (float)v;
        switch (op) {
            case OP_LE: return x <= t;
            case OP_LT: return x < t;
            case OP_GE: return x >= t;
            case OP_GT: return x > t;
            case OP_EQ: return x == t;
            default: return x != t;
        }
    } else {
        /* an integer attribute against the real constant v, compared exactly
         * (every int32 value is a double) */
        double x = (double)ival(r, L->col, row[L->rel]);
        double t = v;
        switch (op) {
            case OP_LE: return x <= t;
            case OP_LT: return x < t;
            case OP_GE: return x >= t;
            case OP_GT: return x > t;
            case OP_EQ: return x == t;
            default: return x != t;
        }
    }
}

/* Evaluate every query on one join tuple (one row id per relation). */
static int eval_tuple(const ctx_t *cx, const int64_t *row, const or_query *qs, int32_t nq, qacc *acc) {
    for (int32_t q = 0; q < nq; ++q) {
        const or_query *Q = &qs[q];
        int ok = 1;
        for (int32_t p = 0; p < Q->n_preds && ok; ++p)
            ok = pred_holds(cx, row, Q->pred_attr[p], Q->pred_op[p], Q->pred_val[p]);
        if (!ok) continue;
        int64_t cell = 0;
        for (int32_t g = 0; g < Q->n_groupby; ++g) {
            const attr_loc *L = &cx->attrs[Q->gb_attr[g]];
            const or_relation *r = &cx->rels[L->rel];
            int64_t v;
            if (Q->gb_nthr[g] == 0) {
                v = ival(r, L->col, row[L->rel]);
                if (v < 0 || v >= Q->gb_dom[g]) return OR_ERR_DOMAIN;
            } else {
                float x = fval(r, L->col, row[L->rel]);
                v = 0;
                for (int32_t k = 0; k < Q->gb_nthr[g]; ++k)
                    if (Q->gb_thr[g][k] < x) ++v;
            }
            cell = cell * Q->gb_dom[g] + v;
        }
        acc[q].counts[cell] += 1;
        int32_t t = 0, f = 0;
        for (int32_t a = 0; a < Q->n_aggs; ++a) {
            size_t s = (size_t)cell * Q->n_aggs + a;
            /* alpha_a = sum_j coeff_j * prod_k X_jk; every term enters the
             * compensated sum on its own */
            for (int32_t j = 0; j < Q->agg_nterms[a]; ++j, ++t) {
                double term = Q->term_coeff[t];
                for (int32_t k = 0; k < Q->term_nfac[t]; ++k, ++f) {
                    const attr_loc *L = &cx->attrs[Q->fac_attr[f]];
                    term *= (double)fval(&cx->rels[L->rel], L->col, row[L->rel]);
                }
                neumaier_add(&acc[q].sum[s], &acc[q].comp[s], term);
                acc[q].abs[s] += fabs(term);
            }
        }
    }
    return OR_OK;
}

/* Enumerate the join below the chosen root row, relation by relation. */
static int enumerate(const ctx_t *cx, int64_t *row, int32_t level, const or_query *qs, int32_t nq, qacc *acc) {
    if (level == cx->n_rels - 1) return eval_tuple(cx, row, qs, nq, acc);
    int32_t r = cx->order[level];
    const or_edge *e = &cx->edges[cx->edge_of[r]];
    const int64_t *idx = cx->index[r];
    int64_t n = cx->rels[r].n_rows;
    int64_t pr = row[e->parent];
    /* first index position whose tuple is >= the parent's */
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cmp_child_parent(cx, e, idx[mid], pr) < 0) lo = mid + 1; else hi = mid;
    }
    for (int64_t i = lo; i < n && cmp_child_parent(cx, e, idx[i], pr) == 0; ++i) {
        row[r] = idx[i];
        int rc = enumerate(cx, row, level + 1, qs, nq, acc);
        if (rc) return rc;
    }
    return OR_OK;
}

static int64_t n_cells_of(const or_query *Q) {
    int64_t n = 1;
    for (int32_t g = 0; g < Q->n_groupby; ++g) n *= Q->gb_dom[g];
    return n;
}

static int alloc_acc(const or_query *qs, int32_t nq, qacc *acc) {
    for (int32_t q = 0; q < nq; ++q) {
        int64_t cells = n_cells_of(&qs[q]);
        size_t ns = (size_t)cells * (size_t)qs[q].n_aggs;
        acc[q].counts = (uint64_t *)calloc((size_t)cells, sizeof(uint64_t));
        acc[q].sum = (double *)calloc(ns + 1, sizeof(double));
        acc[q].comp = (double *)calloc(ns + 1, sizeof(double));
        acc[q].abs = (double *)calloc(ns + 1, sizeof(double));
        if (!acc[q].counts || !acc[q].sum || !acc[q].comp || !acc[q].abs) return OR_ERR_NOMEM;
    }
    return OR_OK;
}

static void free_acc(qacc *acc, int32_t nq) {
    if (!acc) return;
    for (int32_t q = 0; q < nq; ++q) {
        free(acc[q].counts); free(acc[q].sum); free(acc[q].comp); free(acc[q].abs);
    }
}

/*
 * Evaluate `nq` queries over the natural join of `n_rels` relations, whose
 * join tree has `n_edges` = n_rels - 1 edges and whose root is `root`.
 * Only root rows in [root_begin, root_end) are enumerated (the full join when
 * the range covers the root relation).  `attr_rel`/`attr_col` locate every
 * attribute id referenced by a query.  Returns OR_OK or a negative error.
 */
int oracle_evaluate(const or_relation *rels, int32_t n_rels, const or_edge *edges, int32_t n_edges,
                    int32_t root, const int32_t *attr_rel, const int32_t *attr_col, int32_t n_attr_ids,
                    or_query *qs, int32_t nq, int64_t root_begin, int64_t root_end, int32_t n_threads) {
    if (n_rels < 1 || n_edges != n_rels - 1 || root < 0 || root >= n_rels) return OR_ERR_ARG;
    ctx_t cx;
    memset(&cx, 0, sizeof cx);
    cx.rels = rels; cx.n_rels = n_rels; cx.edges = edges; cx.n_edges = n_edges; cx.root = root;
    cx.n_attr_ids = n_attr_ids;
    cx.attrs = (attr_loc *)malloc(sizeof(attr_loc) * (size_t)(n_attr_ids > 0 ? n_attr_ids : 1));
    cx.order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_rels);
    cx.edge_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_rels);
    cx.index = (int64_t **)calloc((size_t)n_rels, sizeof(int64_t *));
    int rc = OR_OK;
    if (!cx.attrs || !cx.order || !cx.edge_of || !cx.index) { rc = OR_ERR_NOMEM; goto done; }
    for (int32_t a = 0; a < n_attr_ids; ++a) { cx.attrs[a].rel = attr_rel[a]; cx.attrs[a].col = attr_col[a]; }

    /* parents-first order of the non-root relations (breadth first from the root) */
    for (int32_t r = 0; r < n_rels; ++r) cx.edge_of[r] = -1;
    for (int32_t e = 0; e < n_edges; ++e) {
        if (cx.edge_of[edges[e].child] != -1 || edges[e].child == root) { rc = OR_ERR_ARG; goto done; }
        cx.edge_of[edges[e].child] = e;
    }
    {
        int32_t head = 0, tail = 0;
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_rels);
        if (!queue) { rc = OR_ERR_NOMEM; goto done; }
        queue[tail++] = root;
        while (head < tail) {
            int32_t p = queue[head++];
            for (int32_t e = 0; e < n_edges; ++e)
                if (edges[e].parent == p) queue[tail++] = edges[e].child;
            if (tail > n_rels) break;
        }
        if (tail != n_rels) { free(queue); rc = OR_ERR_ARG; goto done; }
        for (int32_t i = 1; i < n_rels; ++i) cx.order[i - 1] = queue[i];
        free(queue);
    }
    /* sorted row index of every non-root relation on its shared attributes */
    for (int32_t i = 0; i + 1 < n_rels; ++i) {
        int32_t r = cx.order[i];
        int64_t n = rels[r].n_rows;
        cx.index[r] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        if (!cx.index[r]) { rc = OR_ERR_NOMEM; goto done; }
        for (int64_t k = 0; k < n; ++k) cx.index[r][k] = k;
        g_sort_ctx = &cx;
        g_sort_edge = cx.edge_of[r];
        qsort(cx.index[r], (size_t)n, sizeof(int64_t), cmp_child_rows);
    }
    for (int32_t q = 0; q < nq; ++q) {
        int64_t cells = n_cells_of(&qs[q]);
        memset(qs[q].counts, 0, sizeof(uint64_t) * (size_t)cells);
        memset(qs[q].sums, 0, sizeof(double) * (size_t)cells * (size_t)qs[q].n_aggs);
        memset(qs[q].abs_sums, 0, sizeof(double) * (size_t)cells * (size_t)qs[q].n_aggs);
    }
    if (root_begin < 0) root_begin = 0;
    if (root_end > rels[root].n_rows) root_end = rels[root].n_rows;

    int nt = n_threads > 0 ? n_threads : 1;
    qacc **per = (qacc **)calloc((size_t)nt, sizeof(qacc *));
    int *trc = (int *)calloc((size_t)nt, sizeof(int));
    if (!per || !trc) { free(per); free(trc); rc = OR_ERR_NOMEM; goto done; }
#pragma omp parallel num_threads(nt)
    {
        int t = 0, T = 1;
#ifdef _OPENMP
        t = omp_get_thread_num(); T = omp_get_num_threads();
#endif
        qacc *acc = (qacc *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(qacc));
        per[t] = acc;
        int my = acc ? alloc_acc(qs, nq, acc) : OR_ERR_NOMEM;
        int64_t span = root_end - root_begin;
        int64_t b = root_begin + span * t / T, e = root_begin + span * (t + 1) / T;
        int64_t *row = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_rels);
        if (!row) my = OR_ERR_NOMEM;
        for (int64_t i = b; i < e && my == OR_OK; ++i) {
            row[root] = i;
            my = enumerate(&cx, row, 0, qs, nq, acc);
        }
        free(row);
        trc[t] = my;
    }
    for (int t = 0; t < nt; ++t) if (trc[t] != OR_OK && rc == OR_OK) rc = trc[t];
    if (rc == OR_OK) {
        for (int32_t q = 0; q < nq; ++q) {
            int64_t cells = n_cells_of(&qs[q]);
            size_t ns = (size_t)cells * (size_t)qs[q].n_aggs;
            for (int64_t c = 0; c < cells; ++c) {
                uint64_t cnt = 0;
                for (int t = 0; t < nt; ++t) cnt += per[t][q].counts[c];
                qs[q].counts[c] = cnt;
            }
            for (size_t s = 0; s < ns; ++s) {
                double S = 0.0, C = 0.0, A = 0.0;
                for (int t = 0; t < nt; ++t) {
                    neumaier_add(&S, &C, per[t][q].sum[s]);
                    neumaier_add(&S, &C, per[t][q].comp[s]);
                    A += per[t][q].abs[s];
                }
                qs[q].sums[s] = S + C;
                qs[q].abs_sums[s] = A;
            }
        }
    }
    for (int t = 0; t < nt; ++t) { if (per[t]) { free_acc(per[t], nq); free(per[t]); } }
    free(per);
    free(trc);
done:
    if (cx.index) for (int32_t r = 0; r < n_rels; ++r) free(cx.index[r]);
    free(cx.index); free(cx.order); free(cx.edge_of); free(cx.attrs);
    return rc;
}
