// Host side of the aggregate-batch engine: the C ABI of include/lmfao.h,
// the planner and the executor.
//
// Planning follows the layers of the paper (Section 1.2, Figure 1):
//   join tree      validated tree of single-key edges (Section 3.1); the
//                  root is the relation that is no edge's child;
//   pushdown       every query is decomposed into one view per edge towards
//                  the root (Section 3.2): the view of a child subtree T_i
//                  carries the join key and exactly the parts of the query
//                  that live in T_i -- its continuous factors, its group-by
//                  components and its conjuncts, evaluated once per key
//                  (Appendix C, avoiding repeated UDAF evaluation);
//   merge          views with the same direction and group-by attributes are
//                  merged (Section 3.4, cases 1-3): per child relation the
//                  plan keeps ONE view record holding the union of what all
//                  queries need; at the root, queries with equal group-by
//                  and filter share one table whose aggregate list is the
//                  union of their monomials, and every ungrouped unfiltered
//                  sum shares the covariance block;
//   group          the views leaving one relation form a view group and are
//                  computed by one scan of that relation (Section 3.4);
//   levels         a relation's group depends on its children's groups; the
//                  groups of one tree level are independent (Section 1.2,
//                  parallelization) and run in one launch when batched.
// Code specialisation (Section 3.5, Appendix C) is replaced by templated
// kernels and runtime descriptors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "desc.h"
#include "lmfao.h"

namespace lmfao {
struct FillDesc {
    uint32_t *ptr;
    int64_t n_words;
};
typedef void (*RootKernel)(const RootDesc *);
RootKernel root_kernel(int mode, int p1, bool tables);
hipError_t launch_fill(const void *fills, int n, hipStream_t st);
hipError_t launch_views(const ScanDesc *descs, int n_scans, int64_t max_rows, hipStream_t st);
hipError_t launch_dup(const DupDesc *desc, int64_t n_rows, int64_t n_keys, hipStream_t st);
hipError_t launch_corr(const CorrDesc *desc, int n_pair, hipStream_t st);
hipError_t launch_target(const TargetDesc *descs, int n_targets, int64_t max_items, hipStream_t st);
hipError_t launch_root(RootKernel k, const RootDesc *desc, int grid_x, int parts, int waves, size_t lds_bytes,
                       hipStream_t st);
hipError_t set_root_lds_limit(RootKernel k, size_t bytes);
typedef void (*GramKernel)(const GramDesc *);
GramKernel gram_kernel(int nt, int nf, int pm, bool pr);
hipError_t launch_gram(GramKernel k, const GramDesc *desc, int grid_x, int waves, size_t lds_bytes, hipStream_t st);
hipError_t set_gram_lds_limit(GramKernel k, size_t bytes);
hipError_t set_code_scan_lds_limit(size_t bytes);
hipError_t launch_code_scan(const CodeScanDesc *desc, int grid_x, int parts, size_t lds_bytes, hipStream_t st);
hipError_t set_hist_lds_limit(size_t bytes);
hipError_t launch_hist(const HistDesc *desc, int grid_x, int parts, size_t lds_bytes, hipStream_t st);
hipError_t launch_merge(const MergeDesc *desc, int n_gram, hipStream_t st);
hipError_t launch_assemble(const AssembleDesc *desc, int n_out, int64_t max_cells, hipStream_t st);
hipError_t launch_rollup(const RollupDesc *desc, int n_items, int64_t max_work, hipStream_t st);
// cost-model network (mlp.hip)
hipError_t mlp_forward_dev(int hidden, const float *params, const float *x, int n, float *y, hipStream_t st);
}  // namespace lmfao

using namespace lmfao;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxRecWords = 128;   // largest view record (the zero record stands in for missing keys)
constexpr int kGridMax = 2048;    // workgroups of the general root scan (one covariance partial each)
constexpr int kPartMax = 8192;    // covariance partials (the dedicated scan writes one per wave)

size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int round_up(int x, int m) { return (x + m - 1) / m * m; }

struct Col {
    std::string attr;
    int32_t dtype, kind, domain;
    const void *data;
};

struct Rel {
    std::string name;
    int64_t n_rows = 0;
    std::vector<Col> cols;
    int find(const std::string &a) const {
        for (size_t i = 0; i < cols.size(); ++i)
            if (cols[i].attr == a) return (int)i;
        return -1;
    }
};

struct QGroupBy {
    std::string attr;
    std::vector<float> thr;
};
struct QPred {
    std::string attr;
    int32_t op;
    double value;
};
struct QTerm {
    double coeff;
    std::vector<std::string> f;
};
struct QAgg {
    std::vector<QTerm> terms;
};
struct Query {
    std::vector<QGroupBy> gb;
    std::vector<QPred> preds;
    std::vector<QAgg> aggs;
};

struct ARef {
    int rel = -1, col = -1;
    bool operator<(const ARef &o) const { return rel != o.rel ? rel < o.rel : col < o.col; }
    bool operator==(const ARef &o) const { return rel == o.rel && col == o.col; }
};

struct Comp {              // a group-by component (an attribute, or its buckets)
    ARef src;
    std::vector<float> thr;
    int dom = 0;
    int slot = -1;          // staged component index at the root
};

struct Conj {              // one conjunct of a filter
    ARef src;
    int op;
    double value;
};

struct Table {
    std::vector<int> comps;             // component ids (group-by order)
    int filter = -1;                    // -1: none
    int wdiv = -1;                      // view towards many-to-many child wdiv: rows weighted without its count
    std::vector<std::pair<int, int>> vals;   // monomials (feature a <= b), sorted
    int64_t n_cells = 1;
    // placement
    int part = 0;
    int lds_cnt = -1, lds_val = -1;
    int64_t glb_cnt = 0, glb_val = 0;
    // marginal derivation: summed after the scan from table `from` over its component `drop`
    int from = -1, drop = -1;
    std::vector<int> vmap;              // per value: index in the source table's values
    // uint32 counts, then fp64 sums at an even word offset
    int words() const { return (int)(round_up((int)n_cells, 2) + 2 * n_cells * (int64_t)vals.size()); }
    int val_off() const { return round_up((int)n_cells, 2); }
};

struct Family {
    std::vector<std::pair<int, int>> vals;
    std::vector<std::vector<int>> keys;   // component lists
    std::vector<int> filters;             // ascending filter ids; empty = unfiltered
    std::vector<int> tables;              // index f * n_keys + k -> table id
    bool hist = false;                    // counted by the count-table scan, not the root scan
    int wdiv = -1;                        // as Table::wdiv, shared by the family's tables
};

struct OutTerm {
    int agg;
    int src;          // gram entry / table value index; -1 = count
    double coeff;
};

struct Output {
    bool gram = false;
    int table = -1;
    int target = -1;                   // evaluated at another root: index into Plan::targets
    int64_t n_cells = 1;
    int n_aggs = 0;
    size_t cnt_off = 0, sum_off = 0;   // bytes in the result arena
    std::vector<OutTerm> terms;
};

// A query evaluated at a root R other than the tree root (R a child of it): the view from the
// tree root towards R is the grouped table `table`, keyed by (fk_comp, o_comps); R's side is
// joined by the target scan.
struct TargetPlan {
    int q = -1, rel = -1;
    bool dup = false;                 // R is a many-to-many child: its rows are scanned
    int filter = -1;
    std::vector<int> gb_comp;         // per group-by position of the query: component id
    std::vector<int> gb_o;            // per position: index among o_comps, -1 on R's side
    std::vector<int> o_comps;         // group-by components outside R's subtree
    int fk_comp = -1;
    int table = -1;
    struct Term {
        int agg = 0;
        double coeff = 1.0;
        std::vector<ARef> rfac, ofac; // factors on R's side and outside it
        int val = -1;                 // value of the view summing ofac (-1: its count)
    };
    std::vector<Term> terms;
    int64_t n_cells = 1;
};

struct TileCfg {
    int waves = 0;          // waves per workgroup of the root scan (0 = heuristic)
    int nbuf = 0;           // staging buffers per wave (0 = heuristic)
    int grid_x = 0;         // requested workgroups (0 = heuristic)
    int gram_block = 0;     // fp32 register block edge
    int lds_policy = -1;    // 0 global tables, 1 greedy LDS, 2 partitioned LDS, 3 partitioned LDS with
                            // per-row codes and the count-table scan where they apply (-1 = heuristic)
};

struct RootLaunch {         // one launch of the root scan (batched: one; plain: one per view)
    int mode = 0, p1 = 1;
    bool tables = false;
    int grid_x = 1, parts = 1, waves = 2;
    int resident = 1;        // workgroups one CU holds at once (registers and LDS)
    size_t lds_bytes = 0;
    RootDesc desc;           // pointers filled at bind
    std::vector<int> fam_ids;        // families evaluated (plain: one table view)
    int single_table = -1;           // plain mode: the one table of this launch
    bool with_gram = false;
    size_t desc_off = 0;
    // covariance-only launch on the dedicated BF16 scan (slot tiles gnt, fact tiles gnf)
    bool gram = false;
    bool gpr = false;        // pair-row record buffers (gram_pair_rows)
    int gnt = 0, gnf = 0;
    GramDesc gdesc;
};

struct Plan {
    bool ok = false;
    // tree
    int root = -1;
    std::vector<int> parent, depth, height;
    std::vector<std::vector<int>> children;
    std::vector<int> fk_col;     // per non-root relation: FK column in its parent
    std::vector<int> pk_col;     // per non-root relation: key column in itself
    std::vector<int> n_keys;     // per non-root relation: key domain
    int levels = 0;
    // staged features / components, in DFS order of relations
    std::vector<ARef> feats;                 // [0] = constant 1
    std::vector<std::vector<int>> own_feats; // per relation, feature ids
    std::vector<int> sub_feat_lo, sub_feat_n;   // subtree feature range in staged order
    std::vector<Comp> comps;
    std::vector<std::vector<int>> own_comps;
    std::vector<int> sub_comp_lo, sub_comp_n;
    std::vector<std::vector<Conj>> filters;
    std::vector<std::vector<std::pair<int, int>>> own_preds;   // per relation: (filter, conjunct index)
    int n_mask = 0;
    // record layouts of non-root relations
    std::vector<int> rec_stride, rec_comp_off, rec_feat_off;
    // many-to-many children (join key declared KEY_MANY): count-weighted views.  dup[r]; per such
    // relation the pairs (staged features a <= b, both its own) whose covariance entries take its
    // within-key scatter, weighted by how often the root reaches each key
    std::vector<char> dup;
    std::vector<std::vector<std::pair<int, int>>> dup_pairs;
    bool weighted = false;
    // roots per query (Section 3.3): the relation each query is evaluated at; queries at a child
    // of the tree root are answered by a view towards it and the target scan
    std::vector<int> qroot;
    std::vector<TargetPlan> targets;
    // products of two staged attributes computed per row by the root scan (the degree-2 parts of
    // monomials of degree 3 and 4): staged features n_base .. n_feat-1
    std::vector<std::pair<int, int>> derived;
    int n_base = 1;
    // root outputs
    int n_feat = 1, n_gram = 0;
    bool need_count = false;
    std::vector<Table> tables;
    std::vector<Family> fams;
    std::vector<Output> outs;
    int64_t table_cells = 0, table_vals = 0;
    std::vector<std::vector<int>> rollup_passes;   // derived tables per pass, in execution order
    int n_derived = 0;
    int n_strided = 0;                             // families of root launches with strided LDS layout
    // grouped tables from per-row codes (root scan writes them, a code scan per partition reads)
    bool codes = false;
    int n_mask_codes = 1, n_codes = 0;
    std::vector<int32_t> code_feats;               // staged features summed by the tables
    int code_feat_col = 0;
    int64_t code_pitch = 0;
    int code_grid = 0;
    int64_t code_rows_per_block = 0;
    size_t code_lds_bytes = 0;
    // count tables from 16-bit component codes (unfiltered COUNT-only families beyond the root
    // scan's LDS): the root scan writes the codes, the count-table scan counts them per partition
    bool hist = false;
    std::vector<int> hist_comps;                   // component of each code column
    int64_t hist_pitch = 0;
    std::vector<HistSlice> hist_slices;            // partition by partition
    std::vector<int32_t> hist_part_begin, hist_lds_words;
    int hist_grid = 0;
    int64_t hist_rows_per_block = 0;
    size_t hist_lds_bytes = 0;
    // schedule
    int precision = LMFAO_FP32, schedule = LMFAO_BATCHED, planner = LMFAO_HEURISTIC;
    TileCfg cfg;                      // chosen tile configuration
    int gram_block = 4, n_tiles16 = 1, mode = 0, lds_policy = 0, parts = 1, nbuf = 2, waves = 2;
    int gram_waves = 4;          // waves per workgroup of the dedicated covariance scan
    int grid_x = 1;
    int64_t rows_per_block = kBlock;
    std::vector<RootLaunch> root_launches;
    int app_aggs = 0, inter_aggs = 0, views = 0, groups = 0;
    // sizes
    size_t ws_bytes = 0, res_bytes = 0;
};

}  // namespace

// Workspace for callers that cannot allocate device memory (lmfao_bind_scratch): one array per
// GPU, held until the process ends.  Host code never uses the array's name as an address: the
// device address of each GPU's copy comes from hipGetSymbolAddress (scratch_ptr below).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
struct ScratchSlot {
    std::once_flag once;
    uint8_t *ptr = nullptr;          // device address of this GPU's scratch array
    hipError_t status = hipSuccess;  // result of the symbol lookup
    std::atomic<uint64_t> owner{0};  // binding generation that last bound the array
};
ScratchSlot g_scratch[kMaxDevices];
std::atomic<uint64_t> g_scratch_gen{0};

// Look the array up once per device, with that device current.
hipError_t scratch_ptr(int device, uint8_t **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    ScratchSlot &S = g_scratch[device];
    std::call_once(S.once, [&] {
        int prev = 0;
        S.status = hipGetDevice(&prev);
        if (S.status != hipSuccess) return;
        S.status = hipSetDevice(device);
        if (S.status != hipSuccess) return;
        void *p = nullptr;
        S.status = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (S.status == hipSuccess) S.ptr = static_cast<uint8_t *>(p);
        (void)hipSetDevice(prev);
    });
    *out = S.ptr;
    return S.status;
}
}  // namespace

struct lmfao_ctx {
    int device = 0;
    bool has_device = false;
    int n_cu = 256;
    size_t lds_limit = 160 * 1024;
    std::string err;
    std::vector<Rel> rels;
    std::vector<std::pair<int, int>> edges;
    bool tree_set = false;
    std::vector<Query> queries;
    lmfao_plan_opts opts{};
    Plan plan;
    // binding
    uint64_t scratch_gen = 0;         // nonzero while the workspace is this device's scratch array
    uint8_t *ws = nullptr;
    size_t ws_len = 0;
    uint8_t *res = nullptr;
    size_t res_len = 0;
    bool bound = false;
    // device layout (offsets into ws)
    size_t off_err = 0, off_gcnt = 0, off_gval = 0, off_gpart = 0, off_cpart = 0, off_gsum = 0, off_gram = 0, off_count = 0;
    size_t off_desc = 0, off_mlp = 0, off_zero = 0;
    std::vector<size_t> off_rec, off_seen;
    std::vector<uint8_t> blob;       // descriptor image copied to ws + off_desc
    size_t fill_off = 0;
    int n_fills = 0;
    std::vector<std::vector<int>> level_rels;     // relations per level (non-root)
    std::vector<size_t> view_desc_off;            // per relation: ScanDesc offset in blob
    size_t merge_off = 0, assemble_off = 0;
    int n_assemble = 0;                           // outputs the assemble kernel writes
    size_t target_desc_off = 0;                   // TargetDesc array (one per target query) in blob
    int64_t target_items = 0;                     // most keys or rows of a target scan
    std::vector<size_t> rollup_off;               // per pass: RollupDesc offset in blob
    size_t off_codes = 0;                         // per-row codes
    size_t code_desc_off = 0;                     // CodeScanDesc offset in blob
    size_t off_hcodes = 0;                        // component codes of the count-table scan
    // many-to-many children: per relation the sums, pair sums / scatter and root weights per key
    std::vector<size_t> off_dsum, off_dscat, off_hw;
    std::vector<size_t> dup_desc_off, corr_desc_off;   // per relation: DupDesc / CorrDesc in blob
    size_t hist_desc_off = 0;                     // HistDesc offset in blob
    std::vector<int64_t> rollup_cells;            // per pass: most (cell, sum or count) pairs of a table
    int64_t assemble_cells = 0;                   // most cells of a query result
    // execution
    hipStream_t last_stream = nullptr;
    bool executed = false;
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    hipStream_t graph_stream = nullptr;
};

static lmfao_status fail(lmfao_ctx *c, lmfao_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

// The read-only accessors record their message too (every context is created writable by
// lmfao_create, so the cast is sound).
static lmfao_status fail(const lmfao_ctx *c, lmfao_status s, const std::string &msg) {
    return fail(const_cast<lmfao_ctx *>(c), s, msg);
}

#define HIP_TRY(ctx, call)                                                                                \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return fail((ctx), LMFAO_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ============================================================================
// context, relations, join tree, queries
// ============================================================================

extern "C" lmfao_status lmfao_create(lmfao_ctx **out, int32_t hip_device) {
    if (!out) return LMFAO_ERR_INVALID_ARG;
    *out = nullptr;
    lmfao_ctx *c = new (std::nothrow) lmfao_ctx();
    if (!c) return LMFAO_ERR_INVALID_ARG;
    c->device = hip_device;
    int n = 0;
    if (hipGetDeviceCount(&n) == hipSuccess && n > hip_device && hip_device >= 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) {
            c->has_device = true;
            c->n_cu = prop.multiProcessorCount;
            c->lds_limit = prop.sharedMemPerBlock;
            uint8_t *sp = nullptr;
            (void)scratch_ptr(hip_device, &sp);   // once per device; its status is reported by lmfao_bind_scratch
        }
    } else {
        (void)hipGetLastError();
    }
    *out = c;
    return LMFAO_OK;
}

extern "C" void lmfao_destroy(lmfao_ctx *c) {
    if (!c) return;
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_def) (void)hipGraphDestroy(c->graph_def);
    delete c;
}

extern "C" const char *lmfao_last_error(const lmfao_ctx *c) { return c ? c->err.c_str() : "null context"; }

static void invalidate(lmfao_ctx *c) {
    c->plan.ok = false;
    c->bound = false;
    c->executed = false;
    if (c->graph) { (void)hipGraphExecDestroy(c->graph); c->graph = nullptr; }
    if (c->graph_def) { (void)hipGraphDestroy(c->graph_def); c->graph_def = nullptr; }
}

extern "C" lmfao_status lmfao_add_relation(lmfao_ctx *c, const char *name, int64_t n_rows, int32_t n_cols,
                                           const lmfao_col *cols, int32_t *rel_id) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (c->tree_set) return fail(c, LMFAO_ERR_STATE, "relations must be added before the join tree");
    if (!name || n_rows < 0 || n_cols <= 0 || !cols) return fail(c, LMFAO_ERR_INVALID_ARG, "bad relation arguments");
    if (n_rows > ((int64_t)1 << 40)) return fail(c, LMFAO_ERR_TOO_LARGE, "relation too large");
    Rel r;
    r.name = name;
    r.n_rows = n_rows;
    for (int i = 0; i < n_cols; ++i) {
        const lmfao_col &x = cols[i];
        if (!x.attr || (!x.data && n_rows > 0)) return fail(c, LMFAO_ERR_INVALID_ARG, "column without name or data");
        if (x.kind < LMFAO_KEY || x.kind > LMFAO_KEY_MANY || x.dtype < LMFAO_I32 || x.dtype > LMFAO_F32)
            return fail(c, LMFAO_ERR_INVALID_ARG, std::string("bad kind/dtype for ") + x.attr);
        if ((x.kind == LMFAO_CONT) != (x.dtype == LMFAO_F32))
            return fail(c, LMFAO_ERR_TYPE, std::string("CONT columns are F32, KEY/CAT columns I32: ") + x.attr);
        if (x.kind != LMFAO_CONT && x.domain <= 0)
            return fail(c, LMFAO_ERR_INVALID_ARG, std::string("KEY/CAT column needs a positive domain: ") + x.attr);
        if (r.find(x.attr) >= 0) return fail(c, LMFAO_ERR_INVALID_ARG, std::string("duplicate attribute ") + x.attr);
        r.cols.push_back(Col{x.attr, x.dtype, x.kind, x.domain, x.data});
    }
    for (auto &o : c->rels)
        if (o.name == r.name) return fail(c, LMFAO_ERR_INVALID_ARG, "duplicate relation name " + r.name);
    c->rels.push_back(std::move(r));
    if (rel_id) *rel_id = (int32_t)c->rels.size() - 1;
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_set_join_tree(lmfao_ctx *c, int32_t n_edges, const int32_t *edges) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (c->tree_set) return fail(c, LMFAO_ERR_STATE, "join tree already set");
    const int m = (int)c->rels.size();
    if (m == 0) return fail(c, LMFAO_ERR_STATE, "no relations");
    if (n_edges != m - 1 || (n_edges > 0 && !edges))
        return fail(c, LMFAO_ERR_NOT_ACYCLIC, "a join tree over m relations has m-1 edges");
    std::vector<int> parent(m, -1);
    for (int e = 0; e < n_edges; ++e) {
        const int p = edges[2 * e], ch = edges[2 * e + 1];
        if (p < 0 || p >= m || ch < 0 || ch >= m || p == ch)
            return fail(c, LMFAO_ERR_INVALID_ARG, "edge names an unknown relation");
        if (parent[ch] != -1) return fail(c, LMFAO_ERR_NOT_ACYCLIC, "relation " + c->rels[ch].name + " has two parents");
        parent[ch] = p;
    }
    int root = -1;
    for (int r = 0; r < m; ++r)
        if (parent[r] == -1) {
            if (root != -1) return fail(c, LMFAO_ERR_NOT_ACYCLIC, "edges do not connect all relations");
            root = r;
        }
    if (root == -1) return fail(c, LMFAO_ERR_NOT_ACYCLIC, "edges form a cycle");
    for (int r = 0; r < m; ++r) {   // every relation reaches the root
        int x = r, steps = 0;
        while (x != root && steps <= m) { x = parent[x]; ++steps; }
        if (x != root) return fail(c, LMFAO_ERR_NOT_ACYCLIC, "edges form a cycle");
    }
    // each edge joins on exactly one shared attribute, a KEY of the child
    for (int ch = 0; ch < m; ++ch) {
        if (ch == root) continue;
        const Rel &P = c->rels[parent[ch]], &C = c->rels[ch];
        int shared = 0;
        std::string name;
        for (auto &col : C.cols)
            if (P.find(col.attr) >= 0) { ++shared; name = col.attr; }
        if (shared != 1)
            return fail(c, LMFAO_ERR_UNSUPPORTED, "edge " + P.name + "-" + C.name + " must share exactly one attribute");
        const Col &pc = P.cols[P.find(name)], &cc = C.cols[C.find(name)];
        if (pc.kind != LMFAO_KEY || (cc.kind != LMFAO_KEY && cc.kind != LMFAO_KEY_MANY))
            return fail(c, LMFAO_ERR_TYPE, "join attribute " + name + " must be KEY in the parent and KEY or KEY_MANY in the child");
    }
    // running intersection: the holders of every attribute are connected in the tree
    std::map<std::string, std::vector<int>> holders;
    for (int r = 0; r < m; ++r)
        for (auto &col : c->rels[r].cols) holders[col.attr].push_back(r);
    for (auto &kv : holders) {
        if (kv.second.size() < 2) continue;
        std::set<int> hs(kv.second.begin(), kv.second.end());
        int inner = 0;
        for (int r : kv.second)
            if (r != root && hs.count(parent[r])) ++inner;
        if (inner != (int)hs.size() - 1)
            return fail(c, LMFAO_ERR_NOT_ACYCLIC, "attribute " + kv.first + " violates the running intersection property");
    }
    c->edges.clear();
    for (int e = 0; e < n_edges; ++e) c->edges.push_back({edges[2 * e], edges[2 * e + 1]});
    c->tree_set = true;
    return LMFAO_OK;
}

static bool find_attr(const lmfao_ctx *c, const std::string &a, ARef &out) {
    // a non-key attribute has one holder; a join key is read where it is closest to the root
    const Plan &P = c->plan;
    int best = -1, bestcol = -1, bestdepth = 1 << 30;
    for (int r = 0; r < (int)c->rels.size(); ++r) {
        const int col = c->rels[r].find(a);
        if (col < 0) continue;
        int d = 0, x = r;
        while (x >= 0 && x < (int)P.parent.size() && P.parent[x] >= 0) { x = P.parent[x]; ++d; }
        if (d < bestdepth) { best = r; bestcol = col; bestdepth = d; }
    }
    out.rel = best;
    out.col = bestcol;
    return best >= 0;
}

// The factor 1[X op v] (Section 1.1) on an int32 attribute, for any real v: rewritten as an
// equal test against an int32 constant (X >= v <=> X >= ceil(v), X > v <=> X >= floor(v) + 1,
// X <= v <=> X <= floor(v), X < v <=> X <= ceil(v) - 1; X = v never holds and X != v always
// holds unless v is an int32 value).  Tests that hold for every or for no int32 value become
// X >= INT32_MIN and X < INT32_MIN, so the kernels compare int32 values only.
static void int_predicate(int32_t *op, double *v) {
    const double lo = (double)INT32_MIN, hi = (double)INT32_MAX;
    const bool integral = std::floor(*v) == *v && *v >= lo && *v <= hi;
    auto always = [&] { *op = LMFAO_GE; *v = lo; };
    auto never = [&] { *op = LMFAO_LT; *v = lo; };
    switch (*op) {
        case LMFAO_EQ: if (!integral) never(); return;
        case LMFAO_NE: if (!integral) always(); return;
        case LMFAO_GE:
        case LMFAO_GT: {
            const double t = *op == LMFAO_GE ? std::ceil(*v) : std::floor(*v) + 1.0;
            if (t <= lo) always();
            else if (t > hi) never();
            else { *op = LMFAO_GE; *v = t; }
            return;
        }
        default: {   // LE, LT
            const double t = *op == LMFAO_LE ? std::floor(*v) : std::ceil(*v) - 1.0;
            if (t >= hi) { *op = LMFAO_LE; *v = hi; }
            else if (t < lo) never();
            else { *op = LMFAO_LE; *v = t; }
            return;
        }
    }
}

extern "C" lmfao_status lmfao_add_query(lmfao_ctx *c, const lmfao_query *q, int32_t *qid) {
    if (!c || !q) return LMFAO_ERR_INVALID_ARG;
    if (!c->tree_set) return fail(c, LMFAO_ERR_STATE, "set the join tree before adding queries");
    if (q->n_groupby < 0 || q->n_preds < 0 || q->n_aggs < 0 || (q->n_groupby && !q->groupby) ||
        (q->n_preds && !q->preds) || (q->n_aggs && !q->aggs))
        return fail(c, LMFAO_ERR_INVALID_ARG, "bad query arrays");
    auto holder = [&](const char *a) -> const Col * {
        if (!a) return nullptr;
        for (auto &r : c->rels) {
            const int i = r.find(a);
            if (i >= 0) return &r.cols[i];
        }
        return nullptr;
    };
    Query Q;
    double cells = 1.0;
    for (int g = 0; g < q->n_groupby; ++g) {
        const lmfao_groupby &x = q->groupby[g];
        const Col *col = holder(x.attr);
        if (!col) return fail(c, LMFAO_ERR_UNKNOWN_ATTR, std::string("unknown group-by attribute ") + (x.attr ? x.attr : "(null)"));
        QGroupBy G;
        G.attr = x.attr;
        if (x.n_thresholds < 0 || (x.n_thresholds > 0 && !x.thresholds))
            return fail(c, LMFAO_ERR_INVALID_ARG, "bad thresholds");
        if (col->kind == LMFAO_CONT) {
            if (x.n_thresholds == 0) return fail(c, LMFAO_ERR_TYPE, "a continuous group-by needs thresholds: " + G.attr);
            G.thr.assign(x.thresholds, x.thresholds + x.n_thresholds);
            for (size_t k = 1; k < G.thr.size(); ++k)
                if (!(G.thr[k - 1] < G.thr[k])) return fail(c, LMFAO_ERR_INVALID_ARG, "thresholds must increase strictly");
            cells *= (double)(x.n_thresholds + 1);
        } else {
            if (x.n_thresholds != 0) return fail(c, LMFAO_ERR_TYPE, "thresholds apply to continuous attributes: " + G.attr);
            cells *= (double)col->domain;
        }
        Q.gb.push_back(G);
    }
    if (cells > 2147483647.0) return fail(c, LMFAO_ERR_TOO_LARGE, "query has more than 2^31 cells");
    for (int p = 0; p < q->n_preds; ++p) {
        const lmfao_pred &x = q->preds[p];
        const Col *col = holder(x.attr);
        if (!col) return fail(c, LMFAO_ERR_UNKNOWN_ATTR, std::string("unknown predicate attribute ") + (x.attr ? x.attr : "(null)"));
        if (x.op < LMFAO_LE || x.op > LMFAO_NE) return fail(c, LMFAO_ERR_INVALID_ARG, "bad predicate operator");
        if (std::isnan(x.value)) return fail(c, LMFAO_ERR_INVALID_ARG, "predicate constant is NaN");
        int32_t op = x.op;
        double v = x.value;
        if (col->dtype == LMFAO_I32) int_predicate(&op, &v);
        Q.preds.push_back(QPred{x.attr, op, v});
    }
    for (int a = 0; a < q->n_aggs; ++a) {
        const lmfao_agg &x = q->aggs[a];
        if (x.n_terms < 0 || (x.n_terms && !x.terms)) return fail(c, LMFAO_ERR_INVALID_ARG, "bad aggregate terms");
        QAgg A;
        for (int t = 0; t < x.n_terms; ++t) {
            const lmfao_term &tm = x.terms[t];
            if (tm.n_factors < 0 || tm.n_factors > 4)
                return fail(c, LMFAO_ERR_TOO_LARGE, "terms are products of at most four attributes");
            QTerm T;
            T.coeff = tm.coeff;
            for (int f = 0; f < tm.n_factors; ++f) {
                const Col *col = holder(tm.factors[f]);
                if (!col) return fail(c, LMFAO_ERR_UNKNOWN_ATTR, std::string("unknown factor ") + (tm.factors[f] ? tm.factors[f] : "(null)"));
                if (col->kind != LMFAO_CONT) return fail(c, LMFAO_ERR_TYPE, std::string("factor must be continuous: ") + tm.factors[f]);
                T.f.push_back(tm.factors[f]);
            }
            A.terms.push_back(T);
        }
        Q.aggs.push_back(A);
    }
    c->queries.push_back(std::move(Q));
    invalidate(c);
    if (qid) *qid = (int32_t)c->queries.size() - 1;
    return LMFAO_OK;
}

// ============================================================================
// planner
// ============================================================================

// FP32 register block edge: GB x GB accumulators per lane.  GB = 8 (64
// accumulators plus operands) spills on gfx950, so 6 is the largest used
// unless fewer block pairs than lanes would leave the wave idle.
static int estimate_gram_block(int n_gram) {
    if (n_gram <= 8) return 2;
    if (n_gram <= 24) return 4;
    return 6;
}

static bool gram_block_ok(int n_gram, int gb) {
    if (gb != 2 && gb != 4 && gb != 6 && gb != 8) return false;
    const int ngp = round_up(n_gram, gb);
    const int nb = ngp / gb;
    return nb * (nb + 1) / 2 <= 64;   // block pairs are spread over the 64 lanes of a wave
}

// Decompose the batch into views and tables (pushdown + merge).
static lmfao_status build_logical(lmfao_ctx *c) {
    Plan &P = c->plan;
    const int m = (int)c->rels.size();
    P = Plan();
    P.parent.assign(m, -1);
    for (auto &e : c->edges) P.parent[e.second] = e.first;
    P.children.assign(m, {});
    for (auto &e : c->edges) P.children[e.first].push_back(e.second);
    for (int r = 0; r < m; ++r)
        if (P.parent[r] == -1) P.root = r;
    P.fk_col.assign(m, -1);
    P.pk_col.assign(m, -1);
    P.n_keys.assign(m, 0);
    for (int r = 0; r < m; ++r) {
        if (r == P.root) continue;
        const Rel &Pr = c->rels[P.parent[r]], &C = c->rels[r];
        for (size_t i = 0; i < C.cols.size(); ++i) {
            const int pi = Pr.find(C.cols[i].attr);
            if (pi >= 0) {
                P.fk_col[r] = pi;
                P.pk_col[r] = (int)i;
                P.n_keys[r] = C.cols[i].domain;
            }
        }
    }
    // heights (levels) and DFS order
    P.height.assign(m, 0);
    P.depth.assign(m, 0);
    std::vector<int> order;
    std::vector<int> stack{P.root};
    while (!stack.empty()) {
        const int r = stack.back();
        stack.pop_back();
        order.push_back(r);
        for (int k = (int)P.children[r].size() - 1; k >= 0; --k) {
            P.depth[P.children[r][k]] = P.depth[r] + 1;
            stack.push_back(P.children[r][k]);
        }
    }
    for (int i = (int)order.size() - 1; i >= 0; --i) {
        const int r = order[i];
        for (int ch : P.children[r]) P.height[r] = std::max(P.height[r], P.height[ch] + 1);
    }
    P.levels = P.height[P.root] + 1;

    // ---- resolve queries: features, components, filters ------------------------------
    std::set<ARef> feat_set;
    std::map<std::string, int> comp_ids, filter_ids;
    struct RQ {
        std::vector<int> comps;
        int filter = -1;
        std::vector<std::vector<std::pair<double, std::vector<ARef>>>> aggs;
    };
    std::vector<RQ> rq(c->queries.size());
    for (size_t qi = 0; qi < c->queries.size(); ++qi) {
        const Query &Q = c->queries[qi];
        RQ &R = rq[qi];
        for (auto &g : Q.gb) {
            ARef a;
            find_attr(c, g.attr, a);
            std::string sig = g.attr + "|";
            for (float t : g.thr) { char b[32]; snprintf(b, sizeof b, "%a,", (double)t); sig += b; }
            auto it = comp_ids.find(sig);
            if (it == comp_ids.end()) {
                Comp cp;
                cp.src = a;
                cp.thr = g.thr;
                cp.dom = g.thr.empty() ? c->rels[a.rel].cols[a.col].domain : (int)g.thr.size() + 1;
                it = comp_ids.emplace(sig, (int)P.comps.size()).first;
                P.comps.push_back(cp);
            }
            R.comps.push_back(it->second);
        }
        if (!Q.preds.empty()) {
            std::vector<std::string> parts;
            std::vector<Conj> conj;
            for (auto &p : Q.preds) {
                ARef a;
                find_attr(c, p.attr, a);
                char b[96];
                snprintf(b, sizeof b, "%s|%d|%a", p.attr.c_str(), p.op, p.value);
                parts.push_back(b);
                conj.push_back(Conj{a, p.op, p.value});
            }
            std::vector<size_t> idx(parts.size());
            for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
            std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return parts[x] < parts[y]; });
            std::string sig;
            std::vector<Conj> sorted;
            for (size_t i : idx) { sig += parts[i] + ";"; sorted.push_back(conj[i]); }
            auto it = filter_ids.find(sig);
            if (it == filter_ids.end()) {
                if ((int)P.filters.size() >= kMaxFilters)
                    return fail(c, LMFAO_ERR_TOO_LARGE, "more than 64 distinct WHERE conjunctions");
                it = filter_ids.emplace(sig, (int)P.filters.size()).first;
                P.filters.push_back(sorted);
            }
            R.filter = it->second;
        }
        for (auto &ag : Q.aggs) {
            std::vector<std::pair<double, std::vector<ARef>>> terms;
            for (auto &t : ag.terms) {
                std::vector<ARef> fs;
                for (auto &f : t.f) {
                    ARef a;
                    find_attr(c, f, a);
                    fs.push_back(a);
                    feat_set.insert(a);
                }
                terms.push_back({t.coeff, fs});
            }
            R.aggs.push_back(terms);
        }
    }
    P.n_mask = P.filters.empty() ? 0 : (P.filters.size() <= 32 ? 1 : 2);

    // ---- roots per query (Section 3.3) ----------------------------------------------------------
    const int nq = (int)c->queries.size();
    auto in_sub = [&](int rel, int R) {
        for (int x = rel; x >= 0; x = P.parent[x])
            if (x == R) return true;
        return false;
    };
    auto top_of = [&](int r) {
        while (r != P.root && P.parent[r] != P.root) r = P.parent[r];
        return r;
    };
    auto is_dup = [&](int r) { return r != P.root && c->rels[r].cols[P.pk_col[r]].kind == LMFAO_KEY_MANY; };
    auto gram_q = [&](int q) { return rq[q].comps.empty() && rq[q].filter < 0; };
    P.qroot.assign(nq, P.root);
    if (c->opts.root_policy == LMFAO_ROOT_FIND) {
        // weights: each grouped or filtered query spreads 1 over the relations holding its group-by
        // attributes (over all relations when it has none); roots go by decreasing weight, ties to
        // the larger relation, each to every unassigned query that considered it
        std::vector<double> W(m, 0.0);
        for (int q = 0; q < nq; ++q) {
            if (gram_q(q)) continue;
            if (rq[q].comps.empty())
                for (int r = 0; r < m; ++r) W[r] += 1.0 / m;
            else
                for (int ci : rq[q].comps) W[P.comps[ci].src.rel] += 1.0 / (double)rq[q].comps.size();
        }
        std::vector<int> ord(m);
        for (int r = 0; r < m; ++r) ord[r] = r;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
            if (W[a] != W[b]) return W[a] > W[b];
            return c->rels[a].n_rows > c->rels[b].n_rows;
        });
        std::vector<int> asg(nq, -1);
        for (int R : ord) {
            if (W[R] <= 0.0) continue;
            for (int q = 0; q < nq; ++q) {
                if (gram_q(q) || asg[q] >= 0) continue;
                bool considered = rq[q].comps.empty();
                for (int ci : rq[q].comps) considered = considered || P.comps[ci].src.rel == R;
                if (considered) asg[q] = R;
            }
        }
        for (int q = 0; q < nq; ++q)
            if (asg[q] >= 0) P.qroot[q] = top_of(asg[q]);
    }
    // a query that groups by, filters on, or multiplies attributes of one many-to-many child is
    // evaluated at that child
    std::vector<char> forced(nq, 0);
    for (int q = 0; q < nq; ++q) {
        std::set<int> touched;
        for (int ci : rq[q].comps)
            if (is_dup(P.comps[ci].src.rel)) touched.insert(P.comps[ci].src.rel);
        if (rq[q].filter >= 0)
            for (auto &cj : P.filters[rq[q].filter])
                if (is_dup(cj.src.rel)) touched.insert(cj.src.rel);
        for (auto &ag : rq[q].aggs)
            for (auto &t : ag) {
                std::map<int, int> per;
                for (auto &f : t.second)
                    if (is_dup(f.rel)) ++per[f.rel];
                for (auto &kv : per)
                    if ((!gram_q(q) && kv.second >= 2) || t.second.size() >= 3) touched.insert(kv.first);
            }
        if (touched.size() > 1)
            return fail(c, LMFAO_ERR_UNSUPPORTED, "query " + std::to_string(q) + " groups by, filters on or multiplies "
                                                  "attributes of two many-to-many relations");
        if (touched.size() == 1) {
            P.qroot[q] = *touched.begin();
            forced[q] = 1;
        }
    }
    // views towards each root other than the tree root
    std::map<int, int> fk_comp_of;
    for (int q = 0; q < nq; ++q) {
        const int R = P.qroot[q];
        if (R == P.root) continue;
        TargetPlan T;
        T.q = q;
        T.rel = R;
        T.dup = is_dup(R);
        T.filter = rq[q].filter;
        int64_t ocells = 1;
        for (int ci : rq[q].comps) {
            T.gb_comp.push_back(ci);
            T.n_cells *= P.comps[ci].dom;
            if (in_sub(P.comps[ci].src.rel, R)) {
                T.gb_o.push_back(-1);
            } else {
                T.gb_o.push_back((int)T.o_comps.size());
                T.o_comps.push_back(ci);
                ocells *= P.comps[ci].dom;
            }
        }
        int n_terms = 0;
        for (int a = 0; a < (int)rq[q].aggs.size(); ++a)
            for (auto &t : rq[q].aggs[a]) {
                TargetPlan::Term tt;
                tt.agg = a;
                tt.coeff = t.first;
                for (auto &f : t.second) (in_sub(f.rel, R) ? tt.rfac : tt.ofac).push_back(f);
                T.terms.push_back(tt);
                ++n_terms;
            }
        const bool fits = (int)T.o_comps.size() < kMaxKeyComps && n_terms <= kMaxTargetTerms &&
                          (double)P.n_keys[R] * (double)ocells <= (double)(1 << 24) &&
                          (fk_comp_of.count(R) || (int)P.comps.size() < kMaxComp);
        if (!fits) {
            if (forced[q])
                return fail(c, LMFAO_ERR_TOO_LARGE, "query " + std::to_string(q) + " at many-to-many relation " +
                                                        c->rels[R].name + ": its view would group by more than three "
                                                        "other attributes, exceed 2^24 cells, carry more than 16 terms "
                                                        "or need a 33rd group-by component");
            P.qroot[q] = P.root;
            continue;
        }
        auto it = fk_comp_of.find(R);
        if (it == fk_comp_of.end()) {
            Comp cp;
            cp.src = ARef{P.root, P.fk_col[R]};
            cp.dom = P.n_keys[R];
            it = fk_comp_of.emplace(R, (int)P.comps.size()).first;
            P.comps.push_back(cp);
        }
        T.fk_comp = it->second;
        P.targets.push_back(T);
    }
    if (P.targets.size() > 65535) return fail(c, LMFAO_ERR_TOO_LARGE, "more than 65535 queries at other roots");

    // ---- staged order: DFS over relations, own columns in column order --------------------
    P.feats.assign(1, ARef{});
    P.own_feats.assign(m, {});
    P.own_comps.assign(m, {});
    P.sub_feat_lo.assign(m, 0);
    P.sub_feat_n.assign(m, 0);
    P.sub_comp_lo.assign(m, 0);
    P.sub_comp_n.assign(m, 0);
    std::map<ARef, int> feat_id;
    int comp_slot = 0;
    // recursive DFS assigning contiguous subtree ranges
    std::vector<std::pair<int, int>> st;   // (relation, state)
    std::function<void(int)> visit = [&](int r) {
        P.sub_feat_lo[r] = (int)P.feats.size();
        P.sub_comp_lo[r] = comp_slot;
        for (int col = 0; col < (int)c->rels[r].cols.size(); ++col) {
            ARef a{r, col};
            if (feat_set.count(a)) {
                feat_id[a] = (int)P.feats.size();
                P.own_feats[r].push_back((int)P.feats.size());
                P.feats.push_back(a);
            }
        }
        for (size_t ci = 0; ci < P.comps.size(); ++ci)
            if (P.comps[ci].src.rel == r) {
                P.comps[ci].slot = comp_slot++;
                P.own_comps[r].push_back((int)ci);
            }
        for (int ch : P.children[r]) visit(ch);
        P.sub_feat_n[r] = (int)P.feats.size() - P.sub_feat_lo[r];
        P.sub_comp_n[r] = comp_slot - P.sub_comp_lo[r];
    };
    visit(P.root);
    P.n_base = (int)P.feats.size();
    // monomials of degree 3 and 4 are split, factors sorted by staged id, into a degree-1 or 2 part
    // and a degree-2 part: f1 * (f2 f3) and (f1 f2) * (f3 f4); every degree-2 part becomes a derived
    // feature (one per distinct pair), computed per row by the root scan
    P.derived.clear();
    std::map<std::pair<int, int>, int> der_id;
    auto derived_of = [&](int a, int b) {
        if (a > b) std::swap(a, b);
        auto it = der_id.find({a, b});
        if (it == der_id.end()) {
            it = der_id.emplace(std::make_pair(a, b), P.n_base + (int)P.derived.size()).first;
            P.derived.push_back({a, b});
        }
        return it->second;
    };
    auto derive_for = [&](const std::vector<ARef> &fs) {
        if (fs.size() <= 2) return;
        std::vector<int> ids;
        for (auto &f : fs) ids.push_back(feat_id[f]);
        std::sort(ids.begin(), ids.end());
        if (ids.size() == 3) derived_of(ids[1], ids[2]);
        else { derived_of(ids[0], ids[1]); derived_of(ids[2], ids[3]); }
    };
    for (int q = 0; q < nq; ++q)
        if (P.qroot[q] == P.root)
            for (auto &ag : rq[q].aggs)
                for (auto &t : ag) derive_for(t.second);
    for (auto &T : P.targets)   // a view towards another root sums the factors outside its subtree
        for (auto &t : T.terms) derive_for(t.ofac);
    P.n_feat = P.n_base + (int)P.derived.size();
    if (P.n_feat > kMaxFeat)
        return fail(c, LMFAO_ERR_TOO_LARGE, "more than 63 continuous features and products of two of them");
    if (comp_slot > kMaxComp) return fail(c, LMFAO_ERR_TOO_LARGE, "more than 32 group-by components");
    P.own_preds.assign(m, {});
    for (size_t f = 0; f < P.filters.size(); ++f)
        for (size_t k = 0; k < P.filters[f].size(); ++k) P.own_preds[P.filters[f][k].src.rel].push_back({(int)f, (int)k});

    // ---- outputs: covariance block, tables (merge of same group-by + filter) --------
    auto mono = [&](const std::vector<ARef> &fs) -> std::pair<int, int> {
        std::vector<int> ids;
        for (auto &f : fs) ids.push_back(feat_id[f]);
        std::sort(ids.begin(), ids.end());
        int a = 0, b = 0;
        if (ids.size() == 1) b = ids[0];
        else if (ids.size() == 2) { a = ids[0]; b = ids[1]; }
        else if (ids.size() == 3) { a = ids[0]; b = der_id.at({ids[1], ids[2]}); }
        else { a = der_id.at({ids[0], ids[1]}); b = der_id.at({ids[2], ids[3]}); }
        if (a > b) std::swap(a, b);
        return {a, b};
    };
    std::map<std::tuple<std::vector<int>, int, int>, int> table_ids;
    auto table_of = [&](const std::vector<int> &comps, int filter, int wdiv) {
        auto key = std::make_tuple(comps, filter, wdiv);
        auto it = table_ids.find(key);
        if (it == table_ids.end()) {
            Table T;
            T.comps = comps;
            T.filter = filter;
            T.wdiv = wdiv;
            for (int ci : comps) T.n_cells *= P.comps[ci].dom;
            it = table_ids.emplace(key, (int)P.tables.size()).first;
            P.tables.push_back(T);
        }
        return it->second;
    };
    bool gram_used = false;
    P.outs.resize(c->queries.size());
    for (size_t ti = 0; ti < P.targets.size(); ++ti) {
        TargetPlan &T = P.targets[ti];
        Output &O = P.outs[T.q];
        O.target = (int)ti;
        O.n_aggs = (int)rq[T.q].aggs.size();
        O.n_cells = T.n_cells;
        std::vector<int> key{T.fk_comp};
        key.insert(key.end(), T.o_comps.begin(), T.o_comps.end());
        T.table = table_of(key, T.filter, T.dup ? T.rel : -1);
        for (auto &t : T.terms) {
            if (t.ofac.empty()) continue;
            auto mo = mono(t.ofac);
            auto &v = P.tables[T.table].vals;
            if (std::find(v.begin(), v.end(), mo) == v.end()) v.push_back(mo);
            t.val = mo.first * 1000 + mo.second;   // resolved below
        }
    }
    for (size_t qi = 0; qi < c->queries.size(); ++qi) {
        RQ &R = rq[qi];
        Output &O = P.outs[qi];
        if (O.target >= 0) continue;
        O.n_aggs = (int)R.aggs.size();
        if (R.comps.empty() && R.filter < 0) {
            O.gram = true;
            P.need_count = true;
            for (int a = 0; a < O.n_aggs; ++a)
                for (auto &t : R.aggs[a]) {
                    if (t.second.empty()) O.terms.push_back({a, -1, t.first});
                    else {
                        auto mo = mono(t.second);
                        gram_used = true;
                        O.terms.push_back({a, mo.first * 1000 + mo.second, t.first});   // resolved below
                    }
                }
        } else {
            O.table = table_of(R.comps, R.filter, -1);
            O.n_cells = P.tables[O.table].n_cells;
            for (int a = 0; a < O.n_aggs; ++a)
                for (auto &t : R.aggs[a]) {
                    if (t.second.empty()) O.terms.push_back({a, -1, t.first});
                    else {
                        auto mo = mono(t.second);
                        auto &v = P.tables[O.table].vals;
                        if (std::find(v.begin(), v.end(), mo) == v.end()) v.push_back(mo);
                        O.terms.push_back({a, mo.first * 1000 + mo.second, t.first});
                    }
                }
        }
    }
    P.n_gram = gram_used ? P.n_feat : 0;
    // ---- marginal derivation: a table whose key is another same-filter table's key with one
    // component left out, and whose sums that table already carries, is summed from it after
    // the scan instead of being updated per fact row.  (Adding sums to a finer table would
    // move the coarser table's updates onto more cells, not remove them.)  The source with
    // the smallest dropped domain wins.
    if (!c->opts.scan_every_table) {
        std::vector<int> order(P.tables.size());
        for (size_t t = 0; t < order.size(); ++t) order[t] = (int)t;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return P.tables[a].comps.size() < P.tables[b].comps.size(); });
        for (int t : order) {
            int best = -1, best_pos = -1, best_dom = 0;
            for (size_t u = 0; u < P.tables.size(); ++u) {
                const Table &U = P.tables[u];
                const Table &T = P.tables[t];
                if (U.filter != T.filter || U.wdiv != T.wdiv || U.comps.size() != T.comps.size() + 1) continue;
                bool has_vals = true;
                for (auto &v : T.vals)
                    if (std::find(U.vals.begin(), U.vals.end(), v) == U.vals.end()) has_vals = false;
                if (!has_vals) continue;
                for (size_t d = 0; d < U.comps.size(); ++d) {
                    bool same = true;
                    for (size_t i = 0, j = 0; i < U.comps.size() && same; ++i) {
                        if (i == d) continue;
                        same = U.comps[i] == T.comps[j++];
                    }
                    const int dom = P.comps[U.comps[d]].dom;
                    if (same && (best < 0 || dom < best_dom)) { best = (int)u; best_pos = (int)d; best_dom = dom; }
                }
            }
            if (best < 0) continue;
            Table &T = P.tables[t];
            T.from = best;
            T.drop = best_pos;
            ++P.n_derived;
        }
        // passes: longest derived keys first (their sources are scanned or derived earlier)
        std::map<int, std::vector<int>, std::greater<int>> by_len;
        for (size_t t = 0; t < P.tables.size(); ++t)
            if (P.tables[t].from >= 0) by_len[(int)P.tables[t].comps.size()].push_back((int)t);
        for (auto &kv : by_len) P.rollup_passes.push_back(kv.second);
    }
    for (auto &T : P.tables) std::sort(T.vals.begin(), T.vals.end());
    for (auto &T : P.tables) {
        if (T.from < 0) continue;
        const auto &uv = P.tables[T.from].vals;
        for (auto &v : T.vals) {
            const auto it = std::find(uv.begin(), uv.end(), v);
            if (it == uv.end()) return fail(c, LMFAO_ERR_STATE, "internal: derived table value missing from its source");
            T.vmap.push_back((int)(it - uv.begin()));
        }
    }
    for (auto &T : P.targets)
        for (auto &t : T.terms) {
            if (t.val < 0) continue;
            auto &v = P.tables[T.table].vals;
            t.val = (int)(std::find(v.begin(), v.end(), std::make_pair(t.val / 1000, t.val % 1000)) - v.begin());
        }
    for (auto &O : P.outs)
        for (auto &t : O.terms) {
            if (t.src < 0) continue;
            const int a = t.src / 1000, b = t.src % 1000;
            if (O.gram) t.src = a * P.n_gram + b;
            else {
                auto &v = P.tables[O.table].vals;
                t.src = (int)(std::find(v.begin(), v.end(), std::make_pair(a, b)) - v.begin());
            }
        }
    // ---- families: tables with equal value lists and equal key lists across filters (and equal
    // row weighting) ----
    std::set<int> wdivs;
    for (auto &T : P.tables) wdivs.insert(T.wdiv);
    for (int wd : wdivs) {
        std::map<std::pair<std::vector<std::pair<int, int>>, int>, std::vector<int>> by_vf;
        for (size_t t = 0; t < P.tables.size(); ++t)
            if (P.tables[t].from < 0 && P.tables[t].wdiv == wd) by_vf[{P.tables[t].vals, P.tables[t].filter}].push_back((int)t);
        std::map<std::pair<std::vector<std::pair<int, int>>, std::vector<std::vector<int>>>, std::vector<int>> fam_of;
        for (auto &kv : by_vf) {
            std::vector<std::vector<int>> keys;
            for (int t : kv.second) keys.push_back(P.tables[t].comps);
            auto fk = std::make_pair(kv.first.first, keys);
            if (kv.first.second < 0) {
                Family F;
                F.vals = kv.first.first;
                F.keys = keys;
                F.tables = kv.second;
                F.wdiv = wd;
                P.fams.push_back(F);
            } else {
                fam_of[fk].push_back(kv.first.second);
            }
        }
        for (auto &kv : fam_of) {
            Family F;
            F.vals = kv.first.first;
            F.keys = kv.first.second;
            F.filters = kv.second;
            F.wdiv = wd;
            std::sort(F.filters.begin(), F.filters.end());
            for (int f : F.filters)
                for (auto &k : F.keys) {
                    auto &lst = by_vf[{F.vals, f}];
                    int found = -1;
                    for (int t : lst)
                        if (P.tables[t].comps == k) found = t;
                    F.tables.push_back(found);
                }
            P.fams.push_back(F);
        }
    }
    P.table_cells = 0;
    P.table_vals = 0;
    for (auto &T : P.tables) {
        T.glb_cnt = P.table_cells;
        T.glb_val = P.table_vals;
        P.table_cells += T.n_cells;
        P.table_vals += T.n_cells * (int64_t)T.vals.size();
    }
    // ---- record layouts of non-root relations ------------------------------------------------
    P.rec_stride.assign(m, 0);
    P.rec_comp_off.assign(m, 0);
    P.rec_feat_off.assign(m, 0);
    for (int r = 0; r < m; ++r) {
        if (r == P.root) continue;
        P.rec_comp_off[r] = 1 + P.n_mask;
        P.rec_feat_off[r] = P.rec_comp_off[r] + P.sub_comp_n[r];
        P.rec_stride[r] = round_up(P.rec_feat_off[r] + P.sub_feat_n[r], 4);
        if (P.rec_stride[r] > kMaxRecWords) return fail(c, LMFAO_ERR_TOO_LARGE, "view record of " + c->rels[r].name + " too wide");
    }
    // ---- many-to-many children: count-weighted views (see the header for the supported class) --
    P.dup.assign(m, 0);
    P.dup_pairs.assign(m, {});
    P.weighted = false;
    for (int r = 0; r < m; ++r)
        if (r != P.root && c->rels[r].cols[P.pk_col[r]].kind == LMFAO_KEY_MANY) P.dup[r] = 1;
    for (int r = 0; r < m; ++r) {
        if (!P.dup[r]) continue;
        const std::string nm = c->rels[r].name;
        if (P.parent[r] != P.root || !P.children[r].empty())
            return fail(c, LMFAO_ERR_UNSUPPORTED, "many-to-many relation " + nm + " must be a leaf child of the root");
        // its group-by and predicate attributes belong to queries evaluated at it (the target scan
        // reads them from its rows; its per-key record carries neither)
        auto own = [&](int f) { return f >= P.sub_feat_lo[r] && f < P.sub_feat_lo[r] + P.sub_feat_n[r]; };
        for (auto &d : P.derived)
            if (own(d.first) || own(d.second))
                return fail(c, LMFAO_ERR_UNSUPPORTED, "a product of three or four attributes with one of many-to-many relation " + nm);
        for (auto &T : P.tables)
            for (auto &v : T.vals)
                if (own(v.first) && own(v.second))
                    return fail(c, LMFAO_ERR_UNSUPPORTED, "a grouped sum of two attributes of many-to-many relation " + nm);
        if (P.n_gram > 0) {
            for (int a = P.sub_feat_lo[r]; a < P.sub_feat_lo[r] + P.sub_feat_n[r]; ++a)
                for (int b = a; b < P.sub_feat_lo[r] + P.sub_feat_n[r]; ++b) P.dup_pairs[r].push_back({a, b});
        }
        P.weighted = true;
    }
    // ---- statistics (Table 2 analogue) ---------------------------------------------------------
    P.app_aggs = 0;
    for (auto &Q : c->queries) P.app_aggs += 1 + (int)Q.aggs.size();
    P.inter_aggs = 0;
    for (int r = 0; r < m; ++r)
        if (r != P.root) P.inter_aggs += 1 + (P.n_mask ? 1 : 0) + P.sub_comp_n[r] + P.sub_feat_n[r];
    P.views = (m - 1) + (P.n_gram > 0 || P.need_count ? 1 : 0) + (int)P.tables.size();
    P.groups = m;
    return LMFAO_OK;
}

// LDS layout of the root scan for a tile configuration (32-bit words).
struct Layout {
    int n_fact = 0, n_aux = 0, n_quads = 0, nbuf = 2, waves = 2;
    int w_fact = 0, w_aux = 0, w_rec = 0, w_comp = 0, w_der = 0, w_wgt = 0, wave_words = 0;
    int lds_consts = 0, lds_thr = 0, lds_wave = 0, lds_red = 0, thr_words = 0, ngp = 0;
    int total = 0;
};

static int root_aux_count(const Plan &P) {
    std::set<int> cols;
    for (int ci : P.own_comps[P.root]) cols.insert(P.comps[ci].src.col);
    for (auto &fp : P.own_preds[P.root]) cols.insert(P.filters[fp.first][fp.second].src.col);
    return (int)cols.size();
}

static Layout stage_layout(const Plan &P, int mode, int p1, bool tables, int table_words, int nbuf, int waves) {
    Layout L;
    L.nbuf = nbuf;
    L.waves = waves;
    L.n_fact = (int)P.own_feats[P.root].size();
    L.n_aux = root_aux_count(P);
    for (int ch : P.children[P.root]) L.n_quads += P.rec_stride[ch] / 4;
    int w = 0;
    L.w_fact = w;
    w += nbuf * L.n_fact * kColPitch;
    L.w_aux = w;
    w += nbuf * L.n_aux * kColPitch;
    w = round_up(w, 4);
    L.w_rec = w;
    w += nbuf * L.n_quads * 256;
    L.w_comp = w;
    if (tables) w += (int)P.comps.size() * 64;
    L.w_der = w;
    w += (int)P.derived.size() * kColPitch;
    L.w_wgt = w;
    if (P.weighted) w += 64;
    L.wave_words = round_up(w, 4);
    for (int ci : P.own_comps[P.root]) L.thr_words += (int)P.comps[ci].thr.size();
    int o = round_up(table_words, 4);
    L.lds_consts = o;
    o += 128;
    L.lds_thr = o;
    o += round_up(L.thr_words, 4);
    L.lds_wave = o;
    o += waves * L.wave_words;
    L.lds_red = L.lds_wave;
    int red = 0;
    if (mode == 1) {
        L.ngp = round_up(P.n_gram, p1);
        red = 2 * L.ngp * L.ngp;
    } else if (mode >= 2) {
        red = (mode >= 3 ? 3 : 2) * (16 * p1) * (16 * p1) * 2;
    }
    L.total = std::max(o, L.lds_red + red);
    return L;
}

static int table_words_fit(const lmfao_ctx *c, const Plan &P, int mode, int p1, bool tables, int nbuf, int waves) {
    const Layout L = stage_layout(P, mode, p1, tables, 0, nbuf, waves);
    const int limit = (int)(c->lds_limit / 4) - 64;
    return std::max(0, limit - L.total - 16);
}

// place tables: policy 0 all global; 1 greedy (small first) into one partition's LDS;
// 2 split filtered families' filters (or unfiltered tables) over partitions so all fit
static void place_tables(const lmfao_ctx *c, Plan &P, int policy, int budget_words) {
    for (auto &T : P.tables) { T.part = 0; T.lds_cnt = T.lds_val = -1; }
    P.parts = 1;
    if (P.tables.empty() || policy == 0 || budget_words <= 0) return;
    std::vector<char> in_hist(P.tables.size(), 0);   // tables of the count-table scan stay global
    for (auto &F : P.fams)
        if (F.hist)
            for (int t : F.tables) in_hist[t] = 1;
    if (policy == 1) {
        std::vector<int> idx(P.tables.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return P.tables[a].words() < P.tables[b].words(); });
        int used = 0;
        for (int t : idx) {
            const int w = P.tables[t].words();
            if (P.tables[t].from >= 0 || in_hist[t] || used + w > budget_words) continue;
            P.tables[t].lds_cnt = used;
            P.tables[t].lds_val = used + P.tables[t].val_off();
            used += w;
        }
        return;
    }
    // policy 2: units = (family, filter) groups of tables, or single unfiltered tables
    std::vector<std::vector<int>> units;
    for (auto &F : P.fams) {
        const int nk = (int)F.keys.size();
        if (F.hist) continue;
        if (F.filters.empty()) {
            for (int t : F.tables) units.push_back({t});
        } else {
            for (size_t f = 0; f < F.filters.size(); ++f) {
                std::vector<int> u;
                for (int k = 0; k < nk; ++k) u.push_back(F.tables[f * nk + k]);
                units.push_back(u);
            }
        }
    }
    std::vector<int> used(kMaxParts, 0);
    int parts = 1;
    for (auto &u : units) {
        int w = 0;
        for (int t : u) w += P.tables[t].words();
        if (w > budget_words) {   // too big for any partition: global, evaluated by partition 0
            continue;
        }
        int p = 0;
        while (p < kMaxParts && used[p] + w > budget_words) ++p;
        if (p == kMaxParts) continue;
        for (int t : u) {
            P.tables[t].part = p;
            P.tables[t].lds_cnt = used[p];
            P.tables[t].lds_val = used[p] + P.tables[t].val_off();
            used[p] += P.tables[t].words();
        }
        parts = std::max(parts, p + 1);
    }
    P.parts = parts;
    (void)c;
}

// Kernel mode of the covariance block: 0 none, 1 fp32, 2 BF16X3, 3 BF16X4, 4 BF16X6; and the
// products per tile pair of the dedicated scan in each BF16 mode.
static int precision_mode(const Plan &P) {
    if (P.n_gram == 0) return 0;
    switch (P.precision) {
        case LMFAO_FP32: return 1;
        case LMFAO_BF16X3: return 2;
        case LMFAO_BF16X4: return 3;
        default: return 4;
    }
}
static int gram_products(int mode) { return mode == 3 ? 4 : (mode == 4 ? 6 : 3); }

// The dedicated covariance scan applies to a BF16 covariance block of at most 64
// features (16 to 48 of them from the root relation rounded to whole 16-wide tiles:
// at most 2 such tiles), at most kGramMaxChild children with keys below 2^24, and a
// root of at least 64 rows.  *nt and *nf receive its slot tiles and fact tiles.
static bool gram_eligible(const lmfao_ctx *c, const Plan &P, int *nt, int *nf) {
    if (P.mode < 2 || P.n_gram <= 0 || P.n_gram > kGramMaxSlots || !P.derived.empty() || P.weighted) return false;
    if ((int)P.children[P.root].size() > kGramMaxChild) return false;
    if (c->rels[P.root].n_rows < 64) return false;
    for (int ch : P.children[P.root])
        if (P.n_keys[ch] >= (1 << 24) || P.rec_stride[ch] * 4 > 4096) return false;
    const int n_fact = (int)P.own_feats[P.root].size();
    *nt = (P.n_gram + 15) / 16;
    *nf = (n_fact + 15) / 16;
    return *nf <= 2 && *nf <= *nt && gram_kernel(*nt, *nf, gram_products(P.mode), false) != nullptr;
}

// Pair-row record buffers for the dedicated scan: every child record of at most 8 words (two
// quads), each child given two quads, a row's quads contiguous (32 bytes per row).  A row's
// record is then one contiguous piece for its two neighbouring lanes of a gather request.
static bool gram_pair_rows(const Plan &P) {
    for (int ch : P.children[P.root])
        if (P.rec_stride[ch] > 8) return false;
    return true;
}

static size_t gram_lds_bytes(const Plan &P, int waves, int nf) {
    const bool pr = gram_pair_rows(P);
    int quads = 0;
    for (int ch : P.children[P.root]) quads += pr ? 2 : P.rec_stride[ch] / 4;
    // the constant block (64 rows of 16 or 32 bytes); per wave one record buffer and one fact tile
    return (pr ? 2048 : 1024) + (size_t)waves * ((size_t)quads * kQuadBytes + (size_t)nf * 16 * kFactPitch);
}

// word offset in LDS of the first table of family filter i
static int T_start(const Plan &P, const Family &F, size_t i) { return P.tables[F.tables[i * F.keys.size()]].lds_cnt; }

// Whether a filtered family's LDS layout is strided (see FamilyDesc); fills the
// strided fields when it is.  Checked table by table against the formula the
// kernel uses, so any other layout keeps the per-table descriptors.
static bool family_strided(const Plan &P, const Family &F, FamilyDesc &fd) {
    fd.strided = 0;
    const size_t nk = F.keys.size(), nf = F.filters.size();
    if (nf == 0 || nk == 0) return false;
    int unit = 0;
    for (size_t k = 0; k < nk; ++k) unit += P.tables[F.tables[k]].words();
    for (size_t i = 0; i < nf; ++i) {
        const Table &T0 = P.tables[F.tables[i * nk]];
        for (size_t k = 0; k < nk; ++k) {
            const Table &T = P.tables[F.tables[i * nk + k]];
            const Table &R = P.tables[F.tables[k]];
            if (T.lds_cnt < 0 || T.part != T0.part || T.lds_cnt - T0.lds_cnt != R.lds_cnt - T_start(P, F, 0) ||
                T.lds_val - T0.lds_cnt != R.lds_val - T_start(P, F, 0))
                return false;
        }
    }
    int base[kMaxParts], rank[kMaxParts] = {};
    for (size_t i = 0; i < nf; ++i) {
        const Table &T0 = P.tables[F.tables[i * nk]];
        const int p = T0.part;
        if (rank[p] == 0) base[p] = T0.lds_cnt;
        else if (T0.lds_cnt != base[p] + rank[p] * unit) return false;
        ++rank[p];
    }
    fd.strided = 1;
    fd.unit_words = unit;
    for (int p = 0; p < kMaxParts; ++p) fd.part_base[p] = rank[p] ? base[p] : 0;
    return true;
}

// Per-row codes (see CodeScanDesc): tables that are all filtered, with few sums.
static bool codes_eligible(const Plan &P) {
    int n = 0;
    for (auto &F : P.fams) {
        if (F.hist) continue;
        if (F.filters.empty() || (int)F.vals.size() > kMaxCodeVals) return false;
        ++n;
    }
    return n > 0;
}

static bool all_strided(const Plan &P) {
    for (auto &F : P.fams) {
        if (F.hist) continue;
        FamilyDesc fd{};
        if (!family_strided(P, F, fd)) return false;
    }
    return true;
}

constexpr size_t kMaxCodeBytes = (size_t)16 << 30;   // workspace the per-row codes may take

// The count-table scan (see HistDesc) takes the unfiltered COUNT-only families when the root
// scan, as placed, cannot keep all of their tables in one LDS partition (some are global, or
// the tables need several partitions, each a rescan of the root relation).  Every component of
// those tables must fit a 16-bit code below 0xFFFF.  Slices of at most one LDS of cells are
// packed first-fit, largest first; slices of at most 2048 cells get up to 32 replicas (a power
// of two, odd stride) so that the lanes of a wave spread their updates over LDS banks.
static void plan_hist(const lmfao_ctx *c, Plan &P, int budget) {
    for (auto &F : P.fams) F.hist = false;
    P.hist = false;
    P.hist_comps.clear();
    P.hist_slices.clear();
    P.hist_part_begin.clear();
    P.hist_lds_words.clear();
    const Rel &root = c->rels[P.root];
    if (c->opts.no_hist || P.schedule != LMFAO_BATCHED || P.lds_policy != 3 || root.n_rows <= 0 || P.weighted) return;
    std::vector<int> elig;
    bool spill = P.parts > 1;
    for (size_t f = 0; f < P.fams.size(); ++f) {
        const Family &F = P.fams[f];
        if (!F.filters.empty() || !F.vals.empty()) continue;
        bool ok = true;
        for (int t : F.tables) {
            const Table &T = P.tables[t];
            if ((int)T.comps.size() > kMaxKeyComps || T.n_cells > ((int64_t)1 << 31) - 1) ok = false;
            for (int cp : T.comps)
                if (P.comps[cp].dom >= (int)kNoCode) ok = false;
            if (T.lds_cnt < 0) spill = true;
        }
        if (ok) elig.push_back((int)f);
    }
    if (elig.empty() || !spill) return;
    std::set<int> comps;
    for (int f : elig)
        for (int t : P.fams[f].tables)
            for (int cp : P.tables[t].comps) comps.insert(cp);
    const int64_t pitch = round_up((int)std::min<int64_t>(root.n_rows, 1 << 30), 64);
    if ((size_t)comps.size() * (size_t)pitch * 2 > kMaxCodeBytes) return;
    P.hist_comps.assign(comps.begin(), comps.end());
    P.hist_pitch = pitch;
    // slices of every table
    const int cap = (int)(c->lds_limit / 4) - 64;
    std::vector<HistSlice> sl;
    for (int f : elig)
        for (int t : P.fams[f].tables) {
            const Table &T = P.tables[t];
            HistSlice h{};
            h.n_comp = (int)T.comps.size();
            int64_t stride = 1;
            for (int i = h.n_comp - 1; i >= 0; --i) {
                h.code[i] = (int)(std::find(P.hist_comps.begin(), P.hist_comps.end(), T.comps[i]) - P.hist_comps.begin());
                h.stride[i] = (int32_t)stride;
                stride *= P.comps[T.comps[i]].dom;
            }
            h.glb_cnt = T.glb_cnt;
            const int64_t n = T.n_cells;
            const int64_t k = ceil_div(n, cap);
            for (int64_t j = 0; j < k; ++j) {
                HistSlice x = h;
                x.lo = (int32_t)(n * j / k);
                x.n = (int32_t)(n * (j + 1) / k - x.lo);
                x.reps = 1;
                if (x.n <= 2048)
                    while (x.reps < 32 && (int64_t)(2 * x.reps) * x.n <= 4096) x.reps *= 2;
                x.rep_stride = x.n | 1;
                sl.push_back(x);
            }
        }
    auto words = [](const HistSlice &x) { return (x.reps - 1) * x.rep_stride + x.n; };
    std::stable_sort(sl.begin(), sl.end(), [&](const HistSlice &a, const HistSlice &b) { return words(a) > words(b); });
    std::vector<std::vector<HistSlice>> parts;
    std::vector<int> used;
    for (auto &x : sl) {
        size_t p = 0;
        while (p < parts.size() && used[p] + words(x) > cap) ++p;
        if (p == parts.size()) { parts.emplace_back(); used.push_back(0); }
        x.lds_off = used[p];
        used[p] += round_up(words(x), 4);
        parts[p].push_back(x);
    }
    int max_words = 0;
    for (size_t p = 0; p < parts.size(); ++p) {
        P.hist_part_begin.push_back((int32_t)P.hist_slices.size());
        P.hist_slices.insert(P.hist_slices.end(), parts[p].begin(), parts[p].end());
        P.hist_lds_words.push_back(used[p]);
        max_words = std::max(max_words, used[p]);
    }
    P.hist_part_begin.push_back((int32_t)P.hist_slices.size());
    P.hist_lds_bytes = (size_t)max_words * 4;
    // about two rounds of workgroups over the chip (one resident per CU when a partition fills
    // LDS), with the last round as full as it can be: among 3/4x to 2x that many row blocks per
    // partition, the fewest whose last round leaves under 5% of the chip idle, else the fullest
    // (every block also flushes its partition's nonzero cells, so more blocks cost atomics)
    const int nparts = (int)parts.size();
    const int64_t gmin = std::max<int64_t>(1, std::min<int64_t>(ceil_div(2 * (int64_t)c->n_cu, nparts), ceil_div(root.n_rows, 8192)));
    int64_t gx = gmin;
    double best_idle = 1.0;
    for (int64_t g = std::max<int64_t>(1, 3 * gmin / 4); g <= 2 * gmin && g <= std::max<int64_t>(1, ceil_div(root.n_rows, 8192)); ++g) {
        const double r = (double)(g * nparts) / c->n_cu;
        const double idle = (std::ceil(r) - r) / std::ceil(r);
        if (idle < best_idle - 1e-9) { best_idle = idle; gx = g; }
        if (idle < 0.05) break;
    }
    P.hist_rows_per_block = round_up((int)ceil_div(root.n_rows, gx), 8);
    P.hist_grid = (int)ceil_div(root.n_rows, P.hist_rows_per_block);
    for (int f : elig) P.fams[f].hist = true;
    P.hist = true;
    place_tables(c, P, P.lds_policy, budget);
}

static lmfao_status build_physical(lmfao_ctx *c, const TileCfg &cfg) {
    Plan &P = c->plan;
    const Rel &root = c->rels[P.root];
    P.cfg = cfg;
    if (P.weighted && P.n_gram > 0 && P.precision != LMFAO_FP32)
        return fail(c, LMFAO_ERR_UNSUPPORTED, "many-to-many joins need the FP32 covariance form");
    P.mode = precision_mode(P);
    P.n_tiles16 = (P.n_gram + 15) / 16;
    if (P.mode == 1) {
        int gb = cfg.gram_block > 0 ? cfg.gram_block : estimate_gram_block(P.n_gram);
        if (!gram_block_ok(P.n_gram, gb)) gb = estimate_gram_block(P.n_gram);
        if (!gram_block_ok(P.n_gram, gb)) gb = 8;
        P.gram_block = gb;
    }
    const int p1 = P.mode == 1 ? P.gram_block : (P.mode >= 2 ? P.n_tiles16 : 1);
    const bool has_tables = !P.tables.empty();
    // table placement
    int policy = cfg.lds_policy;
    if (policy < 0) policy = 3;
    P.lds_policy = has_tables ? policy : 0;
    // waves per workgroup and staging buffers: the most resident waves per CU
    // (LDS-limited), two buffers when they fit next to the tables
    {
        const size_t lds_cu = 160 * 1024;
        int best = -1;
        for (int nb : {2, 1})
            for (int wv : {4, 2, 1}) {
                if (cfg.waves > 0 && wv != cfg.waves) continue;
                if (cfg.nbuf > 0 && nb != cfg.nbuf) continue;
                const Layout Ly = stage_layout(P, P.mode, p1, has_tables, 0, nb, wv);
                const size_t bytes = (size_t)Ly.total * 4 + 1024;
                if (bytes > c->lds_limit) continue;
                const int per_cu = (int)std::min<size_t>(8 / wv, lds_cu / bytes) * wv;
                const int score = per_cu * 4 + (nb == 2 ? 2 : 0) + (wv >= 2 ? 1 : 0);
                if (score > best) { best = score; P.nbuf = nb; P.waves = wv; }
            }
        if (best < 0) { P.nbuf = 1; P.waves = 1; }
    }
    const int budget = table_words_fit(c, P, P.mode, p1, has_tables, P.nbuf, P.waves);
    place_tables(c, P, P.lds_policy, budget);
    plan_hist(c, P, budget);
    // COUNT-only filtered tables that need several partitions: the root scan runs once with no
    // tables and writes per-row codes; a code scan per partition, with the whole LDS for its
    // tables, replays them (when the codes fit their workspace cap)
    P.codes = false;
    if (!c->opts.no_row_codes && !P.weighted && P.schedule == LMFAO_BATCHED && P.lds_policy == 3 && P.parts > 1 && root.n_rows > 0 &&
        codes_eligible(P)) {
        P.n_mask_codes = P.filters.size() > 32 ? 2 : 1;
        P.n_codes = P.n_mask_codes;
        for (auto &F : P.fams)
            if (!F.hist) P.n_codes += (int)F.keys.size();
        std::set<int> fs;
        for (auto &F : P.fams)
            for (auto &v : F.vals) {
                if (v.first > 0) fs.insert(v.first);
                if (v.second > 0) fs.insert(v.second);
            }
        P.code_feats.assign(fs.begin(), fs.end());
        P.code_feat_col = P.n_codes;
        P.n_codes += (int)P.code_feats.size();
        P.code_pitch = round_up((int)std::min<int64_t>(root.n_rows, 1 << 30), 64);
        const size_t bytes = (size_t)P.n_codes * (size_t)P.code_pitch * 4;
        place_tables(c, P, 2, (int)(c->lds_limit / 4) - 64);
        if (bytes <= kMaxCodeBytes && all_strided(P)) {
            P.codes = true;
            int words = 0;
            for (auto &T : P.tables)
                if (T.lds_cnt >= 0) words = std::max(words, T.lds_cnt + T.words());
            P.code_lds_bytes = (size_t)words * 4;
            P.code_grid = (int)std::max<int64_t>(1, std::min<int64_t>(c->n_cu, ceil_div(root.n_rows, 1024)));
            P.code_rows_per_block = ceil_div(root.n_rows, P.code_grid);
            P.code_grid = (int)std::max<int64_t>(1, ceil_div(root.n_rows, P.code_rows_per_block));
        } else {
            place_tables(c, P, P.lds_policy, budget);
        }
    }
    int gnt = 0, gnf = 0;
    P.gram_waves = cfg.waves > 0 ? cfg.waves : 4;
    const bool gram_ok = gram_eligible(c, P, &gnt, &gnf) && gram_lds_bytes(P, P.gram_waves, gnf) <= c->lds_limit;
    // root launches
    P.root_launches.clear();
    auto make_launch = [&](bool with_gram, const std::vector<int> &fams, int single_table) {
        RootLaunch L;
        L.with_gram = with_gram;
        L.mode = with_gram ? P.mode : 0;
        L.p1 = with_gram ? p1 : 1;
        // the batched launch computes the components of the count-table scan's codes even when no
        // table of its own is left
        L.tables = !fams.empty() || (P.hist && single_table < 0);
        L.fam_ids = fams;
        L.single_table = single_table;
        int max_words = 0;
        int parts = 1;
        if (single_table >= 0) {
            const Table &T = P.tables[single_table];
            max_words = T.lds_cnt >= 0 ? T.words() : 0;
        } else if (L.tables && P.codes) {
            max_words = 0;   // tables live in the code scan
        } else if (L.tables) {
            std::vector<int> w(kMaxParts, 0);
            for (auto &T : P.tables)
                if (T.lds_cnt >= 0) w[T.part] = std::max(w[T.part], T.lds_cnt + T.words());
            for (int p = 0; p < kMaxParts; ++p) max_words = std::max(max_words, w[p]);
            parts = P.parts;
        }
        L.gram = with_gram && gram_ok && !L.tables;
        int occ_waves = 8;   // resident waves per CU the kernel's registers allow
        if (L.gram) {
            L.gnt = gnt;
            L.gnf = gnf;
            L.gpr = gram_pair_rows(P);
            L.waves = P.gram_waves;
            L.lds_bytes = gram_lds_bytes(P, L.waves, gnf);
            occ_waves = gnt >= 4 || L.mode == 4 ? 8 : 12;
        } else {
            const Layout Ly = stage_layout(P, L.mode, L.p1, L.tables, max_words, P.nbuf, P.waves);
            L.lds_bytes = (size_t)Ly.total * 4;
            L.waves = P.waves;
        }
        L.parts = parts;
        // grid: the general scan covers the chip twice at its residency (its workgroups' costs
        // differ with the tables they update); the dedicated scan gives every workgroup the same
        // rows, so one round of resident workgroups, with no second-round tail, is enough
        const int tile = 64 * L.waves;
        const int64_t blocks_needed = std::max<int64_t>(1, ceil_div(root.n_rows, tile));
        const int occ = (int)std::max<size_t>(1, std::min<size_t>(occ_waves / L.waves, (160 * 1024) / std::max<size_t>(L.lds_bytes + 1024, 1)));
        L.resident = occ;
        int gx = cfg.grid_x > 0 ? cfg.grid_x : (L.gram ? 1 : 2) * c->n_cu * occ;
        gx = (int)std::min<int64_t>(gx, blocks_needed);
        gx = std::max(1, std::min(gx, L.gram ? kPartMax / L.waves : kGridMax));
        const int64_t rpb = round_up((int)std::min<int64_t>(ceil_div(root.n_rows, gx), 1 << 30), tile);
        L.grid_x = (int)std::max<int64_t>(1, ceil_div(root.n_rows, std::max<int64_t>(rpb, tile)));
        L.desc.rows_per_block = std::max<int64_t>(rpb, tile);
        return L;
    };
    std::vector<int> all_fams;
    for (size_t f = 0; f < P.fams.size(); ++f)
        if (!P.fams[f].hist) all_fams.push_back((int)f);
    const bool need_gram_launch = P.n_gram > 0 || P.need_count;
    if (P.schedule == LMFAO_BATCHED) {
        P.root_launches.push_back(make_launch(need_gram_launch, all_fams, -1));
    } else {
        if (need_gram_launch) P.root_launches.push_back(make_launch(true, {}, -1));
        for (size_t f = 0; f < P.fams.size(); ++f)
            for (int t : P.fams[f].tables) P.root_launches.push_back(make_launch(false, {(int)f}, t));
    }
    if (P.root_launches.empty()) P.root_launches.push_back(make_launch(false, {}, -1));
    // the root scan addresses columns and view records with 32-bit byte offsets
    if (root.n_rows > ((int64_t)1 << 30)) return fail(c, LMFAO_ERR_TOO_LARGE, "root relation above 2^30 rows");
    for (int ch : P.children[P.root])
        if ((int64_t)P.n_keys[ch] * P.rec_stride[ch] * 4 >= ((int64_t)1 << 32))
            return fail(c, LMFAO_ERR_TOO_LARGE, "view record array above 4 GiB");
    P.grid_x = P.root_launches[0].grid_x;
    P.rows_per_block = P.root_launches[0].desc.rows_per_block;
    for (auto &L : P.root_launches) {
        if (L.lds_bytes > c->lds_limit) return fail(c, LMFAO_ERR_TOO_LARGE, "root scan exceeds the LDS limit");
        if (!L.gram && !root_kernel(L.mode, L.p1, L.tables))
            return fail(c, LMFAO_ERR_TOO_LARGE, "no kernel variant for this covariance size");
    }
    return LMFAO_OK;
}

// ============================================================================
// device images: workspace layout, descriptors
// ============================================================================

struct Blob {
    std::vector<uint8_t> b;
    size_t put(const void *p, size_t n) {
        const size_t off = align_up(b.size(), 16);
        b.resize(off + n);
        if (n) memcpy(b.data() + off, p, n);
        return off;
    }
    template <class T> size_t vec(const std::vector<T> &v) { return put(v.data(), v.size() * sizeof(T)); }
    template <class T> T *at(size_t off) { return reinterpret_cast<T *>(b.data() + off); }
};

static size_t compute_ws(lmfao_ctx *c) {
    Plan &P = c->plan;
    const int m = (int)c->rels.size();
    size_t o = 0;
    c->off_err = o;
    o += kAlign;
    c->off_rec.assign(m, 0);
    c->off_seen.assign(m, 0);
    c->off_dsum.assign(m, 0);
    c->off_dscat.assign(m, 0);
    c->off_hw.assign(m, 0);
    for (int r = 0; r < m; ++r) {
        if (r == P.root) continue;
        c->off_rec[r] = o;
        o = align_up(o + (size_t)P.n_keys[r] * P.rec_stride[r] * 4);
        c->off_seen[r] = o;
        o = align_up(o + (size_t)P.n_keys[r] * 4);
        if (!P.dup[r]) continue;
        c->off_dsum[r] = o;
        o = align_up(o + (size_t)P.n_keys[r] * P.own_feats[r].size() * 8);
        c->off_dscat[r] = o;
        o = align_up(o + (size_t)P.n_keys[r] * P.dup_pairs[r].size() * 8);
        c->off_hw[r] = o;
        if (!P.dup_pairs[r].empty()) o = align_up(o + (size_t)P.n_keys[r] * 8);
    }
    c->off_gcnt = o;
    o = align_up(o + (size_t)P.table_cells * 8);
    c->off_gval = o;
    o = align_up(o + (size_t)P.table_vals * 8);
    const size_t ntri = (size_t)P.n_gram * (P.n_gram + 1) / 2;
    c->off_gpart = o;
    o = align_up(o + (size_t)kPartMax * ntri * 8);
    c->off_cpart = o;
    o = align_up(o + (size_t)kPartMax * 8);
    c->off_gsum = o;
    o = align_up(o + (size_t)kMergeGroups * (ntri + 1) * 8);
    c->off_gram = o;
    o = align_up(o + (size_t)P.n_gram * P.n_gram * 8 + 8);
    c->off_count = o;
    o = align_up(o + 8);
    c->off_zero = o;
    o = align_up(o + 4 * kMaxRecWords);
    c->off_codes = o;
    if (P.codes) o = align_up(o + (size_t)P.n_codes * (size_t)P.code_pitch * 4);
    c->off_hcodes = o;
    if (P.hist) o = align_up(o + P.hist_comps.size() * (size_t)P.hist_pitch * 2);
    c->off_mlp = o;
    o = align_up(o + ((size_t)1 << 20));
    c->off_desc = o;
    return o;   // descriptor blob size added later
}

static lmfao_status build_blob(lmfao_ctx *c) {
    Plan &P = c->plan;
    const int m = (int)c->rels.size();
    Blob B;
    uint8_t *ws = c->ws;
    const size_t dbase = c->off_desc;
    auto dev = [&](size_t blob_off) -> uint64_t { return (uint64_t)(uintptr_t)(ws + dbase + blob_off); };
    uint32_t *err = reinterpret_cast<uint32_t *>(ws + c->off_err);
    // thresholds of components
    std::vector<size_t> thr_off(P.comps.size(), 0);
    for (size_t i = 0; i < P.comps.size(); ++i)
        if (!P.comps[i].thr.empty()) thr_off[i] = B.vec(P.comps[i].thr);
    auto comp_src = [&](int ci) {
        const Comp &cp = P.comps[ci];
        CompSrc s{};
        s.col = c->rels[cp.src.rel].cols[cp.src.col].data;
        s.thr = cp.thr.empty() ? nullptr : reinterpret_cast<const float *>(dev(thr_off[ci]));
        s.nthr = (int)cp.thr.size();
        s.dom = cp.dom;
        return s;
    };
    auto preds_of = [&](int r) {
        std::vector<PredSrc> v;
        for (auto &fp : P.own_preds[r]) {
            const Conj &cj = P.filters[fp.first][fp.second];
            const Col &col = c->rels[cj.src.rel].cols[cj.src.col];
            PredSrc p{};
            p.col = col.data;
            p.is_float = col.dtype == LMFAO_F32;
            p.op = cj.op;
            p.fval = (float)cj.value;
            p.ival = (int32_t)cj.value;
            p.filter = fp.first;
            v.push_back(p);
        }
        return v;
    };
    uint64_t filter_all = 0;
    for (size_t f = 0; f < P.filters.size(); ++f) filter_all |= 1ull << f;
    auto child_srcs = [&](int r, int feat_base, int comp_base) {
        std::vector<ChildSrc> v;
        for (int ch : P.children[r]) {
            ChildSrc s{};
            s.fk = static_cast<const int32_t *>(c->rels[r].cols[P.fk_col[ch]].data);
            s.rec = reinterpret_cast<const uint32_t *>(ws + c->off_rec[ch]);
            s.n_keys = P.n_keys[ch];
            s.stride = P.rec_stride[ch];
            s.n_mask = P.n_mask;
            s.comp_off = P.rec_comp_off[ch];
            s.n_comp = P.sub_comp_n[ch];
            s.comp_dst = P.sub_comp_lo[ch] - comp_base;
            s.feat_off = P.rec_feat_off[ch];
            s.n_feat = P.sub_feat_n[ch];
            s.feat_dst = P.sub_feat_lo[ch] - feat_base;
            s.hw = P.dup[ch] && !P.dup_pairs[ch].empty() ? reinterpret_cast<double *>(ws + c->off_hw[ch]) : nullptr;
            v.push_back(s);
        }
        return v;
    };
    // ---- view scans of non-root relations, grouped by level ----------------------------
    c->level_rels.assign(P.levels, {});
    c->view_desc_off.assign(m, 0);
    c->dup_desc_off.assign(m, 0);
    c->corr_desc_off.assign(m, 0);
    std::vector<ScanDesc> vdescs(m);
    for (int r = 0; r < m; ++r) {
        if (r == P.root) continue;
        if (P.dup[r]) {
            // many-to-many child: per-key aggregation instead of a one-row-per-key record
            DupDesc d{};
            d.n_rows = c->rels[r].n_rows;
            d.key = static_cast<const int32_t *>(c->rels[r].cols[P.pk_col[r]].data);
            std::vector<FeatSrc> fs;
            for (int f : P.own_feats[r]) {
                FeatSrc x{};
                x.col = static_cast<const float *>(c->rels[r].cols[P.feats[f].col].data);
                x.dst = f - P.sub_feat_lo[r];
                fs.push_back(x);
            }
            std::sort(fs.begin(), fs.end(), [](const FeatSrc &a, const FeatSrc &b) { return a.dst < b.dst; });
            std::vector<int32_t> ab, gab;
            for (auto &pr : P.dup_pairs[r]) {
                ab.push_back(pr.first - P.sub_feat_lo[r]);
                ab.push_back(pr.second - P.sub_feat_lo[r]);
                gab.push_back(pr.first);
                gab.push_back(pr.second);
            }
            if (ab.empty()) ab.assign(2, 0);
            if (gab.empty()) gab.assign(2, 0);
            d.feats = reinterpret_cast<const FeatSrc *>(dev(B.vec(fs)));
            d.pair_ab = reinterpret_cast<const int32_t *>(dev(B.vec(ab)));
            d.n_keys = P.n_keys[r];
            d.n_feat = (int)fs.size();
            d.n_pair = (int)P.dup_pairs[r].size();
            d.rec_stride = P.rec_stride[r];
            d.rec_feat_off = P.rec_feat_off[r];
            d.n_mask = P.n_mask;
            d.filter_all = filter_all;
            d.cnt = reinterpret_cast<uint32_t *>(ws + c->off_seen[r]);
            d.sum = reinterpret_cast<double *>(ws + c->off_dsum[r]);
            d.scat = reinterpret_cast<double *>(ws + c->off_dscat[r]);
            d.rec_out = reinterpret_cast<uint32_t *>(ws + c->off_rec[r]);
            d.err = err;
            c->dup_desc_off[r] = B.put(&d, sizeof d);
            CorrDesc cd{};
            cd.n_keys = P.n_keys[r];
            cd.n_pair = d.n_pair;
            cd.n_gram = P.n_gram;
            cd.hw = reinterpret_cast<const double *>(ws + c->off_hw[r]);
            cd.scat = d.scat;
            cd.gram_ab = reinterpret_cast<const int32_t *>(dev(B.vec(gab)));
            cd.gram = reinterpret_cast<double *>(ws + c->off_gram);
            c->corr_desc_off[r] = B.put(&cd, sizeof cd);
            continue;
        }
        c->level_rels[P.height[r]].push_back(r);
        ScanDesc d{};
        d.n_rows = c->rels[r].n_rows;
        std::vector<FeatSrc> fs;
        for (int f : P.own_feats[r]) {
            FeatSrc s{};
            s.col = static_cast<const float *>(c->rels[r].cols[P.feats[f].col].data);
            s.dst = f - P.sub_feat_lo[r];
            fs.push_back(s);
        }
        std::vector<CompSrc> cs;
        for (int ci : P.own_comps[r]) {
            CompSrc s = comp_src(ci);
            s.dst = P.comps[ci].slot - P.sub_comp_lo[r];
            cs.push_back(s);
        }
        auto ps = preds_of(r);
        auto chs = child_srcs(r, P.sub_feat_lo[r], P.sub_comp_lo[r]);
        d.n_feat = (int)fs.size();
        d.n_comp = (int)cs.size();
        d.n_pred = (int)ps.size();
        d.n_child = (int)chs.size();
        d.n_mask = P.n_mask;
        d.filter_all = filter_all;
        d.feats = reinterpret_cast<const FeatSrc *>(dev(B.vec(fs)));
        d.comps = reinterpret_cast<const CompSrc *>(dev(B.vec(cs)));
        d.preds = reinterpret_cast<const PredSrc *>(dev(B.vec(ps)));
        d.children = reinterpret_cast<const ChildSrc *>(dev(B.vec(chs)));
        d.key = static_cast<const int32_t *>(c->rels[r].cols[P.pk_col[r]].data);
        d.n_keys = P.n_keys[r];
        d.rec_stride = P.rec_stride[r];
        d.rec_comp_off = P.rec_comp_off[r];
        d.rec_feat_off = P.rec_feat_off[r];
        d.rec_n_comp = P.sub_comp_n[r];
        d.rec_n_feat = P.sub_feat_n[r];
        d.rec_out = reinterpret_cast<uint32_t *>(ws + c->off_rec[r]);
        d.seen = reinterpret_cast<uint32_t *>(ws + c->off_seen[r]);
        d.err = err;
        vdescs[r] = d;
    }
    // per level: contiguous arrays of ScanDescs (batched); per relation offsets (plain)
    std::vector<size_t> level_off(P.levels, 0);
    for (int L = 0; L < P.levels; ++L) {
        std::vector<ScanDesc> v;
        for (int r : c->level_rels[L]) v.push_back(vdescs[r]);
        level_off[L] = B.vec(v);
        for (size_t i = 0; i < c->level_rels[L].size(); ++i)
            c->view_desc_off[c->level_rels[L][i]] = level_off[L] + i * sizeof(ScanDesc);
    }
    // ---- root scan ------------------------------------------------------------------------------
    const int r0 = P.root;
    std::vector<FeatSrc> rfs;
    for (int f : P.own_feats[r0]) {
        FeatSrc s{};
        s.col = static_cast<const float *>(c->rels[r0].cols[P.feats[f].col].data);
        s.dst = f;
        rfs.push_back(s);
    }
    // fact columns read by components and predicates are copied into LDS columns ("aux")
    std::vector<int> aux_cols;
    auto aux_of = [&](int col) {
        for (size_t i = 0; i < aux_cols.size(); ++i)
            if (aux_cols[i] == col) return (int)i;
        aux_cols.push_back(col);
        return (int)aux_cols.size() - 1;
    };
    std::vector<float> thr_all;
    std::vector<CompSrc> rcs;
    for (int ci : P.own_comps[r0]) {
        CompSrc s = comp_src(ci);
        s.dst = P.comps[ci].slot;
        s.aux = aux_of(P.comps[ci].src.col);
        s.thr_lds = (int)thr_all.size();
        thr_all.insert(thr_all.end(), P.comps[ci].thr.begin(), P.comps[ci].thr.end());
        rcs.push_back(s);
    }
    auto rps = preds_of(r0);
    {
        size_t k = 0;
        for (auto &fp : P.own_preds[r0]) rps[k++].aux = aux_of(P.filters[fp.first][fp.second].src.col);
    }
    auto rch = child_srcs(r0, 0, 0);
    if ((int)rch.size() > 8) return fail(c, LMFAO_ERR_TOO_LARGE, "the root relation has more than 8 children");
    {
        int qb = 0;
        for (auto &ch : rch) { ch.quad_base = qb; qb += ch.stride / 4; }
    }
    // where each staged feature / component of a tile lives: fact column j (-1 - j) or a
    // word of the row-major record buffer ((quad_base + w / 4) * 256 + w % 4)
    std::vector<int32_t> feat_src(std::max(1, P.n_feat), 0), comp_map(std::max<size_t>(1, P.comps.size()), -1);
    for (size_t j = 0; j < P.own_feats[r0].size(); ++j) feat_src[P.own_feats[r0][j]] = -1 - (int)j;
    std::vector<int32_t> der_ab(std::max<size_t>(2, 2 * P.derived.size()), 0);
    for (size_t j = 0; j < P.derived.size(); ++j) {
        feat_src[P.n_base + j] = kDerivedSrc - (int)j;
        der_ab[2 * j] = P.derived[j].first;
        der_ab[2 * j + 1] = P.derived[j].second;
    }
    for (size_t k = 0; k < P.children[r0].size(); ++k) {
        const int ch = P.children[r0][k];
        for (int i = 0; i < P.sub_feat_n[ch]; ++i) {
            const int w = P.rec_feat_off[ch] + i;
            feat_src[P.sub_feat_lo[ch] + i] = (rch[k].quad_base + w / 4) * 256 + w % 4;
        }
        for (int i = 0; i < P.sub_comp_n[ch]; ++i) {
            const int w = P.rec_comp_off[ch] + i;
            comp_map[P.sub_comp_lo[ch] + i] = (rch[k].quad_base + w / 4) * 256 + w % 4;
        }
    }
    const size_t feat_src_off = B.vec(feat_src), comp_src_off = B.vec(comp_map), der_ab_off = B.vec(der_ab);
    std::vector<uint64_t> fact_ptrs;
    for (int f : P.own_feats[r0]) fact_ptrs.push_back((uint64_t)(uintptr_t)c->rels[r0].cols[P.feats[f].col].data);
    while (fact_ptrs.size() % 16) fact_ptrs.push_back(0);   // the scan preloads 16 entries at a time
    if (fact_ptrs.empty()) fact_ptrs.assign(16, 0);
    const size_t fact_cols_off = B.vec(fact_ptrs);
    std::vector<uint64_t> aux_ptrs;
    for (int col : aux_cols) aux_ptrs.push_back((uint64_t)(uintptr_t)c->rels[r0].cols[col].data);
    while (aux_ptrs.size() % 8) aux_ptrs.push_back(0);
    if (aux_ptrs.empty()) aux_ptrs.assign(8, 0);
    const size_t aux_off = B.vec(aux_ptrs);
    if (thr_all.empty()) thr_all.push_back(0.f);
    const size_t thr_all_off = B.vec(thr_all);
    ScanDesc rs{};
    rs.n_rows = c->rels[r0].n_rows;
    rs.n_feat = (int)rfs.size();
    rs.n_comp = (int)rcs.size();
    rs.n_pred = (int)rps.size();
    rs.n_child = (int)rch.size();
    rs.n_mask = P.n_mask;
    rs.filter_all = filter_all;
    rs.feats = reinterpret_cast<const FeatSrc *>(dev(B.vec(rfs)));
    rs.comps = reinterpret_cast<const CompSrc *>(dev(B.vec(rcs)));
    rs.preds = reinterpret_cast<const PredSrc *>(dev(B.vec(rps)));
    rs.children = reinterpret_cast<const ChildSrc *>(dev(B.vec(rch)));
    rs.err = err;
    // keys and values of all tables
    std::vector<KeyDesc> keys;
    std::vector<ValDesc> vals;
    std::vector<int32_t> fbits;
    auto add_key = [&](const std::vector<int> &comps) {
        KeyDesc k{};
        k.n_comp = (int)comps.size();
        int64_t stride = 1;
        for (int i = (int)comps.size() - 1; i >= 0; --i) {
            k.c[i] = P.comps[comps[i]].slot;
            k.s[i] = (int32_t)stride;
            stride *= P.comps[comps[i]].dom;
        }
        k.n_cells = (int32_t)stride;
        keys.push_back(k);
    };
    unsigned long long *gcnt = reinterpret_cast<unsigned long long *>(ws + c->off_gcnt);
    double *gval = reinterpret_cast<double *>(ws + c->off_gval);
    P.n_strided = 0;
    CodeScanDesc csd{};
    for (auto &L : P.root_launches) {
        int code_col = P.n_mask_codes;
        RootDesc D{};
        D.scan = rs;
        D.n_feat = P.n_feat;
        D.n_gram = L.mode != 0 ? P.n_gram : 0;
        D.n_comp = (int)P.comps.size();
        D.do_count = L.with_gram && P.need_count;
        D.gram_part = 0;
        // families of this launch
        std::vector<FamilyDesc> fdesc;
        std::vector<TabDesc> tdesc;
        std::vector<FlushDesc> flushes[kMaxParts];
        int max_words = 0;
        std::vector<int> pw(kMaxParts, 0);
        for (int fi : L.fam_ids) {
            const Family &F = P.fams[fi];
            FamilyDesc fd{};
            {
                const int wr = L.single_table >= 0 ? P.tables[L.single_table].wdiv : F.wdiv;
                const auto &kids = P.children[P.root];
                fd.wdiv = wr < 0 ? -1 : (int)(std::find(kids.begin(), kids.end(), wr) - kids.begin());
            }
            fd.unfiltered = F.filters.empty();
            fd.n_filt = fd.unfiltered ? 1 : (int)F.filters.size();
            fd.filt_base = (int)fbits.size();
            for (int f : F.filters) { fbits.push_back(f); fd.filt_mask |= 1ull << f; }
            fd.val_base = (int)vals.size();
            for (auto &v : F.vals) vals.push_back(ValDesc{(int16_t)v.first, (int16_t)v.second});
            fd.n_vals = (int)F.vals.size();
            fd.tab_base = (int)tdesc.size();
            fd.key_base = (int)keys.size();
            if (L.single_table >= 0) {
                // plain schedule: this launch computes one table, presented as a 1 x 1 family
                const Table &T = P.tables[L.single_table];
                add_key(T.comps);
                fd.n_keys = 1;
                fd.unfiltered = T.filter < 0;
                fd.n_filt = 1;
                fd.filt_mask = T.filter < 0 ? 0 : (1ull << T.filter);
                fd.filt_base = (int)fbits.size();
                if (T.filter >= 0) fbits.push_back(T.filter);
                TabDesc td{};
                td.part = 0;
                td.lds_cnt = T.lds_cnt >= 0 ? 0 : -1;
                td.lds_val = T.lds_cnt >= 0 ? T.val_off() : -1;
                fd.conv = T.lds_cnt < 0 ? 1 : 0;   // a table in global memory
                td.glb_cnt = T.glb_cnt;
                td.glb_val = T.glb_val;
                tdesc.push_back(td);
                fd.part_mask[0] = fd.filt_mask;
                if (td.lds_cnt >= 0) {
                    flushes[0].push_back(FlushDesc{0, T.val_off(), (int)T.n_cells, (int)T.vals.size(), T.glb_cnt, T.glb_val});
                    pw[0] = T.words();
                }
            } else {
                for (auto &k : F.keys) add_key(k);
                fd.n_keys = (int)F.keys.size();
                fd.code_base = code_col;
                code_col += fd.n_keys;
                for (size_t i = 0; i < F.tables.size(); ++i) {
                    const Table &T = P.tables[F.tables[i]];
                    TabDesc td{};
                    td.part = T.part;
                    td.lds_cnt = T.lds_cnt;
                    td.lds_val = T.lds_val;
                    td.glb_cnt = T.glb_cnt;
                    td.glb_val = T.glb_val;
                    tdesc.push_back(td);
                    if (T.lds_cnt < 0) fd.conv = 1;
                    if (T.filter >= 0) fd.part_mask[T.part] |= 1ull << T.filter;
                    if (T.lds_cnt >= 0) {
                        flushes[T.part].push_back(FlushDesc{T.lds_cnt, T.lds_val, (int)T.n_cells, (int)T.vals.size(), T.glb_cnt, T.glb_val});
                        pw[T.part] = std::max(pw[T.part], T.lds_cnt + T.words());
                    }
                }
                if (family_strided(P, F, fd)) {
                    ++P.n_strided;
                    for (int k = 0; k < fd.n_keys; ++k) {
                        const Table &T = P.tables[F.tables[k]];
                        keys[fd.key_base + k].off_cnt = T.lds_cnt - T_start(P, F, 0);
                        keys[fd.key_base + k].off_val = T.lds_val - T_start(P, F, 0);
                    }
                }
            }
            // the convergent pass takes families with global tables: one atomic per wave on the
            // sorted fact's shared cells (a wave's 64 global atomics on one address serialise);
            // for LDS tables the wave sums cost more than the atomics they save (workload 2:
            // 10.9 -> 14.4 ms when unfiltered LDS families went through it too)
            if (fd.strided) fd.conv = 0;
            if (fd.conv) ++D.conv_fams;
            fdesc.push_back(fd);
        }
        for (int p = 0; p < kMaxParts; ++p) max_words = std::max(max_words, pw[p]);
        std::vector<FlushDesc> fl;
        for (int p = 0; p < kMaxParts; ++p) {
            D.flush_base[p] = (int)fl.size();
            D.n_flush[p] = (int)flushes[p].size();
            D.lds_table_words[p] = pw[p];
            fl.insert(fl.end(), flushes[p].begin(), flushes[p].end());
        }
        const bool codes = P.codes && L.tables && L.single_table < 0;
        if (codes) {
            // the tables move to the code scan; this launch writes the codes
            if (code_col != P.code_feat_col) return fail(c, LMFAO_ERR_STATE, "internal: code columns do not match the plan");
            for (int p = 0; p < kMaxParts; ++p) {
                csd.flush_base[p] = D.flush_base[p];
                csd.n_flush[p] = D.n_flush[p];
                csd.lds_table_words[p] = D.lds_table_words[p];
                if ((size_t)pw[p] * 4 > P.code_lds_bytes) return fail(c, LMFAO_ERR_STATE, "internal: code scan LDS");
                D.n_flush[p] = 0;
                D.lds_table_words[p] = 0;
            }
            max_words = 0;
            D.codes = reinterpret_cast<uint32_t *>(ws + c->off_codes);
            D.code_pitch = P.code_pitch;
            D.n_mask_codes = P.n_mask_codes;
            D.n_code_feats = (int)P.code_feats.size();
            D.code_feats = reinterpret_cast<const int32_t *>(dev(B.vec(P.code_feats)));
            D.code_feat_col = P.code_feat_col;
        }
        if (P.hist && L.tables && L.single_table < 0) {
            std::vector<int32_t> slot;
            for (int cp : P.hist_comps) slot.push_back(P.comps[cp].slot);
            D.n_hcodes = (int)slot.size();
            D.hcodes = reinterpret_cast<uint16_t *>(ws + c->off_hcodes);
            D.hcode_pitch = P.hist_pitch;
            D.hcode_comp = reinterpret_cast<const int32_t *>(dev(B.vec(slot)));
        }
        D.n_fam = (int)fdesc.size();
        D.n_parts = L.parts;
        const Layout Ly = stage_layout(P, L.mode, L.p1, L.tables, max_words, P.nbuf, P.waves);
        D.ngp = Ly.ngp;
        D.n_fact = Ly.n_fact;
        D.n_aux = Ly.n_aux;
        D.n_quads = Ly.n_quads;
        D.nbuf = Ly.nbuf;
        D.lds_tables = 0;
        D.lds_consts = Ly.lds_consts;
        D.lds_thr = Ly.lds_thr;
        D.lds_wave = Ly.lds_wave;
        D.wave_words = Ly.wave_words;
        D.w_fact = Ly.w_fact;
        D.w_aux = Ly.w_aux;
        D.w_rec = Ly.w_rec;
        D.w_comp = Ly.w_comp;
        D.lds_red = Ly.lds_red;
        D.n_thr_words = Ly.thr_words;
        D.fact_cols = reinterpret_cast<const float *const *>(dev(fact_cols_off));
        D.feat_src = reinterpret_cast<const int32_t *>(dev(feat_src_off));
        D.n_der = (int)P.derived.size();
        D.w_der = Ly.w_der;
        D.der_ab = reinterpret_cast<const int32_t *>(dev(der_ab_off));
        D.weighted = P.weighted ? 1 : 0;
        D.w_wgt = Ly.w_wgt;
        // weights up to 2^24 are exact in fp32, and a workgroup's weights add up below 2^32
        // in its uint32 LDS counts
        D.max_weight = (uint32_t)std::min<int64_t>(1 << 24, 0xFFFFFFFFll / std::max<int64_t>(1, L.desc.rows_per_block));
        D.comp_src = reinterpret_cast<const int32_t *>(dev(comp_src_off));
        D.aux_cols = reinterpret_cast<const float *const *>(dev(aux_off));
        D.thr_all = reinterpret_cast<const float *>(dev(thr_all_off));
        D.zero_rec = reinterpret_cast<const uint32_t *>(ws + c->off_zero);
        D.rows_per_block = L.desc.rows_per_block;
        D.fams = reinterpret_cast<const FamilyDesc *>(dev(B.vec(fdesc)));
        D.tabs = reinterpret_cast<const TabDesc *>(dev(B.vec(tdesc)));
        D.flush = reinterpret_cast<const FlushDesc *>(dev(B.vec(fl)));
        if (codes) {
            csd.n_rows = c->rels[r0].n_rows;
            csd.rows_per_block = P.code_rows_per_block;
            csd.pitch = P.code_pitch;
            csd.codes = D.codes;
            csd.n_mask_codes = P.n_mask_codes;
            csd.n_fam = D.n_fam;
            csd.fams = D.fams;
            csd.flush = D.flush;
            csd.g_cnt = gcnt;
            csd.g_val = gval;
        }
        D.g_cnt = gcnt;
        D.g_val = gval;
        D.gram_partial = reinterpret_cast<double *>(ws + c->off_gpart);
        D.count_partial = reinterpret_cast<unsigned long long *>(ws + c->off_cpart);
        D.err = err;
        L.desc = D;
        if (L.gram) {
            GramDesc G{};
            G.n_rows = c->rels[r0].n_rows;
            G.rows_per_block = D.rows_per_block;
            G.n_child = (int)rch.size();
            G.n_fact = (int)P.own_feats[r0].size();
            G.n_gram = P.n_gram;
            G.do_count = D.do_count;
            // record buffer of child k: quad-major from quad quad_base, or (pair rows) two quads from 2k
            G.lds_wave0 = L.gpr ? 2048 : 1024;
            auto quad0 = [&](size_t k) { return L.gpr ? 2 * (int)k : rch[k].quad_base; };
            int quads = 0;
            for (size_t k = 0; k < rch.size(); ++k) {
                G.ch[k].fk = rch[k].fk;
                G.ch[k].rec = rch[k].rec;
                G.ch[k].n_keys = (uint32_t)rch[k].n_keys;
                G.ch[k].rec_bytes = (uint32_t)rch[k].stride * 4u;
                G.ch[k].quad0 = quad0(k);
                G.ch[k].n_quads = rch[k].stride / 4;
                quads += L.gpr ? 2 : rch[k].stride / 4;
            }
            G.fact_off = quads * kQuadBytes;
            G.wave_bytes = G.fact_off + L.gnf * 16 * kFactPitch;
            // slots: fact features, then every child's subtree features, the constant, padding
            int ns = 0;
            for (int j = 0; j < G.n_fact; ++j) G.slot[ns++] = GramSlot{j, 0, 0, P.own_feats[r0][j]};
            for (size_t k = 0; k < P.children[r0].size(); ++k) {
                const int ch = P.children[r0][k];
                for (int i = 0; i < P.sub_feat_n[ch]; ++i) {
                    const int w = P.rec_feat_off[ch] + i;
                    // row 0's word w: quad-major (quad w / 4, word w % 4) or pair rows (word w)
                    const int lds = L.gpr ? quad0(k) * kQuadBytes + 4 * w : (quad0(k) + w / 4) * kQuadBytes + (w % 4) * 4;
                    G.slot[ns++] = GramSlot{-1, lds, 1, P.sub_feat_lo[ch] + i};
                }
            }
            G.slot[ns++] = GramSlot{-1, 0, 0, 0};
            if (ns != P.n_gram) return fail(c, LMFAO_ERR_STATE, "covariance slots do not cover the staged features");
            for (; ns < kGramMaxSlots; ++ns) G.slot[ns] = GramSlot{-1, 4, 0, -1};
            G.fact_cols = D.fact_cols;
            G.gram_partial = D.gram_partial;
            G.count_partial = D.count_partial;
            L.gdesc = G;
        }
    }
    // keys/vals/filter bits are shared by all root launches: patch pointers after all were appended
    const size_t keys_off = B.vec(keys), vals_off = B.vec(vals), fb_off = B.vec(fbits);
    for (auto &L : P.root_launches) {
        L.desc.keys = reinterpret_cast<const KeyDesc *>(dev(keys_off));
        L.desc.vals = reinterpret_cast<const ValDesc *>(dev(vals_off));
        L.desc.filt_bits = reinterpret_cast<const int32_t *>(dev(fb_off));
        L.desc_off = L.gram ? B.put(&L.gdesc, sizeof(GramDesc)) : B.put(&L.desc, sizeof(RootDesc));
    }
    if (P.codes) {
        // each value's factors as code columns (-1: the constant 1)
        std::vector<ValDesc> vcols;
        for (auto &v : vals) {
            int16_t col[2];
            const int f[2] = {v.a, v.b};
            for (int i = 0; i < 2; ++i) {
                if (f[i] == 0) { col[i] = -1; continue; }
                const auto it = std::find(P.code_feats.begin(), P.code_feats.end(), f[i]);
                if (it == P.code_feats.end()) return fail(c, LMFAO_ERR_STATE, "internal: summed feature without a code");
                col[i] = (int16_t)(P.code_feat_col + (it - P.code_feats.begin()));
            }
            vcols.push_back(ValDesc{col[0], col[1]});
        }
        csd.val_cols = reinterpret_cast<const ValDesc *>(dev(B.vec(vcols)));
        csd.keys = reinterpret_cast<const KeyDesc *>(dev(keys_off));
        c->code_desc_off = B.put(&csd, sizeof csd);
    }
    if (P.hist) {
        HistDesc hd{};
        hd.n_rows = c->rels[r0].n_rows;
        hd.rows_per_block = P.hist_rows_per_block;
        hd.pitch = P.hist_pitch;
        hd.codes = reinterpret_cast<const uint16_t *>(ws + c->off_hcodes);
        hd.slices = reinterpret_cast<const HistSlice *>(dev(B.vec(P.hist_slices)));
        hd.part_begin = reinterpret_cast<const int32_t *>(dev(B.vec(P.hist_part_begin)));
        hd.lds_words = reinterpret_cast<const int32_t *>(dev(B.vec(P.hist_lds_words)));
        hd.g_cnt = gcnt;
        c->hist_desc_off = B.put(&hd, sizeof hd);
    }
    // ---- merge and assembly ---------------------------------------------------------------------
    MergeDesc md{};
    md.grid = P.root_launches[0].grid_x;
    for (auto &L : P.root_launches)
        if (L.with_gram) md.grid = L.grid_x;
    md.n_gram = P.n_gram;
    for (auto &L : P.root_launches)
        if (L.with_gram && L.gram) md.grid = L.grid_x * L.waves;   // one partial per wave
    md.group_sum = reinterpret_cast<double *>(ws + c->off_gsum);
    md.group_count = reinterpret_cast<unsigned long long *>(ws + c->off_gsum + (size_t)kMergeGroups *
                                                            ((size_t)P.n_gram * (P.n_gram + 1) / 2) * 8);
    md.gram_partial = reinterpret_cast<const double *>(ws + c->off_gpart);
    md.count_partial = P.need_count ? reinterpret_cast<const unsigned long long *>(ws + c->off_cpart) : nullptr;
    md.gram = reinterpret_cast<double *>(ws + c->off_gram);
    md.count = reinterpret_cast<unsigned long long *>(ws + c->off_count);
    c->merge_off = B.put(&md, sizeof md);
    std::vector<OutDesc> outs;
    std::vector<TermDesc> terms;
    std::vector<int32_t> tcount;
    for (auto &O : P.outs) {
        if (O.target >= 0) continue;   // written by the target scan
        OutDesc od{};
        od.kind = O.gram ? SRC_GRAM : SRC_TABLE;
        od.n_aggs = O.n_aggs;
        od.n_cells = O.n_cells;
        od.dst_cnt = (int64_t)(O.cnt_off / 8);
        od.dst_sum = (int64_t)(O.sum_off / 8);
        if (!O.gram) {
            const Table &T = P.tables[O.table];
            od.src_cnt = T.glb_cnt;
            od.src_val = T.glb_val;
            od.src_nvals = (int)T.vals.size();
        }
        od.term_base = (int)terms.size();
        for (auto &t : O.terms) terms.push_back(TermDesc{t.agg, t.src, t.coeff});
        tcount.push_back((int)O.terms.size());
        outs.push_back(od);
    }
    AssembleDesc ad{};
    ad.n_out = (int)outs.size();
    ad.n_gram = P.n_gram;
    ad.outs = reinterpret_cast<const OutDesc *>(dev(B.vec(outs)));
    ad.terms = reinterpret_cast<const TermDesc *>(dev(B.vec(terms)));
    ad.term_count = reinterpret_cast<const int32_t *>(dev(B.vec(tcount)));
    ad.gram = reinterpret_cast<const double *>(ws + c->off_gram);
    ad.count = reinterpret_cast<const unsigned long long *>(ws + c->off_count);
    ad.g_cnt = gcnt;
    ad.g_val = gval;
    ad.res_cnt = reinterpret_cast<unsigned long long *>(c->res);
    ad.res_sum = reinterpret_cast<double *>(c->res);
    c->assemble_off = B.put(&ad, sizeof ad);
    c->assemble_cells = 0;
    for (auto &O : P.outs)
        if (O.target < 0) c->assemble_cells = std::max(c->assemble_cells, O.n_cells);
    c->n_assemble = (int)outs.size();
    // ---- queries at other roots: the view towards R joined with R's keys or rows -----------
    std::vector<TargetDesc> tdescs;
    c->target_items = 0;
    for (auto &T : P.targets) {
        const int R = T.rel;
        const Output &O = P.outs[T.q];
        const Table &V = P.tables[T.table];
        TargetDesc td{};
        td.dup = T.dup ? 1 : 0;
        td.n_gb = (int)T.gb_comp.size();
        td.n_terms = (int)T.terms.size();
        td.n_aggs = O.n_aggs;
        td.n_items = T.dup ? c->rels[R].n_rows : P.n_keys[R];
        td.n_keys = P.n_keys[R];
        td.key = static_cast<const int32_t *>(c->rels[R].cols[P.pk_col[R]].data);
        td.rec = reinterpret_cast<const uint32_t *>(ws + c->off_rec[R]);
        td.rec_stride = P.rec_stride[R];
        td.mask_word = -1;
        if (!T.dup && T.filter >= 0) {
            td.mask_word = 1 + T.filter / 32;
            td.mask_bit = 1u << (T.filter % 32);
        }
        std::vector<PredSrc> tp;
        if (T.dup)
            for (auto &p : preds_of(R))
                if (p.filter == T.filter) tp.push_back(p);
        td.n_pred = (int)tp.size();
        td.preds = reinterpret_cast<const PredSrc *>(dev(B.vec(tp)));
        std::vector<TargetSrc> gs(T.gb_comp.size());
        int64_t stride = 1;
        for (int i = (int)T.gb_comp.size() - 1; i >= 0; --i) {
            const int ci = T.gb_comp[i];
            TargetSrc &g = gs[i];
            g.from_o = T.gb_o[i];
            g.stride = stride;
            stride *= P.comps[ci].dom;
            if (g.from_o >= 0) continue;
            if (T.dup) g.comp = comp_src(ci);
            else g.rec_word = P.rec_comp_off[R] + P.comps[ci].slot - P.sub_comp_lo[R];
        }
        td.gb = reinterpret_cast<const TargetSrc *>(dev(B.vec(gs)));
        std::vector<TargetTerm> tt;
        for (auto &t : T.terms) {
            TargetTerm x{};
            x.agg = t.agg;
            x.val = t.val;
            x.coeff = t.coeff;
            x.n_fac = (int)t.rfac.size();
            for (size_t j = 0; j < t.rfac.size(); ++j) {
                const ARef &f = t.rfac[j];
                x.col[j] = static_cast<const float *>(c->rels[f.rel].cols[f.col].data);
                int fid = 0;
                for (size_t k = 0; k < P.feats.size(); ++k)
                    if (P.feats[k] == f) fid = (int)k;
                x.rec_word[j] = P.rec_feat_off[R] + fid - P.sub_feat_lo[R];
            }
            tt.push_back(x);
        }
        td.terms = reinterpret_cast<const TargetTerm *>(dev(B.vec(tt)));
        td.n_o = (int)T.o_comps.size();
        td.n_ocells = 1;
        for (int j = 0; j < td.n_o; ++j) {
            td.o_dom[j] = P.comps[T.o_comps[j]].dom;
            td.n_ocells *= td.o_dom[j];
        }
        td.n_vals = (int)V.vals.size();
        td.vcnt = gcnt + V.glb_cnt;
        td.vval = gval + V.glb_val;
        td.n_cells = O.n_cells;
        td.lds = O.n_cells * (1 + (int64_t)O.n_aggs) <= kTargetLdsCells ? 1 : 0;
        td.res_cnt = reinterpret_cast<unsigned long long *>(c->res + O.cnt_off);
        td.res_sum = reinterpret_cast<double *>(c->res + O.sum_off);
        td.err = err;
        tdescs.push_back(td);
        c->target_items = std::max(c->target_items, td.n_items);
    }
    c->target_desc_off = B.vec(tdescs);
    // ---- marginal derivation passes ------------------------------------------------------------
    c->rollup_off.clear();
    c->rollup_cells.clear();
    for (auto &pass : P.rollup_passes) {
        std::vector<RollupItem> items;
        std::vector<int32_t> map;
        int64_t mx = 0;
        for (int t : pass) {
            const Table &T = P.tables[t];
            const Table &U = P.tables[T.from];
            RollupItem it{};
            it.t_cnt = T.glb_cnt;
            it.t_val = T.glb_val;
            it.u_cnt = U.glb_cnt;
            it.u_val = U.glb_val;
            it.t_cells = T.n_cells;
            it.t_nvals = (int)T.vals.size();
            it.u_nvals = (int)U.vals.size();
            it.dom = P.comps[U.comps[T.drop]].dom;
            int64_t suffix = 1;
            for (size_t i = T.drop + 1; i < U.comps.size(); ++i) suffix *= P.comps[U.comps[i]].dom;
            it.suffix = (int32_t)suffix;     // <= T.n_cells < 2^31
            it.map_base = (int)map.size();
            map.insert(map.end(), T.vmap.begin(), T.vmap.end());
            items.push_back(it);
            mx = std::max(mx, T.n_cells * (int64_t)(T.vals.size() + 1));
        }
        RollupDesc rd{};
        rd.n_items = (int)items.size();
        rd.items = reinterpret_cast<const RollupItem *>(dev(B.vec(items)));
        rd.map = reinterpret_cast<const int32_t *>(dev(B.vec(map)));
        rd.g_cnt = gcnt;
        rd.g_val = gval;
        c->rollup_off.push_back(B.put(&rd, sizeof rd));
        c->rollup_cells.push_back(mx);
    }
    // ---- fills: error word, records, seen counters, global tables -----------------------------
    std::vector<FillDesc> fills;
    fills.push_back(FillDesc{err, 1});
    fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(ws + c->off_zero), kMaxRecWords});
    for (int r = 0; r < m; ++r) {
        if (r == P.root) continue;
        fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(ws + c->off_rec[r]), (int64_t)P.n_keys[r] * P.rec_stride[r]});
        fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(ws + c->off_seen[r]), (int64_t)P.n_keys[r]});
        if (!P.dup[r]) continue;
        const int64_t nk = P.n_keys[r];
        fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(ws + c->off_dsum[r]), nk * (int64_t)P.own_feats[r].size() * 2});
        fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(ws + c->off_dscat[r]), nk * (int64_t)P.dup_pairs[r].size() * 2});
        if (!P.dup_pairs[r].empty()) fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(ws + c->off_hw[r]), nk * 2});
    }
    for (auto &T : P.targets) {   // the target scan adds into the query's result
        const Output &O = P.outs[T.q];
        fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(c->res + O.cnt_off), O.n_cells * 2});
        fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(c->res + O.sum_off), O.n_cells * O.n_aggs * 2});
    }
    if (P.table_cells) fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(gcnt), P.table_cells * 2});
    if (P.table_vals) fills.push_back(FillDesc{reinterpret_cast<uint32_t *>(gval), P.table_vals * 2});
    c->n_fills = (int)fills.size();
    c->fill_off = B.vec(fills);
    c->blob = std::move(B.b);
    return LMFAO_OK;
}

static void layout_results(Plan &P) {
    size_t o = 0;
    for (auto &O : P.outs) {
        O.cnt_off = o;
        o = align_up(o + (size_t)O.n_cells * 8, 8);
        O.sum_off = o;
        o = align_up(o + (size_t)O.n_cells * O.n_aggs * 8, 8);
    }
    P.res_bytes = align_up(std::max<size_t>(o, 8));
}

static lmfao_status do_plan(lmfao_ctx *c, const TileCfg &cfg) {
    const int precision = c->plan.precision, schedule = c->plan.schedule, planner = c->plan.planner;
    lmfao_status s = build_logical(c);
    if (s != LMFAO_OK) return s;
    c->plan.precision = precision;
    c->plan.schedule = schedule;
    c->plan.planner = planner;
    s = build_physical(c, cfg);
    if (s != LMFAO_OK) return s;
    layout_results(c->plan);
    // workspace: fixed part + an upper bound of the descriptor image
    const size_t fixed = compute_ws(c);
    // bound the blob by building it against a null base once
    uint8_t *save_ws = c->ws, *save_res = c->res;
    c->ws = nullptr;
    c->res = nullptr;
    s = build_blob(c);
    c->ws = save_ws;
    c->res = save_res;
    if (s != LMFAO_OK) return s;
    c->plan.ws_bytes = align_up(fixed + c->blob.size() + 4096);
    c->plan.ok = true;
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_plan(lmfao_ctx *c, const lmfao_plan_opts *opts) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (!c->tree_set) return fail(c, LMFAO_ERR_STATE, "set the join tree first");
    if (c->queries.empty()) return fail(c, LMFAO_ERR_STATE, "no queries");
    lmfao_plan_opts o{};
    o.precision = LMFAO_FP32;
    o.schedule = LMFAO_BATCHED;
    o.planner = LMFAO_HEURISTIC;
    if (opts) o = *opts;
    if (o.precision < LMFAO_FP32 || o.precision > LMFAO_BF16X6 || o.schedule < LMFAO_PLAIN || o.schedule > LMFAO_BATCHED ||
        o.planner < LMFAO_HEURISTIC || o.planner > LMFAO_LEARNED || o.block_rows != 0 || o.grid_blocks < 0 ||
        o.scan_every_table < 0 || o.scan_every_table > 1 || o.no_row_codes < 0 || o.no_row_codes > 1 ||
        o.no_hist < 0 || o.no_hist > 1 || o.root_policy < LMFAO_ROOT_TREE || o.root_policy > LMFAO_ROOT_FIND ||
        !(o.gram_block == 0 || o.gram_block == 2 || o.gram_block == 4 || o.gram_block == 6 || o.gram_block == 8))
        return fail(c, LMFAO_ERR_INVALID_ARG, "bad plan options");
    invalidate(c);
    c->opts = o;
    c->plan.precision = o.precision;
    c->plan.schedule = o.schedule;
    c->plan.planner = o.planner;
    TileCfg cfg;
    cfg.grid_x = o.grid_blocks;
    cfg.gram_block = o.gram_block;
    cfg.lds_policy = -1;
    return do_plan(c, cfg);
}

extern "C" lmfao_status lmfao_query_root(const lmfao_ctx *c, int32_t qid, int32_t *rel) {
    if (!c || !rel) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    if (qid < 0 || qid >= (int)c->plan.qroot.size()) return fail(c, LMFAO_ERR_INVALID_ARG, "bad query id");
    *rel = c->plan.qroot[qid];
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_plan_stats(const lmfao_ctx *c, lmfao_stats *s) {
    if (!c || !s) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    const Plan &P = c->plan;
    memset(s, 0, sizeof *s);
    s->app_aggregates = P.app_aggs;
    s->inter_aggregates = P.inter_aggs;
    s->views = P.views;
    s->groups = P.groups;
    s->levels = P.levels;
    s->features = P.n_gram;
    s->filters = (int)P.filters.size();
    s->tables = (int)P.tables.size();
    s->derived_tables = P.n_derived;
    s->strided_families = P.n_strided;
    s->code_scan = P.codes ? 1 : 0;
    s->hist_scan = P.hist ? 1 : 0;
    s->hist_parts = P.hist ? (int32_t)P.hist_lds_words.size() : 0;
    s->target_queries = (int32_t)P.targets.size();
    s->table_cells = P.table_cells;
    int launches = 1;   // fill
    for (int L = 0; L < P.levels - 1; ++L) {
        int nrel = 0;
        for (int r = 0; r < (int)c->rels.size(); ++r)
            if (r != P.root && P.height[r] == L && !P.dup[r]) ++nrel;
        launches += P.schedule == LMFAO_BATCHED ? (nrel > 0) : nrel;
    }
    for (int r = 0; r < (int)c->rels.size(); ++r)
        if (P.dup[r]) launches += 2 + (P.n_gram > 0 && !P.dup_pairs[r].empty() ? 1 : 0);   // view build, correction
    launches += P.targets.empty() ? 0 : 1;
    launches += (int)P.root_launches.size() + (P.codes ? 1 : 0) + (P.hist ? 1 : 0);
    if (P.n_gram > 0 || P.need_count) launches += 1;
    launches += (int)P.rollup_passes.size();
    launches += 1;   // assemble
    s->launches = launches;
    s->block_rows = (int32_t)std::min<int64_t>(P.rows_per_block, INT32_MAX);
    s->grid_blocks = P.grid_x;
    s->gram_block = P.mode == 1 ? P.gram_block : (P.mode >= 2 ? 16 * P.n_tiles16 : 0);
    s->lds_tables = P.lds_policy;
    s->waves = P.root_launches[0].waves;
    s->nbuf = P.root_launches[0].gram ? 1 : P.nbuf;
    s->lds_bytes = (int32_t)P.root_launches[0].lds_bytes;
    s->dedicated_scan = 0;
    for (auto &L : P.root_launches)
        if (L.gram) s->dedicated_scan = 1;
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_workspace_size(const lmfao_ctx *c, size_t *bytes) {
    if (!c || !bytes) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    *bytes = c->plan.ws_bytes;
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_result_size(const lmfao_ctx *c, size_t *bytes) {
    if (!c || !bytes) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    *bytes = c->plan.res_bytes;
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_result_layout(const lmfao_ctx *c, int32_t qid, int64_t *n_cells, int32_t *n_sums,
                                            size_t *counts_off, size_t *sums_off) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    if (qid < 0 || qid >= (int)c->plan.outs.size()) return fail(c, LMFAO_ERR_INVALID_ARG, "bad query id");
    const Output &O = c->plan.outs[qid];
    if (n_cells) *n_cells = O.n_cells;
    if (n_sums) *n_sums = O.n_aggs;
    if (counts_off) *counts_off = O.cnt_off;
    if (sums_off) *sums_off = O.sum_off;
    return LMFAO_OK;
}

static lmfao_status upload(lmfao_ctx *c) {
    lmfao_status s = build_blob(c);
    if (s != LMFAO_OK) return s;
    if (c->off_desc + c->blob.size() > c->ws_len) return fail(c, LMFAO_ERR_WORKSPACE, "workspace too small for descriptors");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpy(c->ws + c->off_desc, c->blob.data(), c->blob.size(), hipMemcpyHostToDevice));
    for (auto &L : c->plan.root_launches) {
        if (L.gram) {
            GramKernel k = gram_kernel(L.gnt, L.gnf, gram_products(L.mode), L.gpr);
            if (L.lds_bytes > 64 * 1024) HIP_TRY(c, set_gram_lds_limit(k, L.lds_bytes));
        } else {
            RootKernel k = root_kernel(L.mode, L.p1, L.tables);
            if (L.lds_bytes > 64 * 1024) HIP_TRY(c, set_root_lds_limit(k, L.lds_bytes));
        }
    }
    if (c->plan.codes && c->plan.code_lds_bytes > 64 * 1024) HIP_TRY(c, set_code_scan_lds_limit(c->plan.code_lds_bytes));
    if (c->plan.hist && c->plan.hist_lds_bytes > 64 * 1024) HIP_TRY(c, set_hist_lds_limit(c->plan.hist_lds_bytes));
    return LMFAO_OK;
}

static lmfao_status bind_buffers(lmfao_ctx *c, void *workspace, size_t ws_bytes, void *results, size_t res_bytes);

extern "C" lmfao_status lmfao_bind(lmfao_ctx *c, void *workspace, size_t ws_bytes, void *results, size_t res_bytes) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    return bind_buffers(c, workspace, ws_bytes, results, res_bytes);
}

extern "C" lmfao_status lmfao_bind_scratch(lmfao_ctx *c, void *results, size_t res_bytes) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "plan before binding");
    if (!c->has_device) return fail(c, LMFAO_ERR_HIP, "no HIP device");
    uint8_t *sp = nullptr;
    const hipError_t e = scratch_ptr(c->device, &sp);
    if (e != hipSuccess || !sp)
        return fail(c, LMFAO_ERR_HIP, std::string("scratch array lookup: ") + hipGetErrorString(e));
    if (c->plan.ws_bytes > kScratchBytes)
        return fail(c, LMFAO_ERR_WORKSPACE, "the plan needs " + std::to_string(c->plan.ws_bytes) +
                                                " bytes of workspace; the scratch array holds " +
                                                std::to_string(kScratchBytes));
    return bind_buffers(c, sp, kScratchBytes, results, res_bytes);
}

// Binding generation of the scratch array, checked before every execution: a later binding of
// the array by another context has overwritten this context's descriptors.
static lmfao_status check_scratch_owner(lmfao_ctx *c) {
    if (c->scratch_gen && g_scratch[c->device].owner.load() != c->scratch_gen)
        return fail(c, LMFAO_ERR_STATE, "another context has bound this device's scratch array since; bind again");
    return LMFAO_OK;
}

static lmfao_status bind_buffers(lmfao_ctx *c, void *workspace, size_t ws_bytes, void *results, size_t res_bytes) {
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "plan before binding");
    if (!c->has_device) return fail(c, LMFAO_ERR_HIP, "no HIP device");
    if (!workspace || !results) return fail(c, LMFAO_ERR_WORKSPACE, "null buffer");
    if (((uintptr_t)workspace % kAlign) || ((uintptr_t)results % 8))
        return fail(c, LMFAO_ERR_WORKSPACE, "workspace must be 256-byte aligned, results 8-byte aligned");
    if (ws_bytes < c->plan.ws_bytes || res_bytes < c->plan.res_bytes)
        return fail(c, LMFAO_ERR_WORKSPACE, "bound buffers are smaller than required");
    if (c->graph) { (void)hipGraphExecDestroy(c->graph); c->graph = nullptr; }
    if (c->graph_def) { (void)hipGraphDestroy(c->graph_def); c->graph_def = nullptr; }
    c->ws = static_cast<uint8_t *>(workspace);
    c->ws_len = ws_bytes;
    c->res = static_cast<uint8_t *>(results);
    c->res_len = res_bytes;
    c->scratch_gen = 0;
    uint8_t *sp = nullptr;
    if (scratch_ptr(c->device, &sp) == hipSuccess && sp && c->ws == sp) {
        c->scratch_gen = ++g_scratch_gen;
        g_scratch[c->device].owner.store(c->scratch_gen);
    }
    compute_ws(c);
    lmfao_status s = upload(c);
    if (s != LMFAO_OK) return s;
    c->bound = true;
    c->executed = false;
    return LMFAO_OK;
}

// ============================================================================
// execution
// ============================================================================

static lmfao_status enqueue_root(lmfao_ctx *c, hipStream_t st) {
    for (auto &L : c->plan.root_launches) {
        if (L.gram) {
            GramKernel k = gram_kernel(L.gnt, L.gnf, gram_products(L.mode), L.gpr);
            HIP_TRY(c, launch_gram(k, reinterpret_cast<const GramDesc *>(c->ws + c->off_desc + L.desc_off), L.grid_x,
                                   L.waves, L.lds_bytes, st));
            continue;
        }
        RootKernel k = root_kernel(L.mode, L.p1, L.tables);
        HIP_TRY(c, launch_root(k, reinterpret_cast<const RootDesc *>(c->ws + c->off_desc + L.desc_off), L.grid_x, L.parts,
                               L.waves, L.lds_bytes, st));
    }
    const Plan &P = c->plan;
    if (P.codes)
        HIP_TRY(c, launch_code_scan(reinterpret_cast<const CodeScanDesc *>(c->ws + c->off_desc + c->code_desc_off),
                                    P.code_grid, P.parts, P.code_lds_bytes, st));
    if (P.hist)
        HIP_TRY(c, launch_hist(reinterpret_cast<const HistDesc *>(c->ws + c->off_desc + c->hist_desc_off), P.hist_grid,
                               (int)P.hist_lds_words.size(), P.hist_lds_bytes, st));
    return LMFAO_OK;
}

static lmfao_status enqueue_all(lmfao_ctx *c, hipStream_t st) {
    Plan &P = c->plan;
    uint8_t *db = c->ws + c->off_desc;
    HIP_TRY(c, launch_fill(db + c->fill_off, c->n_fills, st));
    for (size_t r = 0; r < c->rels.size(); ++r)
        if (P.dup[r])
            HIP_TRY(c, launch_dup(reinterpret_cast<const DupDesc *>(db + c->dup_desc_off[r]), c->rels[r].n_rows, P.n_keys[r], st));
    for (int L = 0; L + 1 < P.levels; ++L) {
        const auto &rels = c->level_rels[L];
        if (rels.empty()) continue;
        if (P.schedule == LMFAO_BATCHED) {
            int64_t mx = 0;
            for (int r : rels) mx = std::max(mx, c->rels[r].n_rows);
            HIP_TRY(c, launch_views(reinterpret_cast<const ScanDesc *>(db + c->view_desc_off[rels[0]]), (int)rels.size(), mx, st));
        } else {
            for (int r : rels)
                HIP_TRY(c, launch_views(reinterpret_cast<const ScanDesc *>(db + c->view_desc_off[r]), 1, c->rels[r].n_rows, st));
        }
    }
    lmfao_status s = enqueue_root(c, st);
    if (s != LMFAO_OK) return s;
    if (P.n_gram > 0 || P.need_count)
        HIP_TRY(c, launch_merge(reinterpret_cast<const MergeDesc *>(db + c->merge_off), P.n_gram, st));
    for (size_t r = 0; r < c->rels.size(); ++r)
        if (P.dup[r] && P.n_gram > 0)
            HIP_TRY(c, launch_corr(reinterpret_cast<const CorrDesc *>(db + c->corr_desc_off[r]), (int)P.dup_pairs[r].size(), st));
    for (size_t i = 0; i < c->rollup_off.size(); ++i)
        HIP_TRY(c, launch_rollup(reinterpret_cast<const RollupDesc *>(db + c->rollup_off[i]),
                                 (int)P.rollup_passes[i].size(), c->rollup_cells[i], st));
    if (!P.targets.empty())
        HIP_TRY(c, launch_target(reinterpret_cast<const TargetDesc *>(db + c->target_desc_off), (int)P.targets.size(),
                                 c->target_items, st));
    HIP_TRY(c, launch_assemble(reinterpret_cast<const AssembleDesc *>(db + c->assemble_off), c->n_assemble,
                               c->assemble_cells, st));
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_execute(lmfao_ctx *c, void *hip_stream) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (!c->bound) return fail(c, LMFAO_ERR_STATE, "bind buffers before executing");
    if (check_scratch_owner(c) != LMFAO_OK) return LMFAO_ERR_STATE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(c, hipSetDevice(c->device));
    c->last_stream = st;
    c->executed = true;
    if (c->plan.schedule == LMFAO_BATCHED && st != nullptr) {
        if (c->graph && c->graph_stream != st) {
            (void)hipGraphExecDestroy(c->graph);
            c->graph = nullptr;
            (void)hipGraphDestroy(c->graph_def);
            c->graph_def = nullptr;
        }
        if (!c->graph) {
            HIP_TRY(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            lmfao_status s = enqueue_all(c, st);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(st, &g);
            if (s != LMFAO_OK) { if (g) (void)hipGraphDestroy(g); return s; }
            if (e != hipSuccess) return fail(c, LMFAO_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            c->graph_def = g;
            HIP_TRY(c, hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0));
            c->graph_stream = st;
        }
        HIP_TRY(c, hipGraphLaunch(c->graph, st));
        return LMFAO_OK;
    }
    return enqueue_all(c, st);
}

extern "C" lmfao_status lmfao_sync(lmfao_ctx *c) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (!c->executed) return fail(c, LMFAO_ERR_STATE, "nothing executed");
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->last_stream) HIP_TRY(c, hipStreamSynchronize(c->last_stream));
    else HIP_TRY(c, hipDeviceSynchronize());
    uint32_t flags = 0;
    HIP_TRY(c, hipMemcpy(&flags, c->ws + c->off_err, 4, hipMemcpyDeviceToHost));
    if (flags & kErrDomain) return fail(c, LMFAO_ERR_DOMAIN, "a categorical code lies outside its domain");
    if (flags & kErrKeyRange) return fail(c, LMFAO_ERR_DOMAIN, "a child key lies outside [0, domain)");
    if (flags & kErrDupKey) return fail(c, LMFAO_ERR_UNSUPPORTED, "a child relation has a duplicate join key");
    if (flags & kErrWeight)
        return fail(c, LMFAO_ERR_TOO_LARGE, "a fact row joins more tuples than the root scan counts exactly");
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_time_root_group(lmfao_ctx *c, void *hip_stream, int32_t warmup, int32_t reps, double *ms) {
    if (!c || !ms || reps <= 0 || warmup < 0) return LMFAO_ERR_INVALID_ARG;
    if (!c->bound || !c->executed) return fail(c, LMFAO_ERR_STATE, "execute once before timing");
    if (check_scratch_owner(c) != LMFAO_OK) return LMFAO_ERR_STATE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(c, hipSetDevice(c->device));
    for (int i = 0; i < warmup; ++i) {
        lmfao_status s = enqueue_root(c, st);
        if (s != LMFAO_OK) return s;
    }
    hipEvent_t a, b;
    HIP_TRY(c, hipEventCreate(&a));
    HIP_TRY(c, hipEventCreate(&b));
    HIP_TRY(c, hipEventRecord(a, st));
    for (int i = 0; i < reps; ++i) {
        lmfao_status s = enqueue_root(c, st);
        if (s != LMFAO_OK) return s;
    }
    HIP_TRY(c, hipEventRecord(b, st));
    HIP_TRY(c, hipEventSynchronize(b));
    float t = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = (double)t / reps;
    c->last_stream = st;
    return LMFAO_OK;
}

static lmfao_status select_cfg(lmfao_ctx *c, const TileCfg &t);

// The root of each query chosen by measurement: the plan with every query at the tree root and
// the plan of the paper's root assignment, each with the heuristic configuration, are timed
// whole (every launch of an execution) and the faster is kept.
extern "C" lmfao_status lmfao_choose_root(lmfao_ctx *c, void *hip_stream, int32_t reps, int32_t *policy) {
    if (!c || reps <= 0) return LMFAO_ERR_INVALID_ARG;
    if (!c->bound) return fail(c, LMFAO_ERR_STATE, "bind buffers before choosing");
    if (check_scratch_owner(c) != LMFAO_OK) return LMFAO_ERR_STATE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(c, hipSetDevice(c->device));
    TileCfg heur;
    heur.grid_x = c->opts.grid_blocks;
    heur.gram_block = c->opts.gram_block;
    heur.lds_policy = -1;
    double best_ms = 1e300;
    int best = c->opts.root_policy;
    for (int pol : {LMFAO_ROOT_TREE, LMFAO_ROOT_FIND}) {
        c->opts.root_policy = pol;
        lmfao_status s = select_cfg(c, heur);
        if (s != LMFAO_OK || !c->bound) continue;             // does not fit the bound buffers
        if (pol == LMFAO_ROOT_FIND && c->plan.targets.empty()) continue;   // the same plan as the tree root's
        s = enqueue_all(c, st);
        if (s != LMFAO_OK) continue;
        hipEvent_t a, b;
        HIP_TRY(c, hipEventCreate(&a));
        HIP_TRY(c, hipEventCreate(&b));
        HIP_TRY(c, hipEventRecord(a, st));
        for (int i = 0; i < reps && s == LMFAO_OK; ++i) s = enqueue_all(c, st);
        HIP_TRY(c, hipEventRecord(b, st));
        HIP_TRY(c, hipEventSynchronize(b));
        float t = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&t, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (s == LMFAO_OK && (double)t / reps < best_ms) {
            best_ms = (double)t / reps;
            best = pol;
        }
    }
    c->opts.root_policy = best;
    lmfao_status s = select_cfg(c, heur);
    if (s != LMFAO_OK) return s;
    if (policy) *policy = best;
    if (!c->bound) return LMFAO_OK;   // the chosen plan needs more memory than is bound: bind again
    s = lmfao_execute(c, hip_stream);
    if (s == LMFAO_OK) s = lmfao_sync(c);
    return s;
}

// ============================================================================
// candidates, autotuner, learned choice
// ============================================================================

static std::vector<TileCfg> enumerate_candidates(const lmfao_ctx *c) {
    const Plan &P = c->plan;
    std::vector<TileCfg> out;
    std::vector<int> gbs{0};
    if (P.mode == 1) {
        gbs.clear();
        for (int gb : {2, 4, 6})
            if (gram_block_ok(P.n_gram, gb)) gbs.push_back(gb);
        if (gbs.empty()) gbs.push_back(8);
    }
    std::vector<int> pols{0};
    if (!P.tables.empty()) {
        pols = {0, 1, 2};
        // 3 (partitions with per-row codes or the count-table scan) only where either applies
        bool grouped = false;
        for (auto &F : P.fams) grouped = grouped || F.hist || (F.filters.empty() && F.vals.empty());
        if (grouped || codes_eligible(P)) pols.push_back(3);
    }
    if (!P.root_launches.empty() && P.root_launches[0].gram && P.root_launches.size() == 1) {
        // the dedicated covariance scan: one record buffer, no register blocks or tables
        for (int wv : {1, 2, 4})
            for (int per_cu : {4, 8, 12, 16, 24}) {
                if (per_cu % wv) continue;
                TileCfg t;
                t.waves = wv;
                t.nbuf = 1;
                t.grid_x = per_cu / wv * c->n_cu;
                t.gram_block = 0;
                t.lds_policy = 0;
                out.push_back(t);
            }
        return out;
    }
    for (int wv : {1, 2, 4})
        for (int nb : {1, 2})
            for (int per_cu : {2, 3, 4, 6, 8}) {
                if (per_cu % wv) continue;
                for (int gb : gbs)
                    for (int pl : pols) {
                        TileCfg t;
                        t.waves = wv;
                        t.nbuf = nb;
                        t.grid_x = per_cu / wv * c->n_cu;   // workgroups: a whole number of waves per CU
                        t.gram_block = gb;
                        t.lds_policy = pl;
                        out.push_back(t);
                    }
            }
    return out;
}

extern "C" lmfao_status lmfao_candidates(const lmfao_ctx *c, int32_t *n) {
    if (!c || !n) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    *n = (int32_t)enumerate_candidates(c).size();
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_candidate(const lmfao_ctx *c, int32_t i, int32_t cfg[5]) {
    if (!c || !cfg) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    auto v = enumerate_candidates(c);
    if (i < 0 || i >= (int)v.size()) return fail(c, LMFAO_ERR_INVALID_ARG, "bad candidate index");
    cfg[0] = v[i].waves;
    cfg[1] = v[i].nbuf;
    cfg[2] = v[i].grid_x;
    cfg[3] = v[i].gram_block;
    cfg[4] = v[i].lds_policy;
    return LMFAO_OK;
}

// Rounds of workgroups the root scan takes under candidate t: its workgroups over what the
// chip holds at once.  The plan for t is built in a copy of the context (planning is host-only;
// the copy owns no graph), so the caller's context is not touched.
static double candidate_rounds(const lmfao_ctx *c, const TileCfg &t) {
    lmfao_ctx side = *c;
    side.graph = nullptr;
    side.graph_def = nullptr;
    double rounds = 1.0;
    if (build_logical(&side) == LMFAO_OK) {
        side.plan.precision = c->plan.precision;
        side.plan.schedule = c->plan.schedule;
        side.plan.planner = c->plan.planner;
        if (build_physical(&side, t) == LMFAO_OK && !side.plan.root_launches.empty()) {
            const RootLaunch &L = side.plan.root_launches[0];
            rounds = (double)L.grid_x / ((double)std::max(1, c->n_cu) * std::max(1, L.resident));
        }
    }
    return rounds;
}

static void features_of(const lmfao_ctx *c, const TileCfg &t, float *f) {
    const Plan &P = c->plan;
    const double rows = (double)c->rels[P.root].n_rows;
    int64_t child_keys = 0;
    for (int r = 0; r < (int)c->rels.size(); ++r)
        if (r != P.root) child_keys += P.n_keys[r];
    double upd = 0.0;   // table updates per row (filtered tables counted at half)
    for (auto &T : P.tables) upd += (T.filter < 0 ? 1.0 : 0.5) * (1.0 + (double)T.vals.size());
    const int mode = precision_mode(P);
    f[0] = (float)std::log2(rows + 1.0);
    f[1] = (float)P.n_gram;
    f[2] = (float)std::min(64.0, candidate_rounds(c, t));
    f[3] = (float)P.children[P.root].size();
    f[4] = (float)P.comps.size();
    f[5] = (float)std::log2((double)P.tables.size() + 1.0);
    f[6] = (float)std::log2((double)P.table_cells + 1.0);
    f[7] = (float)std::log2(upd + 1.0);
    f[8] = (float)P.filters.size();
    f[9] = (float)t.lds_policy;
    f[10] = (float)std::log2((double)std::max(1, t.grid_x));
    f[11] = (float)(mode == 1 ? t.gram_block : 0);
    f[12] = (float)mode;
    f[13] = (float)std::log2((double)child_keys + 1.0);
    f[14] = (float)t.waves;
    f[15] = (float)t.nbuf;
}

extern "C" lmfao_status lmfao_candidate_features(const lmfao_ctx *c, int32_t i, float *features) {
    if (!c || !features) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    auto v = enumerate_candidates(c);
    if (i < 0 || i >= (int)v.size()) return fail(c, LMFAO_ERR_INVALID_ARG, "bad candidate index");
    features_of(c, v[i], features);
    return LMFAO_OK;
}

// Re-plan with tile configuration t and re-bind the caller's buffers if the new plan fits them
// (buffers once bound stay known, so one candidate that does not fit leaves later ones bindable).
static lmfao_status select_cfg(lmfao_ctx *c, const TileCfg &t) {
    uint8_t *ws = c->ws, *res = c->res;
    const size_t wl = c->ws_len, rl = c->res_len;
    invalidate(c);
    lmfao_status s = do_plan(c, t);
    if (s != LMFAO_OK) return s;
    if (ws && c->plan.ws_bytes <= wl && c->plan.res_bytes <= rl) {
        s = lmfao_bind(c, ws, wl, res, rl);
        if (s != LMFAO_OK) return s;
    }
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_select_candidate(lmfao_ctx *c, int32_t i) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (!c->plan.ok) return fail(c, LMFAO_ERR_STATE, "no plan: call lmfao_plan first");
    auto v = enumerate_candidates(c);
    if (i < 0 || i >= (int)v.size()) return fail(c, LMFAO_ERR_INVALID_ARG, "bad candidate index");
    return select_cfg(c, v[i]);
}

extern "C" lmfao_status lmfao_autotune(lmfao_ctx *c, void *hip_stream, const char *timing_db, int32_t reps, int32_t *best) {
    if (!c || reps <= 0) return LMFAO_ERR_INVALID_ARG;
    if (!c->bound) return fail(c, LMFAO_ERR_STATE, "bind buffers before autotuning");
    if (check_scratch_owner(c) != LMFAO_OK) return LMFAO_ERR_STATE;
    auto cands = enumerate_candidates(c);
    std::FILE *db = timing_db ? std::fopen(timing_db, "a") : nullptr;
    double best_ms = 1e300;
    int best_i = -1;
    for (size_t i = 0; i < cands.size(); ++i) {
        lmfao_status s = select_cfg(c, cands[i]);
        if (s != LMFAO_OK || !c->bound) continue;   // a candidate that does not fit is skipped
        s = lmfao_execute(c, hip_stream);
        if (s == LMFAO_OK) s = lmfao_sync(c);
        double ms = 0.0;
        if (s == LMFAO_OK) s = lmfao_time_root_group(c, hip_stream, 1, reps, &ms);
        if (s != LMFAO_OK) continue;
        if (db) {
            float f[LMFAO_N_FEATURES];
            features_of(c, cands[i], f);
            for (int k = 0; k < LMFAO_N_FEATURES; ++k) std::fprintf(db, "%.6g,", f[k]);
            std::fprintf(db, "%d,%d,%d,%d,%d,%.6f\n", cands[i].waves, cands[i].nbuf, cands[i].grid_x, cands[i].gram_block,
                         cands[i].lds_policy, ms);
        }
        if (ms < best_ms) { best_ms = ms; best_i = (int)i; }
    }
    if (db) std::fclose(db);
    if (best_i < 0) return fail(c, LMFAO_ERR_HIP, "no candidate ran");
    lmfao_status s = select_cfg(c, cands[best_i]);
    if (s == LMFAO_OK) s = lmfao_execute(c, hip_stream);   // leave the views current for timing
    if (s == LMFAO_OK) s = lmfao_sync(c);
    if (s != LMFAO_OK) return s;
    if (best) *best = best_i;
    return LMFAO_OK;
}

// weights file: "LMFAOMLP" | int32 hidden | float mean[16] | float std[16] | float y_mean | float y_std | params
static bool load_weights(const char *path, int &hidden, std::vector<float> &norm, std::vector<float> &params) {
    std::ifstream in(path, std::ios::binary);
    if (!in) return false;
    char magic[8];
    in.read(magic, 8);
    if (!in || memcmp(magic, "LMFAOMLP", 8) != 0) return false;
    int32_t h = 0;
    in.read(reinterpret_cast<char *>(&h), 4);
    if (!in || h <= 0 || h > 1024) return false;
    norm.resize(2 * LMFAO_N_FEATURES + 2);
    in.read(reinterpret_cast<char *>(norm.data()), norm.size() * 4);
    const int np = lmfao_mlp_param_count(h);
    params.resize(np);
    in.read(reinterpret_cast<char *>(params.data()), (size_t)np * 4);
    if (!in) return false;
    hidden = h;
    return true;
}

// ---- training the cost model from the autotuner's timing file ------------------------------------
//
// One line per timed candidate: LMFAO_N_FEATURES features, the 5 configuration values of
// lmfao_candidate, milliseconds.  Lines whose workload features (those not describing the tile
// candidate) agree belong to one workload; a line's target is min(log(ms / best ms of its
// workload), log 4): only the ranking inside a plan matters, and every candidate 4x slower than
// the best is simply bad.  Features and targets are standardised (a constant feature keeps
// scale 1), the parameters are drawn He-style from a SplitMix64 stream (normal values by
// Box-Muller), and full-batch Adam runs on the device with the network's own kernels.
static const int kWorkloadFeatures[] = {0, 1, 3, 4, 5, 6, 7, 8, 12, 13};

struct Timings {
    std::vector<float> x;        // [n][LMFAO_N_FEATURES]
    std::vector<double> ms;
};

static bool read_timings(const char *path, Timings &T, std::string &err) {
    std::ifstream in(path);
    if (!in) { err = std::string("cannot open ") + path; return false; }
    std::string line;
    int ln = 0;
    while (std::getline(in, line)) {
        ++ln;
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        std::vector<double> v;
        std::stringstream ss(line);
        std::string tok;
        while (std::getline(ss, tok, ',')) {
            char *end = nullptr;
            const double d = strtod(tok.c_str(), &end);
            if (end == tok.c_str()) { err = "bad number on line " + std::to_string(ln); return false; }
            v.push_back(d);
        }
        if ((int)v.size() != LMFAO_N_FEATURES + 6 || !(v.back() > 0.0)) {
            err = "line " + std::to_string(ln) + " is not 16 features, 5 configuration values and milliseconds > 0";
            return false;
        }
        for (int f = 0; f < LMFAO_N_FEATURES; ++f) T.x.push_back((float)v[f]);
        T.ms.push_back(v.back());
    }
    if (T.ms.empty()) { err = "no timings"; return false; }
    return true;
}

static uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double unit_open(uint64_t &s) { return ((double)(splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

static size_t train_ws_bytes(int hidden, int n) {
    const int np = lmfao_mlp_param_count(hidden);
    return align_up((size_t)n * LMFAO_N_FEATURES * 4) + align_up((size_t)n * 4) + 4 * align_up((size_t)np * 4) +
           align_up((size_t)lmfao_mlp_scratch_floats(hidden, n) * 4);
}

extern "C" lmfao_status lmfao_train_workspace_size(const char *timing_db, int32_t hidden, size_t *bytes) {
    if (!timing_db || !bytes || lmfao_mlp_param_count(hidden) <= 0) return LMFAO_ERR_INVALID_ARG;
    Timings T;
    std::string err;
    if (!read_timings(timing_db, T, err)) return LMFAO_ERR_INVALID_ARG;
    *bytes = train_ws_bytes(hidden, (int)T.ms.size()) + (size_t)16 * 4 * 1024;   // + room for the losses
    return LMFAO_OK;
}

extern "C" lmfao_status lmfao_train_cost_model(const char *timing_db, const char *weights_out,
                                               const lmfao_train_opts *opts, void *workspace, size_t ws_bytes,
                                               void *hip_stream, float *final_loss) {
    if (!timing_db || !weights_out || !opts || !workspace || opts->epochs < 1 || opts->epochs > 16 * 1024 ||
        !(opts->lr > 0.f) || lmfao_mlp_param_count(opts->hidden) <= 0)
        return LMFAO_ERR_INVALID_ARG;
    Timings T;
    std::string err;
    if (!read_timings(timing_db, T, err)) return LMFAO_ERR_INVALID_ARG;
    const int n = (int)T.ms.size(), H = opts->hidden, np = lmfao_mlp_param_count(H);
    if ((uintptr_t)workspace % kAlign || ws_bytes < train_ws_bytes(H, n) + (size_t)opts->epochs * 4)
        return LMFAO_ERR_WORKSPACE;
    // workloads and targets
    std::map<std::vector<double>, int> group;
    std::vector<int> g(n);
    for (int i = 0; i < n; ++i) {
        std::vector<double> key;
        for (int f : kWorkloadFeatures) key.push_back(std::round((double)T.x[(size_t)i * LMFAO_N_FEATURES + f] * 1e4));
        auto it = group.emplace(key, (int)group.size()).first;
        g[i] = it->second;
    }
    std::vector<double> best(group.size(), INFINITY), y(n);
    for (int i = 0; i < n; ++i) best[g[i]] = std::min(best[g[i]], std::log(T.ms[i]));
    for (int i = 0; i < n; ++i) y[i] = std::min(std::log(T.ms[i]) - best[g[i]], std::log(4.0));
    // standardisation
    std::vector<float> norm(2 * LMFAO_N_FEATURES + 2);
    for (int f = 0; f < LMFAO_N_FEATURES; ++f) {
        double m = 0.0, q = 0.0;
        for (int i = 0; i < n; ++i) m += T.x[(size_t)i * LMFAO_N_FEATURES + f];
        m /= n;
        for (int i = 0; i < n; ++i) {
            const double d = T.x[(size_t)i * LMFAO_N_FEATURES + f] - m;
            q += d * d;
        }
        double sd = std::sqrt(q / n);
        if (sd == 0.0) sd = 1.0;
        norm[f] = (float)m;
        norm[LMFAO_N_FEATURES + f] = (float)sd;
    }
    double ym = 0.0, yq = 0.0;
    for (double v : y) ym += v;
    ym /= n;
    for (double v : y) yq += (v - ym) * (v - ym);
    double ys = std::sqrt(yq / n);
    if (ys == 0.0) ys = 1.0;
    norm[2 * LMFAO_N_FEATURES] = (float)ym;
    norm[2 * LMFAO_N_FEATURES + 1] = (float)ys;
    std::vector<float> xs((size_t)n * LMFAO_N_FEATURES), ts(n);
    for (int i = 0; i < n; ++i) {
        for (int f = 0; f < LMFAO_N_FEATURES; ++f)
            xs[(size_t)i * LMFAO_N_FEATURES + f] =
                (float)(((double)T.x[(size_t)i * LMFAO_N_FEATURES + f] - norm[f]) / norm[LMFAO_N_FEATURES + f]);
        ts[i] = (float)((y[i] - ym) / ys);
    }
    // parameters: W1[H][16], b1[H], W2[H][H], b2[H], W3[H], b3 (He-style; biases zero)
    std::vector<float> p(np, 0.f);
    uint64_t rs = opts->seed;
    auto normal = [&]() {
        const double u1 = unit_open(rs), u2 = unit_open(rs);
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    size_t o = 0;
    for (int i = 0; i < H * LMFAO_N_FEATURES; ++i) p[o++] = (float)(normal() * std::sqrt(2.0 / LMFAO_N_FEATURES));
    o += H;
    for (int i = 0; i < H * H; ++i) p[o++] = (float)(normal() * std::sqrt(2.0 / H));
    o += H;
    for (int i = 0; i < H; ++i) p[o++] = (float)(normal() * std::sqrt(1.0 / H));
    // device buffers in the caller's workspace
    uint8_t *w = static_cast<uint8_t *>(workspace);
    size_t off = 0;
    auto take = [&](size_t bytes) { uint8_t *q = w + off; off += align_up(bytes); return q; };
    float *dx = reinterpret_cast<float *>(take((size_t)n * LMFAO_N_FEATURES * 4));
    float *dt = reinterpret_cast<float *>(take((size_t)n * 4));
    float *dp = reinterpret_cast<float *>(take((size_t)np * 4));
    float *dm = reinterpret_cast<float *>(take((size_t)np * 4));
    float *dv = reinterpret_cast<float *>(take((size_t)np * 4));
    float *dg = reinterpret_cast<float *>(take((size_t)np * 4));
    float *dscr = reinterpret_cast<float *>(take((size_t)lmfao_mlp_scratch_floats(H, n) * 4));
    float *dl = reinterpret_cast<float *>(w + off);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (hipMemcpyAsync(dx, xs.data(), xs.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dt, ts.data(), ts.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dp, p.data(), p.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(dm, 0, (size_t)np * 4, st) != hipSuccess || hipMemsetAsync(dv, 0, (size_t)np * 4, st) != hipSuccess)
        return LMFAO_ERR_HIP;
    lmfao_status s = lmfao_mlp_train(H, dp, dm, dv, dx, dt, n, opts->epochs, opts->lr, dg, dscr, dl, hip_stream);
    if (s != LMFAO_OK) return s;
    float last = 0.f;
    if (hipMemcpyAsync(p.data(), dp, p.size() * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&last, dl + opts->epochs - 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return LMFAO_ERR_HIP;
    if (final_loss) *final_loss = last;
    std::ofstream out(weights_out, std::ios::binary);
    if (!out) return LMFAO_ERR_INVALID_ARG;
    const int32_t h32 = H;
    out.write("LMFAOMLP", 8);
    out.write(reinterpret_cast<const char *>(&h32), 4);
    out.write(reinterpret_cast<const char *>(norm.data()), norm.size() * 4);
    out.write(reinterpret_cast<const char *>(p.data()), p.size() * 4);
    return out ? LMFAO_OK : LMFAO_ERR_INVALID_ARG;
}

// Cost-model scores of every candidate (inference on the device, in the workspace).  Returns
// false with *st == OK when the model is missing or predicts a non-finite value (the caller
// keeps the heuristic configuration).
static bool predict_candidates(lmfao_ctx *c, const char *weights, void *hip_stream, std::vector<TileCfg> &cands,
                               std::vector<float> &y, lmfao_status *status) {
    *status = LMFAO_OK;
    int hidden = 0;
    std::vector<float> norm, params;
    if (!weights || !load_weights(weights, hidden, norm, params)) return false;
    cands = enumerate_candidates(c);
    const int n = (int)cands.size();
    std::vector<float> x((size_t)n * LMFAO_N_FEATURES);
    for (int i = 0; i < n; ++i) {
        features_of(c, cands[i], &x[(size_t)i * LMFAO_N_FEATURES]);
        for (int k = 0; k < LMFAO_N_FEATURES; ++k) {
            float &v = x[(size_t)i * LMFAO_N_FEATURES + k];
            v = (v - norm[k]) / (norm[LMFAO_N_FEATURES + k] > 0.f ? norm[LMFAO_N_FEATURES + k] : 1.f);
        }
    }
    const size_t need = (params.size() + x.size() + n) * 4;
    if (need > ((size_t)1 << 20)) {
        *status = fail(c, LMFAO_ERR_TOO_LARGE, "cost model too large for its scratch");
        return false;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    float *dp = reinterpret_cast<float *>(c->ws + c->off_mlp);
    float *dx = dp + params.size();
    float *dy = dx + x.size();
    y.assign(n, 0.f);
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = hipMemcpyAsync(dp, params.data(), params.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dx, x.data(), x.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = mlp_forward_dev(hidden, dp, dx, n, dy, st);
    if (e == hipSuccess) e = hipMemcpyAsync(y.data(), dy, (size_t)n * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        *status = fail(c, LMFAO_ERR_HIP, hipGetErrorString(e));
        return false;
    }
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(y[i])) return false;
    return n > 0;
}

extern "C" lmfao_status lmfao_choose_learned(lmfao_ctx *c, const char *weights, void *hip_stream, int32_t *best) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (!c->bound) return fail(c, LMFAO_ERR_STATE, "bind buffers before choosing");
    if (check_scratch_owner(c) != LMFAO_OK) return LMFAO_ERR_STATE;
    if (best) *best = -1;
    std::vector<TileCfg> cands;
    std::vector<float> y;
    lmfao_status s = LMFAO_OK;
    if (!predict_candidates(c, weights, hip_stream, cands, y, &s)) return s;   // heuristic stays unless an error
    const int bi = (int)(std::min_element(y.begin(), y.end()) - y.begin());
    s = select_cfg(c, cands[bi]);
    if (s == LMFAO_OK && !c->bound) {   // needs more workspace or result memory than is bound
        if (best) *best = bi;
        return LMFAO_OK;
    }
    if (s == LMFAO_OK) s = lmfao_execute(c, hip_stream);
    if (s == LMFAO_OK) s = lmfao_sync(c);
    if (s != LMFAO_OK) return s;
    if (best) *best = bi;
    return LMFAO_OK;
}

constexpr double kSwitchMargin = 0.02;

extern "C" lmfao_status lmfao_choose_learned_verified(lmfao_ctx *c, const char *weights, void *hip_stream,
                                                      int32_t top_k, int32_t reps, int32_t *best) {
    if (!c) return LMFAO_ERR_INVALID_ARG;
    if (top_k <= 0 || reps <= 0) return fail(c, LMFAO_ERR_INVALID_ARG, "top_k and reps must be positive");
    if (!c->bound) return fail(c, LMFAO_ERR_STATE, "bind buffers before choosing");
    if (check_scratch_owner(c) != LMFAO_OK) return LMFAO_ERR_STATE;
    if (best) *best = -1;
    std::vector<TileCfg> cands;
    std::vector<float> y;
    lmfao_status s = LMFAO_OK;
    if (!predict_candidates(c, weights, hip_stream, cands, y, &s)) return s;
    std::vector<int> order(cands.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return y[a] < y[b]; });
    order.resize(std::min<size_t>(order.size(), (size_t)top_k));
    // the configuration in place is timed too, and kept when none of the ranked ones beats it
    const TileCfg current = c->plan.cfg;
    double current_ms = 1e300;
    s = lmfao_execute(c, hip_stream);
    if (s == LMFAO_OK) s = lmfao_sync(c);
    if (s == LMFAO_OK) s = lmfao_time_root_group(c, hip_stream, 1, reps, &current_ms);
    if (s != LMFAO_OK) current_ms = 1e300;
    double best_ms = 1e300;
    int best_i = -1;
    for (int i : order) {
        s = select_cfg(c, cands[i]);
        if (s != LMFAO_OK || !c->bound) continue;   // a candidate that does not fit is skipped
        s = lmfao_execute(c, hip_stream);
        if (s == LMFAO_OK) s = lmfao_sync(c);
        double ms = 0.0;
        if (s == LMFAO_OK) s = lmfao_time_root_group(c, hip_stream, 1, reps, &ms);
        if (s != LMFAO_OK) continue;
        if (ms < best_ms) { best_ms = ms; best_i = i; }
    }
    if (best_i < 0 && current_ms >= 1e300) return fail(c, LMFAO_ERR_HIP, "no ranked candidate ran");
    // a ranked candidate replaces the configuration in place only when it is faster by more than
    // the run-to-run spread of these timings (about 2%), so the choice does not follow noise
    const bool keep = best_i < 0 || best_ms >= current_ms * (1.0 - kSwitchMargin);
    s = select_cfg(c, keep ? current : cands[best_i]);
    if (s == LMFAO_OK) s = lmfao_execute(c, hip_stream);
    if (s == LMFAO_OK) s = lmfao_sync(c);
    if (s != LMFAO_OK) return s;
    if (best) *best = keep ? -1 : best_i;
    return LMFAO_OK;
}
