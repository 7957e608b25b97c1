// Device-side descriptors shared by the host planner and the HIP kernels.
//
// A plan is a list of scans.  Each scan reads one relation once (the
// multi-output scan of a view group, paper Section 3.5) and either
//   * builds the key-indexed view record of a non-root relation (leaf and
//     snowflake views, Section 3.2), or
//   * evaluates every outgoing view of the root relation: the covariance
//     block of ungrouped sums, a total count, and grouped tables.
//
// View record layout (32-bit words, one record per key of the relation):
//   [0]                 count of joining rows with this key (0 or 1; for a
//                       many-to-many child the number of its rows with the key)
//   [1 .. 1+n_mask)     filter mask words: bit f = every conjunct of filter f
//                       on an attribute of this subtree holds
//   [comp_off ..)       group-by components of this subtree (int32 cells)
//   [feat_off ..)       continuous features of this subtree (fp32)
//   padded to a multiple of 4 words (one 16-byte load per 4 words).
#pragma once
#include <stdint.h>

namespace lmfao {

constexpr int kMaxFeat = 64;      // staged features per row, including the constant 1
constexpr int kMaxComp = 32;      // staged group-by components per row
constexpr int kMaxFilters = 64;   // distinct WHERE conjunctions
constexpr int kMaxKeyComps = 4;   // components of one group-by key
constexpr int kBlock = 256;       // threads per workgroup of every scan (one row per thread)

// error flags accumulated on the device, reported by lmfao_sync
constexpr uint32_t kErrDomain = 1u;     // categorical code outside [0, domain)
constexpr uint32_t kErrDupKey = 2u;     // two rows of a child relation share a key
constexpr uint32_t kErrKeyRange = 4u;   // a primary key outside [0, n_keys)
constexpr uint32_t kErrWeight = 8u;     // a root row joins more tuples than the root scan counts exactly

enum Op : int32_t { OP_LE = 0, OP_LT = 1, OP_GE = 2, OP_GT = 3, OP_EQ = 4, OP_NE = 5 };

struct FeatSrc {          // continuous attribute of the scanned relation -> staged feature slot
    const float *col;
    int32_t dst;
    int32_t pad;
};

struct CompSrc {          // group-by component of the scanned relation -> staged component slot
    const void *col;      // int32 codes, or fp32 values when nthr > 0
    const float *thr;     // sorted thresholds (device) for a bucketed attribute
    int32_t nthr;         // 0: categorical code
    int32_t dom;          // domain of the cell index
    int32_t dst;
    int32_t aux;          // root scan: LDS column holding this attribute; thresholds at thr_lds
    int32_t thr_lds;      // root scan: word offset of the thresholds in the block's LDS copy
    int32_t pad;
};

struct PredSrc {          // one conjunct 1[X op t] of filter `filter`
    const void *col;
    int32_t is_float;
    int32_t op;
    float fval;
    int32_t ival;
    int32_t filter;
    int32_t aux;          // root scan: LDS column holding this attribute
};

struct ChildSrc {         // a child view gathered through a foreign key of the scanned relation
    const int32_t *fk;    // foreign-key column of the scanned relation
    const uint32_t *rec;  // child view records, indexed by key
    int32_t n_keys;
    int32_t stride;       // words per record
    int32_t n_mask;       // mask words carried by the child record
    int32_t comp_off, n_comp, comp_dst;
    int32_t feat_off, n_feat, feat_dst;
    int32_t quad_base;    // root scan: first 16-byte quad of this child in the record buffer
    double *hw;           // root scan, many-to-many child whose scatter completes the covariance
                          // block: per key, the weight of the root rows reaching it over the
                          // child's count (null otherwise)
};

struct ScanDesc {
    int64_t n_rows;
    int32_t n_feat, n_comp, n_pred, n_child;
    int32_t n_mask;               // mask words in use (0, 1 or 2)
    int32_t pad0;
    uint64_t filter_all;          // bits of every filter of the plan
    const FeatSrc *feats;
    const CompSrc *comps;
    const PredSrc *preds;
    const ChildSrc *children;
    // view building only
    const int32_t *key;           // primary-key column
    int32_t n_keys;               // record count (key domain)
    int32_t rec_stride;
    int32_t rec_comp_off, rec_feat_off;
    int32_t rec_n_comp, rec_n_feat;
    uint32_t *rec_out;
    uint32_t *seen;               // per key: rows seen (duplicate detection)
    uint32_t *err;
};

// ---- root multi-output scan ------------------------------------------------

struct KeyDesc {          // group-by key: cell = sum_i comp[c[i]] * s[i]
    int32_t c[kMaxKeyComps];
    int32_t s[kMaxKeyComps];
    int32_t n_comp;
    int32_t n_cells;
    int32_t off_cnt;      // strided families: word offsets of this key's counts and sums
    int32_t off_val;      // from the start of its filter's group of tables
};

struct ValDesc {          // summed monomial x[a] * x[b]; feature 0 is the constant 1
    int16_t a, b;
};

struct TabDesc {          // one table = (filter, key) of a family
    int32_t part;         // table partition (blockIdx.y) that evaluates it
    int32_t lds_cnt;      // word offset of uint32 counts in LDS, or -1 when global
    int32_t lds_val;      // word offset of fp64 sums in LDS
    int32_t pad;
    int64_t glb_cnt;      // index of the first uint64 count in the global count array
    int64_t glb_val;      // index of the first double sum in the global sum array
};

struct FlushDesc {        // an LDS-resident table of one partition, copied out at the end
    int32_t lds_cnt, lds_val;
    int32_t n_cells, n_vals;
    int64_t glb_cnt, glb_val;
};

constexpr int kMaxParts = 16;

struct FamilyDesc {       // tables sharing one list of summed monomials
    int32_t n_filt;       // filters (1 when the family is unfiltered)
    int32_t unfiltered;
    int32_t filt_base;    // into filt_bits (filter bit of each family filter, ascending)
    int32_t n_keys;
    int32_t key_base;     // into keys
    int32_t n_vals;
    int32_t val_base;     // into vals
    int32_t tab_base;     // table (f, k) = tab_base + f * n_keys + k
    uint64_t filt_mask;   // union of the family's filter bits
    uint64_t part_mask[kMaxParts];   // filter bits whose tables belong to each partition
    // Strided layout (filtered families whose tables all sit in LDS): the tables of one
    // filter are a group of unit_words words, and the groups of the filters of partition
    // p follow each other in filter order from part_base[p].  The group of filter bit b
    // then starts at part_base[p] + popcount(part_mask[p] & (2^b - 1)) * unit_words, so no
    // per-lane table descriptor is read.
    int32_t strided;
    int32_t unit_words;
    int32_t part_base[kMaxParts];
    int32_t code_base;    // per-row codes: column of this family's first key
    int32_t wdiv;         // weighted plans: root child whose record count divides the row weight
                          // (views towards a many-to-many child), -1 none
    int32_t conv;         // updated by the root scan's convergent pass (a non-strided family with
                          // tables in global memory)
    int32_t pad_g;
};

constexpr int kColPitch = 68;     // words per 64-row LDS column (64 rows + 4 words of bank padding)
constexpr int kDerivedSrc = -(1 << 20);   // feat_src of derived feature j: kDerivedSrc - j
constexpr int kMaxWaves = 4;      // waves per workgroup of the root scan

struct RootDesc {
    ScanDesc scan;
    int32_t n_feat;       // staged features (feature 0 = constant 1)
    int32_t n_gram;       // covariance block over features [0, n_gram); 0 = none
    int32_t n_comp;       // staged components
    int32_t n_fam;
    int32_t do_count;     // accumulate the total count
    int32_t n_parts;      // table partitions (grid.y)
    int32_t gram_part;    // partition whose workgroups compute the covariance block and count
    int32_t ngp;          // fp32 covariance: features padded to the register block
    // staged feature order: 0 = constant, [1, 1 + n_fact) fact columns, then child subtrees
    int32_t n_fact;       // fact features (copied straight into LDS columns)
    int32_t n_aux;        // fact columns read by components and predicates
    int32_t n_quads;      // 16-byte record quads over all children
    int32_t nbuf;         // 1 or 2 staging buffers per wave (2: the next tile loads during this one)
    // dynamic LDS layout (32-bit words)
    int32_t lds_tables;   // table storage (lds_table_words[part] words)
    int32_t lds_consts;   // a column of ones and a column of zeros (64 words each)
    int32_t lds_thr;      // thresholds of fact components
    int32_t lds_wave;     // first wave region; wave w at lds_wave + w * wave_words
    int32_t wave_words;
    int32_t w_fact;       // wave-relative: nbuf x n_fact columns
    int32_t w_aux;        // wave-relative: nbuf x n_aux columns
    int32_t w_rec;        // wave-relative: nbuf x n_quads x 64 quads (row-major records)
    int32_t w_comp;       // wave-relative: component columns (tables only)
    int32_t lds_red;      // fp64 reduction scratch at the end (aliases the wave regions)
    int32_t n_thr_words;  // thresholds copied to LDS
    int32_t pad0;
    int32_t lds_table_words[kMaxParts];
    int32_t flush_base[kMaxParts], n_flush[kMaxParts];
    int64_t rows_per_block;    // contiguous rows per workgroup (multiple of 64 * waves)
    const float *const *fact_cols;    // [n_fact] fact feature columns, staged order
    const float *const *aux_cols;     // [n_aux] fact columns (as 32-bit words)
    const int32_t *feat_src;          // [n_feat] child feature f: word offset in one record
                                      // buffer (rows 4 words apart); fact feature: -1 - column
    const int32_t *comp_src;          // [n_comp] child component: record word offset; fact: -1
    const float *thr_all;             // [n_thr_words] thresholds of fact components
    const uint32_t *zero_rec;         // a record of zeros (count 0) for keys without a row
    const FamilyDesc *fams;
    const KeyDesc *keys;
    const ValDesc *vals;
    const TabDesc *tabs;
    const FlushDesc *flush;
    const int32_t *filt_bits;
    unsigned long long *g_cnt;
    double *g_val;
    double *gram_partial;              // [grid.x][n_gram * n_gram]
    unsigned long long *count_partial; // [grid.x]
    uint32_t *err;
    // per-row codes (see CodeScanDesc): when set, the tables are not updated here; each row's
    // filter mask (0 when the row does not join) and the cell of every family key are written
    uint32_t *codes;
    int64_t code_pitch;                // words per code column (rows rounded up to 64)
    int32_t n_mask_codes;              // mask columns: 1, or 2 with more than 32 filters
    int32_t n_code_feats;              // staged features summed by the tables, written as fp32 codes
    const int32_t *code_feats;         // [n_code_feats] their staged feature ids
    int32_t code_feat_col;             // column of the first of them
    int32_t n_der;                     // derived features: products of two staged features per row
    int32_t w_der;                     // wave-relative: n_der LDS columns holding them for the tile
    const int32_t *der_ab;             // [n_der][2] staged features of each product
    int32_t n_hcodes;                  // count-table scan: component code columns to write
    uint16_t *hcodes;                  // [n_hcodes][hcode_pitch] component values, 0xFFFF when the
                                       // row does not join (see HistDesc)
    int64_t hcode_pitch;               // u16 entries per column (rows rounded up to 64)
    const int32_t *hcode_comp;         // [n_hcodes] staged component of each column
    // many-to-many children: each row stands for w = product of its children's record counts
    // joined tuples (count-weighted views); COUNT adds w, sums add w * value, the fp32
    // covariance block weights one factor per row (LDS column w_wgt), hw arrays collect w / count
    int32_t weighted;
    int32_t w_wgt;                     // wave-relative: one LDS column of row weights (fp32)
    uint32_t max_weight;               // larger weights raise kErrWeight (u32 LDS counts, fp32)
    int32_t conv_fams;                 // families updated by the convergent pass (see the root scan)
};

// ---- many-to-many child views ------------------------------------------------------
//
// A child whose join key repeats is summarised per key: its row count, the sum of
// each continuous attribute and the sum of every pair product (dup_agg_kernel, one
// thread per row, fp64 atomics), then per key the record (count, filter bits,
// fp32 means) and the within-key scatter sum_i (x_a - mean_a)(x_b - mean_b) =
// sum x_a x_b - sum x_a sum x_b / count in place of the pair sums
// (dup_final_kernel, one thread per key).
struct DupDesc {
    int64_t n_rows;
    const int32_t *key;
    const FeatSrc *feats;          // [n_feat] continuous attributes; dst = record feature index
    const int32_t *pair_ab;        // [n_pair][2] record feature indices a <= b
    int32_t n_keys, n_feat, n_pair, rec_stride;
    int32_t rec_feat_off, n_mask;
    uint64_t filter_all;           // mask bits of the record (no predicate applies to the child)
    uint32_t *cnt;                 // [n_keys] rows per key
    double *sum;                   // [n_keys][n_feat]
    double *scat;                  // [n_keys][n_pair]
    uint32_t *rec_out;
    uint32_t *err;
};

// ---- queries evaluated at another root (directional views, Section 3.2-3.3) ----------
//
// A query whose root R is a child of the tree root is answered from a grouped table of the
// root scan keyed by (join key of R, the query's group-by components outside R's subtree) --
// the view flowing from the tree root towards R -- joined with R: one thread per key of R
// (its view record carries R's subtree: validity, filter bit, components, features) or, for a
// many-to-many R, per row of R (its columns, predicates evaluated here).  For every cell o of
// the view's other components with a nonzero count, the query's cell gets the view's count and,
// per aggregate, sum over terms of coeff * (R's factors) * (the view's sum of the other factors).
struct TargetSrc {        // one group-by position of the query, in query order
    int32_t from_o;       // >= 0: index among the view's non-key components; -1: R's side
    int32_t rec_word;     // R's side, keyed R: record word of the component
    int64_t stride;       // cell stride of this position in the query's result
    CompSrc comp;         // R's side, many-to-many R: the attribute (column, thresholds, domain)
};

constexpr int kMaxTermFactors = 4;
constexpr int kMaxTargetTerms = 16;   // terms of a query evaluated at another root
constexpr int kTargetLdsCells = 3072; // result words (8 bytes) a target scan workgroup keeps in LDS

struct TargetTerm {
    int32_t agg;
    int32_t val;                          // view value index of the other factors; -1: the view's count
    double coeff;
    int32_t n_fac;                        // factors on R's side (0..4)
    int32_t rec_word[kMaxTermFactors];    // keyed R: record words
    int32_t pad;
    const float *col[kMaxTermFactors];    // many-to-many R: columns
};

struct TargetDesc {
    int32_t dup;                     // 1: iterate R's rows (many-to-many); 0: R's keys
    int32_t n_gb, n_terms, n_aggs;
    int64_t n_items;                 // keys or rows of R
    const int32_t *key;              // many-to-many: R's join key column
    const uint32_t *rec;             // keyed: R's view records
    int32_t rec_stride;
    int32_t mask_word;               // keyed: record word holding the query's filter bit, -1 none
    uint32_t mask_bit;
    int32_t n_pred;
    const PredSrc *preds;            // many-to-many: the query's predicates on R
    const TargetSrc *gb;             // [n_gb]
    const TargetTerm *terms;         // [n_terms]
    int64_t n_ocells;                // view cells per key of R
    int32_t n_o;                     // the view's non-key components
    int32_t o_dom[kMaxKeyComps];     // their domains, in key order
    int32_t n_vals;                  // sums per view cell
    int32_t n_keys;                  // key domain of R
    int32_t lds;                     // 1: the result (cells x (count + aggregates) <= kTargetLdsCells) is
                                     // accumulated per workgroup in LDS and added to global memory once
    int64_t n_cells;                 // cells of the query's result
    const unsigned long long *vcnt;  // the view: counts [n_keys * n_ocells]
    const double *vval;              // sums [n_keys * n_ocells][n_vals]
    unsigned long long *res_cnt;     // the query's result cells
    double *res_sum;                 // [cells][n_aggs]
    uint32_t *err;
};

// Covariance entries of two attributes of one many-to-many child: the merged block
// holds sum_rows w * mean_a * mean_b; adding sum_k hw[k] * scatter_ab[k] completes
// them to the sum over joined tuples of x_a * x_b.  One workgroup per pair.
struct CorrDesc {
    int32_t n_keys, n_pair, n_gram, pad;
    const double *hw;              // [n_keys]
    const double *scat;            // [n_keys][n_pair]
    const int32_t *gram_ab;        // [n_pair][2] staged features (covariance indices)
    double *gram;                  // [n_gram][n_gram]
};

// ---- grouped tables from per-row codes -----------------------------------------
//
// When the root group's tables are filtered, sum at most kMaxCodeVals
// monomials, sit in the strided LDS layout and need more than one partition,
// the root scan runs once with no tables and writes per-row codes instead:
// column-major 32-bit words, column 0 (and 1) the filter mask, then one column
// per family key holding the row's cell, then the fp32 value of every feature
// the tables sum (products are formed here, in fp64, as the root scan would).
// This scan then runs once per partition (blockIdx.y), with the whole LDS for
// that partition's tables, and replays the codes: every partition reads four
// bytes per key and row instead of repeating the root scan's gathers,
// bucketing and predicates.
constexpr int kMaxCodeVals = 4;

struct CodeScanDesc {
    int64_t n_rows;
    int64_t rows_per_block;
    int64_t pitch;                     // words per code column
    const uint32_t *codes;
    int32_t n_mask_codes;
    int32_t n_fam;
    const FamilyDesc *fams;            // strided
    const KeyDesc *keys;
    const ValDesc *val_cols;           // per family value (as vals): code columns of its two
                                       // factors, -1 for the constant 1
    const FlushDesc *flush;
    int32_t lds_table_words[kMaxParts];
    int32_t flush_base[kMaxParts], n_flush[kMaxParts];
    unsigned long long *g_cnt;
    double *g_val;
};

// ---- count tables from component codes ------------------------------------------
//
// Unfiltered COUNT-only grouped tables (the pairwise counts of mutual
// information, Section 2, equation (7)) are kept out of the root scan when
// they do not fit its LDS: the root scan writes each row's group-by component
// values once, as 16-bit codes (0xFFFF when the row does not join), and this
// scan counts them.  A table is cut into slices of consecutive cells that fit
// LDS; slices are packed into partitions (blockIdx.y).  A workgroup of a
// partition counts its rows into LDS (tiny slices in several replicas, so
// that the lanes of a wave spread their updates over banks) and adds its
// nonzero cells to the table's global u64 counts.
constexpr uint16_t kNoCode = 0xFFFFu;

struct HistSlice {
    int32_t n_comp;                 // components of the table's key (1..kMaxKeyComps)
    int32_t code[kMaxKeyComps];     // code column of each component
    int32_t stride[kMaxKeyComps];   // cell = sum code[i] * stride[i]
    int32_t lo;                     // the slice holds cells [lo, lo + n) of its table
    int32_t n;
    int32_t lds_off;                // word offset of its first replica in LDS
    int32_t reps;                   // replicas (a power of two), rep_stride words apart
    int32_t rep_stride;
    int64_t glb_cnt;                // index of the table's first u64 count in g_cnt
};

struct HistDesc {
    int64_t n_rows;
    int64_t rows_per_block;         // multiple of 8
    int64_t pitch;                  // u16 entries per code column
    const uint16_t *codes;
    const HistSlice *slices;
    const int32_t *part_begin;      // [n_parts + 1] slices of partition p: [part_begin[p], part_begin[p+1])
    const int32_t *lds_words;       // [n_parts] LDS words of partition p
    unsigned long long *g_cnt;
};

// ---- covariance-only root scan ------------------------------------------------
//
// When the root group is the covariance block (and the total count) alone and
// the block is computed in BF16 on matrix cores, a dedicated scan runs it.  Its
// features live in "slots": [fact features][child record features][the
// constant 1][zero padding], so that a 16-wide MFMA tile draws all of its
// lanes from one kind of source where the counts allow.  Fact columns are
// loaded from HBM in 256-byte runs per column and staged in a per-wave LDS fact
// tile; child view records are gathered into LDS with buffer loads that bypass
// registers; every slot's operand (fact, record or the constant) is read from
// LDS in the MFMA operand layout.

constexpr int kGramMaxChild = 4;
constexpr int kGramMaxSlots = 64;
constexpr int kQuadBytes = 1040;  // one 16-byte quad of 64 rows, plus 16 bytes of bank skew
constexpr int kFactPitch = 272;   // one fact column of a 64-row tile in LDS, plus 16 bytes of bank skew

struct GramSlot {
    int32_t fact;         // >= 0: fact column of this slot; -1: read from LDS
    int32_t lds;          // LDS byte offset of row 0 (record buffer relative when per_buf)
    int32_t per_buf;      // 1: inside a wave's record buffer; 0: the block's constant quad
    int32_t feat;         // staged feature whose covariance row this slot feeds; -1: padding
};

struct GramChild {
    const int32_t *fk;    // foreign-key column of the root relation
    const uint32_t *rec;  // child view records
    uint32_t n_keys;      // records (keys >= n_keys read as a zero record: no join)
    uint32_t rec_bytes;   // bytes per record (multiple of 16)
    int32_t quad0;        // first quad of this child in a record buffer
    int32_t n_quads;
};

struct GramDesc {
    int64_t n_rows;
    int64_t rows_per_block;      // multiple of 64 * waves
    int32_t n_child;
    int32_t n_fact;              // fact slots [0, n_fact)
    int32_t n_gram;              // staged features (rows of the covariance block)
    int32_t do_count;
    int32_t lds_wave0;           // byte offset of wave 0's region (after the constant block)
    int32_t wave_bytes;          // a wave's region: n_quads * kQuadBytes of records, then the fact tile
    int32_t fact_off;            // offset of the fact tile in a wave's region (16 * NF columns of kFactPitch)
    int32_t pad1;
    GramChild ch[kGramMaxChild];
    GramSlot slot[kGramMaxSlots];
    const float *const *fact_cols;       // [n_fact]
    double *gram_partial;                // [grid][n_gram * n_gram], entries i <= j
    unsigned long long *count_partial;   // [grid]
};

// ---- final merge and result assembly -----------------------------------------

// Covariance partials hold the upper triangle (i <= j) packed row by row:
// entry (i, j) at tri_index(i, j, n).
__host__ __device__ inline int tri_index(int i, int j, int n) { return i * n - (i * (i - 1)) / 2 + (j - i); }

constexpr int kMergeGroups = 64;     // first merge pass: partials summed in this many ordered groups

struct MergeDesc {
    int32_t grid;                      // partials to reduce
    int32_t n_gram;
    const double *gram_partial;        // [grid][n_gram * (n_gram + 1) / 2]
    const unsigned long long *count_partial;   // [grid], or null
    double *group_sum;                 // [kMergeGroups][n_gram * (n_gram + 1) / 2]
    unsigned long long *group_count;   // [kMergeGroups]
    double *gram;                      // [n_gram * n_gram], symmetric
    unsigned long long *count;         // total joined tuples
};

// Marginal derivation: a grouped table T whose key is the key of a table U
// (same filter) with one component d left out is the sum of U over d.  Cells
// are row-major in key order, so with S = cells of the components after d,
// cell t of T is the sum over v < dom(d) of U's cell
// (t / S) * dom(d) * S + v * S + t % S.
struct RollupItem {
    int64_t t_cnt, t_val;     // first global count / sum of T
    int64_t u_cnt, u_val;     // first global count / sum of U
    int64_t t_cells;
    int32_t t_nvals;          // sums per cell of T
    int32_t u_nvals;          // sums per cell of U
    int32_t dom;              // domain of the dropped component
    int32_t suffix;           // S
    int32_t map_base;         // into map: U's value index of each of T's values
    int32_t pad;
};

struct RollupDesc {           // one pass: tables of equal key length, sources already final
    int32_t n_items;
    int32_t pad;
    const RollupItem *items;
    const int32_t *map;
    unsigned long long *g_cnt;
    double *g_val;
};

enum SrcKind : int32_t { SRC_GRAM = 0, SRC_TABLE = 1 };

struct OutDesc {          // one query's result
    int32_t kind;         // SRC_GRAM (ungrouped, unfiltered) or SRC_TABLE
    int32_t n_aggs;
    int64_t n_cells;
    int64_t dst_cnt;      // index into the result arena (uint64 units)
    int64_t dst_sum;      // index into the result arena (double units)
    int64_t src_cnt;      // table: first global count
    int64_t src_val;      // table: first global sum
    int32_t src_nvals;    // table: values per cell
    int32_t term_base;    // into terms
    int32_t pad[2];
};

struct TermDesc {         // alpha_agg += coeff * source value
    int32_t agg;
    int32_t src;          // gram: i * n_gram + j; table: value index; -1: the count
    double coeff;
};

struct AssembleDesc {
    int32_t n_out;
    int32_t n_gram;
    const OutDesc *outs;
    const TermDesc *terms;
    const int32_t *term_count;     // terms per output
    const double *gram;
    const unsigned long long *count;
    const unsigned long long *g_cnt;
    const double *g_val;
    unsigned long long *res_cnt;
    double *res_sum;
};

}  // namespace lmfao
