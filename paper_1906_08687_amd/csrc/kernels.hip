// HIP kernels of the aggregate-batch engine, written for gfx950 (CDNA4).
//
//  * view_build_kernel   key-indexed view records of non-root relations
//                        (leaf views and snowflake views that gather a child
//                        view; paper Section 3.2, Example 3.1)
//  * root_scan_kernel    the multi-output scan of the root relation's view
//                        group (Section 3.5): one coalesced pass over the
//                        sorted, column-major fact table; per row the child
//                        views are looked up by key and every outgoing view
//                        is updated: the covariance block sum x x^T over the
//                        features x = [1, continuous attributes] (Section 2,
//                        equation (2) and Appendix C's lockstep aggregate
//                        arrays), the total count, and grouped tables
//                        (COUNT and SUM of monomials GROUP BY components,
//                        optionally restricted by a filter; equations (3),
//                        (4), (7), (8)).
//  * code_scan_kernel    grouped tables over several LDS partitions, updated
//                        from per-row codes the root scan writes once
//  * merge_kernel        fp64 cross-workgroup reduction of the covariance
//                        partials and counts (the domain-parallel partition
//                        merge implied by Section 1.2)
//  * rollup_kernel       grouped tables derived from a finer table with the
//                        same filter by summing out one component
//  * assemble_kernel     per-query results from the merged views
//
// The covariance-only scan on matrix cores (gram_scan_kernel) is in
// gram_scan.hip; helpers both files use are in device.h.
//
// The covariance block is computed in one of four arithmetics:
//   FP32      register-blocked fp32 FMAs over a row tile staged in LDS;
//   BF16X3    every feature split x = hi + lo (bf16, round to nearest even),
//             hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with fp32
//             accumulation;
//   BF16X4    adds lo*lo;
//   BF16X6    three pieces x = hi + mid + lo: hi*hi + hi*mid + mid*hi + mid*mid
//             + hi*lo + lo*hi, every term down to 2^-16 of a product kept.
// In all, fp32 accumulators are folded every few hundred rows into
// compensated (TwoSum) fp32 pairs; fp64 appears only in the cross-workgroup
// reduction at the end of the scan and in the merge.
#include <hip/hip_runtime.h>

#include "desc.h"
#include "device.h"

namespace lmfao {

// ---------------------------------------------------------------------------
// fills (used instead of memset nodes so the sequence can live in a graph)
// ---------------------------------------------------------------------------

struct FillDesc {
    uint32_t *ptr;
    int64_t n_words;
};

__global__ void multi_fill_kernel(const FillDesc *__restrict__ fills, int n) {
    for (int f = 0; f < n; ++f) {
        uint32_t *p = fills[f].ptr;
        const int64_t m = fills[f].n_words;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
            p[i] = 0u;
    }
}

// ---------------------------------------------------------------------------
// predicates and group-by components
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ bool compare(T x, int op, T t) {
    switch (op) {
        case OP_LE: return x <= t;
        case OP_LT: return x < t;
        case OP_GE: return x >= t;
        case OP_GT: return x > t;
        case OP_EQ: return x == t;
        default: return x != t;
    }
}

template <class PS>   // PredSrc in any address space
__device__ __forceinline__ bool pred_holds(const PS &p, int64_t row) {
    if (p.is_float) return compare(gld(static_cast<const float *>(p.col))[row], p.op, p.fval);
    return compare(gld(static_cast<const int32_t *>(p.col))[row], p.op, p.ival);
}

// categorical code (checked against its domain) or bucket #{k : thr[k] < x}
template <class CS>   // CompSrc in any address space
__device__ __forceinline__ int32_t comp_value(const CS &c, int64_t row, uint32_t *err) {
    if (c.nthr == 0) {
        int32_t v = gld(static_cast<const int32_t *>(c.col))[row];
        if (v < 0 || v >= c.dom) {
            gor(err, kErrDomain);
            v = 0;
        }
        return v;
    }
    const float x = gld(static_cast<const float *>(c.col))[row];
    int lo = 0, hi = c.nthr;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (gld(c.thr)[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// view records of non-root relations (one thread per row; grid.y = relation)
// ---------------------------------------------------------------------------

// One row's record: every word goes through put(w, v).  Records of at most 8 words (REG) are
// assembled in registers and written as one or two 16-byte stores (records are 16-byte aligned;
// words no field fills are written as zeros); wider ones are written word by word.
template <bool REG>
__device__ __forceinline__ void build_record(const AS_CONST ScanDesc &d, int64_t row, uint32_t *rec) {
    uint32_t r[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    auto put = [&](int w, uint32_t v) {
        if (REG) {
#pragma unroll
            for (int k = 0; k < 8; ++k) r[k] = w == k ? v : r[k];
        } else {
            gst(rec)[w] = v;
        }
    };
    uint32_t valid = 1u;
    uint64_t mask = d.filter_all;
    for (int c = 0; c < d.n_child; ++c) {
        const AS_CONST ChildSrc &ch = cst(d.children)[c];
        const int32_t k = gld(ch.fk)[row];
        if (k < 0 || k >= ch.n_keys) { valid = 0u; continue; }
        const AS_GLOBAL uint32_t *cr = gld(ch.rec + (int64_t)k * ch.stride);
        if (cr[0] == 0u) { valid = 0u; continue; }
        if (ch.n_mask > 0) {
            uint64_t m = cr[1];
            if (ch.n_mask > 1) m |= (uint64_t)cr[2] << 32;
            mask &= m;
        }
        for (int i = 0; i < ch.n_comp; ++i) put(d.rec_comp_off + ch.comp_dst + i, cr[ch.comp_off + i]);
        for (int i = 0; i < ch.n_feat; ++i) put(d.rec_feat_off + ch.feat_dst + i, cr[ch.feat_off + i]);
    }
    for (int f = 0; f < d.n_feat; ++f) {
        const AS_CONST FeatSrc &fs = cst(d.feats)[f];
        put(d.rec_feat_off + fs.dst, __float_as_uint(gld(fs.col)[row]));
    }
    for (int c = 0; c < d.n_comp; ++c) {
        const AS_CONST CompSrc &cs = cst(d.comps)[c];
        put(d.rec_comp_off + cs.dst, (uint32_t)comp_value(cs, row, d.err));
    }
    for (int p = 0; p < d.n_pred; ++p) {
        const AS_CONST PredSrc &ps = cst(d.preds)[p];
        if (!pred_holds(ps, row)) mask &= ~(1ull << ps.filter);
    }
    if (d.n_mask > 0) put(1, (uint32_t)mask);
    if (d.n_mask > 1) put(2, (uint32_t)(mask >> 32));
    put(0, valid);
    if (REG) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        AS_GLOBAL u32x4 *o = gst(reinterpret_cast<u32x4 *>(rec));
        o[0] = u32x4{r[0], r[1], r[2], r[3]};
        if (d.rec_stride > 4) o[1] = u32x4{r[4], r[5], r[6], r[7]};
    }
}

__global__ __launch_bounds__(kBlock) void view_build_kernel(const ScanDesc *__restrict__ descs) {
    const AS_CONST ScanDesc &d = cst(descs)[blockIdx.y];
    const int64_t row = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (row >= d.n_rows) return;
    const int32_t key = gld(d.key)[row];
    if (key < 0 || key >= d.n_keys) {
        gor(d.err, kErrKeyRange);
        return;
    }
    // the join key of a child must be unique: the count of rows with this key is checked after the
    // record is written, so the atomic's round trip overlaps the writes (with a duplicate the
    // records are unspecified and the error stops the evaluation at sync)
    const uint32_t seen_before = __hip_atomic_fetch_add(gst(d.seen + key), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t *rec = d.rec_out + (int64_t)key * d.rec_stride;
    if (d.rec_stride <= 8)
        build_record<true>(d, row, rec);
    else
        build_record<false>(d, row, rec);
    if (seen_before != 0u) gor(d.err, kErrDupKey);
}

// ---------------------------------------------------------------------------
// many-to-many child views: per-key count, sums and pair sums (one thread per
// row), then records and within-key scatter (one thread per key)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void dup_agg_kernel(const DupDesc *__restrict__ dp) {
    const AS_CONST DupDesc &d = *cst(dp);
    const int64_t row = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (row >= d.n_rows) return;
    const int32_t k = gld(d.key)[row];
    if (k < 0 || k >= d.n_keys) {
        gor(d.err, kErrKeyRange);
        return;
    }
    __hip_atomic_fetch_add(gst(d.cnt + k), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const AS_CONST FeatSrc *fs = cst(d.feats);
    for (int i = 0; i < d.n_feat; ++i) gadd(d.sum + (int64_t)k * d.n_feat + fs[i].dst, (double)gld(fs[i].col)[row]);
    const AS_CONST int32_t *ab = cst(d.pair_ab);
    for (int p = 0; p < d.n_pair; ++p) {
        // record feature index i is attribute fs[i] (dst == i), so a pair reads its two columns
        const double xa = gld(fs[ab[2 * p]].col)[row], xb = gld(fs[ab[2 * p + 1]].col)[row];
        gadd(d.scat + (int64_t)k * d.n_pair + p, xa * xb);   // a product of two fp32 values is exact in fp64
    }
}

__global__ __launch_bounds__(kBlock) void dup_final_kernel(const DupDesc *__restrict__ dp) {
    const AS_CONST DupDesc &d = *cst(dp);
    const int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (k >= d.n_keys) return;
    const uint32_t n = gld(d.cnt)[k];
    uint32_t *rec = d.rec_out + k * d.rec_stride;
    gst(rec)[0] = n;
    if (d.n_mask > 0) gst(rec)[1] = (uint32_t)d.filter_all;
    if (d.n_mask > 1) gst(rec)[2] = (uint32_t)(d.filter_all >> 32);
    if (n == 0u) return;   // no row with this key: the record stays zero and the key does not join
    const double inv = 1.0 / (double)n;
    const double *sm = d.sum + k * d.n_feat;
    for (int i = 0; i < d.n_feat; ++i) gst(rec)[d.rec_feat_off + i] = __float_as_uint((float)(gld(sm)[i] * inv));
    const AS_CONST int32_t *ab = cst(d.pair_ab);
    double *q = d.scat + k * d.n_pair;
    for (int p = 0; p < d.n_pair; ++p) {
        const double sa = gld(sm)[ab[2 * p]], sb = gld(sm)[ab[2 * p + 1]];
        gst(q)[p] = gld(q)[p] - sa * (sb * inv);
    }
}

// covariance entries of two attributes of a many-to-many child: one workgroup per pair, the
// keys summed in a fixed order (hw holds integers, so the sum does not depend on the run)
__global__ __launch_bounds__(kBlock) void corr_kernel(const CorrDesc *__restrict__ dp) {
    const AS_CONST CorrDesc &d = *cst(dp);
    __shared__ double part[kBlock];
    const int p = blockIdx.x;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < d.n_keys; k += kBlock) {
        const double h = gld(d.hw)[k];
        if (h != 0.0) s += h * gld(d.scat)[k * d.n_pair + p];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int a = cst(d.gram_ab)[2 * p], b = cst(d.gram_ab)[2 * p + 1];
        double *g = d.gram;
        gst(g)[a * d.n_gram + b] += part[0];
        if (a != b) gst(g)[b * d.n_gram + a] += part[0];
    }
}

// ---------------------------------------------------------------------------
// queries at another root: the view from the tree root joined with R's keys
// or rows (grid-stride over R; results accumulated with fp64 / u64 atomics)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void target_scan_kernel(const TargetDesc *__restrict__ dp) {
    const AS_CONST TargetDesc &d = cst(dp)[blockIdx.y];   // one query per grid row
    const AS_CONST TargetSrc *gb = cst(d.gb);
    const AS_CONST TargetTerm *terms = cst(d.terms);
    // small results (a few query cells hit by every item) are summed per workgroup in LDS first:
    // global atomics on a handful of addresses would serialise
    __shared__ unsigned long long lcnt_words[kTargetLdsCells];
    unsigned long long *lcnt = lcnt_words;
    double *lsum = reinterpret_cast<double *>(lcnt_words);   // after the counts
    const int64_t n_res = d.lds ? d.n_cells : 0;
    if (d.lds) {
        for (int i = threadIdx.x; i < kTargetLdsCells; i += kBlock) lcnt_words[i] = 0ull;
        __syncthreads();
    }
    unsigned long long *rcnt = d.lds ? lcnt : d.res_cnt;
    double *rsum = d.lds ? lsum + n_res : d.res_sum;
    for (int64_t item = blockIdx.x * (int64_t)kBlock + threadIdx.x; item < d.n_items;
         item += (int64_t)gridDim.x * kBlock) {
        int64_t k;
        const uint32_t *rec = nullptr;
        if (d.dup) {
            k = gld(d.key)[item];
            if (k < 0 || k >= d.n_keys) continue;   // reported by the many-to-many view build
            bool ok = true;
            for (int p = 0; p < d.n_pred && ok; ++p) ok = pred_holds(cst(d.preds)[p], item);
            if (!ok) continue;
        } else {
            k = item;
            rec = d.rec + k * d.rec_stride;
            if (gld(rec)[0] == 0u) continue;
            if (d.mask_word >= 0 && !(gld(rec)[d.mask_word] & d.mask_bit)) continue;
        }
        // R's side of the cell and of every term
        int64_t base = 0;
        for (int i = 0; i < d.n_gb; ++i) {
            const AS_CONST TargetSrc &g = gb[i];
            if (g.from_o >= 0) continue;
            const int32_t v = d.dup ? comp_value(g.comp, item, d.err) : (int32_t)gld(rec)[g.rec_word];
            base += (int64_t)v * g.stride;
        }
        double rf[kMaxTargetTerms];
        for (int t = 0; t < d.n_terms && t < kMaxTargetTerms; ++t) {
            const AS_CONST TargetTerm &T = terms[t];
            double f = T.coeff;
            for (int j = 0; j < T.n_fac; ++j)
                f *= d.dup ? (double)gld(T.col[j])[item] : (double)__uint_as_float(gld(rec)[T.rec_word[j]]);
            rf[t] = f;
        }
        const int64_t v0 = k * d.n_ocells;
        for (int64_t o = 0; o < d.n_ocells; ++o) {
            const unsigned long long cnt = gld(d.vcnt)[v0 + o];
            if (cnt == 0ull) continue;
            int64_t cell = base, rem = o;
            int digit[kMaxKeyComps];
            for (int j = d.n_o - 1; j >= 0; --j) {
                digit[j] = (int)(rem % d.o_dom[j]);
                rem /= d.o_dom[j];
            }
            for (int i = 0; i < d.n_gb; ++i)
                if (gb[i].from_o >= 0) cell += (int64_t)digit[gb[i].from_o] * gb[i].stride;
            const double *vv = d.vval + (v0 + o) * d.n_vals;
            if (d.lds) atomicAdd(rcnt + cell, cnt);
            else gadd(rcnt + cell, cnt);
            for (int a = 0; a < d.n_aggs; ++a) {
                double s = 0.0;
                for (int t = 0; t < d.n_terms && t < kMaxTargetTerms; ++t) {
                    if (terms[t].agg != a) continue;
                    const int vi = terms[t].val;
                    s += rf[t] * (vi < 0 ? (double)cnt : gld(vv)[vi]);
                }
                if (s == 0.0) continue;
                if (d.lds) atomicAdd(rsum + cell * d.n_aggs + a, s);
                else gadd(rsum + cell * d.n_aggs + a, s);
            }
        }
    }
    if (d.lds) {
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n_res; i += kBlock) {
            if (lcnt[i] == 0ull) continue;
            gadd(d.res_cnt + i, lcnt[i]);
            for (int a = 0; a < d.n_aggs; ++a)
                if (rsum[i * d.n_aggs + a] != 0.0) gadd(d.res_sum + i * d.n_aggs + a, rsum[i * d.n_aggs + a]);
        }
    }
}

template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

// Where a staged feature of a tile lives in LDS: word(row) = base + buf * step + row * stride.
struct FeatLoc {
    int base, step, stride;
};

// f: staged feature; src: its feat_src entry; wave: the wave region's first word
__device__ __forceinline__ FeatLoc feat_loc(const RootDesc &d, int f, int src, int wave) {
    if (f == 0) return {d.lds_consts, 0, 1};                 // constant 1
    if (f >= d.n_feat) return {d.lds_consts + 64, 0, 1};     // padding feature 0
    if (src >= 0) return {wave + d.w_rec + src, d.n_quads * 256, 4};   // child record word
    if (src <= kDerivedSrc) return {wave + d.w_der + (kDerivedSrc - src) * kColPitch, 0, 1};   // product, this tile
    return {wave + d.w_fact + (-1 - src) * kColPitch, d.n_fact * kColPitch, 1};
}

// Root multi-output scan.  Every wave owns a contiguous share of its
// workgroup's rows and walks it in 64-row tiles, one row per lane:
//   * the tile's fact columns and the child view records of its keys are
//     copied straight into LDS (global_load_lds): fact columns
//     feature-major, records row-major; with nbuf = 2 the next tile's copies
//     are in flight while this tile is processed;
//   * covariance: each MFMA lane reads 8 consecutive rows of one feature
//     (from a fact column, or strided out of the records), zeroes rows that
//     do not join, splits into bf16 hi/lo in registers; or fp32 register
//     blocks accumulate per (row phase, block pair);
//   * grouped tables: each lane updates the tables of its own row.
template <int MODE, int P1, bool TABLES>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void root_scan_kernel(
    const RootDesc *__restrict__ dp) {
    extern __shared__ __align__(16) uint32_t smem[];
    const RootDesc &d = *dp;
    const ScanDesc &s = d.scan;
    const AS_CONST CompSrc *comps = cst(s.comps);
    const AS_CONST PredSrc *preds = cst(s.preds);
    const AS_CONST ChildSrc *children = cst(s.children);
    const AS_CONST FamilyDesc *fams = cst(d.fams);
    const AS_CONST KeyDesc *keys = cst(d.keys);
    const AS_CONST ValDesc *vals = cst(d.vals);
    const AS_CONST FlushDesc *flushes = cst(d.flush);
    const AS_CONST int32_t *feat_src = cst(d.feat_src);
    const AS_CONST int32_t *comp_src = cst(d.comp_src);
    const auto fact_cols = cst(d.fact_cols);
    const auto aux_cols = cst(d.aux_cols);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: LDS bases stay scalar
    const int nwaves = blockDim.x >> 6;
    const int part = blockIdx.y;
    const bool do_gram = MODE != 0 && part == d.gram_part && d.n_gram > 0;
    const bool do_count = d.do_count && part == d.gram_part;

    constexpr int GB = MODE == 1 ? P1 : 1;
    constexpr int NT = MODE >= 2 ? P1 : 1;
    constexpr int NHH = NT * (NT + 1) / 2;
    constexpr int NHL = NT * NT;
    constexpr int NLL = MODE >= 3 ? NHH : 1;

    // ---- block set-up: tables zeroed, constant columns, thresholds ------------------
    if (TABLES) {
        const int words = d.lds_table_words[part];
        for (int i = tid; i < words; i += blockDim.x) smem[d.lds_tables + i] = 0u;
    }
    if (tid < 64) {
        smem[d.lds_consts + tid] = __float_as_uint(1.f);
        smem[d.lds_consts + 64 + tid] = 0u;
    }
    for (int i = tid; i < d.n_thr_words; i += blockDim.x) smem[d.lds_thr + i] = __float_as_uint(gld(d.thr_all)[i]);
    __syncthreads();

    const int wbase = d.lds_wave + wave * d.wave_words;
    uint32_t *W = smem + wbase;
    const float *fsm = reinterpret_cast<const float *>(smem);
    const float *thr_lds = reinterpret_cast<const float *>(smem + d.lds_thr);
    const int64_t blk_begin = (int64_t)blockIdx.x * d.rows_per_block;
    const int64_t blk_end = min(blk_begin + d.rows_per_block, s.n_rows);
    const int64_t per_wave = d.rows_per_block / nwaves;
    const int64_t w_begin = blk_begin + wave * per_wave;
    const int64_t w_end = min(w_begin + per_wave, blk_end);
    const int64_t n_tiles = w_end > w_begin ? (w_end - w_begin + 63) / 64 : 0;
    const int64_t last_row = s.n_rows - 1;

    // ---- accumulators and per-lane feature sources ---------------------------------------
    float acc[GB][GB], shi[GB][GB], slo[GB][GB];
    FeatLoc la[GB], lb[GB];
    int gph = 0, nph = 1;
    bool gact = false;
    if (MODE == 1) {
#pragma unroll
        for (int i = 0; i < GB; ++i)
#pragma unroll
            for (int j = 0; j < GB; ++j) acc[i][j] = shi[i][j] = slo[i][j] = 0.f;
        const int nb = d.ngp / GB;
        const int np = nb * (nb + 1) / 2;
        nph = 64 / np;
        int gI = 0, gJ = 0;
        if (lane < np * nph) {
            gact = true;
            int p = lane % np;
            gph = lane / np;
            while (p >= nb - gI) { p -= nb - gI; ++gI; }
            gJ = gI + p;
        }
#pragma unroll
        for (int q = 0; q < GB; ++q) {
            const int fa = gI * GB + q, fb = gJ * GB + q;
            la[q] = feat_loc(d, fa, fa < d.n_feat ? gld(d.feat_src)[fa] : 0, wbase);
            lb[q] = feat_loc(d, fb, fb < d.n_feat ? gld(d.feat_src)[fb] : 0, wbase);
        }
    }
    // hi*hi partials fold into a second fp32 level every kFlushTiles tiles; hi*lo and
    // lo*lo partials are ~2^-8 and ~2^-16 of them, their fp32 chains need no second level
    f32x4 chh[NHH], chl[NHL], cll[NLL], shh[NHH];
    FeatLoc lt[NT];
    if (MODE >= 2) {
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NHH; ++i) chh[i] = shh[i] = z;
#pragma unroll
        for (int i = 0; i < NHL; ++i) chl[i] = z;
#pragma unroll
        for (int i = 0; i < NLL; ++i) cll[i] = z;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int f = 16 * t + (lane & 15);
            lt[t] = feat_loc(d, f, f < d.n_feat ? gld(d.feat_src)[f] : 0, wbase);
        }
    }
    int tiles_since_flush = 0;
    unsigned long long my_count = 0;
    const SplitSel sel = split_sel();

    // ---- tile copies ------------------------------------------------------------------------
    int32_t fk[kMaxChild];
    auto load_keys = [&](int64_t tile) {
        const int64_t row = min(w_begin + tile * 64 + lane, last_row);
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c)
            if (c < s.n_child) fk[c] = gld(children[c].fk)[row];
    };
    // copies address scalar bases plus 32-bit per-lane byte offsets (row * 4 and
    // key * record bytes stay below 4 GiB: the planner bounds table sizes)
    auto issue = [&](int64_t tile, int buf) {
        const uint32_t roff = (uint32_t)min(w_begin + tile * 64 + lane, last_row) * 4u;
        uint32_t *fb = W + d.w_fact + buf * d.n_fact * kColPitch;
        // the pointer array is padded to 16 entries: the first 16 bases load together,
        // unconditionally, before any copy is issued
        const char *fp[16];
#pragma unroll
        for (int f = 0; f < 16; ++f) fp[f] = reinterpret_cast<const char *>(fact_cols[f]);
#pragma unroll
        for (int f = 0; f < 16; ++f)
            if (f < d.n_fact) lds_dma4(fp[f] + roff, fb + f * kColPitch);
        for (int f = 16; f < d.n_fact; ++f) lds_dma4(reinterpret_cast<const char *>(fact_cols[f]) + roff, fb + f * kColPitch);
        uint32_t *ab = W + d.w_aux + buf * d.n_aux * kColPitch;
        const char *ap[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) ap[a] = reinterpret_cast<const char *>(aux_cols[a]);
#pragma unroll
        for (int a = 0; a < 8; ++a)
            if (a < d.n_aux) lds_dma4(ap[a] + roff, ab + a * kColPitch);
        for (int a = 8; a < d.n_aux; ++a) lds_dma4(reinterpret_cast<const char *>(aux_cols[a]) + roff, ab + a * kColPitch);
        uint32_t *rb = W + d.w_rec + buf * d.n_quads * 256;
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c) {
            if (c < s.n_child) {
                const AS_CONST ChildSrc &ch = children[c];
                const int32_t k = fk[c];
                const bool hit = k >= 0 && k < ch.n_keys;
                const char *base = reinterpret_cast<const char *>(hit ? ch.rec : d.zero_rec);
                const uint32_t koff = hit ? (uint32_t)k * (uint32_t)ch.stride * 4u : 0u;
                const int nq = ch.stride >> 2;
                uint32_t *dst = rb + ch.quad_base * 256;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q < nq) lds_dma16(base + koff + 16 * q, dst + q * 256);
                for (int q = 4; q < nq; ++q) lds_dma16(base + koff + 16 * q, dst + q * 256);
            }
        }
    };

    if (n_tiles > 0) {
        load_keys(0);
        if (d.nbuf == 2) {
            __builtin_amdgcn_s_waitcnt(0);
            issue(0, 0);
            if (n_tiles > 1) load_keys(1);
        }
    }

    for (int64_t t = 0; t < n_tiles; ++t) {
        const int buf = d.nbuf == 2 ? (int)(t & 1) : 0;
        if (d.nbuf == 1) {
            __builtin_amdgcn_s_waitcnt(0);
            wave_sync();       // the previous tile's reads of the single buffer are done
            issue(t, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);   // this tile's copies and the next tile's keys have landed
        wave_sync();
        if (d.nbuf == 2 && t + 1 < n_tiles) {
            issue(t + 1, buf ^ 1);
            if (t + 2 < n_tiles) load_keys(t + 2);
        } else if (d.nbuf == 1 && t + 1 < n_tiles) {
            load_keys(t + 1);
        }

        // ---- per-row validity, filters, components --------------------------------------------
        const int64_t row = w_begin + t * 64 + lane;
        bool valid = row < w_end;
        uint64_t mask = s.filter_all;
        const uint32_t *rb = W + d.w_rec + buf * d.n_quads * 256;
        const uint32_t *ab = W + d.w_aux + buf * d.n_aux * kColPitch;
        unsigned long long w64 = 1ull;   // joined tuples this row stands for (weighted plans)
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c) {
            if (c < s.n_child) {
                const uint4 q0 = *reinterpret_cast<const uint4 *>(rb + (children[c].quad_base * 64 + lane) * 4);
                if (q0.x == 0u) valid = false;
                if (s.n_mask > 0) mask &= (uint64_t)q0.y | (s.n_mask > 1 ? (uint64_t)q0.z << 32 : 0ull);
                if (d.weighted) w64 = min(w64, 1ull << 32) * q0.x;
            }
        }
        uint32_t wt = 1u;
        if (d.weighted) {
            if (valid && w64 > d.max_weight) gor(d.err, kErrWeight);
            wt = valid ? (uint32_t)min(w64, (unsigned long long)d.max_weight) : 0u;
            if (MODE == 1 && do_gram) W[d.w_wgt + lane] = __float_as_uint((float)wt);
            if (do_gram) {
                // per key of a many-to-many child: the tuples reaching it over its own count.  The
                // fact is sorted by its keys, so a tile's valid rows mostly share one key: then the
                // wave adds once (a wave's 64 atomics on one address would serialise)
#pragma unroll
                for (int c = 0; c < kMaxChild; ++c) {
                    if (c < s.n_child && children[c].hw) {
                        const uint32_t n = rb[(children[c].quad_base * 64 + lane) * 4];
                        const int32_t k = gld(children[c].fk)[min(row, last_row)];
                        const double h = valid ? (double)wt / (double)n : 0.0;
                        const uint64_t vb = __ballot(valid);
                        if (vb == 0ull) continue;
                        const int32_t k0 = __builtin_amdgcn_readlane(k, __ffsll((long long)vb) - 1);
                        if (__ballot(valid && k != k0) == 0ull) {
                            const double tot = wave_sum_f64(h);
                            if (lane == 0) gadd(children[c].hw + k0, tot);
                        } else if (valid) {
                            gadd(children[c].hw + k, h);
                        }
                    }
                }
            }
        }
        for (int p = 0; p < s.n_pred; ++p) {
            const AS_CONST PredSrc &ps = preds[p];
            const uint32_t raw = ab[ps.aux * kColPitch + lane];
            const bool ok = ps.is_float ? compare(__uint_as_float(raw), ps.op, ps.fval) : compare((int32_t)raw, ps.op, ps.ival);
            if (!ok) mask &= ~(1ull << ps.filter);
        }
        if (TABLES) {
            for (int c = 0; c < d.n_comp; ++c) {
                const int src = comp_src[c];
                if (src >= 0) W[d.w_comp + c * 64 + lane] = rb[src + lane * 4];
            }
            for (int c = 0; c < s.n_comp; ++c) {
                const AS_CONST CompSrc &cs = comps[c];
                const uint32_t raw = ab[cs.aux * kColPitch + lane];
                int32_t v;
                if (cs.nthr == 0) {
                    v = (int32_t)raw;
                    if (valid && (v < 0 || v >= cs.dom)) gor(d.err, kErrDomain);
                    if (v < 0 || v >= cs.dom) v = 0;
                } else {
                    const float x = __uint_as_float(raw);
                    v = 0;
                    for (int k = 0; k < cs.nthr; ++k) v += thr_lds[cs.thr_lds + k] < x ? 1 : 0;
                }
                W[d.w_comp + cs.dst * 64 + lane] = (uint32_t)v;
            }
        }
        const uint64_t vm = __ballot(valid);
        if (do_count) my_count += valid ? (unsigned long long)wt : 0ull;
        // derived features: the row's products of two staged features (fp32), one LDS column each
        if (d.n_der > 0) {
            const AS_CONST int32_t *ab = cst(d.der_ab);
            for (int j = 0; j < d.n_der; ++j) {
                const int fa = ab[2 * j], fb = ab[2 * j + 1];
                const FeatLoc La = feat_loc(d, fa, gld(d.feat_src)[fa], wbase);
                const FeatLoc Lb = feat_loc(d, fb, gld(d.feat_src)[fb], wbase);
                const float v = fsm[La.base + buf * La.step + lane * La.stride] * fsm[Lb.base + buf * Lb.step + lane * Lb.stride];
                W[d.w_der + j * kColPitch + lane] = __float_as_uint(v);
            }
            wave_sync();
        }

        // ---- covariance block ---------------------------------------------------------------
        if (MODE == 1 && do_gram && d.weighted) wave_sync();   // the tile's row weights are in LDS
        if (MODE == 1 && do_gram && gact) {
            int pa[GB], pb[GB];
#pragma unroll
            for (int q = 0; q < GB; ++q) {
                pa[q] = la[q].base + buf * la[q].step;
                pb[q] = lb[q].base + buf * lb[q].step;
            }
            auto rows = [&](auto weighted) {
                for (int r = gph; r < 64; r += nph) {
                    if (!((vm >> r) & 1ull)) continue;
                    float a[GB], b[GB];
#pragma unroll
                    for (int q = 0; q < GB; ++q) { a[q] = fsm[pa[q] + r * la[q].stride]; b[q] = fsm[pb[q] + r * lb[q].stride]; }
                    if (decltype(weighted)::value) {
                        const float wr = fsm[wbase + d.w_wgt + r];
#pragma unroll
                        for (int q = 0; q < GB; ++q) a[q] *= wr;
                    }
#pragma unroll
                    for (int i = 0; i < GB; ++i)
#pragma unroll
                        for (int j = 0; j < GB; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
                }
            };
            if (d.weighted) rows(BoolTag<true>{});
            else rows(BoolTag<false>{});
            if (++tiles_since_flush == 4) {
#pragma unroll
                for (int i = 0; i < GB; ++i)
#pragma unroll
                    for (int j = 0; j < GB; ++j) { two_sum_acc(shi[i][j], slo[i][j], acc[i][j]); acc[i][j] = 0.f; }
                tiles_since_flush = 0;
            }
        }
        if (MODE >= 2 && do_gram) {
            const bool all_rows = vm == ~0ull;   // wave-uniform: the common case needs no masking
#pragma unroll 1
            for (int ks = 0; ks < 2; ++ks) {
                const int row0 = 32 * ks + 8 * (lane >> 4);
                const uint32_t vbits = (uint32_t)(vm >> row0) & 0xFFu;
                bf16x8 fh[NT], fl[NT], fm[MODE == 4 ? NT : 1];
#pragma unroll
                for (int t2 = 0; t2 < NT; ++t2) {
                    const int st = lt[t2].stride;
                    const float *p = fsm + lt[t2].base + buf * lt[t2].step + row0 * st;
                    float x[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) { x[i] = *p; p += st; }
                    if (!all_rows) {
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (!((vbits >> i) & 1u)) x[i] = 0.f;
                    }
                    if (MODE == 4) split3_bf16x8(sel, x, fh[t2], fm[MODE == 4 ? t2 : 0], fl[t2]);
                    else split_bf16x8(sel, x, fh[t2], fl[t2]);
                }
                int ih = 0;
#pragma unroll
                for (int t2 = 0; t2 < NT; ++t2)
#pragma unroll
                    for (int u = t2; u < NT; ++u, ++ih) {
                        chh[ih] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[t2], fh[u], chh[ih], 0, 0, 0);
                        if (MODE == 3) cll[ih] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fl[t2], fl[u], cll[ih], 0, 0, 0);
                        if (MODE == 4) cll[ih] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fm[MODE == 4 ? t2 : 0], fm[MODE == 4 ? u : 0], cll[ih], 0, 0, 0);
                    }
#pragma unroll
                for (int t2 = 0; t2 < NT; ++t2)
#pragma unroll
                    for (int u = 0; u < NT; ++u)
                        chl[t2 * NT + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[t2], fl[u], chl[t2 * NT + u], 0, 0, 0);
#pragma unroll
                for (int t2 = 0; t2 < NT; ++t2)
#pragma unroll
                    for (int u = 0; u < NT; ++u)
                        if (MODE == 4)   // hi*mid and hi*lo share the full-square accumulators
                            chl[t2 * NT + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[t2], fm[MODE == 4 ? u : 0], chl[t2 * NT + u], 0, 0, 0);
            }
            if (++tiles_since_flush == kFlushTiles) {
                const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < NHH; ++i) { shh[i] += chh[i]; chh[i] = z; }
                tiles_since_flush = 0;
            }
        }

        // ---- grouped tables (this lane's own row) ---------------------------------------------
        if (TABLES && d.hcodes && row < w_end) {
            // component codes for the count-table scan: every row of the range once, 0xFFFF when
            // the row does not join
            const AS_CONST int32_t *hcomp = cst(d.hcode_comp);
            uint16_t *hc = d.hcodes + row;
            for (int j = 0; j < d.n_hcodes; ++j) {
                const uint32_t v = valid ? W[d.w_comp + hcomp[j] * 64 + lane] : (uint32_t)kNoCode;
                gst(hc)[(int64_t)j * d.hcode_pitch] = (uint16_t)v;
            }
        }
        if (TABLES && !d.codes && d.conv_fams > 0) {
            // families with global tables, in code every lane runs: on the sorted fact the rows of
            // a wave often update one cell (a table keyed by the key a run shares), and then the
            // wave sums its rows and adds once instead of 64 atomics on one address, which
            // serialise
            const uint32_t *cr = W + d.w_comp + lane;
            auto fval = [&](int f) -> double {
                const FeatLoc L = feat_loc(d, f, f < d.n_feat ? feat_src[f] : 0, wbase);
                return (double)fsm[L.base + buf * L.step + lane * L.stride];
            };
            for (int fi = 0; fi < d.n_fam; ++fi) {
                const AS_CONST FamilyDesc &F = fams[fi];
                if (!F.conv) continue;
                uint32_t wf = 0u;
                if (valid) wf = F.wdiv >= 0 ? wt / rb[(children[F.wdiv].quad_base * 64 + lane) * 4] : wt;
                const double wd = (double)wf;
                for (int j = 0; j < F.n_filt; ++j) {
                    const bool on = valid && (F.unfiltered || ((mask >> cst(d.filt_bits)[F.filt_base + j]) & 1ull));
                    const uint64_t ob = __ballot(on);
                    if (ob == 0ull) continue;
                    for (int k = 0; k < F.n_keys; ++k) {
                        const AS_GLOBAL TabDesc &T = gld(d.tabs)[F.tab_base + j * F.n_keys + k];
                        if (T.part != part) continue;
                        const AS_CONST KeyDesc &K = keys[F.key_base + k];
                        int32_t cell = 0;
                        for (int c = 0; c < K.n_comp; ++c) cell += (int32_t)cr[K.c[c] * 64] * K.s[c];
                        const bool lds = T.lds_cnt >= 0;
                        unsigned long long *gc = d.g_cnt + T.glb_cnt;
                        double *gv = d.g_val + T.glb_val;
                        uint32_t *lc = smem + d.lds_tables + T.lds_cnt;
                        double *lv = reinterpret_cast<double *>(smem + d.lds_tables + T.lds_val);
                        const int32_t c0 = __builtin_amdgcn_readlane(cell, __ffsll((long long)ob) - 1);
                        if (__ballot(on && cell != c0) == 0ull) {
                            const unsigned long long tc = wave_sum_u64(on ? (unsigned long long)wf : 0ull);
                            if (lane == 0) {
                                if (lds) atomicAdd(lc + c0, (uint32_t)tc);
                                else gadd(gc + c0, tc);
                            }
                            for (int v = 0; v < F.n_vals; ++v) {
                                const AS_CONST ValDesc &vd = vals[F.val_base + v];
                                const double tv = wave_sum_f64(on ? fval(vd.a) * fval(vd.b) * wd : 0.0);
                                if (lane == 0) {
                                    if (lds) atomicAdd(lv + (int64_t)c0 * F.n_vals + v, tv);
                                    else gadd(gv + (int64_t)c0 * F.n_vals + v, tv);
                                }
                            }
                        } else if (on) {
                            if (lds) atomicAdd(lc + cell, wf);
                            else gadd(gc + cell, (unsigned long long)wf);
                            for (int v = 0; v < F.n_vals; ++v) {
                                const AS_CONST ValDesc &vd = vals[F.val_base + v];
                                const double x = fval(vd.a) * fval(vd.b) * wd;
                                if (lds) atomicAdd(lv + (int64_t)cell * F.n_vals + v, x);
                                else gadd(gv + (int64_t)cell * F.n_vals + v, x);
                            }
                        }
                    }
                }
            }
        }
        if (TABLES && d.codes) {
            // per-row codes for the partitioned table scan; rows past the range write nothing
            if (row < w_end) {
                const uint64_t m = valid ? mask : 0ull;
                uint32_t *cd = d.codes + row;
                gst(cd)[0] = (uint32_t)m;
                if (d.n_mask_codes > 1) gst(cd)[d.code_pitch] = (uint32_t)(m >> 32);
                const uint32_t *cr = W + d.w_comp + lane;
                for (int fi = 0; fi < d.n_fam; ++fi) {
                    const AS_CONST FamilyDesc &F = fams[fi];
                    for (int k = 0; k < F.n_keys; ++k) {
                        const AS_CONST KeyDesc &K = keys[F.key_base + k];
                        int32_t cell = 0;
                        for (int c = 0; c < K.n_comp; ++c) cell += (int32_t)cr[K.c[c] * 64] * K.s[c];
                        gst(cd)[(int64_t)(F.code_base + k) * d.code_pitch] = (uint32_t)cell;
                    }
                }
                for (int j = 0; j < d.n_code_feats; ++j) {
                    const int f = cst(d.code_feats)[j];
                    const FeatLoc L = feat_loc(d, f, f < d.n_feat ? feat_src[f] : 0, wbase);
                    gst(cd)[(int64_t)(d.code_feat_col + j) * d.code_pitch] =
                        __float_as_uint(fsm[L.base + buf * L.step + lane * L.stride]);
                }
            }
        } else if (TABLES && valid) {
            const uint32_t *cr = W + d.w_comp + lane;
            auto fval = [&](int f) -> double {
                const FeatLoc L = feat_loc(d, f, f < d.n_feat ? feat_src[f] : 0, wbase);
                return (double)fsm[L.base + buf * L.step + lane * L.stride];
            };
            for (int fi = 0; fi < d.n_fam; ++fi) {
                const AS_CONST FamilyDesc &F = fams[fi];
                // the row's weight: 1 unless the plan is weighted; a view towards a many-to-many
                // child leaves that child's own count out (products stay exact in fp64)
                const uint32_t wf = F.wdiv >= 0 ? wt / rb[(children[F.wdiv].quad_base * 64 + lane) * 4] : wt;
                const double wd = (double)wf;
                if (F.strided) {
                    // the cell of each key once per row, then one update per filter this row
                    // satisfies, at an address computed from the filter's rank in the partition
                    const uint64_t pm = F.part_mask[part];
                    const uint64_t rb = mask & pm;
                    if (rb) {
                        const uint32_t tb = (uint32_t)(d.lds_tables + F.part_base[part]);
                        for (int k = 0; k < F.n_keys; ++k) {
                            const AS_CONST KeyDesc &K = keys[F.key_base + k];
                            int32_t cell = 0;
                            for (int c = 0; c < K.n_comp; ++c) cell += (int32_t)cr[K.c[c] * 64] * K.s[c];
                            uint64_t b = rb;
                            while (b) {
                                const int bi = __ffsll((long long)b) - 1;
                                b &= b - 1;
                                const uint32_t u = tb + (uint32_t)__popcll(pm & ((1ull << bi) - 1ull)) * (uint32_t)F.unit_words;
                                atomicAdd(&smem[u + K.off_cnt + cell], wf);
                                if (F.n_vals) {
                                    double *vs = reinterpret_cast<double *>(smem + u + K.off_val) + (int64_t)cell * F.n_vals;
                                    for (int v = 0; v < F.n_vals; ++v) {
                                        const AS_CONST ValDesc &vd = vals[F.val_base + v];
                                        atomicAdd(vs + v, fval(vd.a) * fval(vd.b) * wd);
                                    }
                                }
                            }
                        }
                    }
                    continue;
                }
                if (F.conv) continue;   // done by the convergent pass
                uint64_t bits = F.unfiltered ? 1ull : (mask & F.part_mask[part]);
                while (bits) {
                    int f;
                    if (F.unfiltered) {
                        f = 0;
                        bits = 0;
                    } else {
                        const int b = __ffsll((long long)bits) - 1;
                        bits &= bits - 1;
                        f = __popcll(F.filt_mask & ((1ull << b) - 1ull));
                    }
                    for (int k = 0; k < F.n_keys; ++k) {
                        const AS_GLOBAL TabDesc &T = gld(d.tabs)[F.tab_base + f * F.n_keys + k];
                        if (T.part != part) continue;
                        const AS_CONST KeyDesc &K = keys[F.key_base + k];
                        int32_t cell = 0;
                        for (int c = 0; c < K.n_comp; ++c) cell += (int32_t)cr[K.c[c] * 64] * K.s[c];
                        // a product of two fp32 values is exact in fp64; cell sums accumulate
                        // in fp64 (runs of one dimension key repeat a value thousands of
                        // times in a row, beyond what fp32 sums exactly)
                        if (T.lds_cnt >= 0) {
                            atomicAdd(&smem[d.lds_tables + T.lds_cnt + cell], wf);
                            double *vs = reinterpret_cast<double *>(smem + d.lds_tables + T.lds_val) + (int64_t)cell * F.n_vals;
                            for (int v = 0; v < F.n_vals; ++v) {
                                const AS_CONST ValDesc &vd = vals[F.val_base + v];
                                atomicAdd(vs + v, fval(vd.a) * fval(vd.b) * wd);
                            }
                        } else {
                            gadd(d.g_cnt + T.glb_cnt + cell, (unsigned long long)wf);
                            double *vs = d.g_val + T.glb_val + (int64_t)cell * F.n_vals;
                            for (int v = 0; v < F.n_vals; ++v) {
                                const AS_CONST ValDesc &vd = vals[F.val_base + v];
                                gadd(vs + v, fval(vd.a) * fval(vd.b) * wd);
                            }
                        }
                    }
                }
            }
        }
    }

    // ---- end of scan: workgroup reduction in fp64, partials out ------------------------
    __syncthreads();   // every wave is done with its region; the reduction scratch aliases them
    double *red = reinterpret_cast<double *>(smem + d.lds_red);
    if (MODE == 1 && do_gram) {
        const int ngp = d.ngp;
        for (int i = tid; i < ngp * ngp; i += blockDim.x) red[i] = 0.0;
        __syncthreads();
        if (gact) {
            const int nb = d.ngp / GB;
            int p = lane % (nb * (nb + 1) / 2), gI = 0;
            while (p >= nb - gI) { p -= nb - gI; ++gI; }
            const int gJ = gI + p;
#pragma unroll
            for (int i = 0; i < GB; ++i)
#pragma unroll
                for (int j = 0; j < GB; ++j) {
                    two_sum_acc(shi[i][j], slo[i][j], acc[i][j]);
                    const int gi = gI * GB + i, gj = gJ * GB + j;
                    if (gi <= gj) atomicAdd(&red[gi * ngp + gj], (double)shi[i][j] + (double)slo[i][j]);
                }
        }
        __syncthreads();
        const int ntri = d.n_gram * (d.n_gram + 1) / 2;
        double *out = d.gram_partial + (int64_t)blockIdx.x * ntri;
        for (int e = tid; e < d.n_gram * d.n_gram; e += blockDim.x) {
            const int i = e / d.n_gram, j = e % d.n_gram;
            if (i <= j) gst(out)[tri_index(i, j, d.n_gram)] = red[i * ngp + j];
        }
    }
    if (MODE >= 2 && do_gram) {
        const int n16 = NT * 16;
        double *rhh = red, *rhl = red + n16 * n16, *rll = red + 2 * n16 * n16;
        const int nred = (MODE >= 3 ? 3 : 2) * n16 * n16;
        for (int i = tid; i < nred; i += blockDim.x) red[i] = 0.0;
        __syncthreads();
        const int ci = 4 * (lane >> 4), cj = lane & 15;
        int ih = 0;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int u = t; u < NT; ++u, ++ih)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    atomicAdd(&rhh[(16 * t + ci + e) * n16 + 16 * u + cj], (double)shh[ih][e] + (double)chh[ih][e]);
                    if (MODE >= 3) atomicAdd(&rll[(16 * t + ci + e) * n16 + 16 * u + cj], (double)cll[ih][e]);
                }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    atomicAdd(&rhl[(16 * t + ci + e) * n16 + 16 * u + cj], (double)chl[t * NT + u][e]);
        __syncthreads();
        const int ntri = d.n_gram * (d.n_gram + 1) / 2;
        double *out = d.gram_partial + (int64_t)blockIdx.x * ntri;
        for (int e = tid; e < d.n_gram * d.n_gram; e += blockDim.x) {
            const int i = e / d.n_gram, j = e % d.n_gram;
            if (i <= j) {
                double v = rhh[i * n16 + j] + rhl[i * n16 + j] + rhl[j * n16 + i];
                if (MODE >= 3) v += rll[i * n16 + j];
                gst(out)[tri_index(i, j, d.n_gram)] = v;
            }
        }
    }
    if (do_count) {
        __shared__ unsigned long long wcount[kMaxWaves];
        const unsigned long long w = wave_sum_u64(my_count);
        if (lane == 0) wcount[wave] = w;
        __syncthreads();
        if (tid == 0) {
            unsigned long long t = 0;
            for (int i = 0; i < nwaves; ++i) t += wcount[i];
            gst(d.count_partial)[blockIdx.x] = t;
        }
    }
    if (TABLES) {
        const int nf = d.n_flush[part];
        for (int t = 0; t < nf; ++t) {
            const AS_CONST FlushDesc &F = flushes[d.flush_base[part] + t];
            const uint32_t *cnt = smem + d.lds_tables + F.lds_cnt;
            const double *val = reinterpret_cast<const double *>(smem + d.lds_tables + F.lds_val);
            for (int cell = tid; cell < F.n_cells; cell += blockDim.x) {
                const uint32_t c = cnt[cell];
                if (c == 0u) continue;
                gadd(d.g_cnt + F.glb_cnt + cell, (unsigned long long)c);
                for (int v = 0; v < F.n_vals; ++v) {
                    const double x = val[(int64_t)cell * F.n_vals + v];
                    if (x != 0.0) gadd(d.g_val + F.glb_val + (int64_t)cell * F.n_vals + v, x);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// grouped tables from per-row codes: one workgroup of 1024 threads per (row
// block, partition); the partition's tables in LDS, a thread per row, the
// strided addressing and the fp64 products of the root scan
// ---------------------------------------------------------------------------

constexpr int kCodeBatch = 8;   // key cells of one row requested together by the code scan

__global__ __launch_bounds__(1024) void code_scan_kernel(const CodeScanDesc *__restrict__ dp) {
    extern __shared__ __align__(16) uint32_t smem[];
    const AS_CONST CodeScanDesc &d = *cst(dp);
    const AS_CONST FamilyDesc *fams = cst(d.fams);
    const AS_CONST KeyDesc *keys = cst(d.keys);
    const AS_CONST ValDesc *vcols = cst(d.val_cols);
    const int part = blockIdx.y;
    const int tid = threadIdx.x;
    const int words = d.lds_table_words[part];
    for (int i = tid; i < words; i += blockDim.x) smem[i] = 0u;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * d.rows_per_block;
    const int64_t r1 = r0 + d.rows_per_block < d.n_rows ? r0 + d.rows_per_block : d.n_rows;
    const uint32_t *codes = d.codes;
    for (int64_t r = r0 + tid; r < r1; r += blockDim.x) {
        uint64_t mask = gld(codes)[r];
        if (d.n_mask_codes > 1) mask |= (uint64_t)gld(codes)[d.pitch + r] << 32;
        for (int fi = 0; fi < d.n_fam; ++fi) {
            const AS_CONST FamilyDesc &F = fams[fi];
            const uint64_t pm = F.part_mask[part];
            const uint64_t rb = mask & pm;
            if (!rb) continue;
            const uint32_t tb = (uint32_t)F.part_base[part];
            // the row's summed monomials, products of two fp32 codes formed in fp64
            double pv[kMaxCodeVals];
#pragma unroll
            for (int v = 0; v < kMaxCodeVals; ++v) {
                pv[v] = 0.0;
                if (v < F.n_vals) {
                    const AS_CONST ValDesc &vc = vcols[F.val_base + v];
                    const float xa = vc.a < 0 ? 1.f : __uint_as_float(gld(codes)[(int64_t)vc.a * d.pitch + r]);
                    const float xb = vc.b < 0 ? 1.f : __uint_as_float(gld(codes)[(int64_t)vc.b * d.pitch + r]);
                    pv[v] = (double)xa * (double)xb;
                }
            }
            // the cells of kCodeBatch keys are requested together, then their updates made
            for (int k0 = 0; k0 < F.n_keys; k0 += kCodeBatch) {
                uint32_t cells[kCodeBatch];
#pragma unroll
                for (int j = 0; j < kCodeBatch; ++j)
                    cells[j] = k0 + j < F.n_keys ? gld(codes)[(int64_t)(F.code_base + k0 + j) * d.pitch + r] : 0u;
#pragma unroll
                for (int j = 0; j < kCodeBatch; ++j) {
                    if (k0 + j >= F.n_keys) break;
                    const AS_CONST KeyDesc &K = keys[F.key_base + k0 + j];
                    const uint32_t cell = cells[j];
                    uint64_t b = rb;
                    while (b) {
                        const int bi = __ffsll((long long)b) - 1;
                        b &= b - 1;
                        const uint32_t u = tb + (uint32_t)__popcll(pm & ((1ull << bi) - 1ull)) * (uint32_t)F.unit_words;
                        atomicAdd(&smem[u + K.off_cnt + cell], 1u);
                        if (F.n_vals) {
                            double *vs = reinterpret_cast<double *>(smem + u + K.off_val) + (int64_t)cell * F.n_vals;
#pragma unroll
                            for (int v = 0; v < kMaxCodeVals; ++v)
                                if (v < F.n_vals) atomicAdd(vs + v, pv[v]);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    const int nf = d.n_flush[part];
    for (int t = 0; t < nf; ++t) {
        const AS_CONST FlushDesc &F = cst(d.flush)[d.flush_base[part] + t];
        const double *val = reinterpret_cast<const double *>(smem + F.lds_val);
        for (int cell = tid; cell < F.n_cells; cell += blockDim.x) {
            const uint32_t c = smem[F.lds_cnt + cell];
            if (c == 0u) continue;
            gadd(d.g_cnt + F.glb_cnt + cell, (unsigned long long)c);
            for (int v = 0; v < F.n_vals; ++v) {
                const double x = val[(int64_t)cell * F.n_vals + v];
                if (x != 0.0) gadd(d.g_val + F.glb_val + (int64_t)cell * F.n_vals + v, x);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// count tables from 16-bit component codes (see HistDesc): one workgroup of
// 1024 threads per (row block, partition); a thread takes eight consecutive
// rows per step (one 16-byte load per code column) and counts each row into
// the slices of its partition that hold its cell
// ---------------------------------------------------------------------------

constexpr int kHistChunks = 4;   // 8-row chunks per thread and slice whose loads are issued together

__global__ __launch_bounds__(1024) void hist_scan_kernel(const HistDesc *__restrict__ dp) {
    extern __shared__ __align__(16) uint32_t smem[];
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const AS_CONST HistDesc &d = *cst(dp);
    const int part = blockIdx.y;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int s0 = cst(d.part_begin)[part], s1 = cst(d.part_begin)[part + 1];
    const int words = cst(d.lds_words)[part];
    for (int i = tid; i < words; i += blockDim.x) smem[i] = 0u;
    __syncthreads();
    const AS_CONST HistSlice *sl = cst(d.slices);
    const int64_t r0 = (int64_t)blockIdx.x * d.rows_per_block;
    const int64_t r1 = r0 + d.rows_per_block < d.n_rows ? r0 + d.rows_per_block : d.n_rows;
    const uint16_t *codes = d.codes;
    // per step the workgroup covers kHistChunks consecutive stretches of 8 * blockDim rows; thread
    // t takes 8 rows of each, so every load instruction of a wave reads 1 KiB contiguous, and the
    // loads of all chunks and components of a slice are in flight together
    const int64_t span = 8 * (int64_t)blockDim.x;
    for (int64_t r = r0; r < r1; r += kHistChunks * span) {
        for (int si = s0; si < s1; ++si) {
            const AS_CONST HistSlice &S = sl[si];
            u32x4 v[kHistChunks][kMaxKeyComps];
#pragma unroll
            for (int j = 0; j < kHistChunks; ++j) {
                const int64_t row = r + j * span + 8 * tid;
#pragma unroll
                for (int c = 0; c < kMaxKeyComps; ++c) {
                    // rows at or past the block's end are not loaded (a chunk that starts before it
                    // ends inside the column: columns are padded to 64 rows)
                    if (c < S.n_comp && row < r1)
                        v[j][c] = gld(reinterpret_cast<const u32x4 *>(codes + (int64_t)S.code[c] * d.pitch + row))[0];
                    else
                        v[j][c] = u32x4{0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
                }
            }
            const uint32_t base = (uint32_t)S.lds_off + (uint32_t)(lane & (S.reps - 1)) * (uint32_t)S.rep_stride;
#pragma unroll
            for (int j = 0; j < kHistChunks; ++j) {
                const int64_t row = r + j * span + 8 * tid;
                const int nv = row >= r1 ? 0 : (r1 - row < 8 ? (int)(r1 - row) : 8);
                uint32_t cell[8];
                bool ok[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    cell[i] = 0u;
                    ok[i] = i < nv;
                }
#pragma unroll
                for (int c = 0; c < kMaxKeyComps; ++c) {
                    if (c >= S.n_comp) break;
                    const uint32_t st = (uint32_t)S.stride[c];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const uint32_t x = (v[j][c][i >> 1] >> (16 * (i & 1))) & 0xFFFFu;
                        if (x == kNoCode) ok[i] = false;
                        cell[i] += x * st;
                    }
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t k = cell[i] - (uint32_t)S.lo;
                    if (ok[i] && k < (uint32_t)S.n) atomicAdd(&smem[base + k], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int si = s0; si < s1; ++si) {
        const AS_CONST HistSlice &S = sl[si];
        for (int k = tid; k < S.n; k += blockDim.x) {
            uint32_t c = 0u;
            for (int rp = 0; rp < S.reps; ++rp) c += smem[S.lds_off + rp * S.rep_stride + k];
            if (c) gadd(d.g_cnt + S.glb_cnt + S.lo + k, (unsigned long long)c);
        }
    }
}

hipError_t set_hist_lds_limit(size_t bytes) {
    return hipFuncSetAttribute((const void *)hist_scan_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_hist(const HistDesc *desc, int grid_x, int parts, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(hist_scan_kernel, dim3(grid_x, parts), dim3(1024), lds_bytes, st, desc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cross-workgroup merge (fp64, fixed order: deterministic)
// ---------------------------------------------------------------------------

// Two passes in a fixed order, so the result does not depend on scheduling.
// Pass 1: workgroup (x, g) sums partials g*P/G .. (g+1)*P/G - 1 for 64
// consecutive packed entries (lane = entry: every load is one coalesced
// 512-byte row), in eight interleaved running sums added in a fixed order.
// Pass 2: each entry sums its G group sums the same way and is written to both
// (i, j) and (j, i).
__global__ void merge_groups_kernel(const MergeDesc *__restrict__ dp) {
    const MergeDesc &d = *dp;
    const int ntri = d.n_gram * (d.n_gram + 1) / 2;
    const int e = blockIdx.x * 64 + threadIdx.x;
    const int g = blockIdx.y;
    const int p0 = (int)((int64_t)d.grid * g / kMergeGroups), p1 = (int)((int64_t)d.grid * (g + 1) / kMergeGroups);
    if (e < ntri) {
        // eight running sums (partial p goes to sum p % 8), added in a fixed order at the end:
        // eight loads in flight per lane, and the same result on every run
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int p = p0;
        for (; p + 8 <= p1; p += 8)
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] += gld(d.gram_partial)[(int64_t)(p + k) * ntri + e];
        for (int k = 0; p < p1; ++p, ++k) a[k] += gld(d.gram_partial)[(int64_t)p * ntri + e];
        gst(d.group_sum)[(int64_t)g * ntri + e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    if (blockIdx.x == 0 && d.count_partial) {
        unsigned long long t = 0;
        for (int p = p0 + threadIdx.x; p < p1; p += 64) t += gld(d.count_partial)[p];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (threadIdx.x == 0) gst(d.group_count)[g] = t;
    }
}

__global__ void merge_final_kernel(const MergeDesc *__restrict__ dp) {
    const MergeDesc &d = *dp;
    const int n = d.n_gram;
    const int ntri = n * (n + 1) / 2;
    const int e = blockIdx.x * 64 + threadIdx.x;
    if (e < ntri) {
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        static_assert(kMergeGroups % 8 == 0, "group sums are taken eight at a time");
        for (int g = 0; g < kMergeGroups; g += 8)
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] += gld(d.group_sum)[(int64_t)(g + k) * ntri + e];
        const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        int i = 0;
        while (tri_index(i + 1, i + 1, n) <= e) ++i;
        const int j = i + (e - tri_index(i, i, n));
        gst(d.gram)[i * n + j] = s;
        gst(d.gram)[j * n + i] = s;
    }
    if (e == 0 && d.count_partial) {
        unsigned long long t = 0;
        for (int g = 0; g < kMergeGroups; ++g) t += gld(d.group_count)[g];
        *gst(d.count) = t;
    }
}

// ---------------------------------------------------------------------------
// marginal derivation of grouped tables: one pass per key length, longest
// first, so every source table is final when it is read; items on blockIdx.y,
// cells of the derived table on threads; each cell sums its source cells in
// ascending order of the dropped component (a fixed order: deterministic)
// ---------------------------------------------------------------------------

__global__ void rollup_kernel(const RollupDesc *__restrict__ dp) {
    const AS_CONST RollupDesc &d = *cst(dp);
    for (int i = blockIdx.y; i < d.n_items; i += gridDim.y) {
        const AS_CONST RollupItem &it = cst(d.items)[i];
        const int64_t S = it.suffix, D = it.dom;
        const int tn = it.t_nvals, un = it.u_nvals;
        const int64_t per = tn + 1;             // the cell's sums, then its count
        const int32_t *map = d.map + it.map_base;
        const unsigned long long *ucnt = d.g_cnt + it.u_cnt;
        const double *uval = d.g_val + it.u_val;
        for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < it.t_cells * per;
             w += (int64_t)gridDim.x * blockDim.x) {
            const int64_t t = w / per;
            const int j = (int)(w - t * per);
            const int64_t u0 = (t / S) * D * S + t % S;
            if (j == tn) {
                unsigned long long cnt = 0;
#pragma unroll 4
                for (int64_t v = 0; v < D; ++v) cnt += gld(ucnt)[u0 + v * S];
                gst(d.g_cnt)[it.t_cnt + t] = cnt;
            } else {
                const int k = gld(map)[j];
                double s = 0.0;
#pragma unroll 4
                for (int64_t v = 0; v < D; ++v) s += gld(uval)[(u0 + v * S) * un + k];
                gst(d.g_val)[it.t_val + t * tn + j] = s;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// result assembly: queries on blockIdx.y, cells on threads
// ---------------------------------------------------------------------------

__global__ void assemble_kernel(const AssembleDesc *__restrict__ dp) {
    const AS_CONST AssembleDesc &d = *cst(dp);
    for (int o = blockIdx.y; o < d.n_out; o += gridDim.y) {
        const AS_CONST OutDesc &O = cst(d.outs)[o];
        const AS_CONST TermDesc *terms = cst(d.terms) + O.term_base;
        const int nt = cst(d.term_count)[o];
        const bool gram = O.kind == SRC_GRAM;
        for (int64_t cell = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; cell < O.n_cells;
             cell += (int64_t)gridDim.x * blockDim.x) {
            const unsigned long long cnt = gram ? *gld(d.count) : gld(d.g_cnt)[O.src_cnt + cell];
            gst(d.res_cnt)[O.dst_cnt + cell] = cnt;
            const double *vals = d.g_val + O.src_val + cell * O.src_nvals;
            // each aggregate summed in registers, its terms in list order
            for (int a = 0; a < O.n_aggs; ++a) {
                double s = 0.0;
                for (int t = 0; t < nt; ++t) {
                    if (terms[t].agg != a) continue;
                    const int src = terms[t].src;
                    const double v = src < 0 ? (double)cnt : (gram ? gld(d.gram)[src] : gld(vals)[src]);
                    s += terms[t].coeff * v;
                }
                gst(d.res_sum)[O.dst_sum + cell * O.n_aggs + a] = s;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// kernel table for the host
// ---------------------------------------------------------------------------

typedef void (*RootKernel)(const RootDesc *);

template <int MODE, int P1>
static RootKernel pick_tables(bool tables) {
    return tables ? (RootKernel)root_scan_kernel<MODE, P1, true> : (RootKernel)root_scan_kernel<MODE, P1, false>;
}

// mode 0: no covariance; 1: fp32 with p1 = register block edge; 2/3: bf16x3/bf16x4 with p1 = 16-wide tiles
RootKernel root_kernel(int mode, int p1, bool tables) {
    switch (mode) {
        case 0: return pick_tables<0, 1>(tables);
        case 1:
            switch (p1) {
                case 2: return pick_tables<1, 2>(tables);
                case 4: return pick_tables<1, 4>(tables);
                case 6: return pick_tables<1, 6>(tables);
                case 8: return pick_tables<1, 8>(tables);
            }
            return nullptr;
        case 2:
            switch (p1) {
                case 1: return pick_tables<2, 1>(tables);
                case 2: return pick_tables<2, 2>(tables);
                case 3: return pick_tables<2, 3>(tables);
                case 4: return pick_tables<2, 4>(tables);
            }
            return nullptr;
        case 3:
            switch (p1) {
                case 1: return pick_tables<3, 1>(tables);
                case 2: return pick_tables<3, 2>(tables);
                case 3: return pick_tables<3, 3>(tables);
                case 4: return pick_tables<3, 4>(tables);
            }
            return nullptr;
        case 4:
            switch (p1) {
                case 1: return pick_tables<4, 1>(tables);
                case 2: return pick_tables<4, 2>(tables);
                case 3: return pick_tables<4, 3>(tables);
                case 4: return pick_tables<4, 4>(tables);
            }
            return nullptr;
    }
    return nullptr;
}

hipError_t launch_fill(const void *fills, int n, hipStream_t st) {
    hipLaunchKernelGGL(multi_fill_kernel, dim3(1024), dim3(256), 0, st, (const FillDesc *)fills, n);
    return hipGetLastError();
}

hipError_t launch_views(const ScanDesc *descs, int n_scans, int64_t max_rows, hipStream_t st) {
    const int64_t blocks = (max_rows + kBlock - 1) / kBlock;
    if (blocks == 0 || n_scans == 0) return hipSuccess;
    hipLaunchKernelGGL(view_build_kernel, dim3((unsigned)blocks, (unsigned)n_scans), dim3(kBlock), 0, st, descs);
    return hipGetLastError();
}

hipError_t launch_dup(const DupDesc *desc, int64_t n_rows, int64_t n_keys, hipStream_t st) {
    const int64_t rb = (n_rows + kBlock - 1) / kBlock, kb = (n_keys + kBlock - 1) / kBlock;
    if (rb > 0) hipLaunchKernelGGL(dup_agg_kernel, dim3((unsigned)rb), dim3(kBlock), 0, st, desc);
    if (kb > 0) hipLaunchKernelGGL(dup_final_kernel, dim3((unsigned)kb), dim3(kBlock), 0, st, desc);
    return hipGetLastError();
}

hipError_t launch_target(const TargetDesc *descs, int n_targets, int64_t max_items, hipStream_t st) {
    const int64_t b = (max_items + kBlock - 1) / kBlock;
    if (b > 0 && n_targets > 0)
        hipLaunchKernelGGL(target_scan_kernel, dim3(b < 1024 ? (unsigned)b : 1024u, (unsigned)n_targets), dim3(kBlock), 0,
                           st, descs);
    return hipGetLastError();
}

hipError_t launch_corr(const CorrDesc *desc, int n_pair, hipStream_t st) {
    if (n_pair > 0) hipLaunchKernelGGL(corr_kernel, dim3(n_pair), dim3(kBlock), 0, st, desc);
    return hipGetLastError();
}

hipError_t launch_root(RootKernel k, const RootDesc *desc, int grid_x, int parts, int waves, size_t lds_bytes,
                       hipStream_t st) {
    hipLaunchKernelGGL(k, dim3(grid_x, parts), dim3(64 * waves), lds_bytes, st, desc);
    return hipGetLastError();
}

hipError_t set_root_lds_limit(RootKernel k, size_t bytes) {
    return hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_merge(const MergeDesc *desc, int n_gram, hipStream_t st) {
    const int ntri = n_gram > 0 ? n_gram * (n_gram + 1) / 2 : 1;
    const int bx = (ntri + 63) / 64;
    hipLaunchKernelGGL(merge_groups_kernel, dim3(bx, kMergeGroups), dim3(64), 0, st, desc);
    hipLaunchKernelGGL(merge_final_kernel, dim3(bx), dim3(64), 0, st, desc);
    return hipGetLastError();
}

hipError_t set_code_scan_lds_limit(size_t bytes) {
    return hipFuncSetAttribute((const void *)code_scan_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_code_scan(const CodeScanDesc *desc, int grid_x, int parts, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(code_scan_kernel, dim3(grid_x, parts), dim3(1024), lds_bytes, st, desc);
    return hipGetLastError();
}

hipError_t launch_rollup(const RollupDesc *desc, int n_items, int64_t max_work, hipStream_t st) {
    if (n_items == 0 || max_work <= 0) return hipSuccess;
    const int64_t bx = (max_work + 255) / 256;
    hipLaunchKernelGGL(rollup_kernel, dim3(bx < 1024 ? (unsigned)bx : 1024u, n_items < 1024 ? n_items : 1024), dim3(256),
                       0, st, desc);
    return hipGetLastError();
}

hipError_t launch_assemble(const AssembleDesc *desc, int n_out, int64_t max_cells, hipStream_t st) {
    if (n_out == 0 || max_cells <= 0) return hipSuccess;
    const int bs = max_cells < 256 ? 64 : 256;
    const int64_t bx = (max_cells + bs - 1) / bs;
    hipLaunchKernelGGL(assemble_kernel, dim3(bx < 1024 ? (unsigned)bx : 1024u, n_out < 4096 ? n_out : 4096), dim3(bs), 0,
                       st, desc);
    return hipGetLastError();
}

}  // namespace lmfao
