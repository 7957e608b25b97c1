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
//  * merge_kernel        fp64 cross-workgroup reduction of the covariance
//                        partials and counts (the domain-parallel partition
//                        merge implied by Section 1.2)
//  * rollup_kernel       grouped tables derived from a finer table with the
//                        same filter by summing out one component
//  * assemble_kernel     per-query results from the merged views
//
// The covariance block is computed in one of three arithmetics:
//   FP32      register-blocked fp32 FMAs over a row tile staged in LDS;
//   BF16X3    every feature split x = hi + lo (bf16, round to nearest even),
//             hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with fp32
//             accumulation;
//   BF16X4    adds lo*lo.
// In both, fp32 accumulators are folded every few hundred rows into
// compensated (TwoSum) fp32 pairs; fp64 appears only in the cross-workgroup
// reduction at the end of the scan and in the merge.
#include <hip/hip_runtime.h>

#include "desc.h"

namespace lmfao {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxChild = 8;

// Address-space views.  Descriptor arrays are read through the constant
// space (scalar loads that wait on lgkmcnt only); per-lane data and atomics
// go through the global space.  Generic (flat) accesses would count against
// both wait counters and serialise the asynchronous LDS copies.
#define AS_GLOBAL __attribute__((address_space(1)))
#define AS_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const AS_CONST T *cst(const T *p) { return (const AS_CONST T *)p; }
template <class T>
__device__ __forceinline__ const AS_GLOBAL T *gld(const T *p) { return (const AS_GLOBAL T *)p; }
template <class T>
__device__ __forceinline__ AS_GLOBAL T *gst(T *p) { return (AS_GLOBAL T *)p; }
template <class T>
__device__ __forceinline__ void gadd(T *p, T v) {
    __hip_atomic_fetch_add(gst(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gor(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_or(gst(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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
// helpers of the root scan
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// s + e += x with TwoSum (Knuth): s is the fp32 sum, e its running error
__device__ __forceinline__ void two_sum_acc(float &s, float &e, float x) {
    const float t = s + x;
    const float bp = t - s;
    e += (s - (t - bp)) + (x - bp);
    s = t;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) void lds_void;

// Asynchronous global -> LDS copies (no registers): every lane's 4 or 16
// bytes land at lds_base + lane * size.  lds_base must be wave-uniform.
__device__ __forceinline__ void lds_dma4(const void *g, uint32_t *lds_base) {
    __builtin_amdgcn_global_load_lds(g, (lds_void *)lds_base, 4, 0, 0);
}
__device__ __forceinline__ void lds_dma16(const void *g, uint32_t *lds_base) {
    __builtin_amdgcn_global_load_lds(g, (lds_void *)lds_base, 16, 0, 0);
}

// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), both round-to-nearest-even
__device__ __forceinline__ void split_bf16x8(const float *x, bf16x8 &hi, bf16x8 &lo) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const f32x2 v = {x[2 * i], x[2 * i + 1]};
        const bf16x2 hb = __builtin_convertvector(v, bf16x2);
        const f32x2 hf = __builtin_convertvector(hb, f32x2);
        const bf16x2 lb = __builtin_convertvector(v - hf, bf16x2);
        h[i] = __builtin_bit_cast(uint32_t, hb);
        l[i] = __builtin_bit_cast(uint32_t, lb);
    }
    hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
    lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

constexpr int kFlushTiles = 16;   // mfma accumulators fold into fp32 sums every 16 tiles (1024 rows per wave)

// Where a staged feature of a tile lives in LDS: word(row) = base + buf * step + row * stride.
struct FeatLoc {
    int base, step, stride;
};

// f: staged feature; src: its feat_src entry; wave: the wave region's first word
__device__ __forceinline__ FeatLoc feat_loc(const RootDesc &d, int f, int src, int wave) {
    if (f == 0) return {d.lds_consts, 0, 1};                 // constant 1
    if (f >= d.n_feat) return {d.lds_consts + 64, 0, 1};     // padding feature 0
    if (src >= 0) return {wave + d.w_rec + src, d.n_quads * 256, 4};   // child record word
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
    constexpr int NLL = MODE == 3 ? NHH : 1;

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
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c) {
            if (c < s.n_child) {
                const uint4 q0 = *reinterpret_cast<const uint4 *>(rb + (children[c].quad_base * 64 + lane) * 4);
                if (q0.x == 0u) valid = false;
                if (s.n_mask > 0) mask &= (uint64_t)q0.y | (s.n_mask > 1 ? (uint64_t)q0.z << 32 : 0ull);
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
        if (do_count) my_count += valid ? 1ull : 0ull;

        // ---- covariance block ---------------------------------------------------------------
        if (MODE == 1 && do_gram && gact) {
            int pa[GB], pb[GB];
#pragma unroll
            for (int q = 0; q < GB; ++q) {
                pa[q] = la[q].base + buf * la[q].step;
                pb[q] = lb[q].base + buf * lb[q].step;
            }
            for (int r = gph; r < 64; r += nph) {
                if (!((vm >> r) & 1ull)) continue;
                float a[GB], b[GB];
#pragma unroll
                for (int q = 0; q < GB; ++q) { a[q] = fsm[pa[q] + r * la[q].stride]; b[q] = fsm[pb[q] + r * lb[q].stride]; }
#pragma unroll
                for (int i = 0; i < GB; ++i)
#pragma unroll
                    for (int j = 0; j < GB; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
            }
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
                bf16x8 fh[NT], fl[NT];
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
                    split_bf16x8(x, fh[t2], fl[t2]);
                }
                int ih = 0;
#pragma unroll
                for (int t2 = 0; t2 < NT; ++t2)
#pragma unroll
                    for (int u = t2; u < NT; ++u, ++ih) {
                        chh[ih] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[t2], fh[u], chh[ih], 0, 0, 0);
                        if (MODE == 3) cll[ih] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fl[t2], fl[u], cll[ih], 0, 0, 0);
                    }
#pragma unroll
                for (int t2 = 0; t2 < NT; ++t2)
#pragma unroll
                    for (int u = 0; u < NT; ++u)
                        chl[t2 * NT + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[t2], fl[u], chl[t2 * NT + u], 0, 0, 0);
            }
            if (++tiles_since_flush == kFlushTiles) {
                const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < NHH; ++i) { shh[i] += chh[i]; chh[i] = z; }
                tiles_since_flush = 0;
            }
        }

        // ---- grouped tables (this lane's own row) ---------------------------------------------
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
                                atomicAdd(&smem[u + K.off_cnt + cell], 1u);
                                if (F.n_vals) {
                                    double *vs = reinterpret_cast<double *>(smem + u + K.off_val) + (int64_t)cell * F.n_vals;
                                    for (int v = 0; v < F.n_vals; ++v) {
                                        const AS_CONST ValDesc &vd = vals[F.val_base + v];
                                        atomicAdd(vs + v, fval(vd.a) * fval(vd.b));
                                    }
                                }
                            }
                        }
                    }
                    continue;
                }
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
                            atomicAdd(&smem[d.lds_tables + T.lds_cnt + cell], 1u);
                            double *vs = reinterpret_cast<double *>(smem + d.lds_tables + T.lds_val) + (int64_t)cell * F.n_vals;
                            for (int v = 0; v < F.n_vals; ++v) {
                                const AS_CONST ValDesc &vd = vals[F.val_base + v];
                                atomicAdd(vs + v, fval(vd.a) * fval(vd.b));
                            }
                        } else {
                            gadd(d.g_cnt + T.glb_cnt + cell, 1ull);
                            double *vs = d.g_val + T.glb_val + (int64_t)cell * F.n_vals;
                            for (int v = 0; v < F.n_vals; ++v) {
                                const AS_CONST ValDesc &vd = vals[F.val_base + v];
                                gadd(vs + v, fval(vd.a) * fval(vd.b));
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
        const int nred = (MODE == 3 ? 3 : 2) * n16 * n16;
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
                    if (MODE == 3) atomicAdd(&rll[(16 * t + ci + e) * n16 + 16 * u + cj], (double)cll[ih][e]);
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
                if (MODE == 3) v += rll[i * n16 + j];
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
            for (int k = 0; k < F.n_keys; ++k) {
                const AS_CONST KeyDesc &K = keys[F.key_base + k];
                const uint32_t cell = gld(codes)[(int64_t)(F.code_base + k) * d.pitch + r];
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
// covariance-only root scan (BF16 hi+lo split on matrix cores)
// ---------------------------------------------------------------------------

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
    // raw buffer: stride 0, range `bytes`; loads beyond the range return zeros
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// One wave scans its rows in 64-row tiles.  Lane (i, g) = (lane % 16,
// lane / 16) feeds slot i of each 16-slot tile; in k-step ks (32 rows) it
// holds rows 32ks + 4g + {0..3} and 32ks + 16 + 4g + {0..3}.  (Any pairing of
// rows to MFMA k-indices is valid as long as every operand uses the same one;
// this one keeps the four lane groups on different LDS banks and lets every
// fact chunk be one 16-byte load.)  Per tile t:
//   1. wait until tile t's records and facts and tile t+1's keys have landed;
//   2. spread records gathered once for a uniform key to every row; write tile
//      t's facts (loaded as 256 contiguous bytes per column) from registers to
//      the wave's LDS fact tile, and request tile t+1's facts into them;
//   3. find the tile's valid rows and split every slot value x = hi + lo in
//      bf16 into operand registers (from the fact tile, the record buffer and
//      the constant block);
//   4. gather tile t+1's child records into the record buffer with buffer
//      loads that bypass registers (a key outside [0, n_keys) reads past the
//      buffer range and lands as zeros: no join), then request the keys of
//      tile t+2 (after the last tile these requests repeat it, unused);
//   5. accumulate hi*hi + hi*lo + lo*hi (+ lo*lo) for every upper-triangle
//      16x16 tile pair on MFMA while those copies are in flight.
// Fact columns and keys are streamed once: their loads are non-temporal, so
// they do not push the gathered view records out of the caches.  Each wave
// writes its own fp64 partial of the upper triangle (no LDS reduction).
template <int NT, int NF, bool X4, bool PR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NT >= 4 ? 2 : 3))) void gram_scan_kernel(
    const GramDesc *__restrict__ dp) {
    extern __shared__ __align__(16) uint32_t smem[];
    const AS_CONST GramDesc &d = *cst(dp);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    constexpr int NP = NT * (NT + 1) / 2;
    constexpr int NFA = NF > 0 ? NF : 1;

    // the constant block: 64 rows of [1, 0, 0, 0] (pair rows: [1, 0, ..., 0] of 8 words), laid out
    // like the record rows so that constant and padding slots read it with the records' stride
    constexpr int kRowWords = PR ? 8 : 4;
    if (tid < 64) {
        smem[kRowWords * tid] = __float_as_uint(1.f);
#pragma unroll
        for (int w = 1; w < kRowWords; ++w) smem[kRowWords * tid + w] = 0u;
    }
    __syncthreads();

    // row indices fit 32 bits: the planner refuses a root above 2^30 rows
    const int n_rows = (int)d.n_rows;
    const int rpb = (int)d.rows_per_block;
    const int blk_begin = (int)blockIdx.x * rpb;
    const int blk_end = min(blk_begin + rpb, n_rows);
    // the waves of a workgroup take its 64-row tiles in turn, so that at any time they stream
    // neighbouring stretches of every column (DRAM pages are opened once for several waves)
    const int blk_tiles = blk_end > blk_begin ? (blk_end - blk_begin + 63) / 64 : 0;
    const int n_tiles = blk_tiles > wave ? (blk_tiles - wave + nwaves - 1) / nwaves : 0;
    const int n_child = d.n_child;
    const int rbase = d.lds_wave0 + wave * d.wave_bytes;     // this wave's record buffer (bytes)
    const uint32_t last_row = (uint32_t)(n_rows - 1);

    // per-lane sources of the NT slots this lane feeds (in fact tiles, fact lanes read the
    // fact tile in LDS at lds_off; other lanes their record word or the constant quad)
    bool is_fact[NT];
    int lds_off[NT];
    const int fbase = rbase + d.fact_off;                      // this wave's fact tile in LDS
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int s = 16 * t + li;
        const int fc = gld(&dp->slot[s].fact)[0];
        is_fact[t] = fc >= 0;
        const int off = gld(&dp->slot[s].lds)[0];       // row 0 of the slot's word
        lds_off[t] = fc >= 0 ? fbase + s * kFactPitch : (gld(&dp->slot[s].per_buf)[0] ? rbase + off : off);
    }
    // fact loads: in load q of fact tile f, lane (i, g) reads rows 4i..4i+3 of fact column
    // 16f + 4q + g, so 16 lanes read 256 contiguous bytes of one column.  Lanes past the last
    // fact column read column 0 (ignored), so every load is issued by the whole wave.
    const char *fld[NFA][4];
    int fst[NFA][4];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 16 * f + 4 * q + lg;
            fld[f][q] = reinterpret_cast<const char *>(gld(d.fact_cols)[c < d.n_fact ? c : 0]) + 16 * li;
            fst[f][q] = fbase + c * kFactPitch + 16 * li;
        }
    const bool mixed = NF > 0 && d.n_fact < 16 * NF;   // wave-uniform: the last fact tile has LDS lanes too

    // per-child constants, hoisted out of the tile loop (wave-uniform)
    __amdgpu_buffer_rsrc_t rrs[kGramMaxChild];
    const int32_t *fkp[kGramMaxChild];
    uint32_t nkey[kGramMaxChild], rbytes[kGramMaxChild];
    int cdst[kGramMaxChild], cnq[kGramMaxChild];
#pragma unroll
    for (int c = 0; c < kGramMaxChild; ++c)
        if (c < n_child) {
            const AS_CONST GramChild &ch = d.ch[c];
            nkey[c] = ch.n_keys;
            rbytes[c] = ch.rec_bytes;
            rrs[c] = buffer_rsrc(ch.rec, nkey[c] * rbytes[c]);
            fkp[c] = ch.fk;
            cdst[c] = rbase + ch.quad0 * kQuadBytes;
            cnq[c] = ch.n_quads;
        }

    f32x4 acc[NP], sacc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        acc[p] = f32x4{0.f, 0.f, 0.f, 0.f};
        sacc[p] = acc[p];
    }
    unsigned long long count = 0;
    int since_flush = 0;

    uint32_t key[kGramMaxChild];
    // children whose keys are equal on all 64 rows of the next / this tile (the fact is sorted
    // by its keys, so long runs are common): their record is gathered by one lane into row 0
    // and copied to the other rows inside LDS, which costs the memory pipeline one request
    uint32_t uni_next = 0u, uni_cur = 0u;
    // children whose record buffer holds one record in every row (a uniform tile, spread), and
    // that record's key: a next tile with the same uniform key needs no copy at all
    uint32_t held_ok = 0u;
    uint32_t held[kGramMaxChild];
    f32x4 F[NFA][4];      // the next tile's fact chunks, in flight (see fld)

    auto tile_row = [&](int t) -> int { return blk_begin + 64 * (wave + t * nwaves); };
    auto load_keys = [&](int t) {
        const uint32_t row = min((uint32_t)(tile_row(t) + lane), last_row);
#pragma unroll
        for (int c = 0; c < kGramMaxChild; ++c)
            if (c < n_child) key[c] = (uint32_t)__builtin_nontemporal_load(gld(fkp[c]) + row);
    };
    auto issue_rec = [&]() {
        uni_next = 0u;
#pragma unroll
        for (int c = 0; c < kGramMaxChild; ++c)
            if (c < n_child) {
                const uint32_t k0 = __builtin_amdgcn_readfirstlane(key[c]);
                const bool uni = __ballot(key[c] != k0) == 0ull;
                uint32_t koff = __umul24(min(key[c], nkey[c]), rbytes[c]);
                char *dst = reinterpret_cast<char *>(smem) + cdst[c];
                if (uni && ((held_ok >> c) & 1u) && held[c] == k0) {
                    // already in every row (the fact is sorted, so the small dimensions' keys
                    // stay the same over many tiles)
                } else if (uni) {
                    uni_next |= 1u << c;
                    held[c] = k0;
                    held_ok |= 1u << c;
                    if (PR) {
                        // lanes 0 and 1: the record's two quads land in row 0 (a one-quad
                        // record's second lane reads past the buffer range: zeros)
                        if (lane < 2) {
                            const uint32_t ko = lane < cnq[c] ? koff + 16u * (uint32_t)lane : nkey[c] * rbytes[c];
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(rrs[c], (lds_void *)dst, 16, ko, 0, 0, 0);
                        }
                    } else if (lane == 0) {
                        // one lane: the record lands in row 0 of each quad
#pragma unroll 1
                        for (int q = 0; q < cnq[c]; ++q, koff += 16u, dst += kQuadBytes)
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(rrs[c], (lds_void *)dst, 16, koff, 0, 0, 0);
                    }
                } else {
                    held_ok &= ~(1u << c);
                    if (PR) {
                        // lane l of request i reads quad l % 2 of row 32 i + l / 2: a row's two
                        // quads are one contiguous 32-byte piece on neighbouring lanes, so the
                        // memory pipeline handles one address per row, not one per row and quad
#pragma unroll
                        for (int i = 0; i < 2; ++i) {
                            const uint32_t f = 64u * (uint32_t)i + (uint32_t)lane;
                            const uint32_t kr = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(4u * (f >> 1)), (int)key[c]);
                            const uint32_t ko = (f & 1u) < (uint32_t)cnq[c] ? __umul24(min(kr, nkey[c]), rbytes[c]) + 16u * (f & 1u)
                                                                           : nkey[c] * rbytes[c];
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(rrs[c], (lds_void *)(dst + 1024 * i), 16, ko, 0, 0, 0);
                        }
                    } else {
                        // a rolled loop: per-quad conditions and addresses stay out of the scalar registers
#pragma unroll 1
                        for (int q = 0; q < cnq[c]; ++q, koff += 16u, dst += kQuadBytes)
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(rrs[c], (lds_void *)dst, 16, koff, 0, 0, 0);
                    }
                }
            }
    };
    // fact chunks of tile t into F: always four loads per fact tile by the whole wave, so the
    // count of operations in flight never depends on the data.  A tile that ends past the
    // last row loads clamped (in-bounds) chunks; its rows are re-read one by one before use.
    auto load_fact = [&](int t) {
        const int r0 = tile_row(t);
        if (r0 + 64 <= n_rows) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    F[f][q] = __builtin_nontemporal_load(gld(reinterpret_cast<const f32x4 *>(fld[f][q] + (uint32_t)r0 * 4u)));
        } else {
            const int rq = min(r0 + 4 * li, n_rows - 4);
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    F[f][q] = gld(reinterpret_cast<const f32x4 *>(fld[f][q] - 16 * li + (uint32_t)rq * 4u))[0];
        }
    };
    // the tile's facts from F into the wave's LDS fact tile (a tile ending past the last row
    // is re-read row by row first, waited for here so no load stays pending)
    auto store_fact = [&](int t) {
        const int r0 = tile_row(t);
        if (r0 + 64 > n_rows) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float *p = reinterpret_cast<const float *>(fld[f][q] - 16 * li) + r0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) F[f][q][e] = r0 + 4 * li + e < n_rows ? gld(p)[4 * li + e] : 0.f;
                }
            __builtin_amdgcn_s_waitcnt(0x0F70);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int q = 0; q < 4; ++q) *reinterpret_cast<f32x4 *>(reinterpret_cast<char *>(smem) + fst[f][q]) = F[f][q];
    };

    // Phase 1 of a tile: validity, then every operand of both k-steps split into bf16 hi/lo
    // registers.  After it the tile needs neither its LDS record buffer nor its fact
    // registers, so the next copies can be issued before phase 2 (the MFMAs) runs.
    bf16x8 oph[2][NT], opl[2][NT];
    auto phase1 = [&](int t) -> bool {
        const int r0 = tile_row(t);
        bool valid = r0 + lane < blk_end;
        uint32_t cnt[kGramMaxChild];
#pragma unroll
        for (int c = 0; c < kGramMaxChild; ++c) cnt[c] = c < n_child ? smem[cdst[c] / 4 + kRowWords * lane] : 1u;
#pragma unroll
        for (int c = 0; c < kGramMaxChild; ++c)
            if (cnt[c] == 0u) valid = false;
        const uint64_t vm = __ballot(valid);
        count += (unsigned long long)__popcll(vm);
        const bool all_rows = vm == ~0ull;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const uint32_t vbits = (uint32_t)((vm >> (32 * ks + 4 * lg)) & 0xFull) |
                                   ((uint32_t)((vm >> (32 * ks + 16 + 4 * lg)) & 0xFull) << 4);
#pragma unroll
            for (int t2 = 0; t2 < NT; ++t2) {
                float x[8];
                if (t2 < NF && is_fact[t2]) {
                    // rows 32ks + 4g + {0..3} and 32ks + 16 + 4g + {0..3} of the slot's column
                    const char *base = reinterpret_cast<const char *>(smem) + lds_off[t2] + 128 * ks + 16 * lg;
                    const f32x4 lo4 = *reinterpret_cast<const f32x4 *>(base);
                    const f32x4 hi4 = *reinterpret_cast<const f32x4 *>(base + 64);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        x[e] = lo4[e];
                        x[4 + e] = hi4[e];
                    }
                }
                if (t2 >= NF || (t2 == NF - 1 && mixed)) {
                    if (t2 >= NF || !is_fact[t2]) {
                        const float *p = reinterpret_cast<const float *>(reinterpret_cast<const char *>(smem) +
                                                                         lds_off[t2] + 16 * kRowWords * lg + 128 * kRowWords * ks);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            x[i] = p[kRowWords * i];
                            x[4 + i] = p[16 * kRowWords + kRowWords * i];
                        }
                    }
                }
                if (!all_rows) {
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (!((vbits >> i) & 1u)) x[i] = 0.f;
                }
                split_bf16x8(x, oph[ks][t2], opl[ks][t2]);
            }
        }
        return true;
    };
    // Phase 2: the MFMAs of both k-steps, from registers only.
    auto phase2 = [&]() {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            int p = 0;
#pragma unroll
            for (int a = 0; a < NT; ++a)
#pragma unroll
                for (int b = a; b < NT; ++b, ++p)
                    acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(oph[ks][a], oph[ks][b], acc[p], 0, 0, 0);
            p = 0;
#pragma unroll
            for (int a = 0; a < NT; ++a)
#pragma unroll
                for (int b = a; b < NT; ++b, ++p)
                    acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(oph[ks][a], opl[ks][b], acc[p], 0, 0, 0);
            p = 0;
#pragma unroll
            for (int a = 0; a < NT; ++a)
#pragma unroll
                for (int b = a; b < NT; ++b, ++p)
                    acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(opl[ks][a], oph[ks][b], acc[p], 0, 0, 0);
            if (X4) {
                p = 0;
#pragma unroll
                for (int a = 0; a < NT; ++a)
#pragma unroll
                    for (int b = a; b < NT; ++b, ++p)
                        acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(opl[ks][a], opl[ks][b], acc[p], 0, 0, 0);
            }
        }
        if (++since_flush == kFlushTiles) {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                sacc[p] += acc[p];
                acc[p] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
            since_flush = 0;
        }
    };

    // Every step issues the same operations whether or not a further tile exists (past the
    // end they re-read the last tile, in bounds, and nothing uses the result): the count of
    // operations after any load is then the same on every path, and the compiler's own
    // waits before a register's first use never reach past the newest fact loads.
    auto step = [&](int t) {
        // this tile's records and facts and the next keys have landed
        __builtin_amdgcn_s_waitcnt(0x0F70);
        wave_sync();
        uni_cur = uni_next;
        const bool live = t < n_tiles;
        if (live && uni_cur) {
            // records gathered once: row 0 to the other rows of each quad
#pragma unroll
            for (int c = 0; c < kGramMaxChild; ++c)
                if (c < n_child && ((uni_cur >> c) & 1u)) {
                    char *q0 = reinterpret_cast<char *>(smem) + cdst[c];
                    if (PR) {
                        const f32x4 v0 = *reinterpret_cast<const f32x4 *>(q0);
                        const f32x4 v1 = *reinterpret_cast<const f32x4 *>(q0 + 16);
                        if (lane > 0) {
                            *reinterpret_cast<f32x4 *>(q0 + 32 * lane) = v0;
                            *reinterpret_cast<f32x4 *>(q0 + 32 * lane + 16) = v1;
                        }
                    } else {
#pragma unroll 1
                        for (int q = 0; q < cnq[c]; ++q, q0 += kQuadBytes) {
                            const f32x4 v = *reinterpret_cast<const f32x4 *>(q0);
                            if (lane > 0) *reinterpret_cast<f32x4 *>(q0 + 16 * lane) = v;
                        }
                    }
                }
        }
        if (live) store_fact(t);
        load_fact(min(t + 1, n_tiles - 1));             // in flight for the rest of the step
        wave_sync();
        if (live) phase1(t);
        __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this tile's LDS reads are done
        wave_sync();
        issue_rec();                                    // tile t+1 (keys loaded last step)
        load_keys(min(t + 2, n_tiles - 1));
        if (live) phase2();                             // MFMAs while the copies are in flight
    };

    if (n_tiles > 0) {
        load_keys(0);
        __builtin_amdgcn_s_waitcnt(0x0F70);
        issue_rec();
        load_keys(min(1, n_tiles - 1));
        load_fact(0);
    }
    for (int t = 0; t < n_tiles; ++t) step(t);
    __builtin_amdgcn_s_waitcnt(0);

    // ---- every wave writes its own partial: fp64 upper triangle, staged feature order ------
    // (each unordered feature pair is one slot pair: one lane of one accumulator owns it)
    const int ng = d.n_gram;
    const int pidx = blockIdx.x * nwaves + wave;
    double *out = d.gram_partial + (int64_t)pidx * (ng * (ng + 1) / 2);
    {
        int p = 0;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int b = a; b < NT; ++b, ++p) {
                const int sb = 16 * b + li;
                const int fb = gld(&dp->slot[sb].feat)[0];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int sa = 16 * a + 4 * lg + e;
                    if (a == b && sa > sb) continue;
                    const int fa = gld(&dp->slot[sa].feat)[0];
                    if (fa < 0 || fb < 0) continue;
                    gst(out)[tri_index(min(fa, fb), max(fa, fb), ng)] = (double)sacc[p][e] + (double)acc[p][e];
                }
            }
    }
    if (d.do_count && lane == 0) gst(d.count_partial)[pidx] = count;
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
    }
    return nullptr;
}

typedef void (*GramKernel)(const GramDesc *);

template <int NT, int NF>
static GramKernel pick_gram(bool x4, bool pr) {
    if (pr) return x4 ? (GramKernel)gram_scan_kernel<NT, NF, true, true> : (GramKernel)gram_scan_kernel<NT, NF, false, true>;
    return x4 ? (GramKernel)gram_scan_kernel<NT, NF, true, false> : (GramKernel)gram_scan_kernel<NT, NF, false, false>;
}

// nt: 16-wide slot tiles (1..4); nf: tiles holding fact slots (0..min(nt, 2)); pr: pair-row record
// buffers (every child record at most two quads, a row's quads contiguous) instead of quad-major ones
GramKernel gram_kernel(int nt, int nf, bool x4, bool pr) {
    if (nf < 0 || nf > 2 || nf > nt) return nullptr;
    switch (nt * 4 + nf) {
        case 4: return pick_gram<1, 0>(x4, pr);
        case 5: return pick_gram<1, 1>(x4, pr);
        case 8: return pick_gram<2, 0>(x4, pr);
        case 9: return pick_gram<2, 1>(x4, pr);
        case 10: return pick_gram<2, 2>(x4, pr);
        case 12: return pick_gram<3, 0>(x4, pr);
        case 13: return pick_gram<3, 1>(x4, pr);
        case 14: return pick_gram<3, 2>(x4, pr);
        case 16: return pick_gram<4, 0>(x4, pr);
        case 17: return pick_gram<4, 1>(x4, pr);
        case 18: return pick_gram<4, 2>(x4, pr);
    }
    return nullptr;
}

hipError_t launch_gram(GramKernel k, const GramDesc *desc, int grid_x, int waves, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(k, dim3(grid_x), dim3(64 * waves), lds_bytes, st, desc);
    return hipGetLastError();
}

hipError_t set_gram_lds_limit(GramKernel k, size_t bytes) {
    return hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
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
