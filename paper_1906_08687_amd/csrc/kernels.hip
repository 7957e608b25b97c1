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
//                        equation (2) and Appendix D's lockstep aggregate
//                        arrays), the total count, and grouped tables
//                        (COUNT and SUM of monomials GROUP BY components,
//                        optionally restricted by a filter; equations (3),
//                        (4), (5), (8)).
//  * merge_kernel        fp64 cross-workgroup reduction of the covariance
//                        partials and counts (the domain-parallel partition
//                        merge implied by Section 1.2)
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

__device__ __forceinline__ bool pred_holds(const PredSrc &p, int64_t row) {
    if (p.is_float) return compare(static_cast<const float *>(p.col)[row], p.op, p.fval);
    return compare(static_cast<const int32_t *>(p.col)[row], p.op, p.ival);
}

// categorical code (checked against its domain) or bucket #{k : thr[k] < x}
__device__ __forceinline__ int32_t comp_value(const CompSrc &c, int64_t row, uint32_t *err) {
    if (c.nthr == 0) {
        int32_t v = static_cast<const int32_t *>(c.col)[row];
        if (v < 0 || v >= c.dom) {
            atomicOr(err, kErrDomain);
            v = 0;
        }
        return v;
    }
    const float x = static_cast<const float *>(c.col)[row];
    int lo = 0, hi = c.nthr;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c.thr[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// view records of non-root relations (one thread per row; grid.y = relation)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void view_build_kernel(const ScanDesc *__restrict__ descs) {
    const ScanDesc &d = descs[blockIdx.y];
    const int64_t row = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (row >= d.n_rows) return;
    const int32_t key = d.key[row];
    if (key < 0 || key >= d.n_keys) {
        atomicOr(d.err, kErrKeyRange);
        return;
    }
    if (atomicAdd(&d.seen[key], 1u) != 0u) {   // the join key of a child must be unique
        atomicOr(d.err, kErrDupKey);
        return;
    }
    uint32_t *rec = d.rec_out + (int64_t)key * d.rec_stride;
    uint32_t valid = 1u;
    uint64_t mask = d.filter_all;
    for (int c = 0; c < d.n_child; ++c) {
        const ChildSrc &ch = d.children[c];
        const int32_t k = ch.fk[row];
        if (k < 0 || k >= ch.n_keys) { valid = 0u; continue; }
        const uint32_t *cr = ch.rec + (int64_t)k * ch.stride;
        if (cr[0] == 0u) { valid = 0u; continue; }
        if (ch.n_mask > 0) {
            uint64_t m = cr[1];
            if (ch.n_mask > 1) m |= (uint64_t)cr[2] << 32;
            mask &= m;
        }
        for (int i = 0; i < ch.n_comp; ++i) rec[d.rec_comp_off + ch.comp_dst + i] = cr[ch.comp_off + i];
        for (int i = 0; i < ch.n_feat; ++i) rec[d.rec_feat_off + ch.feat_dst + i] = cr[ch.feat_off + i];
    }
    for (int f = 0; f < d.n_feat; ++f) rec[d.rec_feat_off + d.feats[f].dst] = __float_as_uint(d.feats[f].col[row]);
    for (int c = 0; c < d.n_comp; ++c) rec[d.rec_comp_off + d.comps[c].dst] = (uint32_t)comp_value(d.comps[c], row, d.err);
    for (int p = 0; p < d.n_pred; ++p)
        if (!pred_holds(d.preds[p], row)) mask &= ~(1ull << d.preds[p].filter);
    if (d.n_mask > 0) rec[1] = (uint32_t)mask;
    if (d.n_mask > 1) rec[2] = (uint32_t)(mask >> 32);
    rec[0] = valid;
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

__device__ __forceinline__ void two_sum_acc4(f32x4 &s, f32x4 &e, f32x4 x) {
    const f32x4 t = s + x;
    const f32x4 bp = t - s;
    e += (s - (t - bp)) + (x - bp);
    s = t;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// bf16 fragment layout of one wave (64 rows = two 32-row k-steps):
// dword((kstep*2 + part) * frag_sp + tile*272 + group*68 + feat*4 + slot/2)
// holds rows 8*group + slot, slot+1 of feature 16*tile + feat; part 0 = hi, 1 = lo.
constexpr int kTileWords = 272;
constexpr int kGroupWords = 68;

template <int MODE, int P1, bool TABLES>
__global__ __launch_bounds__(kBlock) void root_scan_kernel(const RootDesc *__restrict__ dp) {
    extern __shared__ __align__(16) uint32_t smem[];
    const RootDesc &d = *dp;
    const ScanDesc &s = d.scan;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int part = blockIdx.y;
    const bool do_gram = MODE != 0 && part == d.gram_part && d.n_gram > 0;
    const bool do_count = d.do_count && part == d.gram_part;

    constexpr int GB = MODE == 1 ? P1 : 1;
    constexpr int NT = MODE >= 2 ? P1 : 1;
    constexpr int NHH = NT * (NT + 1) / 2;
    constexpr int NHL = NT * NT;
    constexpr int NLL = MODE == 3 ? NHH : 0;

    // ---- LDS set-up --------------------------------------------------------
    if (TABLES) {
        const int words = d.lds_table_words[part];
        for (int i = tid; i < words; i += kBlock) smem[d.lds_tables + i] = 0u;
    }
    if (MODE >= 2 && do_gram) {   // padding features stay zero for the whole scan
        for (int i = tid; i < 4 * d.frag_wave_words; i += kBlock) smem[d.lds_frag + i] = 0u;
    }
    if (MODE == 1 && do_gram) {
        for (int i = tid; i < kBlock * d.ngp; i += kBlock) smem[d.lds_xs + i] = 0u;
    }

    // ---- fp32 covariance: thread -> (row phase, GB x GB block pair) ------------
    int gI = 0, gJ = 0, gph = 0, nph = 1;
    bool gact = false;
    float acc[GB][GB], shi[GB][GB], slo[GB][GB];
    if (MODE == 1) {
#pragma unroll
        for (int i = 0; i < GB; ++i)
#pragma unroll
            for (int j = 0; j < GB; ++j) acc[i][j] = shi[i][j] = slo[i][j] = 0.f;
        const int nb = d.ngp / GB;
        const int np = nb * (nb + 1) / 2;
        nph = kBlock / np;
        if (tid < np * nph) {
            gact = true;
            int p = tid % np;
            gph = tid / np;
            int I = 0;
            while (p >= nb - I) { p -= nb - I; ++I; }
            gI = I;
            gJ = I + p;
        }
    }
    // ---- bf16 covariance accumulators ---------------------------------------------
    f32x4 chh[NHH], chl[NHL], cll[NLL > 0 ? NLL : 1];
    f32x4 shh[NHH], ehh[NHH], shl[NHL], ehl[NHL], sll[NLL > 0 ? NLL : 1], ell[NLL > 0 ? NLL : 1];
    if (MODE >= 2) {
#pragma unroll
        for (int i = 0; i < NHH; ++i) chh[i] = shh[i] = ehh[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < NHL; ++i) chl[i] = shl[i] = ehl[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < (NLL > 0 ? NLL : 1); ++i) cll[i] = sll[i] = ell[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    int rows_since_flush = 0;

    unsigned long long my_count = 0;
    const int64_t row_begin = (int64_t)blockIdx.x * d.rows_per_block;
    const int64_t row_end = min(row_begin + d.rows_per_block, s.n_rows);
    float *xs = reinterpret_cast<float *>(smem + d.lds_xs);
    float *tfeat = reinterpret_cast<float *>(smem + d.lds_tfeat);
    int32_t *tcomp = reinterpret_cast<int32_t *>(smem + d.lds_tcomp);
    uint32_t *frag = smem + d.lds_frag + wave * d.frag_wave_words;
    // this lane's slot in the fragment layout (row = lane of the wave)
    const int f_ks = lane >> 5, f_grp = (lane >> 3) & 3, f_half = (lane & 7) >> 1, f_part = lane & 1;
    const int f_wbase = (f_ks * 2 + f_part) * d.frag_sp + f_grp * kGroupWords + f_half;
    __syncthreads();

    for (int64_t base = row_begin; base < row_end; base += kBlock) {
        const int64_t row = base + tid;
        const bool in = row < row_end;
        bool valid = in;
        uint64_t mask = s.filter_all;

        // child views: validity, filter masks (one record per key, Section 3.2)
        const uint32_t *rp[kMaxChild];
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c) {
            rp[c] = nullptr;
            if (c < s.n_child) {
                const ChildSrc &ch = s.children[c];
                if (in) {
                    const int32_t k = ch.fk[row];
                    if (k >= 0 && k < ch.n_keys) {
                        const uint32_t *r = ch.rec + (int64_t)k * ch.stride;
                        if (r[0] != 0u) {
                            rp[c] = r;
                            if (ch.n_mask > 0) {
                                uint64_t m = r[1];
                                if (ch.n_mask > 1) m |= (uint64_t)r[2] << 32;
                                mask &= m;
                            }
                        } else valid = false;
                    } else valid = false;
                }
            }
        }
        if (in)
            for (int p = 0; p < s.n_pred; ++p)
                if (!pred_holds(s.preds[p], row)) mask &= ~(1ull << s.preds[p].filter);
        if (do_count) my_count += valid ? 1ull : 0ull;

        if (MODE >= 2 && do_gram) wave_sync();   // previous fragments consumed

        // ---- stage features: x[0] = 1, own columns, child record features -------
        auto put = [&](int dst, float v) {
            if (MODE == 1 && do_gram && dst < d.n_gram) xs[tid * d.ngp + dst] = v;
            if (MODE >= 2 && do_gram && dst < d.n_gram) {
                const uint32_t hi = bf16_rne(v);
                const uint32_t lo = bf16_rne(v - __uint_as_float(hi << 16));
                const uint32_t send = (lane & 1) ? hi : lo;
                const uint32_t recv = (uint32_t)__shfl_xor((int)send, 1);
                const uint32_t word = (lane & 1) ? (recv | (lo << 16)) : (hi | (recv << 16));
                frag[f_wbase + (dst >> 4) * kTileWords + (dst & 15) * 4] = word;
            }
            if (TABLES && dst < d.n_tfeat) tfeat[tid * d.n_tfeat + dst] = v;
        };
        put(0, valid ? 1.f : 0.f);
        for (int f = 0; f < s.n_feat; ++f) {
            const FeatSrc &fs = s.feats[f];
            float v = 0.f;
            if (valid) v = fs.col[row];
            put(fs.dst, v);
        }
#pragma unroll
        for (int c = 0; c < kMaxChild; ++c) {
            if (c < s.n_child) {
                const ChildSrc &ch = s.children[c];
                const uint32_t *r = rp[c];
                for (int i = 0; i < ch.n_feat; ++i) {
                    float v = 0.f;
                    if (valid) v = __uint_as_float(r[ch.feat_off + i]);
                    put(ch.feat_dst + i, v);
                }
                if (TABLES && valid)
                    for (int i = 0; i < ch.n_comp; ++i) tcomp[tid * d.n_comp + ch.comp_dst + i] = (int32_t)r[ch.comp_off + i];
            }
        }
        if (TABLES && valid)
            for (int c = 0; c < s.n_comp; ++c) tcomp[tid * d.n_comp + s.comps[c].dst] = comp_value(s.comps[c], row, d.err);

        // ---- grouped tables (this thread's own row) ------------------------------------
        if (TABLES && valid) {
            const float *xr = tfeat + tid * d.n_tfeat;
            const int32_t *cr = tcomp + tid * d.n_comp;
            for (int fi = 0; fi < d.n_fam; ++fi) {
                const FamilyDesc &F = d.fams[fi];
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
                        const TabDesc &T = d.tabs[F.tab_base + f * F.n_keys + k];
                        if (T.part != part) continue;
                        const KeyDesc &K = d.keys[F.key_base + k];
                        int32_t cell = 0;
                        for (int c = 0; c < K.n_comp; ++c) cell += cr[K.c[c]] * K.s[c];
                        // a product of two fp32 values is exact in fp64; the cell sums
                        // accumulate in fp64 (runs of one dimension key repeat a value
                        // thousands of times in a row, beyond what fp32 sums exactly)
                        if (T.lds_cnt >= 0) {
                            atomicAdd(&smem[d.lds_tables + T.lds_cnt + cell], 1u);
                            double *vs = reinterpret_cast<double *>(smem + d.lds_tables + T.lds_val) + (int64_t)cell * F.n_vals;
                            for (int v = 0; v < F.n_vals; ++v) {
                                const ValDesc vd = d.vals[F.val_base + v];
                                atomicAdd(vs + v, (double)xr[vd.a] * (double)xr[vd.b]);
                            }
                        } else {
                            atomicAdd(&d.g_cnt[T.glb_cnt + cell], 1ull);
                            double *vs = d.g_val + T.glb_val + (int64_t)cell * F.n_vals;
                            for (int v = 0; v < F.n_vals; ++v) {
                                const ValDesc vd = d.vals[F.val_base + v];
                                atomicAdd(vs + v, (double)xr[vd.a] * (double)xr[vd.b]);
                            }
                        }
                    }
                }
            }
        }

        // ---- covariance block --------------------------------------------------------
        if (MODE == 1) {
            __syncthreads();
            if (do_gram && gact) {
                for (int r = gph; r < kBlock; r += nph) {
                    const float *xr = xs + r * d.ngp;
                    float a[GB], b[GB];
#pragma unroll
                    for (int q = 0; q < GB; ++q) { a[q] = xr[gI * GB + q]; b[q] = xr[gJ * GB + q]; }
#pragma unroll
                    for (int i = 0; i < GB; ++i)
#pragma unroll
                        for (int j = 0; j < GB; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
                }
                rows_since_flush += kBlock / nph;
                if (rows_since_flush >= 128) {
#pragma unroll
                    for (int i = 0; i < GB; ++i)
#pragma unroll
                        for (int j = 0; j < GB; ++j) { two_sum_acc(shi[i][j], slo[i][j], acc[i][j]); acc[i][j] = 0.f; }
                    rows_since_flush = 0;
                }
            }
            __syncthreads();
        }
        if (MODE >= 2 && do_gram) {
            wave_sync();
            const uint32_t *fr = smem + d.lds_frag + wave * d.frag_wave_words + (lane >> 4) * kGroupWords + (lane & 15) * 4;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                bf16x8 fh[NT], fl[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const uint4 h = *reinterpret_cast<const uint4 *>(fr + (ks * 2 + 0) * d.frag_sp + t * kTileWords);
                    const uint4 l = *reinterpret_cast<const uint4 *>(fr + (ks * 2 + 1) * d.frag_sp + t * kTileWords);
                    fh[t] = __builtin_bit_cast(bf16x8, h);
                    fl[t] = __builtin_bit_cast(bf16x8, l);
                }
                int ih = 0;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int u = t; u < NT; ++u, ++ih) {
                        chh[ih] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[t], fh[u], chh[ih], 0, 0, 0);
                        if (MODE == 3) cll[ih] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fl[t], fl[u], cll[ih], 0, 0, 0);
                    }
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int u = 0; u < NT; ++u)
                        chl[t * NT + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fh[t], fl[u], chl[t * NT + u], 0, 0, 0);
            }
            rows_since_flush += 64;
            if (rows_since_flush >= 512) {
const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < NHH; ++i) { two_sum_acc4(shh[i], ehh[i], chh[i]); chh[i] = zero4; }
#pragma unroll
                for (int i = 0; i < NHL; ++i) { two_sum_acc4(shl[i], ehl[i], chl[i]); chl[i] = zero4; }
                if (MODE == 3) {
#pragma unroll
                    for (int i = 0; i < NHH; ++i) { two_sum_acc4(sll[i], ell[i], cll[i]); cll[i] = zero4; }
                }
                rows_since_flush = 0;
            }
        }
    }

    // ---- end of scan: workgroup reduction in fp64, partials out --------------------
    __syncthreads();
    double *red = reinterpret_cast<double *>(smem + d.lds_red);
    if (MODE == 1 && do_gram) {
        const int ngp = d.ngp;
        for (int i = tid; i < ngp * ngp; i += kBlock) red[i] = 0.0;
        __syncthreads();
        if (gact) {
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
        double *out = d.gram_partial + (int64_t)blockIdx.x * d.n_gram * d.n_gram;
        for (int e = tid; e < d.n_gram * d.n_gram; e += kBlock) {
            const int i = e / d.n_gram, j = e % d.n_gram;
            if (i <= j) out[e] = red[i * ngp + j];
        }
    }
    if (MODE >= 2 && do_gram) {
        const int n16 = NT * 16;
        double *rhh = red, *rhl = red + n16 * n16, *rll = red + 2 * n16 * n16;
        const int nred = (MODE == 3 ? 3 : 2) * n16 * n16;
        for (int i = tid; i < nred; i += kBlock) red[i] = 0.0;
        __syncthreads();
        const int ci = 4 * (lane >> 4), cj = lane & 15;
#pragma unroll
        for (int i = 0; i < NHH; ++i) {
            two_sum_acc4(shh[i], ehh[i], chh[i]);
            if (MODE == 3) two_sum_acc4(sll[i], ell[i], cll[i]);
        }
#pragma unroll
        for (int i = 0; i < NHL; ++i) two_sum_acc4(shl[i], ehl[i], chl[i]);
        int ih = 0;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int u = t; u < NT; ++u, ++ih)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    atomicAdd(&rhh[(16 * t + ci + e) * n16 + 16 * u + cj], (double)shh[ih][e] + (double)ehh[ih][e]);
                    if (MODE == 3) {
                        atomicAdd(&rll[(16 * t + ci + e) * n16 + 16 * u + cj], (double)sll[ih][e] + (double)ell[ih][e]);
                    }
                }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    atomicAdd(&rhl[(16 * t + ci + e) * n16 + 16 * u + cj],
                              (double)shl[t * NT + u][e] + (double)ehl[t * NT + u][e]);
                }
        __syncthreads();
        double *out = d.gram_partial + (int64_t)blockIdx.x * d.n_gram * d.n_gram;
        for (int e = tid; e < d.n_gram * d.n_gram; e += kBlock) {
            const int i = e / d.n_gram, j = e % d.n_gram;
            if (i <= j) {
                double v = rhh[i * n16 + j] + rhl[i * n16 + j] + rhl[j * n16 + i];
                if (MODE == 3) v += rll[i * n16 + j];
                out[e] = v;
            }
        }
    }
    if (do_count) {
        __shared__ unsigned long long wcount[kBlock / 64];
        const unsigned long long w = wave_sum_u64(my_count);
        if (lane == 0) wcount[wave] = w;
        __syncthreads();
        if (tid == 0) {
            unsigned long long t = 0;
            for (int i = 0; i < kBlock / 64; ++i) t += wcount[i];
            d.count_partial[blockIdx.x] = t;
        }
    }
    if (TABLES) {
        const int nf = d.n_flush[part];
        const FlushDesc *fl = d.flush + d.flush_base[part];
        for (int t = 0; t < nf; ++t) {
            const FlushDesc F = fl[t];
            const uint32_t *cnt = smem + d.lds_tables + F.lds_cnt;
            const double *val = reinterpret_cast<const double *>(smem + d.lds_tables + F.lds_val);
            for (int cell = tid; cell < F.n_cells; cell += kBlock) {
                const uint32_t c = cnt[cell];
                if (c == 0u) continue;
                atomicAdd(&d.g_cnt[F.glb_cnt + cell], (unsigned long long)c);
                for (int v = 0; v < F.n_vals; ++v) {
                    const double x = val[(int64_t)cell * F.n_vals + v];
                    if (x != 0.0) atomicAdd(&d.g_val[F.glb_val + (int64_t)cell * F.n_vals + v], x);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// cross-workgroup merge (fp64, fixed order: deterministic)
// ---------------------------------------------------------------------------

__global__ void merge_kernel(const MergeDesc *__restrict__ dp) {
    const MergeDesc &d = *dp;
    const int n = d.n_gram;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n * n) {
        const int i = e / n, j = e % n;
        if (i <= j) {
            double s = 0.0;
            for (int b = 0; b < d.grid; ++b) s += d.gram_partial[(int64_t)b * n * n + e];
            d.gram[i * n + j] = s;
            d.gram[j * n + i] = s;
        }
    }
    if (e == 0 && d.count_partial) {
        unsigned long long t = 0;
        for (int b = 0; b < d.grid; ++b) t += d.count_partial[b];
        *d.count = t;
    }
}

// ---------------------------------------------------------------------------
// result assembly: one workgroup per query, threads over cells
// ---------------------------------------------------------------------------

__global__ void assemble_kernel(const AssembleDesc *__restrict__ dp) {
    const AssembleDesc &d = *dp;
    for (int o = blockIdx.x; o < d.n_out; o += gridDim.x) {
        const OutDesc &O = d.outs[o];
        const TermDesc *terms = d.terms + O.term_base;
        const int nt = d.term_count[o];
        for (int64_t cell = threadIdx.x; cell < O.n_cells; cell += blockDim.x) {
            unsigned long long cnt;
            if (O.kind == SRC_GRAM) cnt = *d.count;
            else cnt = d.g_cnt[O.src_cnt + cell];
            d.res_cnt[O.dst_cnt + cell] = cnt;
            double *sum = d.res_sum + O.dst_sum + cell * O.n_aggs;
            for (int a = 0; a < O.n_aggs; ++a) sum[a] = 0.0;
            for (int t = 0; t < nt; ++t) {
                const TermDesc T = terms[t];
                double v;
                if (T.src < 0) v = (double)cnt;
                else if (O.kind == SRC_GRAM) v = d.gram[T.src];
                else v = d.g_val[O.src_val + cell * O.src_nvals + T.src];
                sum[T.agg] += T.coeff * v;
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

hipError_t launch_root(RootKernel k, const RootDesc *desc, int grid_x, int parts, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL(k, dim3(grid_x, parts), dim3(kBlock), lds_bytes, st, desc);
    return hipGetLastError();
}

hipError_t set_root_lds_limit(RootKernel k, size_t bytes) {
    return hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_merge(const MergeDesc *desc, int n_gram, hipStream_t st) {
    const int n = n_gram * n_gram > 0 ? n_gram * n_gram : 1;
    hipLaunchKernelGGL(merge_kernel, dim3((n + 255) / 256), dim3(256), 0, st, desc);
    return hipGetLastError();
}

hipError_t launch_assemble(const AssembleDesc *desc, int n_out, hipStream_t st) {
    if (n_out == 0) return hipSuccess;
    hipLaunchKernelGGL(assemble_kernel, dim3(n_out < 4096 ? n_out : 4096), dim3(256), 0, st, desc);
    return hipGetLastError();
}

}  // namespace lmfao
