// The covariance-only root scan of the aggregate-batch engine, written for
// gfx950 (CDNA4): when the root relation's view group is the covariance
// block (Section 2, equation (2)) and the total count alone, computed from
// bf16 pieces of every value (hi + lo, or hi + mid + lo) on matrix cores,
// this kernel scans the fact once, gathers the child view records, and
// accumulates the block on v_mfma_f32_16x16x32_bf16 (see the per-tile steps
// below).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "desc.h"
#include "device.h"

namespace lmfao {

// ---------------------------------------------------------------------------
// covariance-only root scan (bf16 pieces on matrix cores)
// ---------------------------------------------------------------------------

// Pair-row record buffers hold row r = 16b + 4g + i at position 16b + 4i + g (a transpose of
// each 4 x 4 block of rows; the map is its own inverse).  The four lane groups g of an MFMA
// operand read rows 4g + i together: at positions 4i + g they are 8 words apart instead of 32,
// on different LDS banks.
__device__ __forceinline__ int pair_row_of(int p) { return (p & ~15) | ((p & 3) << 2) | ((p >> 2) & 3); }

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
//   3. find the tile's valid rows and read every slot value of both k-steps
//      into registers, from the fact tile, the record buffer and the constant
//      block (values of rows outside the valid ones are zeroed, in a branch
//      that only tiles with such rows take);
//   4. gather tile t+1's child records into the record buffer with buffer
//      loads that bypass registers (a key outside [0, n_keys) reads past the
//      buffer range and lands as zeros: no join), then request the keys of
//      tile t+2 (after the last tile these requests repeat it, unused);
//   5. split every value into its bf16 pieces (x = hi + lo, or hi + mid + lo)
//      and accumulate their products (see PM) for every upper-triangle 16x16
//      tile pair on MFMA while those copies are in flight.
// Fact columns and keys are streamed once: their loads are non-temporal, so
// they do not push the gathered view records out of the caches.  Each wave
// writes its own fp64 partial of the upper triangle (no LDS reduction).
// PM: products per tile pair: 3 (hi*hi + hi*lo + lo*hi), 4 (adds lo*lo), or 6 (three pieces
// hi, mid, lo: hi*hi + hi*mid + mid*hi + mid*mid + hi*lo + lo*hi, every term down to 2^-16 of a
// product kept; the six-product form holds three operand registers per slot tile and runs two
// waves per SIMD)
template <int NT, int NF, int PM, bool PR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NT >= 4 || PM == 6 ? 2 : 3))) void gram_scan_kernel(
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
    // six products: on a diagonal tile pair (a, a) the cross terms hi*mid + mid*hi and hi*lo + lo*hi
    // are the transposes of each other, so hi*mid and hi*lo alone are accumulated here (one MFMA
    // each instead of two) and added to their transposes when the partial is written; they are
    // 2^-8 and 2^-16 of the block, so their fp32 chains need no second level
    constexpr int NX = PM == 6 ? NT : 1;
    f32x4 accx[NX];
#pragma unroll
    for (int a = 0; a < NX; ++a) accx[a] = f32x4{0.f, 0.f, 0.f, 0.f};
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
                        // lane l of request i reads quad l % 2 of the row kept at position
                        // 32 i + l / 2 (pair_row_of): a row's two quads are one contiguous 32-byte
                        // piece on neighbouring lanes, so the memory pipeline handles one address
                        // per row, not one per row and quad
#pragma unroll
                        for (int i = 0; i < 2; ++i) {
                            const uint32_t f = 64u * (uint32_t)i + (uint32_t)lane;
                            const uint32_t kr = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(4u * pair_row_of(f >> 1)), (int)key[c]);
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

    // the operands of both k-steps: bf16 pieces of every slot value (hi, lo, and mid in the
    // six-product form)
    constexpr int NMID = PM == 6 ? NT : 1;
    bf16x8 oph[2][NT], opl[2][NT], opm[2][NMID];
    const SplitSel sel = split_sel();
    // The 8 values of slot tile t2 this lane feeds in k-step ks: rows 32ks + 4g + {0..3} and
    // 32ks + 16 + 4g + {0..3} of its slot.  Whole fact tiles and record tiles read one source for
    // every lane; only the last fact tile of a fact whose features do not fill it (wave-uniform
    // `mixed`) chooses per lane.
    auto read_slot = [&](int ks, int t2, float *x) {
        const char *sm = reinterpret_cast<const char *>(smem);
        auto read_fact = [&]() {
            const char *base = sm + lds_off[t2] + 128 * ks + 16 * lg;
            const f32x4 lo4 = *reinterpret_cast<const f32x4 *>(base);
            const f32x4 hi4 = *reinterpret_cast<const f32x4 *>(base + 64);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                x[e] = lo4[e];
                x[4 + e] = hi4[e];
            }
        };
        auto read_rec = [&]() {
            if (PR) {
                // row 32ks + 4g + i sits at position 32ks + 4i + g (see pair_row_of)
                const float *p = reinterpret_cast<const float *>(sm + lds_off[t2]) + 8 * lg + 256 * ks;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    x[i] = p[32 * i];
                    x[4 + i] = p[128 + 32 * i];
                }
            } else {
                const float *p = reinterpret_cast<const float *>(sm + lds_off[t2] + 16 * kRowWords * lg + 128 * kRowWords * ks);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    x[i] = p[kRowWords * i];
                    x[4 + i] = p[16 * kRowWords + kRowWords * i];
                }
            }
        };
        if (t2 >= NF) read_rec();
        else if (!(t2 == NF - 1 && mixed)) read_fact();
        else if (is_fact[t2]) read_fact();
        else read_rec();
    };
    // Phase 1 reads every operand value of both k-steps out of LDS (then the tile's LDS buffers
    // are free for the next copies) and zeroes the values of rows outside the tile's valid rows,
    // in a branch that tiles whose 64 rows are all valid, nearly all of them, skip; the split
    // into bf16 pieces follows the copies, where the compiler interleaves it with the MFMAs.
    float xv[2][NT][8];
    auto phase1 = [&](int t) {
        const int r0 = tile_row(t);
        bool valid = r0 + lane < blk_end;
        uint32_t cnt[kGramMaxChild];
#pragma unroll
        for (int c = 0; c < kGramMaxChild; ++c)
            cnt[c] = c < n_child ? smem[cdst[c] / 4 + kRowWords * (PR ? pair_row_of(lane) : lane)] : 1u;
#pragma unroll
        for (int c = 0; c < kGramMaxChild; ++c)
            if (cnt[c] == 0u) valid = false;
        const uint64_t vm = __ballot(valid);
        count += (unsigned long long)__popcll(vm);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int t2 = 0; t2 < NT; ++t2) read_slot(ks, t2, xv[ks][t2]);
        if (vm != ~0ull) {
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const uint32_t vbits = (uint32_t)((vm >> (32 * ks + 4 * lg)) & 0xFull) |
                                       ((uint32_t)((vm >> (32 * ks + 16 + 4 * lg)) & 0xFull) << 4);
#pragma unroll
                for (int t2 = 0; t2 < NT; ++t2)
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (!((vbits >> i) & 1u)) xv[ks][t2][i] = 0.f;
            }
        }
    };
    auto split_all = [&]() {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int t2 = 0; t2 < NT; ++t2) {
                if (PM == 6) split3_bf16x8(sel, xv[ks][t2], oph[ks][t2], opm[ks][t2 < NMID ? t2 : 0], opl[ks][t2]);
                else split_bf16x8(sel, xv[ks][t2], oph[ks][t2], opl[ks][t2]);
            }
    };
    // Phase 2: the MFMAs of both k-steps, from registers only.
    auto mfma_pass = [&](const bf16x8 *A, const bf16x8 *B) {
        int p = 0;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int b = a; b < NT; ++b, ++p)
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a], B[b], acc[p], 0, 0, 0);
    };
    // off-diagonal tile pairs (a < b) only
    auto mfma_cross = [&](const bf16x8 *A, const bf16x8 *B) {
        int p = 0;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int b = a; b < NT; ++b, ++p)
                if (b > a) acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[a], B[b], acc[p], 0, 0, 0);
    };
    auto phase2 = [&]() {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            mfma_pass(oph[ks], oph[ks]);
            if (PM == 6) {
                mfma_cross(oph[ks], opm[ks]);
                mfma_cross(opm[ks], oph[ks]);
                mfma_pass(opm[ks], opm[ks]);
                mfma_cross(oph[ks], opl[ks]);
                mfma_cross(opl[ks], oph[ks]);
#pragma unroll
                for (int a = 0; a < NX; ++a) {
                    accx[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(oph[ks][a], opm[ks][a < NMID ? a : 0], accx[a], 0, 0, 0);
                    accx[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(oph[ks][a], opl[ks][a], accx[a], 0, 0, 0);
                }
            } else {
                mfma_pass(oph[ks], opl[ks]);
                mfma_pass(opl[ks], oph[ks]);
                if (PM == 4) mfma_pass(opl[ks], opl[ks]);
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
        if (live) {
            split_all();
            phase2();                                   // MFMAs while the copies are in flight
        }
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
    // The diagonal cross terms go through the wave's own LDS region (free after the last tile)
    // so that each lane can read the transposed entry: xt[a][e] = accx[a] at (column, row).
    float xt[NX][4];
    if (PM == 6) {
        float *tr = reinterpret_cast<float *>(reinterpret_cast<char *>(smem) + rbase);
        wave_sync();
#pragma unroll
        for (int a = 0; a < NX; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) tr[a * 256 + (4 * lg + e) * 16 + li] = accx[a][e];
        wave_sync();
#pragma unroll
        for (int a = 0; a < NX; ++a)
#pragma unroll
            for (int e = 0; e < 4; ++e) xt[a][e] = tr[a * 256 + li * 16 + 4 * lg + e];
    }
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
                    double v = (double)sacc[p][e] + (double)acc[p][e];
                    if (PM == 6 && a == b) v += (double)accx[a < NX ? a : 0][e] + (double)xt[a < NX ? a : 0][e];
                    gst(out)[tri_index(min(fa, fb), max(fa, fb), ng)] = v;
                }
            }
    }
    if (d.do_count && lane == 0) gst(d.count_partial)[pidx] = count;
}

typedef void (*GramKernel)(const GramDesc *);

template <int NT, int NF, int PM>
static GramKernel pick_pr(bool pr) {
    return pr ? (GramKernel)gram_scan_kernel<NT, NF, PM, true> : (GramKernel)gram_scan_kernel<NT, NF, PM, false>;
}

template <int NT, int NF>
static GramKernel pick_gram(int pm, bool pr) {
    if (pm == 6) return pick_pr<NT, NF, 6>(pr);
    return pm == 4 ? pick_pr<NT, NF, 4>(pr) : pick_pr<NT, NF, 3>(pr);
}

// nt: 16-wide slot tiles (1..4); nf: tiles holding fact slots (0..min(nt, 2)); pm: products per tile
// pair (3, 4 or 6); pr: pair-row record buffers (every child record at most two quads, a row's quads
// contiguous) instead of quad-major ones
GramKernel gram_kernel(int nt, int nf, int pm, bool pr) {
    if (nf < 0 || nf > 2 || nf > nt || (pm != 3 && pm != 4 && pm != 6)) return nullptr;
    switch (nt * 4 + nf) {
        case 4: return pick_gram<1, 0>(pm, pr);
        case 5: return pick_gram<1, 1>(pm, pr);
        case 8: return pick_gram<2, 0>(pm, pr);
        case 9: return pick_gram<2, 1>(pm, pr);
        case 10: return pick_gram<2, 2>(pm, pr);
        case 12: return pick_gram<3, 0>(pm, pr);
        case 13: return pick_gram<3, 1>(pm, pr);
        case 14: return pick_gram<3, 2>(pm, pr);
        case 16: return pick_gram<4, 0>(pm, pr);
        case 17: return pick_gram<4, 1>(pm, pr);
        case 18: return pick_gram<4, 2>(pm, pr);
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

}  // namespace lmfao
