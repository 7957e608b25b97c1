// Device-side helpers shared by the engine's HIP sources (gfx950): vector
// types, address-space views, wave helpers, asynchronous LDS copies and the
// bf16 hi/lo split.
#pragma once
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
// helpers of the scans
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

// sum over the 64 lanes of a wave (every lane active); the same value on every lane
__device__ __forceinline__ double wave_sum_f64(double v) {
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

// Residuals of the split: x - hi for a packed pair hi = (bf16(x0), bf16(x1)) as one
// v_dot2c_f32_bf16 per value, hi . (-1, 0) + x0 and hi . (0, -1) + x1, instead of unpacking hi
// to fp32 and subtracting (two instructions per value).  x - hi is exact in fp32, and the dot
// product returns it bit for bit: checked on the device for every finite fp32 x below bf16's
// overflow threshold (about 3.39e38, where hi becomes infinite in either form).  The two
// selector constants live in registers, made opaque to the compiler, which would otherwise fold
// them into an inline constant that the instruction reads as (0, -1) for both.
struct SplitSel {
    bf16x2 lo, hi;   // (-1, 0) and (0, -1)
};
__device__ __forceinline__ SplitSel split_sel() {
    uint32_t a = 0x0000BF80u, b = 0xBF800000u;
    asm("" : "+v"(a), "+v"(b));
    return SplitSel{__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b)};
}
__device__ __forceinline__ f32x2 residual(const SplitSel &k, bf16x2 h, f32x2 v) {
    return f32x2{__builtin_amdgcn_fdot2_f32_bf16(h, k.lo, v.x, false), __builtin_amdgcn_fdot2_f32_bf16(h, k.hi, v.y, false)};
}

// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), both round-to-nearest-even
__device__ __forceinline__ void split_bf16x8(const SplitSel &k, const float *x, bf16x8 &hi, bf16x8 &lo) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const f32x2 v = {x[2 * i], x[2 * i + 1]};
        const bf16x2 hb = __builtin_convertvector(v, bf16x2);
        const bf16x2 lb = __builtin_convertvector(residual(k, hb, v), bf16x2);
        h[i] = __builtin_bit_cast(uint32_t, hb);
        l[i] = __builtin_bit_cast(uint32_t, lb);
    }
    hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
    lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

// x = hi + mid + lo with hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid), each round to
// nearest even; x - hi and x - hi - mid are exact in fp32, and hi + mid + lo carries x to within
// 2^-24 |x| (8 significant bits per piece)
__device__ __forceinline__ void split3_bf16x8(const SplitSel &k, const float *x, bf16x8 &hi, bf16x8 &mid, bf16x8 &lo) {
    uint32_t h[4], m[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const f32x2 v = {x[2 * i], x[2 * i + 1]};
        const bf16x2 hb = __builtin_convertvector(v, bf16x2);
        const f32x2 r1 = residual(k, hb, v);
        const bf16x2 mb = __builtin_convertvector(r1, bf16x2);
        const bf16x2 lb = __builtin_convertvector(residual(k, mb, r1), bf16x2);
        h[i] = __builtin_bit_cast(uint32_t, hb);
        m[i] = __builtin_bit_cast(uint32_t, mb);
        l[i] = __builtin_bit_cast(uint32_t, lb);
    }
    hi = __builtin_bit_cast(bf16x8, make_uint4(h[0], h[1], h[2], h[3]));
    mid = __builtin_bit_cast(bf16x8, make_uint4(m[0], m[1], m[2], m[3]));
    lo = __builtin_bit_cast(bf16x8, make_uint4(l[0], l[1], l[2], l[3]));
}

constexpr int kFlushTiles = 16;   // mfma accumulators fold into fp32 sums every 16 tiles (1024 rows per wave)

}  // namespace lmfao
