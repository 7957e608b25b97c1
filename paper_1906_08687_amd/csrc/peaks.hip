// Throughput probes of the units the scans are bound by, for the roofline of
// each kernel: a streaming HBM read, LDS atomic adds (u32 at random and at
// conflict-free addresses, fp64 at random addresses) and device-scope u64
// atomic adds on a table resident in the caches.  Each probe is one timed
// launch that touches only the caller's buffer and its own LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "lmfao.h"

namespace lmfao {

constexpr int kPeakThreads = 1024;
constexpr uint32_t kLdsWords = 32768;     // 128 KiB table in LDS

__device__ __forceinline__ uint32_t lcg(uint32_t x) { return x * 1664525u + 1013904223u; }
static size_t align_up_16(size_t x) { return (x + 15) / 16 * 16; }

// every thread reads 16-byte chunks, grid-stride; the XOR of what it read goes to out[block]
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kPeakThreads) void peak_read_kernel(const u32x4 *__restrict__ p, int64_t n16, uint32_t *out) {
    uint32_t acc = 0u;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x) {
        const u32x4 v = __builtin_nontemporal_load(p + i);
        acc ^= v[0] ^ v[1] ^ v[2] ^ v[3];
    }
    __shared__ uint32_t red[kPeakThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t r = 0u;
        for (int i = 0; i < kPeakThreads; ++i) r ^= red[i];
        out[blockIdx.x] = r;
    }
}

// iters LDS atomic adds per thread; RANDOM: addresses from a per-thread LCG over the table,
// else lane-distinct banks (lane + 64 * (i & 31)); F64: ds_add_f64 on 8-byte cells
template <bool RANDOM, bool F64>
__global__ __launch_bounds__(kPeakThreads) void peak_lds_kernel(int iters, uint32_t *out) {
    extern __shared__ __align__(16) uint32_t smem[];
    constexpr uint32_t cells = F64 ? kLdsWords / 2 : kLdsWords;
    for (uint32_t i = threadIdx.x; i < kLdsWords; i += blockDim.x) smem[i] = 0u;
    __syncthreads();
    uint32_t x = lcg(blockIdx.x * 7919u + threadIdx.x * 104729u + 1u);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (int i = 0; i < iters; ++i) {
        uint32_t a;
        if (RANDOM) {
            x = lcg(x);
            a = (x >> 7) & (cells - 1u);
        } else {
            a = (lane + 64u * ((uint32_t)i & 31u) + 2048u * wave) & (cells - 1u);
        }
        if (F64) atomicAdd(reinterpret_cast<double *>(smem) + a, 1.0);
        else atomicAdd(&smem[a], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t r = 0u;
        for (uint32_t i = 0; i < kLdsWords; i += 97u) r += smem[i];
        out[blockIdx.x] = r;
    }
}

// iters device-scope u64 atomic adds per thread at LCG addresses over `cells` counters
__global__ __launch_bounds__(kPeakThreads) void peak_global_kernel(unsigned long long *tab, uint32_t cells, int iters) {
    uint32_t x = lcg(blockIdx.x * 7919u + threadIdx.x * 104729u + 3u);
    for (int i = 0; i < iters; ++i) {
        x = lcg(x);
        gadd(tab + (x >> 4) % cells, 1ull);
    }
}

}  // namespace lmfao

using namespace lmfao;

extern "C" lmfao_status lmfao_measure_peak(int32_t kind, void *buf, size_t buf_bytes, int32_t iters, void *hip_stream,
                                           double *ms, double *units) {
    if (!ms || !units || iters < 1 || kind < LMFAO_PEAK_READ || kind > LMFAO_PEAK_GLOBAL_U64) return LMFAO_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int n_cu = 256, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LMFAO_ERR_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n_cu = prop.multiProcessorCount;
    const int grid = 4 * n_cu;
    // the caller's buffer: the data read (READ), the counters (GLOBAL_U64), or room for one result
    // word per workgroup (LDS probes)
    if (!buf || buf_bytes < (size_t)grid * 4 || (kind == LMFAO_PEAK_READ && buf_bytes < (size_t)grid * 4 + 16))
        return LMFAO_ERR_WORKSPACE;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LMFAO_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return LMFAO_ERR_HIP; }
    uint32_t *out = static_cast<uint32_t *>(buf);
    const int lds_bytes = (int)(kLdsWords * 4);
    if (hipFuncSetAttribute((const void *)peak_lds_kernel<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes) != hipSuccess ||
        hipFuncSetAttribute((const void *)peak_lds_kernel<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes) != hipSuccess ||
        hipFuncSetAttribute((const void *)peak_lds_kernel<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return LMFAO_ERR_HIP;
    }
    (void)hipEventRecord(e0, st);
    for (int rep = 0; rep < (kind == LMFAO_PEAK_READ ? iters : 1); ++rep) {
        switch (kind) {
            case LMFAO_PEAK_READ: {
                // the first grid words receive the per-block results; the rest is read
                const size_t skip = align_up_16((size_t)grid * 4);
                const int64_t n16 = (int64_t)((buf_bytes - skip) / 16);
                hipLaunchKernelGGL(peak_read_kernel, dim3(grid), dim3(kPeakThreads), 0, st,
                                   reinterpret_cast<const u32x4 *>(static_cast<char *>(buf) + skip), n16, out);
                *units = (double)n16 * 16.0 * iters;
                break;
            }
            case LMFAO_PEAK_LDS_U32:
                hipLaunchKernelGGL((peak_lds_kernel<true, false>), dim3(grid), dim3(kPeakThreads), kLdsWords * 4, st, iters, out);
                *units = (double)grid * kPeakThreads * iters;
                break;
            case LMFAO_PEAK_LDS_U32_SPREAD:
                hipLaunchKernelGGL((peak_lds_kernel<false, false>), dim3(grid), dim3(kPeakThreads), kLdsWords * 4, st, iters, out);
                *units = (double)grid * kPeakThreads * iters;
                break;
            case LMFAO_PEAK_LDS_F64:
                hipLaunchKernelGGL((peak_lds_kernel<true, true>), dim3(grid), dim3(kPeakThreads), kLdsWords * 4, st, iters, out);
                *units = (double)grid * kPeakThreads * iters;
                break;
            default: {
                const uint32_t cells = (uint32_t)std::min<size_t>(buf_bytes / 8, 0xFFFFFFFFu);
                hipLaunchKernelGGL(peak_global_kernel, dim3(grid), dim3(kPeakThreads), 0, st,
                                   static_cast<unsigned long long *>(buf), cells, iters);
                *units = (double)grid * kPeakThreads * iters;
                break;
            }
        }
    }
    (void)hipEventRecord(e1, st);
    hipError_t e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return LMFAO_ERR_HIP;
    *ms = (double)t;
    return LMFAO_OK;
}
