// Cost-model network of the learned planner: a fully connected network
//   x(16) -> H (ReLU) -> H (ReLU) -> 1
// predicting log(milliseconds) of a view-group scan from plan features.
// Forward, backward and Adam are hand-written kernels; gradients are sums
// over samples computed per parameter in a fixed order (deterministic).
//
// Parameter layout (fp32): W1[H][16], b1[H], W2[H][H], b2[H], W3[H], b3.
#include <hip/hip_runtime.h>

#include "lmfao.h"

namespace lmfao {

constexpr int kIn = LMFAO_N_FEATURES;

struct MlpView {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};

__host__ __device__ inline int mlp_params(int H) { return H * kIn + H + H * H + H + H + 1; }

__device__ inline MlpView mlp_view(const float *p, int H) {
    MlpView v;
    v.W1 = p;
    v.b1 = v.W1 + H * kIn;
    v.W2 = v.b1 + H;
    v.b2 = v.W2 + H * H;
    v.W3 = v.b2 + H;
    v.b3 = v.W3 + H;
    return v;
}

template <int H>
__device__ inline float mlp_eval(const MlpView &w, const float *x, float *z1, float *a1, float *z2, float *a2) {
    for (int j = 0; j < H; ++j) {
        float s = w.b1[j];
        for (int k = 0; k < kIn; ++k) s = fmaf(w.W1[j * kIn + k], x[k], s);
        z1[j] = s;
        a1[j] = s > 0.f ? s : 0.f;
    }
    for (int j = 0; j < H; ++j) {
        float s = w.b2[j];
        for (int k = 0; k < H; ++k) s = fmaf(w.W2[j * H + k], a1[k], s);
        z2[j] = s;
        a2[j] = s > 0.f ? s : 0.f;
    }
    float y = w.b3[0];
    for (int k = 0; k < H; ++k) y = fmaf(w.W3[k], a2[k], y);
    return y;
}

template <int H>
__global__ void mlp_forward_kernel(const float *__restrict__ params, const float *__restrict__ x, int n,
                                   float *__restrict__ y) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const MlpView w = mlp_view(params, H);
    float xs[kIn], z1[H], a1[H], z2[H], a2[H];
    for (int k = 0; k < kIn; ++k) xs[k] = x[(int64_t)s * kIn + k];
    y[s] = mlp_eval<H>(w, xs, z1, a1, z2, a2);
}

// per sample: forward, squared error, and the back-propagated deltas
// scratch layout: a1[n][H], a2[n][H], d1[n][H], d2[n][H], d3[n], e2[n]
template <int H>
__global__ void mlp_backprop_kernel(const float *__restrict__ params, const float *__restrict__ x,
                                    const float *__restrict__ target, int n, float *__restrict__ scratch) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const MlpView w = mlp_view(params, H);
    float xs[kIn], z1[H], a1[H], z2[H], a2[H], d2[H];
    for (int k = 0; k < kIn; ++k) xs[k] = x[(int64_t)s * kIn + k];
    const float y = mlp_eval<H>(w, xs, z1, a1, z2, a2);
    const float e = y - target[s];
    const float d3 = 2.f * e / (float)n;          // d(mean e^2)/dy
    float *A1 = scratch, *A2 = A1 + (int64_t)n * H, *D1 = A2 + (int64_t)n * H, *D2 = D1 + (int64_t)n * H;
    float *D3 = D2 + (int64_t)n * H, *E2 = D3 + n;
    for (int j = 0; j < H; ++j) {
        d2[j] = z2[j] > 0.f ? w.W3[j] * d3 : 0.f;
        A1[(int64_t)s * H + j] = a1[j];
        A2[(int64_t)s * H + j] = a2[j];
        D2[(int64_t)s * H + j] = d2[j];
    }
    for (int k = 0; k < H; ++k) {
        float t = 0.f;
        for (int j = 0; j < H; ++j) t = fmaf(w.W2[j * H + k], d2[j], t);
        D1[(int64_t)s * H + k] = z1[k] > 0.f ? t : 0.f;
    }
    D3[s] = d3;
    E2[s] = e * e;
}

// one thread per parameter (plus one for the loss): sum over samples in order
template <int H>
__global__ void mlp_grad_kernel(const float *__restrict__ x, int n, const float *__restrict__ scratch,
                                float *__restrict__ grad, float *__restrict__ loss) {
    const int P = mlp_params(H);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    const float *A1 = scratch, *A2 = A1 + (int64_t)n * H, *D1 = A2 + (int64_t)n * H, *D2 = D1 + (int64_t)n * H;
    const float *D3 = D2 + (int64_t)n * H, *E2 = D3 + n;
    float g = 0.f;
    if (p == P) {
        for (int s = 0; s < n; ++s) g += E2[s];
        *loss = g / (float)n;
        return;
    }
    int q = p;
    if (q < H * kIn) {                       // W1[j][k]
        const int j = q / kIn, k = q % kIn;
        for (int s = 0; s < n; ++s) g = fmaf(D1[(int64_t)s * H + j], x[(int64_t)s * kIn + k], g);
    } else if ((q -= H * kIn) < H) {         // b1[j]
        for (int s = 0; s < n; ++s) g += D1[(int64_t)s * H + q];
    } else if ((q -= H) < H * H) {           // W2[j][k]
        const int j = q / H, k = q % H;
        for (int s = 0; s < n; ++s) g = fmaf(D2[(int64_t)s * H + j], A1[(int64_t)s * H + k], g);
    } else if ((q -= H * H) < H) {           // b2[j]
        for (int s = 0; s < n; ++s) g += D2[(int64_t)s * H + q];
    } else if ((q -= H) < H) {               // W3[k]
        for (int s = 0; s < n; ++s) g = fmaf(D3[s], A2[(int64_t)s * H + q], g);
    } else {                                 // b3
        for (int s = 0; s < n; ++s) g += D3[s];
    }
    grad[p] = g;
}

// Adam (Kingma & Ba, 2015) with bias-corrected moments
__global__ void adam_kernel(int n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static bool hidden_ok(int H) { return H == 8 || H == 16 || H == 32 || H == 64; }

hipError_t mlp_forward_dev(int hidden, const float *params, const float *x, int n, float *y, hipStream_t st) {
    const dim3 b(128), g((n + 127) / 128);
    if (n <= 0) return hipSuccess;
    switch (hidden) {
        case 8: hipLaunchKernelGGL(mlp_forward_kernel<8>, g, b, 0, st, params, x, n, y); break;
        case 16: hipLaunchKernelGGL(mlp_forward_kernel<16>, g, b, 0, st, params, x, n, y); break;
        case 32: hipLaunchKernelGGL(mlp_forward_kernel<32>, g, b, 0, st, params, x, n, y); break;
        case 64: hipLaunchKernelGGL(mlp_forward_kernel<64>, g, b, 0, st, params, x, n, y); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int H>
static hipError_t loss_grad_t(const float *params, const float *x, const float *t, int n, float *loss, float *grad,
                              float *scratch, hipStream_t st) {
    hipLaunchKernelGGL(mlp_backprop_kernel<H>, dim3((n + 127) / 128), dim3(128), 0, st, params, x, t, n, scratch);
    const int P = mlp_params(H) + 1;
    hipLaunchKernelGGL(mlp_grad_kernel<H>, dim3((P + 127) / 128), dim3(128), 0, st, x, n, scratch, grad, loss);
    return hipGetLastError();
}

hipError_t mlp_loss_grad_dev(int hidden, const float *params, const float *x, const float *t, int n, float *loss,
                             float *grad, float *scratch, hipStream_t st) {
    switch (hidden) {
        case 8: return loss_grad_t<8>(params, x, t, n, loss, grad, scratch, st);
        case 16: return loss_grad_t<16>(params, x, t, n, loss, grad, scratch, st);
        case 32: return loss_grad_t<32>(params, x, t, n, loss, grad, scratch, st);
        case 64: return loss_grad_t<64>(params, x, t, n, loss, grad, scratch, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace lmfao

using namespace lmfao;

extern "C" int32_t lmfao_mlp_param_count(int32_t hidden) { return hidden > 0 ? mlp_params(hidden) : 0; }

extern "C" int64_t lmfao_mlp_scratch_floats(int32_t hidden, int32_t n) {
    return (int64_t)n * (4 * (int64_t)hidden + 2);
}

extern "C" lmfao_status lmfao_mlp_forward(int32_t hidden, const float *params, const float *x, int32_t n, float *y,
                                          void *hip_stream) {
    if (!hidden_ok(hidden) || !params || !x || !y || n < 0) return LMFAO_ERR_INVALID_ARG;
    return mlp_forward_dev(hidden, params, x, n, y, (hipStream_t)hip_stream) == hipSuccess ? LMFAO_OK : LMFAO_ERR_HIP;
}

extern "C" lmfao_status lmfao_mlp_loss_grad(int32_t hidden, const float *params, const float *x, const float *target,
                                            int32_t n, float *loss, float *grad, float *scratch, void *hip_stream) {
    if (!hidden_ok(hidden) || !params || !x || !target || !loss || !grad || !scratch || n <= 0)
        return LMFAO_ERR_INVALID_ARG;
    return mlp_loss_grad_dev(hidden, params, x, target, n, loss, grad, scratch, (hipStream_t)hip_stream) == hipSuccess
               ? LMFAO_OK
               : LMFAO_ERR_HIP;
}

extern "C" lmfao_status lmfao_adam_step(int32_t n_params, float *params, const float *grad, float *m, float *v,
                                        int32_t step, float lr, float beta1, float beta2, float eps, void *hip_stream) {
    if (n_params <= 0 || !params || !grad || !m || !v || step <= 0) return LMFAO_ERR_INVALID_ARG;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n_params + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, n_params, params,
                       grad, m, v, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? LMFAO_OK : LMFAO_ERR_HIP;
}

extern "C" lmfao_status lmfao_mlp_train(int32_t hidden, float *params, float *m, float *v, const float *x,
                                        const float *target, int32_t n, int32_t epochs, float lr, float *grad,
                                        float *scratch, float *losses, void *hip_stream) {
    if (!hidden_ok(hidden) || epochs <= 0 || !losses) return LMFAO_ERR_INVALID_ARG;
    const int P = mlp_params(hidden);
    for (int e = 0; e < epochs; ++e) {
        lmfao_status s = lmfao_mlp_loss_grad(hidden, params, x, target, n, losses + e, grad, scratch, hip_stream);
        if (s != LMFAO_OK) return s;
        s = lmfao_adam_step(P, params, grad, m, v, e + 1, lr, 0.9f, 0.999f, 1e-8f, hip_stream);
        if (s != LMFAO_OK) return s;
    }
    return LMFAO_OK;
}
