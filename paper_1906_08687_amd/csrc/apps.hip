// Application loops on a batch's results, run on the device without host
// round trips (Section 2, the three application families of the batches):
//
//  * ridge linear regression by batch gradient descent over the non-centred
//    covariance matrix (Section 2, linear regression: the gradient is a
//    product of the covariance matrix with the parameter vector), with
//    Barzilai-Borwein step sizes, until the gradient norm falls below a
//    tolerance relative to its first value;
//  * mutual information of two categorical attributes from their pairwise
//    counts (Section 2, equation (7) and the 4-ary aggregate f = delta/alpha *
//    log(alpha * delta / (beta * gamma))), and the Chow-Liu tree: edges taken
//    by decreasing mutual information, each joining two components;
//  * the best split of every node of a decision-tree level from its
//    histograms (Section 2, decision trees): variance of the label on both
//    sides for regression trees (from COUNT, SUM(y), SUM(y^2)), count-weighted
//    Gini index for classification trees (from COUNT GROUP BY label).
// Each reduction runs in a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.h"
#include "lmfao.h"

namespace lmfao {

constexpr int kAppThreads = 256;
constexpr int kRidgeMax = 64;        // features of the covariance matrix (with the constant and the label)

// block-wide sum in a fixed order: per-thread values to LDS, then a binary tree
__device__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// ---- ridge regression ---------------------------------------------------------------------
// C: n x n covariance over the staged vector (index 0 the constant 1, C[0][0] = |D|), label
// index `label`.  Parameters theta over every index but the label, whose coefficient is fixed at
// -1; J = 1/(2|D|) sum (theta . X)^2 + lambda/2 |theta_free|^2, gradient_k = (C theta)_k / |D| +
// lambda theta_k for free k.
__global__ __launch_bounds__(kAppThreads) void ridge_bgd_kernel(const double *__restrict__ cov, int n, int label,
                                                                double lambda, int max_iters, double tol,
                                                                double *theta_out, double *info) {
    __shared__ double C[kRidgeMax * kRidgeMax];
    __shared__ double th[kRidgeMax], g[kRidgeMax], th0[kRidgeMax], g0[kRidgeMax];
    __shared__ double red[kAppThreads];
    const int t = threadIdx.x;
    for (int i = t; i < n * n; i += blockDim.x) C[i] = cov[i];
    __syncthreads();
    const double inv_n = 1.0 / C[0];
    if (t < n) th[t] = t == label ? -1.0 : 0.0;
    __syncthreads();
    auto gradient = [&]() {       // g = C theta / |D| + lambda theta (free indices), 0 at the label
        if (t < n) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += C[t * n + j] * th[j];
            g[t] = t == label ? 0.0 : s * inv_n + lambda * th[t];
        }
        __syncthreads();
    };
    gradient();
    const double gn0 = sqrt(block_sum(t < n ? g[t] * g[t] : 0.0, red));
    // first step 1/L with L an upper bound of the Hessian's largest eigenvalue (trace / |D| + lambda)
    double tr = block_sum(t < n && t != label ? C[t * n + t] : 0.0, red);
    double step = 1.0 / (tr * inv_n + lambda);
    int it = 0;
    double gn = gn0;
    while (it < max_iters && gn > tol * gn0 && gn > 0.0) {
        if (t < n) {
            th0[t] = th[t];
            g0[t] = g[t];
            if (t != label) th[t] -= step * g[t];
        }
        __syncthreads();
        gradient();
        // Barzilai-Borwein: step = (dtheta . dtheta) / (dtheta . dg)
        const double dth = t < n ? th[t] - th0[t] : 0.0, dg = t < n ? g[t] - g0[t] : 0.0;
        const double ss = block_sum(dth * dth, red), sy = block_sum(dth * dg, red);
        if (sy > 0.0) step = ss / sy;
        gn = sqrt(block_sum(t < n ? g[t] * g[t] : 0.0, red));
        ++it;
    }
    // objective: 1/(2|D|) theta^T C theta + lambda/2 |theta_free|^2
    double q = 0.0;
    if (t < n) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += C[t * n + j] * th[j];
        q = th[t] * s * inv_n + (t == label ? 0.0 : lambda * th[t] * th[t]);
    }
    const double obj = 0.5 * block_sum(q, red);
    if (t < n) theta_out[t] = th[t];
    if (t == 0) {
        info[0] = obj;
        info[1] = (double)it;
        info[2] = gn;
    }
}

// ---- mutual information ---------------------------------------------------------------------
constexpr int kMiMaxDom = 2048;

// one workgroup per pair table: marginals from its row and column sums, then the sum of
// delta/alpha * log(alpha * delta / (beta * gamma)) over its nonzero cells
__global__ __launch_bounds__(kAppThreads) void mutual_information_kernel(const unsigned long long *const *__restrict__ tabs,
                                                                         const int32_t *__restrict__ doms, double *mi) {
    __shared__ double beta[kMiMaxDom], gamma_[kMiMaxDom];
    __shared__ double red[kAppThreads];
    const int p = blockIdx.x, t = threadIdx.x;
    const unsigned long long *d = tabs[p];
    const int da = doms[2 * p], db = doms[2 * p + 1];
    for (int a = t; a < da; a += blockDim.x) {
        unsigned long long s = 0;
        for (int b = 0; b < db; ++b) s += d[(int64_t)a * db + b];
        beta[a] = (double)s;
    }
    for (int b = t; b < db; b += blockDim.x) {
        unsigned long long s = 0;
        for (int a = 0; a < da; ++a) s += d[(int64_t)a * db + b];
        gamma_[b] = (double)s;
    }
    __syncthreads();
    double part = 0.0;
    for (int a = t; a < da; a += blockDim.x) part += beta[a];
    const double alpha = block_sum(part, red);
    double acc = 0.0;
    const int64_t cells = (int64_t)da * db;
    for (int64_t c = t; c < cells; c += blockDim.x) {
        const unsigned long long x = d[c];
        if (x == 0) continue;
        const double delta = (double)x;
        acc += delta / alpha * log(alpha * delta / (beta[c / db] * gamma_[c % db]));
    }
    const double r = block_sum(acc, red);
    if (t == 0) mi[p] = alpha > 0.0 ? r : 0.0;
}

// ---- Chow-Liu tree ------------------------------------------------------------------------------
constexpr int kClMax = 64;

// one workgroup: the pairs ranked by decreasing mutual information (ties: lower pair index first)
// by counting, then one lane joins components in that order (union-find)
__global__ __launch_bounds__(kAppThreads) void chow_liu_kernel(const double *__restrict__ mi, int n, int32_t *edges,
                                                               double *total) {
    __shared__ int order[kClMax * (kClMax - 1) / 2];
    __shared__ int comp[kClMax];
    const int t = threadIdx.x;
    const int np = n * (n - 1) / 2;
    auto pair_of = [&](int k, int &i, int &j) {
        i = 0;
        while (k >= n - 1 - i) { k -= n - 1 - i; ++i; }
        j = i + 1 + k;
    };
    for (int k = t; k < np; k += blockDim.x) {
        int i, j;
        pair_of(k, i, j);
        const double w = mi[i * n + j];
        int rank = 0;
        for (int k2 = 0; k2 < np; ++k2) {
            int i2, j2;
            pair_of(k2, i2, j2);
            const double w2 = mi[i2 * n + j2];
            if (w2 > w || (w2 == w && k2 < k)) ++rank;
        }
        order[rank] = k;
    }
    for (int i = t; i < n; i += blockDim.x) comp[i] = i;
    __syncthreads();
    if (t == 0) {
        int taken = 0;
        double sum = 0.0;
        for (int r = 0; r < np && taken < n - 1; ++r) {
            int i, j;
            pair_of(order[r], i, j);
            int a = i, b = j;
            while (comp[a] != a) a = comp[a];
            while (comp[b] != b) b = comp[b];
            if (a == b) continue;
            comp[a < b ? b : a] = a < b ? a : b;
            edges[2 * taken] = i;
            edges[2 * taken + 1] = j;
            sum += mi[i * n + j];
            ++taken;
        }
        for (int k = taken; k < n - 1; ++k) edges[2 * k] = edges[2 * k + 1] = -1;
        total[0] = sum;
    }
}

// ---- decision-tree splits ---------------------------------------------------------------------
constexpr int kMaxLabels = 16;

__device__ __forceinline__ double variance_cost(double n, double s1, double s2) { return n > 0.0 ? s2 - s1 * s1 / n : 0.0; }

// one workgroup (one wave) per node; lane i takes inputs i, i + 64, ... of that node and every
// split of each; the lowest (cost, input, cell) wins
__global__ __launch_bounds__(64) void best_split_kernel(const lmfao_split_input *__restrict__ in, int n_in, int criterion,
                                                        int n_labels, lmfao_split_result *out) {
    __shared__ double lab[64][2][kMaxLabels];   // per lane: left and total label counts (classification)
    const int node = blockIdx.x, lane = threadIdx.x;
    double best = INFINITY;
    int best_in = -1, best_cell = -1;
    for (int k = lane; k < n_in; k += 64) {
        const lmfao_split_input &I = in[k];
        if (I.node != node) continue;
        const int nc = I.n_cells;
        if (criterion == LMFAO_SPLIT_VARIANCE) {
            double N = 0.0, S1 = 0.0, S2 = 0.0;
            for (int c = 0; c < nc; ++c) {
                N += (double)I.counts[c];
                S1 += I.sums[(int64_t)c * I.sum_stride];
                S2 += I.sums[(int64_t)c * I.sum_stride + 1];
            }
            double n = 0.0, s1 = 0.0, s2 = 0.0;
            for (int c = 0; c < (I.categorical ? nc : nc - 1); ++c) {
                const double cn = (double)I.counts[c], c1 = I.sums[(int64_t)c * I.sum_stride],
                             c2 = I.sums[(int64_t)c * I.sum_stride + 1];
                double ln, l1, l2;
                if (I.categorical) { ln = cn; l1 = c1; l2 = c2; }
                else { n += cn; s1 += c1; s2 += c2; ln = n; l1 = s1; l2 = s2; }
                if (ln <= 0.0 || N - ln <= 0.0) continue;
                const double cost = variance_cost(ln, l1, l2) + variance_cost(N - ln, S1 - l1, S2 - l2);
                if (cost < best) { best = cost; best_in = k; best_cell = c; }
            }
        } else {
            // counts[label][cell]; left = buckets <= c (continuous) or cell c (categorical)
            for (int l = 0; l < n_labels; ++l) {
                unsigned long long s = 0;
                for (int c = 0; c < nc; ++c) s += I.counts[(int64_t)l * nc + c];
                lab[lane][1][l] = (double)s;
                lab[lane][0][l] = 0.0;
            }
            double N = 0.0;
            for (int l = 0; l < n_labels; ++l) N += lab[lane][1][l];
            for (int c = 0; c < (I.categorical ? nc : nc - 1); ++c) {
                double ln = 0.0;
                for (int l = 0; l < n_labels; ++l) {
                    const double x = (double)I.counts[(int64_t)l * nc + c];
                    lab[lane][0][l] = I.categorical ? x : lab[lane][0][l] + x;
                    ln += lab[lane][0][l];
                }
                const double rn = N - ln;
                if (ln <= 0.0 || rn <= 0.0) continue;
                double ql = 0.0, qr = 0.0;
                for (int l = 0; l < n_labels; ++l) {
                    const double a = lab[lane][0][l], b = lab[lane][1][l] - a;
                    ql += a * a;
                    qr += b * b;
                }
                // n_L * gini_L + n_R * gini_R = n_L - sum a^2 / n_L + n_R - sum b^2 / n_R
                const double cost = (ln - ql / ln) + (rn - qr / rn);
                if (cost < best) { best = cost; best_in = k; best_cell = c; }
            }
        }
    }
    // lowest (cost, input, cell) over the wave, in a fixed order
    for (int o = 32; o > 0; o >>= 1) {
        const double oc = __shfl_xor(best, o);
        const int oi = __shfl_xor(best_in, o), ol = __shfl_xor(best_cell, o);
        const bool take = oi >= 0 && (best_in < 0 || oc < best || (oc == best && (oi < best_in || (oi == best_in && ol < best_cell))));
        if (take) { best = oc; best_in = oi; best_cell = ol; }
    }
    if (lane == 0) {
        out[node].cost = best_in >= 0 ? best : 0.0;
        out[node].input = best_in;
        out[node].cell = best_cell;
        out[node].pad = 0;
    }
}

}  // namespace lmfao

using namespace lmfao;

extern "C" lmfao_status lmfao_ridge_bgd(const double *cov, int32_t n, int32_t label, double lambda, int32_t max_iters,
                                        double tol, double *theta, double *info, void *hip_stream) {
    if (!cov || !theta || !info || n < 2 || n > kRidgeMax || label <= 0 || label >= n || lambda < 0.0 ||
        max_iters < 0 || !(tol >= 0.0))
        return LMFAO_ERR_INVALID_ARG;
    hipLaunchKernelGGL(ridge_bgd_kernel, dim3(1), dim3(kAppThreads), 0, static_cast<hipStream_t>(hip_stream), cov, n,
                       label, lambda, max_iters, tol, theta, info);
    return hipGetLastError() == hipSuccess ? LMFAO_OK : LMFAO_ERR_HIP;
}

extern "C" lmfao_status lmfao_mutual_information(const unsigned long long *const *tables, const int32_t *doms,
                                                 int32_t n_pairs, int32_t max_dom, double *mi, void *hip_stream) {
    if (!tables || !doms || !mi || n_pairs < 0 || max_dom < 1) return LMFAO_ERR_INVALID_ARG;
    if (max_dom > kMiMaxDom) return LMFAO_ERR_TOO_LARGE;
    if (n_pairs == 0) return LMFAO_OK;
    hipLaunchKernelGGL(mutual_information_kernel, dim3(n_pairs), dim3(kAppThreads), 0,
                       static_cast<hipStream_t>(hip_stream), tables, doms, mi);
    return hipGetLastError() == hipSuccess ? LMFAO_OK : LMFAO_ERR_HIP;
}

extern "C" lmfao_status lmfao_chow_liu(const double *mi, int32_t n, int32_t *edges, double *total, void *hip_stream) {
    if (!mi || !edges || !total || n < 2) return LMFAO_ERR_INVALID_ARG;
    if (n > kClMax) return LMFAO_ERR_TOO_LARGE;
    hipLaunchKernelGGL(chow_liu_kernel, dim3(1), dim3(kAppThreads), 0, static_cast<hipStream_t>(hip_stream), mi, n,
                       edges, total);
    return hipGetLastError() == hipSuccess ? LMFAO_OK : LMFAO_ERR_HIP;
}

extern "C" lmfao_status lmfao_best_splits(const lmfao_split_input *inputs, int32_t n_inputs, int32_t n_nodes,
                                          int32_t criterion, int32_t n_labels, lmfao_split_result *out,
                                          void *hip_stream) {
    if (!inputs || !out || n_inputs < 0 || n_nodes < 0 ||
        (criterion != LMFAO_SPLIT_VARIANCE && criterion != LMFAO_SPLIT_GINI) ||
        (criterion == LMFAO_SPLIT_GINI && n_labels < 1))
        return LMFAO_ERR_INVALID_ARG;
    if (criterion == LMFAO_SPLIT_GINI && n_labels > kMaxLabels) return LMFAO_ERR_TOO_LARGE;
    if (n_nodes == 0) return LMFAO_OK;
    hipLaunchKernelGGL(best_split_kernel, dim3(n_nodes), dim3(64), 0, static_cast<hipStream_t>(hip_stream), inputs,
                       n_inputs, criterion, n_labels, out);
    return hipGetLastError() == hipSuccess ? LMFAO_OK : LMFAO_ERR_HIP;
}
