// Cost-model MLP kernels: forward, backward, gradient reduction, Adam.
//
// The model maps the feature vector of one kernel step to the natural log
// of its duration:  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
// y = w3 . h2 + b3, with F inputs, H = 64 hidden units per layer, FP32
// throughout.  Flat parameter layout: W1 [H][F], b1 [H], W2 [H][H], b2 [H],
// w3 [H], b3 [1].
//
// A sample costs about F*H + H*H = 5.6e3 multiply-adds, so a launch over a
// few thousand samples is bound by launch latency, not by arithmetic: one
// thread per sample with the weights broadcast from LDS keeps the kernels
// short and every reduction in a fixed order (the gradients are
// bit-reproducible).  Training loss: mean squared error over the batch.
#include <hip/hip_runtime.h>

#include <cmath>

#include "htn.h"
#include "kernels.hpp"

namespace htn {
namespace kern {

namespace {
constexpr int MF = HTN_MODEL_FEATURES, MH = HTN_MODEL_HIDDEN;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MH * MF;
constexpr int OFF_W2 = OFF_B1 + MH;
constexpr int OFF_B2 = OFF_W2 + MH * MH;
constexpr int OFF_W3 = OFF_B2 + MH;
constexpr int OFF_B3 = OFF_W3 + MH;
constexpr int NPARAM = OFF_B3 + 1;
constexpr int TPB = 256;
}  // namespace

int64_t model_param_count() { return NPARAM; }

// One thread per sample (sample s reads row idx[s] of x when idx is given).
// With z1/z2 non-null the pre-activations are kept for the backward pass,
// as [s][H] rows.
__global__ __launch_bounds__(TPB) void k_mlp_fwd(const float *__restrict__ prm, const float *__restrict__ x,
                                                const int32_t *__restrict__ idx, int n, float *__restrict__ y,
                                                float *__restrict__ z1, float *__restrict__ z2) {
    __shared__ float w[NPARAM];
    for (int i = threadIdx.x; i < NPARAM; i += TPB) w[i] = prm[i];
    __syncthreads();
    const int s = blockIdx.x * TPB + threadIdx.x;
    if (s >= n) return;
    const int64_t src = idx ? idx[s] : s;
    float xv[MF];
#pragma unroll
    for (int f = 0; f < MF; ++f) xv[f] = x[src * MF + f];
    float h1[MH];
#pragma unroll
    for (int j = 0; j < MH; ++j) {
        float a = w[OFF_B1 + j];
#pragma unroll
        for (int f = 0; f < MF; ++f) a = fmaf(w[OFF_W1 + j * MF + f], xv[f], a);
        if (z1) z1[(int64_t)s * MH + j] = a;
        h1[j] = fmaxf(a, 0.0f);
    }
    float out = w[OFF_B3];
    for (int j = 0; j < MH; ++j) {
        float a = w[OFF_B2 + j];
#pragma unroll
        for (int i = 0; i < MH; ++i) a = fmaf(w[OFF_W2 + j * MH + i], h1[i], a);
        if (z2) z2[(int64_t)s * MH + j] = a;
        out = fmaf(w[OFF_W3 + j], fmaxf(a, 0.0f), out);
    }
    y[s] = out;
}

// Per-sample backward: with loss (1/n) sum_s (y_s - t_s)^2,
//   dy_s = 2 (y_s - t_s) / n,  dz2 = dy_s w3 * [z2 > 0],  dz1 = W2^T dz2 * [z1 > 0].
__global__ __launch_bounds__(TPB) void k_mlp_bwd(const float *__restrict__ prm, const float *__restrict__ t,
                                                const int32_t *__restrict__ idx, int n, float scale,
                                                const float *__restrict__ y, const float *__restrict__ z1,
                                                const float *__restrict__ z2, float *__restrict__ d1,
                                                float *__restrict__ d2, float *__restrict__ dy) {
    __shared__ float w[NPARAM];
    for (int i = threadIdx.x; i < NPARAM; i += TPB) w[i] = prm[i];
    __syncthreads();
    const int s = blockIdx.x * TPB + threadIdx.x;
    if (s >= n) return;
    const int64_t src = idx ? idx[s] : s;
    const float g = scale * (y[s] - t[src]);
    dy[s] = g;
    float dz2[MH];
#pragma unroll
    for (int j = 0; j < MH; ++j) {
        dz2[j] = z2[(int64_t)s * MH + j] > 0.0f ? g * w[OFF_W3 + j] : 0.0f;
        d2[(int64_t)s * MH + j] = dz2[j];
    }
    for (int i = 0; i < MH; ++i) {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < MH; ++j) a = fmaf(w[OFF_W2 + j * MH + i], dz2[j], a);
        d1[(int64_t)s * MH + i] = z1[(int64_t)s * MH + i] > 0.0f ? a : 0.0f;
    }
}

// Gradient of the loss: one thread per parameter, summing its per-sample
// terms over s = 0..n-1 in order.
__global__ __launch_bounds__(TPB) void k_mlp_grad(const float *__restrict__ x, const int32_t *__restrict__ idx, int n,
                                                 const float *__restrict__ z1, const float *__restrict__ z2,
                                                 const float *__restrict__ d1, const float *__restrict__ d2,
                                                 const float *__restrict__ dy, float *__restrict__ grad) {
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= NPARAM) return;
    float acc = 0.0f;
    if (p < OFF_B1) {
        const int j = p / MF, f = p - j * MF;
        for (int s = 0; s < n; ++s) {
            const int64_t src = idx ? idx[s] : s;
            acc = fmaf(d1[(int64_t)s * MH + j], x[src * MF + f], acc);
        }
    } else if (p < OFF_W2) {
        const int j = p - OFF_B1;
        for (int s = 0; s < n; ++s) acc += d1[(int64_t)s * MH + j];
    } else if (p < OFF_B2) {
        const int q = p - OFF_W2, j = q / MH, i = q - j * MH;
        for (int s = 0; s < n; ++s) acc = fmaf(d2[(int64_t)s * MH + j], fmaxf(z1[(int64_t)s * MH + i], 0.0f), acc);
    } else if (p < OFF_W3) {
        const int j = p - OFF_B2;
        for (int s = 0; s < n; ++s) acc += d2[(int64_t)s * MH + j];
    } else if (p < OFF_B3) {
        const int j = p - OFF_W3;
        for (int s = 0; s < n; ++s) acc = fmaf(dy[s], fmaxf(z2[(int64_t)s * MH + j], 0.0f), acc);
    } else {
        for (int s = 0; s < n; ++s) acc += dy[s];
    }
    grad[p] = acc;
}

// Mean squared error of a batch (one workgroup, fixed summation order).
__global__ __launch_bounds__(TPB) void k_mlp_loss(const float *__restrict__ y, const float *__restrict__ t,
                                                 const int32_t *__restrict__ idx, int n, float *__restrict__ loss) {
    __shared__ float red[TPB];
    float a = 0.0f;
    for (int s = threadIdx.x; s < n; s += TPB) {
        const int64_t src = idx ? idx[s] : s;
        const float d = y[s] - t[src];
        a = fmaf(d, d, a);
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int m = TPB / 2; m > 0; m >>= 1) {
        if (threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)n;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
__global__ __launch_bounds__(TPB) void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                             const float *__restrict__ g, int np, float lr, float b1, float b2,
                                             float c1, float c2, float eps) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

hipError_t launch_mlp_forward(const float *prm, const float *x, const int32_t *idx, int n, float *y, float *z1,
                              float *z2, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_fwd, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, st, prm, x, idx, n, y, z1, z2);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *prm, const float *x, const float *t, const int32_t *idx, int n,
                               const float *y, const float *z1, const float *z2, float *d1, float *d2, float *dy,
                               float *grad, float *loss, hipStream_t st) {
    if (n <= 0) return hipErrorInvalidValue;
    const dim3 gs((n + TPB - 1) / TPB);
    hipLaunchKernelGGL(k_mlp_bwd, gs, dim3(TPB), 0, st, prm, t, idx, n, 2.0f / (float)n, y, z1, z2, d1, d2, dy);
    hipLaunchKernelGGL(k_mlp_grad, dim3((NPARAM + TPB - 1) / TPB), dim3(TPB), 0, st, x, idx, n, z1, z2, d1, d2, dy,
                       grad);
    if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(TPB), 0, st, y, t, idx, n, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, float *m, float *v, const float *g, float lr, int64_t step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const double c1 = 1.0 / (1.0 - std::pow(0.9, (double)step));
    const double c2 = 1.0 / (1.0 - std::pow(0.999, (double)step));
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + TPB - 1) / TPB), dim3(TPB), 0, st, p, m, v, g, NPARAM, lr, b1, b2,
                       (float)c1, (float)c2, eps);
    return hipGetLastError();
}

}  // namespace kern
}  // namespace htn
