// mlp.hip -- training and inference kernels of the learned cost model: a
// three-layer perceptron  x[D0] -> relu(x W1 + b1)[H1] -> relu(. W2 + b2)[H2]
// -> (. W3 + b3)  predicting log(kernel time) from (shape, tile config)
// features.  Sizes are tiny (D0 ~ 24, H ~ 64, a few thousand rows), so each
// kernel maps one thread to one output value and sums in a fixed order: the
// results are reproducible run to run.
//
// Parameter vector layout (fp32): W1 (D0 x H1, row-major), b1 (H1),
// W2 (H1 x H2), b2 (H2), W3 (H2), b3 (1).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.hpp"

namespace mlk {

namespace {

constexpr int kT = 256;

inline int blocks(int64_t n) { return (int)((n + kT - 1) / kT); }

// z[r, j] = b[j] + sum_i in[r, i] W[i, j];  a = relu(z) when a != null
__global__ __launch_bounds__(kT) void k_layer(const float* __restrict__ in, int64_t B, int64_t I,
                                              const float* __restrict__ W,
                                              const float* __restrict__ b, int64_t J,
                                              float* __restrict__ z, float* __restrict__ a) {
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= B * J) return;
    const int64_t r = idx / J, j = idx % J;
    float s = b[j];
    for (int64_t i = 0; i < I; ++i) s += in[r * I + i] * W[i * J + j];
    if (z) z[idx] = s;
    if (a) a[idx] = s > 0.0f ? s : 0.0f;
}

// loss = (1/B) sum_r (y_r - t_r)^2 and dy_r = 2 (y_r - t_r) / B  (one block)
__global__ __launch_bounds__(kT) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                            int64_t B, float* __restrict__ dy,
                                            float* __restrict__ loss) {
    __shared__ float sh[kT];
    float s = 0.0f;
    for (int64_t r = threadIdx.x; r < B; r += kT) {
        const float e = y[r] - t[r];
        s += e * e;
        dy[r] = 2.0f * e / (float)B;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = sh[0] / (float)B;
}

// d[r, i] = (z[r, i] > 0) * sum_j W[i, j] dn[r, j]
__global__ __launch_bounds__(kT) void k_backprop(const float* __restrict__ W, int64_t I, int64_t J,
                                                 const float* __restrict__ dn,
                                                 const float* __restrict__ z, int64_t B,
                                                 float* __restrict__ d) {
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= B * I) return;
    const int64_t r = idx / I, i = idx % I;
    float s = 0.0f;
    if (z[idx] > 0.0f)
        for (int64_t j = 0; j < J; ++j) s += W[i * J + j] * dn[r * J + j];
    d[idx] = s;
}

// G[i, j] = sum_r P[r, i] Q[r, j];  and, from the threads of row i == 0,
// g[j] = sum_r Q[r, j] (bias gradient)
__global__ __launch_bounds__(kT) void k_weight_grad(const float* __restrict__ P, int64_t I,
                                                    const float* __restrict__ Q, int64_t J,
                                                    int64_t B, float* __restrict__ G,
                                                    float* __restrict__ g) {
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= I * J) return;
    const int64_t i = idx / J, j = idx % J;
    float s = 0.0f;
    for (int64_t r = 0; r < B; ++r) s += P[r * I + i] * Q[r * J + j];
    G[idx] = s;
    if (i == 0) {
        float sb = 0.0f;
        for (int64_t r = 0; r < B; ++r) sb += Q[r * J + j];
        g[j] = sb;
    }
}

__global__ __launch_bounds__(kT) void k_adam(int64_t n, float* __restrict__ p,
                                             const float* __restrict__ g, float* __restrict__ m,
                                             float* __restrict__ v, float lr, float b1, float b2,
                                             float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct Offsets {
    int64_t W1, b1, W2, b2, W3, b3;
};

Offsets offsets(int64_t D0, int64_t H1, int64_t H2) {
    Offsets o;
    o.W1 = 0;
    o.b1 = o.W1 + D0 * H1;
    o.W2 = o.b1 + H1;
    o.b2 = o.W2 + H1 * H2;
    o.W3 = o.b2 + H2;
    o.b3 = o.W3 + H2;
    return o;
}

}  // namespace

hipError_t launch_mlp_forward(int64_t B, int64_t D0, int64_t H1, int64_t H2, const float* p,
                              const float* X, float* y, float* ws, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    const Offsets o = offsets(D0, H1, H2);
    float* a1 = ws;
    float* a2 = ws + B * H1;
    hipLaunchKernelGGL(k_layer, dim3(blocks(B * H1)), dim3(kT), 0, s, X, B, D0, p + o.W1, p + o.b1,
                       H1, (float*)nullptr, a1);
    hipLaunchKernelGGL(k_layer, dim3(blocks(B * H2)), dim3(kT), 0, s, (const float*)a1, B, H1,
                       p + o.W2, p + o.b2, H2, (float*)nullptr, a2);
    // output layer: linear, no activation
    hipLaunchKernelGGL(k_layer, dim3(blocks(B)), dim3(kT), 0, s, (const float*)a2, B, H2, p + o.W3,
                       p + o.b3, (int64_t)1, y, (float*)nullptr);
    return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(int64_t B, int64_t D0, int64_t H1, int64_t H2, const float* p,
                                const float* X, const float* t, float* grad, float* loss, float* ws,
                                hipStream_t s) {
    if (B <= 0) return hipErrorInvalidValue;
    const Offsets o = offsets(D0, H1, H2);
    float* z1 = ws;
    float* a1 = z1 + B * H1;
    float* d1 = a1 + B * H1;
    float* z2 = d1 + B * H1;
    float* a2 = z2 + B * H2;
    float* d2 = a2 + B * H2;
    float* y = d2 + B * H2;
    float* dy = y + B;
    // forward, keeping pre-activations
    hipLaunchKernelGGL(k_layer, dim3(blocks(B * H1)), dim3(kT), 0, s, X, B, D0, p + o.W1, p + o.b1,
                       H1, z1, a1);
    hipLaunchKernelGGL(k_layer, dim3(blocks(B * H2)), dim3(kT), 0, s, (const float*)a1, B, H1,
                       p + o.W2, p + o.b2, H2, z2, a2);
    // output layer: linear, no activation
    hipLaunchKernelGGL(k_layer, dim3(blocks(B)), dim3(kT), 0, s, (const float*)a2, B, H2, p + o.W3,
                       p + o.b3, (int64_t)1, y, (float*)nullptr);
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(kT), 0, s, (const float*)y, t, B, dy, loss);
    // backward: deltas of the two hidden layers
    hipLaunchKernelGGL(k_backprop, dim3(blocks(B * H2)), dim3(kT), 0, s, p + o.W3, H2, (int64_t)1,
                       (const float*)dy, (const float*)z2, B, d2);
    hipLaunchKernelGGL(k_backprop, dim3(blocks(B * H1)), dim3(kT), 0, s, p + o.W2, H1, H2,
                       (const float*)d2, (const float*)z1, B, d1);
    // parameter gradients
    hipLaunchKernelGGL(k_weight_grad, dim3(blocks(H2)), dim3(kT), 0, s, (const float*)a2, H2,
                       (const float*)dy, (int64_t)1, B, grad + o.W3, grad + o.b3);
    hipLaunchKernelGGL(k_weight_grad, dim3(blocks(H1 * H2)), dim3(kT), 0, s, (const float*)a1, H1,
                       (const float*)d2, H2, B, grad + o.W2, grad + o.b2);
    hipLaunchKernelGGL(k_weight_grad, dim3(blocks(D0 * H1)), dim3(kT), 0, s, X, D0,
                       (const float*)d1, H1, B, grad + o.W1, grad + o.b1);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr,
                       float b1, float b2, float eps, int64_t t, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const float c1 = (float)(1.0 - pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(kT), 0, s, n, p, g, m, v, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

}  // namespace mlk
