// mlp.hip -- training and inference kernels of the placement cost model, a
// 3-layer perceptron d -> 64 -> 64 -> 1 (ReLU) that predicts the log run time
// of a placement from (op, n, batch, scope, pack) features.  The paper picks
// placements by measurement only (Sec. III-A, Sec. IV-A); this model proposes
// placements for shapes that were not measured, with measured search as the
// fallback and as what decides among its picks.
//
// Parameter vector (flat): W1 [64][d], b1 [64], W2 [64][64], b2 [64],
// w3 [64], b3 [1].  One wavefront works on a group of samples; lane j owns
// hidden unit j.  The backward pass writes per-block partial gradients that a
// second kernel sums over blocks in a fixed order, so training is
// deterministic (no floating-point atomics).
#include "device_common.hpp"
#include "glass_internal.hpp"

namespace glass {
namespace {

constexpr int kH = 64;
constexpr int kMaxD = 32;
constexpr int kFwdSamples = 16;
constexpr int kBwdSamples = 32;

GLASS_DEV float wave_sum(float v) {
    // butterfly over the 64 lanes; every lane ends with the same total
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct Off {
    int W1, b1, W2, b2, w3, b3, total;
};

__host__ __device__ inline Off offsets(int d) {
    Off o;
    o.W1 = 0;
    o.b1 = kH * d;
    o.W2 = o.b1 + kH;
    o.b2 = o.W2 + kH * kH;
    o.w3 = o.b2 + kH;
    o.b3 = o.w3 + kH;
    o.total = o.b3 + 1;
    return o;
}

__global__ void __launch_bounds__(64) mlp_forward_k(int N, int d, const float* __restrict__ X,
                                                     const float* __restrict__ P, float* __restrict__ H1,
                                                     float* __restrict__ H2, float* __restrict__ Y) {
    __shared__ float xs[kMaxD];
    __shared__ float h1s[kH];
    const int j = threadIdx.x;
    const Off o = offsets(d);
    float w1[kMaxD];
#pragma unroll
    for (int i = 0; i < kMaxD; ++i) w1[i] = i < d ? P[o.W1 + j * d + i] : 0.f;
    float w2[kH];
#pragma unroll
    for (int k = 0; k < kH; ++k) w2[k] = P[o.W2 + j * kH + k];
    const float b1 = P[o.b1 + j], b2 = P[o.b2 + j], w3 = P[o.w3 + j], b3 = P[o.b3];
    const int s0 = blockIdx.x * kFwdSamples;
    for (int s = s0; s < min(s0 + kFwdSamples, N); ++s) {
        if (j < d) xs[j] = X[(size_t)s * d + j];
        wave_sync();
        float a = b1;
#pragma unroll
        for (int i = 0; i < kMaxD; ++i)
            if (i < d) a = fmaf(w1[i], xs[i], a);
        const float h1 = fmaxf(a, 0.f);
        h1s[j] = h1;
        wave_sync();
        float a2 = b2;
#pragma unroll
        for (int k = 0; k < kH; ++k) a2 = fmaf(w2[k], h1s[k], a2);
        const float h2 = fmaxf(a2, 0.f);
        const float y = wave_sum(w3 * h2) + b3;
        if (H1) H1[(size_t)s * kH + j] = h1;
        if (H2) H2[(size_t)s * kH + j] = h2;
        if (j == 0) Y[s] = y;
        wave_sync();
    }
}

// Partial gradients of L = (1/N) sum (y - t)^2 over this block's samples.
__global__ void __launch_bounds__(64) mlp_backward_k(int N, int d, const float* __restrict__ X,
                                                      const float* __restrict__ P, const float* __restrict__ H1,
                                                      const float* __restrict__ H2, const float* __restrict__ Y,
                                                      const float* __restrict__ T, float* __restrict__ part) {
    __shared__ float xs[kMaxD];
    __shared__ float h1s[kH];
    __shared__ float d2s[kH];
    const int j = threadIdx.x;
    const Off o = offsets(d);
    float w2c[kH];  // column j of W2 (for dh1_j)
#pragma unroll
    for (int k = 0; k < kH; ++k) w2c[k] = P[o.W2 + k * kH + j];
    const float w3 = P[o.w3 + j];
    float gW2[kH], gW1[kMaxD];
#pragma unroll
    for (int k = 0; k < kH; ++k) gW2[k] = 0.f;
#pragma unroll
    for (int i = 0; i < kMaxD; ++i) gW1[i] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f;
    const float scale = 2.0f / (float)N;
    const int s0 = blockIdx.x * kBwdSamples;
    for (int s = s0; s < min(s0 + kBwdSamples, N); ++s) {
        if (j < d) xs[j] = X[(size_t)s * d + j];
        const float h1 = H1[(size_t)s * kH + j];
        const float h2 = H2[(size_t)s * kH + j];
        h1s[j] = h1;
        const float dy = scale * (Y[s] - T[s]);
        gw3 = fmaf(dy, h2, gw3);
        gb3 += dy;
        const float dh2 = h2 > 0.f ? dy * w3 : 0.f;
        d2s[j] = dh2;
        gb2 += dh2;
        wave_sync();
#pragma unroll
        for (int k = 0; k < kH; ++k) gW2[k] = fmaf(dh2, h1s[k], gW2[k]);
        float a = 0.f;
#pragma unroll
        for (int k = 0; k < kH; ++k) a = fmaf(w2c[k], d2s[k], a);
        const float dh1 = h1 > 0.f ? a : 0.f;
        gb1 += dh1;
#pragma unroll
        for (int i = 0; i < kMaxD; ++i)
            if (i < d) gW1[i] = fmaf(dh1, xs[i], gW1[i]);
        wave_sync();
    }
    float* out = part + (size_t)blockIdx.x * o.total;
#pragma unroll
    for (int i = 0; i < kMaxD; ++i)
        if (i < d) out[o.W1 + j * d + i] = gW1[i];
    out[o.b1 + j] = gb1;
#pragma unroll
    for (int k = 0; k < kH; ++k) out[o.W2 + j * kH + k] = gW2[k];
    out[o.b2 + j] = gb2;
    out[o.w3 + j] = gw3;
    if (j == 0) out[o.b3] = gb3;
}

__global__ void __launch_bounds__(256) mlp_reduce_k(int nblocks, int P, const float* __restrict__ part,
                                                    float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * P + i];
    grad[i] = s;
}

__global__ void __launch_bounds__(256) mlp_adam_k(int P, float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                  float b2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

}  // namespace

size_t mlp_num_params(int d) { return (size_t)offsets(d).total; }

size_t mlp_backward_workspace_bytes(int N, int d) {
    const int nb = (N + kBwdSamples - 1) / kBwdSamples;
    return sizeof(float) * (size_t)nb * offsets(d).total;
}

int launch_mlp_forward(int N, int d, const float* X, const float* P, float* H1, float* H2, float* Y, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipLaunchKernelGGL(mlp_forward_k, dim3((N + kFwdSamples - 1) / kFwdSamples), dim3(64), 0, (hipStream_t)stream, N,
                       d, X, P, H1, H2, Y);
    return (int)hipGetLastError();
}

int launch_mlp_backward(int N, int d, const float* X, const float* P, const float* H1, const float* H2,
                        const float* Y, const float* T, float* grad, void* workspace, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    const int nb = (N + kBwdSamples - 1) / kBwdSamples;
    const int np = offsets(d).total;
    float* part = reinterpret_cast<float*>(workspace);
    hipLaunchKernelGGL(mlp_backward_k, dim3(nb), dim3(64), 0, (hipStream_t)stream, N, d, X, P, H1, H2, Y, T, part);
    hipLaunchKernelGGL(mlp_reduce_k, dim3((np + 255) / 256), dim3(256), 0, (hipStream_t)stream, nb, np, part, grad);
    return (int)hipGetLastError();
}

int launch_mlp_adam(int P, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                    float bc1, float bc2, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier runtime call is not ours
    hipLaunchKernelGGL(mlp_adam_k, dim3((P + 255) / 256), dim3(256), 0, (hipStream_t)stream, P, p, g, m, v, lr, b1,
                       b2, eps, bc1, bc2);
    return (int)hipGetLastError();
}

}  // namespace glass
