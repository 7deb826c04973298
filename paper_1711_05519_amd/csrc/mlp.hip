// The threshold network of the learned schedule (not part of the paper):
// o = w3 . relu(W2 relu(W1 phi + b1) + b2) + b3 with phi in R^4, 32 hidden
// units per layer; the loop uses it as a multiplicative correction of
// Algorithm 1's threshold, zeta = beta (sigma_{r+1} + gamma^{k+1} sigma_1)
// exp(clip(o, -5, 5)) (the single-wave tail of the gather). Parameters are one
// FP32 vector of MLP_PARAMS values: W1 (32 x 4, row-major), b1, W2 (32 x 32),
// b2, w3, b3. These kernels train it: a batched forward pass, the gradient
// of sum_b g_b o_b summed over the batch in a fixed order, and Adam.

#include "launch.hpp"

namespace rpca {
namespace {

constexpr int OFF_W1 = 0, OFF_B1 = MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H,
              OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H;
static_assert(OFF_B3 + 1 == MLP_PARAMS, "parameter layout");

// Activations of one sample, computed by the 64 lanes of a wave (lane j < 32
// owns hidden unit j); results in LDS.
__device__ inline void mlp_act(const float* __restrict__ th, const float* ph, float* a1, float* h1, float* a2,
                               float* h2, float* o) {
    const int lane = threadIdx.x & (WAVE - 1);
    if (lane < MLP_H) {
        float v = th[OFF_B1 + lane];
        for (int i = 0; i < MLP_IN; ++i) v = fmaf(th[OFF_W1 + lane * MLP_IN + i], ph[i], v);
        a1[lane] = v;
        h1[lane] = fmaxf(v, 0.f);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float c = 0.f;
    if (lane < MLP_H) {
        float v = th[OFF_B2 + lane];
        for (int i = 0; i < MLP_H; ++i) v = fmaf(th[OFF_W2 + lane * MLP_H + i], h1[i], v);
        a2[lane] = v;
        h2[lane] = fmaxf(v, 0.f);
        c = th[OFF_W3 + lane] * h2[lane];
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, WAVE);
    if (lane == 0) *o = c + th[OFF_B3];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// one wave per sample
__global__ __launch_bounds__(WAVE) void k_mlp_forward(const float* __restrict__ th, const float* __restrict__ phi,
                                                     float* __restrict__ o, int B) {
    const int b = blockIdx.x;
    if (b >= B) return;
    __shared__ float ph[MLP_IN], a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H], out;
    if (threadIdx.x < MLP_IN) ph[threadIdx.x] = phi[(size_t)b * MLP_IN + threadIdx.x];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    mlp_act(th, ph, a1, h1, a2, h2, &out);
    if (threadIdx.x == 0) o[b] = out;
}

// grad = sum over b (in order) of g_b d o_b / d theta; one workgroup, each
// thread owns parameters t, t + 256, ...; wave 0 recomputes the activations.
__global__ __launch_bounds__(256) void k_mlp_backward(const float* __restrict__ th, const float* __restrict__ phi,
                                                     const float* __restrict__ g, int B, float* __restrict__ grad) {
    __shared__ float ph[MLP_IN], a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H], out;
    __shared__ float ga2[MLP_H], ga1[MLP_H];
    float acc[(MLP_PARAMS + 255) / 256];
    for (int u = 0; u < (MLP_PARAMS + 255) / 256; ++u) acc[u] = 0.f;
    for (int b = 0; b < B; ++b) {
        const float gb = g[b];
        if (threadIdx.x < MLP_IN) ph[threadIdx.x] = phi[(size_t)b * MLP_IN + threadIdx.x];
        __syncthreads();
        if (threadIdx.x < WAVE) mlp_act(th, ph, a1, h1, a2, h2, &out);
        __syncthreads();
        if (threadIdx.x < MLP_H) {
            const int j = threadIdx.x;
            ga2[j] = a2[j] > 0.f ? gb * th[OFF_W3 + j] : 0.f;   // d/d a2_j
        }
        __syncthreads();
        if (threadIdx.x < MLP_H) {
            const int i = threadIdx.x;
            float v = 0.f;
            for (int j = 0; j < MLP_H; ++j) v = fmaf(th[OFF_W2 + j * MLP_H + i], ga2[j], v);
            ga1[i] = a1[i] > 0.f ? v : 0.f;                    // d/d a1_i
        }
        __syncthreads();
        for (int u = 0; u < (MLP_PARAMS + 255) / 256; ++u) {
            const int t = threadIdx.x + 256 * u;
            if (t >= MLP_PARAMS) break;
            float d;
            if (t < OFF_B1) d = ga1[t / MLP_IN] * ph[t % MLP_IN];
            else if (t < OFF_W2) d = ga1[t - OFF_B1];
            else if (t < OFF_B2) d = ga2[(t - OFF_W2) / MLP_H] * h1[(t - OFF_W2) % MLP_H];
            else if (t < OFF_W3) d = ga2[t - OFF_B2];
            else if (t < OFF_B3) d = gb * h2[t - OFF_W3];
            else d = gb;
            acc[u] += d;
        }
        __syncthreads();
    }
    for (int u = 0; u < (MLP_PARAMS + 255) / 256; ++u) {
        const int t = threadIdx.x + 256 * u;
        if (t < MLP_PARAMS) grad[t] = acc[u];
    }
}

// Adam (Kingma and Ba, Algorithm 1), step t >= 1, elementwise
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                                 const float* __restrict__ g, int n, int t, float lr, float b1,
                                                 float b2, float eps) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float mi = b1 * m[i] + (1.f - b1) * g[i];
    const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - powf(b1, (float)t));
    const float vh = vi / (1.f - powf(b2, (float)t));
    th[i] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

hipError_t launch_mlp_forward(const float* th, const float* phi, float* o, int B, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(WAVE), 0, s, th, phi, o, B);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* th, const float* phi, const float* g, int B, float* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_backward, dim3(1), dim3(256), 0, s, th, phi, g, B, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* th, float* m, float* v, const float* g, int t, float lr, float b1, float b2,
                           float eps, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, s, th, m, v, g, MLP_PARAMS, t, lr,
                       b1, b2, eps);
    return hipGetLastError();
}

}  // namespace rpca
