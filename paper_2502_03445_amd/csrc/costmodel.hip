// Learned cost model: a small MLP that predicts the log device time of one
// pairwise-contraction launch from its shape features, trained on timings
// of the plain contractor and used to rank candidate plans.  (The paper
// notes that flops over peak over-estimates GPU time and that GPU-specific
// profiling is needed; this is that profiling, learned.)
//
//   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 . w3 + b3
//   x: kFeat features, hidden width kHid, float32.
//
// Layout of the lanes: one wavefront per input row, lane j computes hidden
// unit j of both layers; the rows of a wave are processed in a fixed order
// and the gradient of each parameter is owned by exactly one lane of each
// wave, so gradients are reduced without atomics (deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "costmodel.hpp"

namespace tqc {

static_assert(kHid == 64, "one lane per hidden unit");

__device__ inline float wave_sum(float v) {
  // fixed butterfly: every lane ends with the same, order-defined sum
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline void load_params(const float *theta, float *s) {
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) s[i] = theta[i];
  __syncthreads();
}

// offsets in the parameter vector
constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kFeat * kHid;
constexpr int oW2 = oB1 + kHid;
constexpr int oB2 = oW2 + kHid * kHid;
constexpr int oW3 = oB2 + kHid;
constexpr int oB3 = oW3 + kHid;

__global__ void __launch_bounds__(256) mlp_forward_kernel(const float *theta, const float *X,
                                                          int64_t n, float *y) {
  __shared__ float s[kParams];
  load_params(theta, s);
  const int lane = threadIdx.x & 63;
  const int64_t wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t r = wave; r < n; r += nw) {
    const float *x = X + r * kFeat;
    float z1 = s[oB1 + lane];
    for (int f = 0; f < kFeat; ++f) z1 += x[f] * s[oW1 + f * kHid + lane];
    const float h1 = z1 > 0.f ? z1 : 0.f;
    float z2 = s[oB2 + lane];
    for (int i = 0; i < kHid; ++i) z2 += __shfl(h1, i, 64) * s[oW2 + i * kHid + lane];
    const float h2 = z2 > 0.f ? z2 : 0.f;
    const float out = wave_sum(h2 * s[oW3 + lane]) + s[oB3];
    if (lane == 0) y[r] = out;
  }
}

// Per-wave gradient partials of L = mean_r (y_r - t_r)^2.  Wave w handles
// rows w, w + nw, ... in order; partial[w][p] holds its contribution.
__global__ void __launch_bounds__(256) mlp_grad_kernel(const float *theta, const float *X,
                                                       const float *t, const int32_t *rows,
                                                       int64_t n, float inv_n, float *partial) {
  __shared__ float s[kParams];
  load_params(theta, s);
  const int lane = threadIdx.x & 63;
  const int64_t wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * 4;
  float gW1[kFeat], gW2[kHid];
  for (int f = 0; f < kFeat; ++f) gW1[f] = 0.f;
  for (int i = 0; i < kHid; ++i) gW2[i] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f;
  for (int64_t q = wave; q < n; q += nw) {
    const int64_t r = rows ? rows[q] : q;
    const float *x = X + r * kFeat;
    float z1 = s[oB1 + lane];
    for (int f = 0; f < kFeat; ++f) z1 += x[f] * s[oW1 + f * kHid + lane];
    const float h1 = z1 > 0.f ? z1 : 0.f;
    float z2 = s[oB2 + lane];
    for (int i = 0; i < kHid; ++i) z2 += __shfl(h1, i, 64) * s[oW2 + i * kHid + lane];
    const float h2 = z2 > 0.f ? z2 : 0.f;
    const float yv = wave_sum(h2 * s[oW3 + lane]) + s[oB3];
    const float dy = 2.f * (yv - t[r]) * inv_n;
    gw3 += dy * h2;
    gb3 += dy;  // identical in every lane; lane 0's copy is written
    const float dz2 = z2 > 0.f ? dy * s[oW3 + lane] : 0.f;
    gb2 += dz2;
    for (int i = 0; i < kHid; ++i) gW2[i] += __shfl(h1, i, 64) * dz2;
    // dz1_lane = [z1 > 0] * sum_j W2[lane][j] dz2_j
    float acc = 0.f;
    for (int j = 0; j < kHid; ++j) acc += s[oW2 + lane * kHid + j] * __shfl(dz2, j, 64);
    const float dz1 = z1 > 0.f ? acc : 0.f;
    gb1 += dz1;
    for (int f = 0; f < kFeat; ++f) gW1[f] += x[f] * dz1;
  }
  float *P = partial + wave * (int64_t)kParams;
  for (int f = 0; f < kFeat; ++f) P[oW1 + f * kHid + lane] = gW1[f];
  P[oB1 + lane] = gb1;
  for (int i = 0; i < kHid; ++i) P[oW2 + i * kHid + lane] = gW2[i];
  P[oB2 + lane] = gb2;
  P[oW3 + lane] = gw3;
  if (lane == 0) P[oB3] = gb3;
}

__global__ void __launch_bounds__(256) mlp_reduce_kernel(const float *partial, int nwaves, float *g) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  float acc = 0.f;
  for (int w = 0; w < nwaves; ++w) acc += partial[(int64_t)w * kParams + p];
  g[p] = acc;
}

__global__ void __launch_bounds__(256) adam_kernel(float *theta, const float *g, float *m, float *v,
                                                   float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  theta[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

hipError_t launch_mlp_forward(const float *theta, const float *X, int64_t n, float *y, hipStream_t s) {
  int64_t blocks = (n + 3) / 4;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, s, theta, X, n, y);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *theta, const float *X, const float *t, const int32_t *rows,
                           int64_t n, float *partial, float *g, hipStream_t s) {
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(kGradBlocks), dim3(256), 0, s, theta, X, t, rows, n,
                     1.0f / (float)n, partial);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, partial,
                     kGradBlocks * 4, g);
  return hipGetLastError();
}

hipError_t launch_adam(float *theta, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, theta, g, m, v, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace tqc
