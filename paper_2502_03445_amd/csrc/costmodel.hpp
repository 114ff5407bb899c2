// Cost-model MLP: sizes and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tqc {

constexpr int kFeat = 16;
constexpr int kHid = 64;
constexpr int kParams = kFeat * kHid + kHid + kHid * kHid + kHid + kHid + 1;
constexpr int kGradBlocks = 64;  // fixed, so gradient sums have a fixed order

hipError_t launch_mlp_forward(const float *theta, const float *X, int64_t n, float *y, hipStream_t s);
// g = dL/dtheta of L = mean over rows (rows[] selects, or all n rows if null)
hipError_t launch_mlp_grad(const float *theta, const float *X, const float *t, const int32_t *rows,
                           int64_t n, float *partial, float *g, hipStream_t s);
hipError_t launch_adam(float *theta, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);

}  // namespace tqc
