// The selector's network (11 -> 64 -> 64 -> 7, ReLU) in FP32: forward, backward and Adam.
//
// Parameters are one flat vector: W1 (64 x 11, row-major), b1, W2 (64 x 64), b2, W3 (7 x 64),
// b3.  Forward: one thread per sample, parameters staged in LDS.  Backward: one thread per
// sample for the per-sample error signals, then one thread per parameter summing its gradient
// over the samples in order (deterministic; no atomics).  Loss: mean softmax cross-entropy.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace smx {

namespace {

constexpr int kIn = kMlpIn, kH = 64, kOut = 7;
constexpr int kW1 = 0, kB1 = kW1 + kH * kIn, kW2 = kB1 + kH, kB2 = kW2 + kH * kH,
              kW3 = kB2 + kH, kB3 = kW3 + kOut * kH;
static_assert(kB3 + kOut == kMlpParams, "layout");

__device__ __forceinline__ void stage_params(const float* params, float* sp) {
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) sp[i] = params[i];
  __syncthreads();
}

// Forward for sample s; a1 / a2 keep the pre-activations (for the ReLU masks).
__device__ __forceinline__ void forward_one(const float* sp, const float* x, float* a1, float* a2,
                                            float* z) {
  float h1[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float a = sp[kB1 + j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) a = __builtin_fmaf(sp[kW1 + j * kIn + i], x[i], a);
    a1[j] = a;
    h1[j] = a > 0.f ? a : 0.f;
  }
  float h2[kH];
#pragma unroll 4
  for (int j = 0; j < kH; ++j) {
    float a = sp[kB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) a = __builtin_fmaf(sp[kW2 + j * kH + i], h1[i], a);
    a2[j] = a;
    h2[j] = a > 0.f ? a : 0.f;
  }
#pragma unroll
  for (int o = 0; o < kOut; ++o) {
    float a = sp[kB3 + o];
#pragma unroll
    for (int i = 0; i < kH; ++i) a = __builtin_fmaf(sp[kW3 + o * kH + i], h2[i], a);
    z[o] = a;
  }
}

// logits (n x 7); when `work` is given also the pre-activations A1 (n x 64), A2 (n x 64).
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* params, const float* X,
                                                          int n, float* logits, float* A1,
                                                          float* A2) {
  __shared__ float sp[kMlpParams];
  stage_params(params, sp);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[kIn], a1[kH], a2[kH], z[kOut];
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = X[s * kIn + i];
  forward_one(sp, x, a1, a2, z);
#pragma unroll
  for (int o = 0; o < kOut; ++o) logits[(size_t)s * kOut + o] = z[o];
  if (A1) {
#pragma unroll
    for (int j = 0; j < kH; ++j) {
      A1[(size_t)s * kH + j] = a1[j];
      A2[(size_t)s * kH + j] = a2[j];
    }
  }
}

// Per-sample error signals: dZ = (softmax(z) - onehot(y)) / n, D2 = (dZ W3) * [a2 > 0],
// D1 = (D2 W2) * [a1 > 0]; per-sample loss -log softmax(z)[y].
__global__ __launch_bounds__(256) void mlp_delta_kernel(const float* params, const float* Z,
                                                        const float* A1, const float* A2,
                                                        const int* y, int n, float* DZ, float* D1,
                                                        float* D2, float* Ls) {
  __shared__ float sp[kMlpParams];
  stage_params(params, sp);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float z[kOut], zmax = -3.0e38f;
#pragma unroll
  for (int o = 0; o < kOut; ++o) {
    z[o] = Z[(size_t)s * kOut + o];
    zmax = fmaxf(zmax, z[o]);
  }
  float se = 0.f;
#pragma unroll
  for (int o = 0; o < kOut; ++o) se += __expf(z[o] - zmax);
  const float lse = zmax + __logf(se);
  const int lab = y[s];
  const float inv_n = 1.0f / (float)n;
  float dz[kOut];
#pragma unroll
  for (int o = 0; o < kOut; ++o) {
    dz[o] = (__expf(z[o] - lse) - (o == lab ? 1.f : 0.f)) * inv_n;
    DZ[(size_t)s * kOut + o] = dz[o];
  }
  float zl = z[0];
#pragma unroll
  for (int o = 1; o < kOut; ++o) zl = o == lab ? z[o] : zl;
  Ls[s] = lse - zl;
  float d2[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    float a = 0.f;
#pragma unroll
    for (int o = 0; o < kOut; ++o) a = __builtin_fmaf(dz[o], sp[kW3 + o * kH + j], a);
    d2[j] = A2[(size_t)s * kH + j] > 0.f ? a : 0.f;
    D2[(size_t)s * kH + j] = d2[j];
  }
#pragma unroll 4
  for (int i = 0; i < kH; ++i) {
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < kH; ++j) a = __builtin_fmaf(d2[j], sp[kW2 + j * kH + i], a);
    D1[(size_t)s * kH + i] = A1[(size_t)s * kH + i] > 0.f ? a : 0.f;
  }
}

// One thread per parameter: its gradient summed over the samples in order; thread kMlpParams
// writes the mean loss.
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* X, const float* A1,
                                                       const float* A2, const float* DZ,
                                                       const float* D1, const float* D2,
                                                       const float* Ls, int n, float* grad,
                                                       float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  float acc = 0.f;
  if (p == kMlpParams) {
    for (int s = 0; s < n; ++s) acc += Ls[s];
    *loss = acc / (float)n;
    return;
  }
  if (p < kB1) {                     // W1[j][i]: D1[s][j] * x[s][i]
    const int j = p / kIn, i = p % kIn;
    for (int s = 0; s < n; ++s) acc = __builtin_fmaf(D1[(size_t)s * kH + j], X[s * kIn + i], acc);
  } else if (p < kW2) {              // b1[j]
    const int j = p - kB1;
    for (int s = 0; s < n; ++s) acc += D1[(size_t)s * kH + j];
  } else if (p < kB2) {              // W2[j][i]: D2[s][j] * relu(a1[s][i])
    const int j = (p - kW2) / kH, i = (p - kW2) % kH;
    for (int s = 0; s < n; ++s) {
      const float h = fmaxf(A1[(size_t)s * kH + i], 0.f);
      acc = __builtin_fmaf(D2[(size_t)s * kH + j], h, acc);
    }
  } else if (p < kW3) {              // b2[j]
    const int j = p - kB2;
    for (int s = 0; s < n; ++s) acc += D2[(size_t)s * kH + j];
  } else if (p < kB3) {              // W3[o][i]: dZ[s][o] * relu(a2[s][i])
    const int o = (p - kW3) / kH, i = (p - kW3) % kH;
    for (int s = 0; s < n; ++s) {
      const float h = fmaxf(A2[(size_t)s * kH + i], 0.f);
      acc = __builtin_fmaf(DZ[(size_t)s * kOut + o], h, acc);
    }
  } else {                           // b3[o]
    const int o = p - kB3;
    for (int s = 0; s < n; ++s) acc += DZ[(size_t)s * kOut + o];
  }
  grad[p] = acc;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float* params, const float* grad, float* m,
                                                       float* v, float lr, float b1, float b2,
                                                       float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm * c1) / (__builtin_sqrtf(vv * c2) + eps);
}

}  // namespace

hipError_t launch_mlp_forward(const float* params, const float* X, int n, float* logits,
                              float* A1, float* A2, hipStream_t s) {
  const int grid = (n + 255) / 256;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(256), 0, s, params, X, n, logits, A1, A2);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* params, const float* X, const int* y, int n,
                               float* work, float* grad, float* loss, hipStream_t s) {
  // work: Z (7n), A1 (64n), A2 (64n), DZ (7n), D1 (64n), D2 (64n), Ls (n)
  float* Z = work;
  float* A1 = Z + (size_t)kOut * n;
  float* A2 = A1 + (size_t)kH * n;
  float* DZ = A2 + (size_t)kH * n;
  float* D1 = DZ + (size_t)kOut * n;
  float* D2 = D1 + (size_t)kH * n;
  float* Ls = D2 + (size_t)kH * n;
  const int grid = (n + 255) / 256;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(256), 0, s, params, X, n, Z, A1, A2);
  hipLaunchKernelGGL(mlp_delta_kernel, dim3(grid), dim3(256), 0, s, params, Z, A1, A2, y, n, DZ,
                     D1, D2, Ls);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s, X, A1,
                     A2, DZ, D1, D2, Ls, n, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, params,
                     grad, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace smx
