// Measured matrix-core issue rates (measurement support): the rates that a kernel's MFMA
// fraction is quoted against beside the datasheet peaks.  Every wave issues `CH` independent
// chains of the instruction the library's kernels use (FP64: v_mfma_f64_16x16x4_f64, BF16:
// v_mfma_f32_16x16x32_bf16), eight waves per SIMD, no memory traffic but one store per lane of
// the summed accumulators (so the work is kept).  No launch bounds: with them the compiler
// moves the accumulators to AGPRs at three waves per SIMD, which measured 49 instead of 78
// TFLOP/s for FP64.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace smx {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int kChains = 8;

__global__ void rate_f64_kernel(double* out, int iters) {
  const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
  d4_t acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = (d4_t){0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void rate_bf16_kernel(double* out, int iters) {
  bf8_t a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1.0f + (threadIdx.x + e) * 1e-3f);
    b[e] = (__bf16)(1.0f - (threadIdx.x + e) * 1e-3f);
  }
  f4_t acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = (f4_t){0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (double)s;
}

}  // namespace

int probe_grid(int cus) { return 8 * cus; }   // 8 workgroups of 4 waves per CU: 8 waves per SIMD

hipError_t launch_rate_probe(int kind, double* out, int grid, int iters, hipStream_t s) {
  if (kind == 0) hipLaunchKernelGGL(rate_f64_kernel, dim3(grid), dim3(256), 0, s, out, iters);
  else hipLaunchKernelGGL(rate_bf16_kernel, dim3(grid), dim3(256), 0, s, out, iters);
  return hipGetLastError();
}

double probe_flops_per_wave_iter(int kind) {
  // kChains instructions of 16x16x4 (FP64) or 16x16x32 (BF16) multiply-adds
  return kind == 0 ? kChains * 2.0 * 16 * 16 * 4 : kChains * 2.0 * 16 * 16 * 32;
}

}  // namespace smx
