// Small kernels of the LU factorization without pivoting (strassen_dgetrf_nopiv) and of the
// Cholesky factorization (strassen_dpotrf_lower): the base cases of their recursive panel
// factorizations and triangular solves.  Everything above them is cast as
// matrix products (the rank-k updates that the paper's future work, Sec. 6, proposes to run with
// Strassen), which the library's own GEMM computes.
//
// Each kernel performs the elimination's operations in the order of plain right-looking
// elimination (a multiplier is a quotient by the pivot; an entry is reduced by one product per
// earlier pivot, in increasing pivot order, each product and difference rounded separately), so
// where no product is computed elsewhere the results are those of the plain algorithm.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace smx {

namespace {

constexpr int kLuB = 64;   // largest base-case block

// In-place LU of the w x w block at P (w <= 64) by one workgroup through LDS.
__global__ __launch_bounds__(256) void lu_base_kernel(double* P, int64_t ld, int w) {
  __shared__ double t[kLuB * (kLuB + 1)];
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += 256) {
    const int i = e % w, j = e / w;
    t[j * (kLuB + 1) + i] = P[i + (int64_t)j * ld];
  }
  __syncthreads();
  for (int p = 0; p < w; ++p) {
    const double piv = t[p * (kLuB + 1) + p];
    for (int i = p + 1 + tid; i < w; i += 256) t[p * (kLuB + 1) + i] = t[p * (kLuB + 1) + i] / piv;
    __syncthreads();
    const int r = w - p - 1;
    for (int e = tid; e < r * r; e += 256) {
      const int i = p + 1 + e % r, j = p + 1 + e / r;
      const double prod = t[p * (kLuB + 1) + i] * t[j * (kLuB + 1) + p];
      t[j * (kLuB + 1) + i] = t[j * (kLuB + 1) + i] - prod;
    }
    __syncthreads();
  }
  for (int e = tid; e < w * w; e += 256) {
    const int i = e % w, j = e / w;
    P[i + (int64_t)j * ld] = t[j * (kLuB + 1) + i];
  }
}

// X (rows x w) := X U^{-1} with U upper triangular w x w (w <= 64; unit: ones on the diagonal,
// not read): one thread per row (64 per workgroup, so that the rows spread over many CUs),
// x_j = (b_j - sum_{p<j} x_p u_pj) / u_jj with the sum subtracted term by term in p order.
// Element (r, j) of X is at B + r * xr + j * xc and u_pj at U + p * ur + j * uc, so the same
// kernel solves B := B U^{-1} (xr = 1, xc = ldb) and, on the transposed view, B := L^{-1} B for
// a unit lower L (U = L^T: ur = ldl, uc = 1; X = B^T: xr = ldb, xc = 1).
__global__ __launch_bounds__(64) void trsm_rows_upper_kernel(const double* U, int64_t ur,
                                                            int64_t uc, int w, int unit, double* B,
                                                            int64_t xr, int64_t xc, int64_t rows) {
  __shared__ double u[kLuB * (kLuB + 1)];
  for (int e = threadIdx.x; e < kLuB * kLuB; e += 64) {   // entries past w read as zero
    const int i = e % kLuB, j = e / kLuB;
    u[j * (kLuB + 1) + i] = (i < w && j < w && i <= j) ? U[i * ur + (int64_t)j * uc] : 0.0;
  }
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (row >= rows) return;
  double* b = B + row * xr;
  // (bounds known at compile time, so the row stays in registers; columns past w stay zero)
  double x[kLuB];
#pragma unroll
  for (int j = 0; j < kLuB; ++j) x[j] = j < w ? b[j * xc] : 0.0;
#pragma unroll
  for (int j = 0; j < kLuB; ++j) {
    double v = x[j];
#pragma unroll
    for (int p = 0; p < j; ++p) {
      const double prod = x[p] * u[j * (kLuB + 1) + p];
      v = v - prod;
    }
    x[j] = j < w ? (unit ? v : v / u[j * (kLuB + 1) + j]) : 0.0;
  }
#pragma unroll
  for (int j = 0; j < kLuB; ++j)
    if (j < w) b[j * xc] = x[j];
}

// In-place Cholesky factor of the w x w block at P (w <= 64; lower triangle only) by one
// workgroup through LDS: for each p, l_pp = sqrt(a_pp), the column below divided by it, then
// the trailing lower triangle reduced by one product per earlier column, in column order.  A
// pivot that is not positive records its column (col0 + p) in *info by an atomic minimum.
__global__ __launch_bounds__(256) void chol_base_kernel(double* P, int64_t ld, int w, int* info,
                                                       int col0) {
  __shared__ double t[kLuB * (kLuB + 1)];
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += 256) {
    const int i = e % w, j = e / w;
    t[j * (kLuB + 1) + i] = i >= j ? P[i + (int64_t)j * ld] : 0.0;   // upper: never read
  }
  __syncthreads();
  for (int p = 0; p < w; ++p) {
    const double d = t[p * (kLuB + 1) + p];
    if (tid == 0 && !(d > 0.0)) atomicMin(info, col0 + p);
    const double l = __builtin_sqrt(d);
    __syncthreads();   // every thread has read the pivot
    if (tid == 0) t[p * (kLuB + 1) + p] = l;
    for (int i = p + 1 + tid; i < w; i += 256) t[p * (kLuB + 1) + i] = t[p * (kLuB + 1) + i] / l;
    __syncthreads();
    const int r = w - p - 1;
    for (int e = tid; e < r * r; e += 256) {
      const int i = p + 1 + e % r, j = p + 1 + e / r;
      if (i < j) continue;
      const double prod = t[p * (kLuB + 1) + i] * t[p * (kLuB + 1) + j];
      t[j * (kLuB + 1) + i] = t[j * (kLuB + 1) + i] - prod;
    }
    __syncthreads();
  }
  for (int e = tid; e < w * w; e += 256) {
    const int i = e % w, j = e / w;
    if (i >= j) P[i + (int64_t)j * ld] = t[j * (kLuB + 1) + i];
  }
}

// C := C - W on the lower triangle of the n x n block C (W n x n, leading dimension ldw).
__global__ __launch_bounds__(256) void sub_lower_kernel(double* C, int64_t ldc, const double* W,
                                                       int64_t ldw, int64_t n) {
  const int64_t j = blockIdx.y;
  const int64_t i = j + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  C[i + j * ldc] = C[i + j * ldc] - W[i + j * ldw];
}

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

}  // namespace

hipError_t launch_chol_base(double* P, int64_t ld, int w, int* info, int col0, hipStream_t s) {
  if (w < 1 || w > kLuB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_base_kernel, dim3(1), dim3(256), 0, s, P, ld, w, info, col0);
  return hipGetLastError();
}

hipError_t launch_sub_lower(double* C, int64_t ldc, const double* W, int64_t ldw, int64_t n,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n >= 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sub_lower_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256),
                     0, s, C, ldc, W, ldw, n);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

// B (rows x w) := B L^{-T} for a lower triangular L (w <= 64): the row solve on U = L^T
// (u_pj = l_jp: strides ldl, 1), dividing by the diagonal.
hipError_t launch_trsm_rows_lower_t(const double* L, int64_t ldl, int w, double* B, int64_t ldb,
                                    int64_t rows, hipStream_t s) {
  if (w < 1 || w > kLuB) return hipErrorInvalidValue;
  if (rows <= 0) return hipSuccess;
  const int64_t grid = (rows + 63) / 64;
  if (grid >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(trsm_rows_upper_kernel, dim3((unsigned)grid), dim3(64), 0, s, L, ldl,
                     int64_t(1), w, 0, B, int64_t(1), ldb, rows);
  return hipGetLastError();
}

hipError_t launch_lu_base(double* P, int64_t ld, int w, hipStream_t s) {
  if (w < 1 || w > kLuB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lu_base_kernel, dim3(1), dim3(256), 0, s, P, ld, w);
  return hipGetLastError();
}

hipError_t launch_trsm_rows_upper(const double* U, int64_t ldu, int w, double* B, int64_t ldb,
                                  int64_t rows, hipStream_t s) {
  if (w < 1 || w > kLuB) return hipErrorInvalidValue;
  if (rows <= 0) return hipSuccess;
  const int64_t grid = (rows + 63) / 64;
  if (grid >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(trsm_rows_upper_kernel, dim3((unsigned)grid), dim3(64), 0, s, U, int64_t(1),
                     ldu, w, 0, B, int64_t(1), ldb, rows);
  return hipGetLastError();
}

hipError_t launch_trsm_cols_lower_unit(const double* L, int64_t ldl, int k, double* B,
                                       int64_t ldb, int64_t cols, hipStream_t s) {
  if (k < 1 || k > kLuB) return hipErrorInvalidValue;
  if (cols <= 0) return hipSuccess;
  const int64_t grid = (cols + 63) / 64;
  if (grid >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  // B := L^{-1} B is B^T := B^T L^{-T}: rows of B^T are the columns of B, L^T is unit upper
  hipLaunchKernelGGL(trsm_rows_upper_kernel, dim3((unsigned)grid), dim3(64), 0, s, L, ldl,
                     int64_t(1), k, 1, B, ldb, int64_t(1), cols);
  return hipGetLastError();
}

}  // namespace smx
