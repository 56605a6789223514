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

#include <algorithm>

#include "launch.h"

namespace smx {

namespace {

constexpr int kLuB = 64;   // largest base-case block

constexpr int kAhead = 12;   // LDS reads in flight ahead of the one being consumed
constexpr int kGroup = 4;    // reads issued together between scheduling fences

// Reads of an LDS vector of 64 doubles that every lane needs in full: pairs c0 .. 31 are read
// 16 bytes at a time into a ring of registers kAhead pairs ahead of their use, with scheduling
// fences every kGroup reads keeping each read at its place, and f(j, value) is called for
// j = 2 c0 .. 63 in order.
template <int C0, class F>
__device__ __attribute__((always_inline)) inline void stream_pairs(const double* v, F&& f) {
  constexpr int n = kLuB / 2 - C0;
  constexpr int ring_n = kAhead + kGroup;
  const double2* v2 = reinterpret_cast<const double2*>(v);
  double2 ring[ring_n];
#pragma unroll
  for (int q = 0; q < kAhead && q < n; ++q) ring[q] = v2[C0 + q];
#pragma unroll
  for (int q = 0; q < n; ++q) {
    if (q % kGroup == 0) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int g = 0; g < kGroup; ++g) {
        const int c = q + kAhead + g;
        if (c < n) ring[c % ring_n] = v2[C0 + c];
      }
    }
    f(2 * (C0 + q), ring[q % ring_n].x);
    f(2 * (C0 + q) + 1, ring[q % ring_n].y);
  }
}

template <int P>
struct StepIndex {
  static constexpr int value = P;
};

// Runs f(StepIndex<0>{}), ..., f(StepIndex<N - 1>{}): a loop whose index is a compile-time
// constant in the body, as the register-resident rows below need.
template <int I, int N, class F>
__device__ __attribute__((always_inline)) inline void static_for(F&& f) {
  if constexpr (I < N) {
    f(StepIndex<I>{});
    static_for<I + 1, N>(f);
  }
}

// 64-bit DPP broadcast of lane Q of each group of four lanes to the whole group.
template <int Q>
__device__ __attribute__((always_inline)) inline double quad_bcast(double v) {
  constexpr int ctrl = Q * 0x55;   // quad_perm [Q, Q, Q, Q]
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, ctrl, 0xf, 0xf, false);
  const uint32_t hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), ctrl, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

// In-place LU of the w x w block at P (w <= 64) by a workgroup of 256 threads, four lanes per
// row: lane q of row i's group holds a_ij for the 16 columns j = q (mod 4) in registers.  For
// each p the pivot row is published through LDS (two buffers, so one barrier per step), the lane
// holding a_ip (i > p) forms the multiplier a_ip / a_pp, a DPP broadcast hands it to the group,
// and each lane reduces its own a_ij (j > p) by it times a_pj: the operations of plain
// elimination, in its order, for every entry.
__global__ __launch_bounds__(256) void lu_base_kernel(double* P, int64_t ld, int w) {
  constexpr int kPer = kLuB / 4;
  __shared__ double prow[2][kLuB];
  const int tid = threadIdx.x, row = tid >> 2, q = tid & 3;
  const int rc = std::min(row, w - 1);
  double a[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int j = 4 * k + q;
    const double v = P[rc + (int64_t)std::min(j, w - 1) * ld];
    a[k] = (row < w && j < w) ? v : 0.0;
  }
  static_for<0, kLuB>([&](auto step) {
    constexpr int p = decltype(step)::value, q0 = p % 4, k0 = p / 4, b = p % 2;
    if (p < w) {   // (uniform)
      if (row == p) {
#pragma unroll
        for (int k = 0; k < kPer; ++k) prow[b][4 * k + q] = a[k];
      }
      __syncthreads();   // the pivot row is published; the buffer of step p - 1 stays intact
      const double l = quad_bcast<q0>(a[k0] / prow[b][p]);   // a_ip / a_pp, from lane q0
      if (row > p) {
        if (q == q0) a[k0] = l;
        if (q > q0) {
          const double prod = l * prow[b][4 * k0 + q];
          a[k0] = a[k0] - prod;
        }
#pragma unroll
        for (int k = k0 + 1; k < kPer; ++k) {
          const double prod = l * prow[b][4 * k + q];
          a[k] = a[k] - prod;
        }
      }
    }
  });
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int j = 4 * k + q;
    if (row < w && j < w) P[row + (int64_t)j * ld] = a[k];
  }
}

// X (rows x w) := X U^{-1} with U upper triangular w x w (w <= 64; unit: ones on the diagonal,
// not read).  Each row of X is solved right-looking: for p = 0, 1, ...: x_p := x_p * (1 / u_pp),
// then every later x_j is reduced by x_p u_pj.  Each x_j thus receives its products in increasing
// p and is scaled last, the order of x_j = (b_j - sum_{p<j} x_p u_pj) / u_jj summed term by term,
// with the division done as LAPACK's unblocked factorizations do it: by the rounded reciprocal
// of the diagonal (the same value as the quotient where u_jj is a power of two).  The 64
// reciprocals are formed once, in parallel, before the solve, so the chain of dependent
// operations from one step to the next holds a multiplication where a division would stand.
// Element (r, j) of X is at B + r * xr + j * xc and u_pj at U + p * ur + j * uc, so the same
// kernel solves B := B U^{-1} (xr = 1, xc = ldb), B := B L^{-T} (U = L^T: ur = ldl, uc = 1) and,
// on the transposed view, B := L^{-1} B for a unit lower L (U = L^T; X = B^T: xr = ldb, xc = 1).
//
// A workgroup of 256 threads solves 64 rows, four lanes per row: lane q of a row's group holds
// x_j for the 16 columns j = q (mod 4) in registers.  At step p the lane holding x_p divides it
// and a DPP broadcast hands it to the other three, which then reduce their own columns, so the
// reductions of a step are spread over four lanes.  U and the 64 x 64 block of X go through LDS
// (loaded and stored with the contiguous index across the lanes; loads use indices clamped into
// the matrix and then select zero, so that a batch of loads is in flight at once), and the U
// entries of step p + 1 are read while step p computes.
__global__ __launch_bounds__(256) void trsm_rows_upper_kernel(const double* U, int64_t ur,
                                                             int64_t uc, int w, int unit, double* B,
                                                             int64_t xr, int64_t xc, int64_t rows) {
  constexpr int kS = kLuB + 2;    // row stride of the U copy
  constexpr int kX = kLuB + 1;    // row stride of the X block
  constexpr int kPer = kLuB / 4;  // columns per lane
  __shared__ double u[kLuB * kS];
  __shared__ double xs[kLuB * kX];
  __shared__ double uinv[kLuB];   // 1 / u_pp
  const int tid = threadIdx.x;
  const bool col_major_u = ur == 1;
  const bool rows_contiguous = xc == 1 && xr != 1;   // X^T is column-major
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int64_t last = rows - 1;
  {
    // 4096 entries of each matrix, 16 per thread: element e = it * 256 + tid has fast index
    // e % 64 (contiguous in memory) and slow index e / 64.
    double uv[16], bv[16];
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int e = it * 256 + tid, fast = e % kLuB, slow = e / kLuB;
      const int i = col_major_u ? fast : slow, j = col_major_u ? slow : fast;
      uv[it] = U[std::min(i, w - 1) * ur + (int64_t)std::min(j, w - 1) * uc];
      const int r = rows_contiguous ? slow : fast, c = rows_contiguous ? fast : slow;
      bv[it] = B[std::min(r0 + r, last) * xr + std::min(c, w - 1) * xc];
    }
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int e = it * 256 + tid, fast = e % kLuB, slow = e / kLuB;
      const int i = col_major_u ? fast : slow, j = col_major_u ? slow : fast;
      // past w: the identity, so that x_j stays zero there; unit: ones on the diagonal
      const double d = (j < w && !unit) ? uv[it] : 1.0;
      u[i * kS + j] = i == j ? d : ((i < j && j < w) ? uv[it] : 0.0);
      const int r = rows_contiguous ? slow : fast, c = rows_contiguous ? fast : slow;
      xs[r * kX + c] = (r0 + r < rows && c < w) ? bv[it] : 0.0;
    }
  }
  __syncthreads();
  if (tid < kLuB) uinv[tid] = 1.0 / u[tid * kS + tid];
  __syncthreads();
  const int row = tid >> 2, q = tid & 3;
  const double* uq = u + q;   // lane q reads columns 4k + q of U
  double x[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) x[k] = xs[row * kX + 4 * k + q];
  // U entries of one step: 1 / u_pp, then u_{p, 4k+q} for k = p / 4 .. 15
  double cur[kPer + 1];
  cur[0] = uinv[0];
#pragma unroll
  for (int k = 0; k < kPer; ++k) cur[1 + k] = uq[4 * k];
  static_for<0, kLuB>([&](auto step) {
    constexpr int p = decltype(step)::value, q0 = p % 4, k0 = p / 4;
    double nxt[kPer + 1];
    __builtin_amdgcn_sched_barrier(0);
    if (p + 1 < kLuB) {
      constexpr int pn = p + 1, kn = pn / 4;
      nxt[0] = uinv[pn];
#pragma unroll
      for (int k = kn; k < kPer; ++k) nxt[1 + k - kn] = uq[pn * kS + 4 * k];
    }
    const double piv = x[k0] * cur[0];        // meaningful on lane q0 of each group
    const double xp = quad_bcast<q0>(piv);    // x_p, final
    if (q == q0) x[k0] = xp;
    if (q > q0) {
      const double prod = xp * cur[1];
      x[k0] = x[k0] - prod;
    }
#pragma unroll
    for (int k = k0 + 1; k < kPer; ++k) {
      const double prod = xp * cur[1 + k - k0];
      x[k] = x[k] - prod;
    }
    if (p + 1 < kLuB) {
      constexpr int kn = (p + 1) / 4;
#pragma unroll
      for (int k = 0; k <= kPer - kn; ++k) cur[k] = nxt[k];
    }
  });
#pragma unroll
  for (int k = 0; k < kPer; ++k) xs[row * kX + 4 * k + q] = x[k];
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int e = it * 256 + tid, fast = e % kLuB, slow = e / kLuB;
    const int r = rows_contiguous ? slow : fast, c = rows_contiguous ? fast : slow;
    const double v = xs[r * kX + c];
    if (r0 + r < rows && c < w) B[(r0 + r) * xr + c * xc] = v;
  }
}

// In-place Cholesky factor of the w x w block at P (w <= 64; lower triangle only) by one
// wave, lane i holding row i in registers: for each p, the pivot a_pp is read from lane p,
// l_pp = sqrt(a_pp), lane i > p divides a_ip by it, the column is published through LDS, and
// lane i reduces a_ij (p < j <= i) by l_ip l_jp: one product per earlier column, in column
// order.  The reductions run unpredicated over every j > p: for j > i they touch only the
// unused strict upper part of the row (zero on entry, never stored), and a lane i <= p reduces
// only such entries, so the lower triangle receives exactly the operations above.  A pivot that
// is not positive records its column (col0 + p) in *info by an atomic minimum.
__global__ __launch_bounds__(64) void chol_base_kernel(double* P, int64_t ld, int w, int* info,
                                                      int col0) {
  __shared__ __attribute__((aligned(16))) double col[kLuB];
  const int lane = threadIdx.x;
  const int ln = std::min(lane, w - 1);
  double a[kLuB];   // row `lane`: the lower part, then scratch (the strict upper part)
#pragma unroll
  for (int j = 0; j < kLuB; ++j) {
    const double v = P[ln + (int64_t)std::min(j, ln) * ld];
    a[j] = (lane < w && j < w && j <= lane) ? v : 0.0;
  }
  static_for<0, kLuB>([&](auto step) {
    constexpr int p = decltype(step)::value;
    if (p < w) {   // (uniform)
      const double d = __builtin_bit_cast(
          double, (uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                      (int)__builtin_bit_cast(uint64_t, a[p]), p) |
                      ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                           (int)(__builtin_bit_cast(uint64_t, a[p]) >> 32), p)
                       << 32));
      if (lane == 0 && !(d > 0.0)) atomicMin(info, col0 + p);
      const double l = __builtin_sqrt(d);
      const double q = a[p] / l;
      a[p] = lane == p ? l : (lane > p ? q : a[p]);
      col[lane] = a[p];
      __syncthreads();   // one wave: orders the column's publication before its reads
      const double lip = a[p];
      stream_pairs<(p + 1) / 2>(col, [&](int j, double ljp) {
        if (j > p) {
          const double prod = lip * ljp;
          a[j] = a[j] - prod;
        }
      });
      __syncthreads();   // every lane has read the column before the next one is published
    }
  });
#pragma unroll
  for (int j = 0; j < kLuB; ++j)
    if (lane < w && j < w && j <= lane) P[lane + (int64_t)j * ld] = a[j];
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
  hipLaunchKernelGGL(chol_base_kernel, dim3(1), dim3(64), 0, s, P, ld, w, info, col0);
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
  hipLaunchKernelGGL(trsm_rows_upper_kernel, dim3((unsigned)grid), dim3(256), 0, s, L, ldl,
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
  hipLaunchKernelGGL(trsm_rows_upper_kernel, dim3((unsigned)grid), dim3(256), 0, s, U,
                     int64_t(1), ldu, w, 0, B, int64_t(1), ldb, rows);
  return hipGetLastError();
}

hipError_t launch_trsm_cols_lower_unit(const double* L, int64_t ldl, int k, double* B,
                                       int64_t ldb, int64_t cols, hipStream_t s) {
  if (k < 1 || k > kLuB) return hipErrorInvalidValue;
  if (cols <= 0) return hipSuccess;
  const int64_t grid = (cols + 63) / 64;
  if (grid >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  // B := L^{-1} B is B^T := B^T L^{-T}: rows of B^T are the columns of B, L^T is unit upper
  hipLaunchKernelGGL(trsm_rows_upper_kernel, dim3((unsigned)grid), dim3(256), 0, s, L, ldl,
                     int64_t(1), k, 1, B, ldb, int64_t(1), cols);
  return hipGetLastError();
}

}  // namespace smx
