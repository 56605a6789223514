// Host-side helpers shared by the library's translation units (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "plan.h"

namespace smx {

// Records a message for strassen_last_error and returns `code`.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
void clear_error();

#define SMX_HIP(call)                                      \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return smx::hip_fail(e_, #call); \
  } while (0)

// The kNumTables operation tables (host copies; the device copies are uploaded per device).
const TableDev* host_tables();
// The product-side table for 0..kMaxLevelsAbc levels (host only).
const std::vector<Product>& host_table(int levels);
// Current device checked (gfx950) and its constant tables uploaded; returns 0 or an error code.
int device_ready(int* dev_out);

// Where a call's workspace comes from.  fixed: the buffer [ptr, ptr + bytes) (a caller's
// workspace, or the library's static scratch), nothing is allocated; otherwise the
// library-owned workspace, grown on demand up to `bytes` (the limit).  fits(b): a workspace of
// b bytes can be had without exceeding the buffer or the limit (a library-owned allocation can
// still fail).
struct WsSource {
  bool fixed = false;
  void* ptr = nullptr;
  size_t bytes = 0;
  const char* what = nullptr;   // name used in error messages (fixed buffers)
  // fixed buffer whose device address is resolved on first use (ptr == nullptr), on the
  // current device
  int (*resolve)(int dev, void** ptr) = nullptr;
  bool fits(size_t b) const { return b <= bytes; }
};
// The workspace of the ordinary entry points: the caller's (strassen_set_workspace) if set,
// else library-owned under the current limit.
WsSource default_workspace();

// Suspends (true) or resumes the kernel-timing event pairs on the calling thread (launches
// recorded into a graph by stream capture must not carry them).
void suspend_timing(bool on);

// Whether one-level ABC stages its sums and runs its products on the classical kernel for
// this shape (given aligned operands with even leading dimensions and the workspace).
bool one_level_staged_shape(int64_t m, int64_t n, int64_t k);

// C := alpha*A*B + beta*C (strassen_dgemm) with its workspace taken from `ws`.
int dgemm(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
          const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int levels,
          int variant, const WsSource& ws, hipStream_t stream);

// C := alpha*op(A)*op(B) + beta*C (strassen_gemm; op = N, T or C) with its workspace from `ws`.
int gemm_t(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
           const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
           int64_t ldc, int levels, int variant, const WsSource& ws, hipStream_t stream);

// One launch of the all-products kernel (operand terms per side: na, nb).
struct ApLaunch {
  FusedArgs f;
  int na, nb;
};
// Whether ABC at `levels` can run on the all-products kernel for these operands, and its
// launches with the outer sums formed in the load (one at one level, seven at two; stream order
// gives every C element its updates in product order).  Returns 0 or an error code.
bool all_products_ok(int64_t m, int64_t k, const double* A, int64_t lda, const double* B,
                     int64_t ldb, const double* C, int64_t ldc, int levels);
int all_products_plan(int64_t m, int64_t n, int64_t k, int levels, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double* C, int64_t ldc, double alpha,
                      double beta, std::vector<ApLaunch>* out);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

}  // namespace smx
