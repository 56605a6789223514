// libstrassen_blas.so: a drop-in BLAS level-3 dgemm on top of libstrassen.
//
// The paper's implementations are plug-compatible with dgemm (Introduction; Sec. 2.2 states the
// operation with its BLAS interface).  This library exports the two standard entry points with
// their usual signatures, so a program that calls dgemm can be linked against it (or have it
// preloaded) instead of a CPU BLAS, much as NVBLAS sits in front of a GPU BLAS:
//   dgemm_       Fortran calling convention (every argument by reference; hidden string
//                lengths, if the caller passes them, are ignored);
//   cblas_dgemm  the C interface (column- or row-major).
// The member of the Strassen family (classical, one or two levels, ABC / AB / Naive) is chosen
// per call by strassen_select.  A, B and C may be host or device memory (each pointer is
// classified by hipPointerGetAttributes): host operands are copied to the device, the product
// runs on the GPU and C is copied back; the call returns when C holds the result, as a BLAS
// call does.  Invalid arguments are reported as BLAS's xerbla does ("On entry to DGEMM
// parameter number i had an illegal value" on stderr) and C is left unchanged; runtime failures
// (no device, no memory) print the library's message and leave C unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>

#include "../../include/strassen.h"

namespace {

bool is_device(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();   // plain host memory: not an error to keep
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

void illegal(int info) {
  std::fprintf(stderr, " ** On entry to DGEMM  parameter number %2d had an illegal value\n", info);
}

bool trans_of(char t, bool* out) {
  if (t == 'N' || t == 'n') *out = false;
  else if (t == 'T' || t == 't' || t == 'C' || t == 'c') *out = true;
  else return false;
  return true;
}

// A rows x cols column-major matrix (leading dimension ld) on the device: the caller's pointer
// when it is device memory, else a packed device copy (leading dimension rows).
struct DevMat {
  const double* host = nullptr;
  double* dev = nullptr;
  int64_t ld = 0;
  bool owned = false;
};

int to_device(const double* p, int64_t rows, int64_t cols, int64_t ld, bool copy_in, DevMat* out) {
  out->host = p;
  if (is_device(p)) {
    out->dev = const_cast<double*>(p);
    out->ld = ld;
    return 0;
  }
  const int64_t ldd = std::max<int64_t>(1, rows);
  if (hipMalloc(&out->dev, (size_t)ldd * cols * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    std::fprintf(stderr, "strassen dgemm: no device memory for a %lld x %lld operand\n",
                 (long long)rows, (long long)cols);
    return STRASSEN_ERR_ALLOC;
  }
  out->owned = true;
  out->ld = ldd;
  if (copy_in && rows > 0 && cols > 0 &&
      hipMemcpy2D(out->dev, ldd * sizeof(double), p, ld * sizeof(double), rows * sizeof(double),
                  cols, hipMemcpyHostToDevice) != hipSuccess) {
    std::fprintf(stderr, "strassen dgemm: copy to the device failed\n");
    return STRASSEN_ERR_HIP;
  }
  return 0;
}

void release(DevMat* d) {
  if (d->owned && d->dev) (void)hipFree(d->dev);
  d->dev = nullptr;
}

void run(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
         const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
         int64_t ldc) {
  bool ta = false, tb = false;
  int info = 0;
  if (!trans_of(transa, &ta)) info = 1;
  else if (!trans_of(transb, &tb)) info = 2;
  else if (m < 0) info = 3;
  else if (n < 0) info = 4;
  else if (k < 0) info = 5;
  else if (lda < std::max<int64_t>(1, ta ? k : m)) info = 8;
  else if (ldb < std::max<int64_t>(1, tb ? n : k)) info = 10;
  else if (ldc < std::max<int64_t>(1, m)) info = 13;
  if (info) {
    illegal(info);
    return;
  }
  if (m == 0 || n == 0 || ((alpha == 0.0 || k == 0) && beta == 1.0)) return;
  const bool reads_ab = alpha != 0.0 && k > 0;
  DevMat a, b, c;
  int rc = 0;
  if (reads_ab) rc = to_device(A, ta ? k : m, ta ? m : k, lda, true, &a);
  if (!rc && reads_ab) rc = to_device(B, tb ? n : k, tb ? k : n, ldb, true, &b);
  if (!rc) rc = to_device(C, m, n, ldc, beta != 0.0, &c);
  if (!rc) {
    rc = strassen_gemm(transa, transb, m, n, k, alpha, a.dev, reads_ab ? a.ld : std::max<int64_t>(1, ta ? k : m),
                       b.dev, reads_ab ? b.ld : std::max<int64_t>(1, tb ? n : k), beta, c.dev, c.ld,
                       -1, STRASSEN_ABC, nullptr);
    if (rc) std::fprintf(stderr, "strassen dgemm: %s (code %d)\n", strassen_last_error(), rc);
  }
  if (!rc && hipStreamSynchronize(nullptr) != hipSuccess) {
    std::fprintf(stderr, "strassen dgemm: %s\n", hipGetErrorString(hipGetLastError()));
    rc = STRASSEN_ERR_HIP;
  }
  if (!rc && c.owned &&
      hipMemcpy2D(C, ldc * sizeof(double), c.dev, c.ld * sizeof(double), m * sizeof(double), n,
                  hipMemcpyDeviceToHost) != hipSuccess)
    std::fprintf(stderr, "strassen dgemm: copy of C back to the host failed\n");
  release(&a);
  release(&b);
  release(&c);
}

}  // namespace

extern "C" {

void dgemm_(const char* transa, const char* transb, const int* m, const int* n, const int* k,
            const double* alpha, const double* A, const int* lda, const double* B, const int* ldb,
            const double* beta, double* C, const int* ldc) {
  run(*transa, *transb, *m, *n, *k, *alpha, A, *lda, B, *ldb, *beta, C, *ldc);
}

// CBLAS enumerations (values of the reference cblas.h).
enum { kCblasRowMajor = 101, kCblasColMajor = 102 };
enum { kCblasNoTrans = 111, kCblasTrans = 112, kCblasConjTrans = 113 };

void cblas_dgemm(int order, int transa, int transb, int m, int n, int k, double alpha,
                 const double* A, int lda, const double* B, int ldb, double beta, double* C,
                 int ldc) {
  auto code = [](int t) { return t == kCblasNoTrans ? 'N' : (t == kCblasTrans || t == kCblasConjTrans) ? 'T' : '?'; };
  if (order == kCblasColMajor) {
    run(code(transa), code(transb), m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  } else if (order == kCblasRowMajor) {
    // row-major C = op(A) op(B) is column-major C^T = op(B)^T op(A)^T
    run(code(transb), code(transa), n, m, k, alpha, B, ldb, A, lda, beta, C, ldc);
  } else {
    std::fprintf(stderr, " ** On entry to cblas_dgemm parameter number  1 had an illegal value\n");
  }
}

}  // extern "C"
