// LU factorization without pivoting with Strassen in its rank-k updates (strassen_dgetrf_nopiv).
//
// The paper's future work (Sec. 6) notes that the blocked algorithms underneath LAPACK cast
// most of their computation as rank-k updates, and asks how ABC Strassen can accelerate them.
// This is the right-looking blocked LU: for each block column of width nb, the panel below the
// diagonal is factored, the block row to its right is solved against the panel's unit lower
// triangle, and the trailing matrix receives the rank-nb update  A22 := A22 - L21 U12, a GEMM
// of shape (n - j - nb) x (n - j - nb) x nb that runs through strassen_dgemm.  The panel and the
// triangular solves are recursive (halving the width down to 64 columns), so they too are mostly
// matrix products, which run on the same GEMM; their 64-wide base cases are small kernels
// (kernels_lu.hip).
//
// No pivoting: every leading principal minor must be nonzero, as it is for diagonally dominant
// matrices; a zero pivot is not detected (it yields infinities or NaNs).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/strassen.h"
#include "internal.h"
#include "launch.h"

namespace smx {

namespace {

constexpr int64_t kBase = 64;

struct LuCtx {
  int levels;          // Strassen levels of the large updates (-1: strassen_select per update)
  hipStream_t stream;
  WsSource ws;
};

// C := C - A B.  Updates whose output and inner dimension are large (min(m, n) >= 2048 and
// k >= 1024, the shapes where Strassen can pay on this GPU) use the requested levels; smaller
// ones the classical product.
int update(const LuCtx& c, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
           const double* B, int64_t ldb, double* C, int64_t ldc) {
  if (m <= 0 || n <= 0 || k <= 0) return 0;
  int levels = 0, variant = STRASSEN_ABC;
  if (std::min(m, n) >= 2048 && k >= 1024) {
    if (c.levels >= 0) {
      levels = c.levels;
    } else if (int rc = strassen_select(m, n, k, 0, &levels, &variant)) {
      return rc;
    }
  }
  return dgemm(m, n, k, -1.0, A, lda, B, ldb, 1.0, C, ldc, levels, variant, c.ws, c.stream);
}

// Split of a width above the base case: half, rounded down to a multiple of 64.
int64_t split(int64_t w) { return std::max<int64_t>(kBase, (w / 2) / kBase * kBase); }

// B (k x cols) := L^{-1} B, L unit lower triangular.
int trsm_lower_unit(const LuCtx& c, const double* L, int64_t ldl, int64_t k, double* B,
                    int64_t ldb, int64_t cols) {
  if (k <= kBase) {
    SMX_HIP(launch_trsm_cols_lower_unit(L, ldl, (int)k, B, ldb, cols, c.stream));
    return 0;
  }
  const int64_t k1 = split(k);
  if (int rc = trsm_lower_unit(c, L, ldl, k1, B, ldb, cols)) return rc;
  if (int rc = update(c, k - k1, cols, k1, L + k1, ldl, B, ldb, B + k1, ldb)) return rc;
  return trsm_lower_unit(c, L + k1 + k1 * ldl, ldl, k - k1, B + k1, ldb, cols);
}

// B (rows x w) := B U^{-1}, U upper triangular.
int trsm_upper_right(const LuCtx& c, const double* U, int64_t ldu, int64_t w, double* B,
                     int64_t ldb, int64_t rows) {
  if (w <= kBase) {
    SMX_HIP(launch_trsm_rows_upper(U, ldu, (int)w, B, ldb, rows, c.stream));
    return 0;
  }
  const int64_t w1 = split(w);
  if (int rc = trsm_upper_right(c, U, ldu, w1, B, ldb, rows)) return rc;
  if (int rc = update(c, rows, w - w1, w1, B, ldb, U + w1 * ldu, ldu, B + w1 * ldb, ldb)) return rc;
  return trsm_upper_right(c, U + w1 + w1 * ldu, ldu, w - w1, B + w1 * ldb, ldb, rows);
}

// The m x w panel at P (m >= w): its top w x w block becomes L11 \ U11, the rows below L21.
int panel(const LuCtx& c, double* P, int64_t ld, int64_t m, int64_t w) {
  if (w <= kBase) {
    SMX_HIP(launch_lu_base(P, ld, (int)w, c.stream));
    if (m > w) return trsm_upper_right(c, P, ld, w, P + w, ld, m - w);
    return 0;
  }
  const int64_t w1 = split(w);
  if (int rc = panel(c, P, ld, m, w1)) return rc;
  if (int rc = trsm_lower_unit(c, P, ld, w1, P + w1 * ld, ld, w - w1)) return rc;
  if (int rc = update(c, m - w1, w - w1, w1, P + w1, ld, P + w1 * ld, ld, P + w1 + w1 * ld, ld))
    return rc;
  return panel(c, P + w1 + w1 * ld, ld, m - w1, w - w1);
}

}  // namespace

int getrf_nopiv(int64_t n, double* A, int64_t lda, int64_t nb, int levels, const WsSource& ws,
                hipStream_t stream) {
  clear_error();
  if (n < 0) return fail(-1, "n = %lld < 0", (long long)n);
  if (n > 0 && A == nullptr) return fail(-2, "A is NULL");
  if (lda < std::max<int64_t>(1, n)) return fail(-3, "lda = %lld < max(1, n)", (long long)lda);
  if (nb < kBase || nb % kBase != 0) return fail(-4, "nb = %lld is not a positive multiple of 64", (long long)nb);
  if (levels < -1 || levels > kMaxLevelsAbc) return fail(-5, "levels = %d not in -1..%d", levels, kMaxLevelsAbc);
  if (n == 0) return 0;
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  const LuCtx c{levels, stream, ws};
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t jb = std::min(nb, n - j);
    double* Ajj = A + j + j * lda;
    if (int rc = panel(c, Ajj, lda, n - j, jb)) return rc;
    const int64_t rest = n - j - jb;
    if (rest <= 0) break;
    // U12 := L11^{-1} A12, then the rank-jb update of the trailing matrix
    if (int rc = trsm_lower_unit(c, Ajj, lda, jb, Ajj + jb * lda, lda, rest)) return rc;
    if (int rc = update(c, rest, rest, jb, Ajj + jb, lda, Ajj + jb * lda, lda,
                        Ajj + jb + jb * lda, lda))
      return rc;
  }
  return 0;
}

}  // namespace smx

extern "C" int strassen_dgetrf_nopiv(int64_t n, double* A, int64_t lda, int64_t nb, int levels,
                                     void* stream) {
  return smx::getrf_nopiv(n, A, lda, nb, levels, smx::default_workspace(),
                          static_cast<hipStream_t>(stream));
}
