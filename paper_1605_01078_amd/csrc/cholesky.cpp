// Cholesky factorization A = L L^T with Strassen in its trailing updates (strassen_dpotrf_lower).
//
// The paper's future work (Sec. 6) points at the rank-k updates inside LAPACK's blocked
// algorithms; in Cholesky the trailing matrix of every block column receives the symmetric
// rank-nb update  A22 := A22 - L21 L21^T  (lower triangle).  Here that update is split into
// block columns of width bs: below each diagonal block one GEMM  C(i, J) -= L21(i) L21(J)^T  of
// shape (rest) x bs x nb runs through the library's GEMM (Strassen for the large ones, the
// transposed operand packed as strassen_gemm does), and each bs x bs diagonal block is formed
// as a product into a scratch block whose lower triangle is then subtracted (the strict upper
// triangle of A is never written).  The panel factorization and the triangular solve
// L21 := A21 L11^{-T} recurse by halving the width down to 64 columns, so they too are mostly
// products; their base cases are small kernels (kernels_lu.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <mutex>
#include <vector>

#include "../../include/strassen.h"
#include "internal.h"
#include "launch.h"

namespace smx {

namespace {

constexpr int64_t kBase = 64;        // width of the base-case kernels
constexpr int64_t kDiagBlock = 2048; // largest diagonal block of a symmetric update

// Per-device buffers of the factorization: the first failing column (an int) and the scratch
// block the diagonal blocks of the symmetric updates are formed in (grown on demand).
struct CholDevice {
  int* info = nullptr;
  double* w = nullptr;
  size_t w_elems = 0;
};
std::mutex g_chol_mu;
std::vector<CholDevice> g_chol;

int chol_buffers(int dev, size_t w_elems, CholDevice* out) {
  std::lock_guard<std::mutex> lk(g_chol_mu);
  if ((int)g_chol.size() <= dev) g_chol.resize(dev + 1);
  CholDevice& d = g_chol[dev];
  if (!d.info) SMX_HIP(hipMalloc(&d.info, 256));
  if (d.w_elems < w_elems) {
    if (d.w) SMX_HIP(hipFree(d.w));
    d.w = nullptr;
    d.w_elems = 0;
    SMX_HIP(hipMalloc(&d.w, w_elems * sizeof(double)));
    d.w_elems = w_elems;
  }
  *out = d;
  return 0;
}

struct CholCtx {
  int levels;          // Strassen levels of the large updates (-1: strassen_select per update)
  hipStream_t stream;
  WsSource ws;
  int* info;
  double* w;           // scratch for a diagonal block, kDiagBlock^2 doubles
};

// Levels of one update C (m x n) -= A B^T with inner dimension k: large updates (min(m, n) >=
// 2048 and k >= 1024, the shapes where Strassen can pay on this GPU) use the requested levels,
// smaller ones the classical product.
int levels_of(const CholCtx& c, int64_t m, int64_t n, int64_t k, int* variant) {
  *variant = STRASSEN_ABC;
  if (std::min(m, n) < 2048 || k < 1024) return 0;
  if (c.levels >= 0) return c.levels;
  int lv = 0;
  if (strassen_select(m, n, k, 0, &lv, variant) != 0) return -1;
  return lv;
}

// C (m x n) := C - A B^T, A m x k, B n x k.
int update_t(const CholCtx& c, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
             const double* B, int64_t ldb, double* C, int64_t ldc) {
  if (m <= 0 || n <= 0 || k <= 0) return 0;
  int variant = STRASSEN_ABC;
  const int levels = levels_of(c, m, n, k, &variant);
  if (levels < 0) return fail(STRASSEN_ERR_HIP, "selector failed");
  return gemm_t('N', 'T', m, n, k, -1.0, A, lda, B, ldb, 1.0, C, ldc, levels, variant, c.ws,
                c.stream);
}

// Lower triangle of C (n x n) := C - A A^T, A n x k: block columns of width at most
// kDiagBlock; the part below each diagonal block is one product, the diagonal block a product
// into the scratch block followed by the subtraction of its lower triangle.
int syrk_lower(const CholCtx& c, double* C, int64_t ldc, int64_t n, const double* A,
               int64_t lda, int64_t k) {
  if (n <= 0 || k <= 0) return 0;
  for (int64_t j = 0; j < n; j += kDiagBlock) {
    const int64_t bs = std::min(kDiagBlock, n - j);
    int variant = STRASSEN_ABC;
    const int levels = levels_of(c, bs, bs, k, &variant);
    if (levels < 0) return fail(STRASSEN_ERR_HIP, "selector failed");
    if (int rc = gemm_t('N', 'T', bs, bs, k, 1.0, A + j, lda, A + j, lda, 0.0, c.w, bs, levels,
                        variant, c.ws, c.stream))
      return rc;
    SMX_HIP(launch_sub_lower(C + j + j * ldc, ldc, c.w, bs, bs, c.stream));
    if (int rc = update_t(c, n - j - bs, bs, k, A + j + bs, lda, A + j, lda, C + j + bs + j * ldc,
                          ldc))
      return rc;
  }
  return 0;
}

// Split of a width above the base case: half, rounded down to a multiple of 64.
int64_t split(int64_t w) { return std::max<int64_t>(kBase, (w / 2) / kBase * kBase); }

// B (rows x w) := B L^{-T}, L lower triangular w x w.
int trsm_lower_t(const CholCtx& c, const double* L, int64_t ldl, int64_t w, double* B,
                 int64_t ldb, int64_t rows) {
  if (rows <= 0) return 0;
  if (w <= kBase) {
    SMX_HIP(launch_trsm_rows_lower_t(L, ldl, (int)w, B, ldb, rows, c.stream));
    return 0;
  }
  const int64_t w1 = split(w);
  if (int rc = trsm_lower_t(c, L, ldl, w1, B, ldb, rows)) return rc;
  // B2 := B2 - B1 L21^T, L21 = L(w1:w, 0:w1)
  if (int rc = update_t(c, rows, w - w1, w1, B, ldb, L + w1, ldl, B + w1 * ldb, ldb)) return rc;
  return trsm_lower_t(c, L + w1 + w1 * ldl, ldl, w - w1, B + w1 * ldb, ldb, rows);
}

// The w x w diagonal block at P (global column col0): L11 in its lower triangle.
int potrf_block(const CholCtx& c, double* P, int64_t ld, int64_t w, int64_t col0) {
  if (w <= kBase) {
    SMX_HIP(launch_chol_base(P, ld, (int)w, c.info, (int)col0, c.stream));
    return 0;
  }
  const int64_t w1 = split(w);
  if (int rc = potrf_block(c, P, ld, w1, col0)) return rc;
  if (int rc = trsm_lower_t(c, P, ld, w1, P + w1, ld, w - w1)) return rc;
  if (int rc = syrk_lower(c, P + w1 + w1 * ld, ld, w - w1, P + w1, ld, w1)) return rc;
  return potrf_block(c, P + w1 + w1 * ld, ld, w - w1, col0 + w1);
}

}  // namespace

int potrf_lower(int64_t n, double* A, int64_t lda, int64_t nb, int levels, const WsSource& ws,
                hipStream_t stream, int64_t* info_out) {
  clear_error();
  *info_out = 0;
  if (n < 0) return fail(-1, "n = %lld < 0", (long long)n);
  if (n > 0 && A == nullptr) return fail(-2, "A is NULL");
  if (lda < std::max<int64_t>(1, n)) return fail(-3, "lda = %lld < max(1, n)", (long long)lda);
  if (nb < kBase || nb % kBase != 0) return fail(-4, "nb = %lld is not a positive multiple of 64", (long long)nb);
  if (levels < -1 || levels > kMaxLevelsAbc) return fail(-5, "levels = %d not in -1..%d", levels, kMaxLevelsAbc);
  if (n >= INT_MAX) return fail(STRASSEN_ERR_UNSUPPORTED, "n = %lld too large", (long long)n);
  if (n == 0) return 0;
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  CholDevice d;
  if (int rc = chol_buffers(dev, (size_t)kDiagBlock * kDiagBlock, &d)) return rc;
  SMX_HIP(launch_set_int(d.info, INT_MAX, stream));
  const CholCtx c{levels, stream, ws, d.info, d.w};
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t jb = std::min(nb, n - j);
    double* Ajj = A + j + j * lda;
    if (int rc = potrf_block(c, Ajj, lda, jb, j)) return rc;
    const int64_t rest = n - j - jb;
    if (rest <= 0) break;
    // L21 := A21 L11^{-T}, then the symmetric rank-jb update of the trailing lower triangle
    if (int rc = trsm_lower_t(c, Ajj, lda, jb, Ajj + jb, lda, rest)) return rc;
    if (int rc = syrk_lower(c, Ajj + jb + jb * lda, lda, rest, Ajj + jb, lda, jb)) return rc;
  }
  int first = INT_MAX;
  SMX_HIP(hipMemcpyAsync(&first, d.info, sizeof(int), hipMemcpyDeviceToHost, stream));
  SMX_HIP(hipStreamSynchronize(stream));
  *info_out = first == INT_MAX ? 0 : (int64_t)first + 1;
  return 0;
}

}  // namespace smx

extern "C" int strassen_dpotrf_lower(int64_t n, double* A, int64_t lda, int64_t nb, int levels,
                                     int64_t* info, void* stream) {
  int64_t dummy = 0;
  return smx::potrf_lower(n, A, lda, nb, levels, smx::default_workspace(),
                          static_cast<hipStream_t>(stream), info ? info : &dummy);
}
