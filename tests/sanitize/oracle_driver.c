/* The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every function on small
 * ragged shapes with exactly sized heap operands (so that a read or write one element past a
 * matrix is reported), checked against each other.  Exit status 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_dgemm(int64_t m, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double beta, double *C, int64_t ldc);
int oracle_strassen(int64_t m, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double beta, double *C, int64_t ldc, int levels);
int oracle_winograd(int64_t m, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double beta, double *C, int64_t ldc, int levels);
int oracle_lu_nopiv(int64_t n, double *A, int64_t lda);
int oracle_dgemm_dot2(int64_t m, int64_t n, int64_t k, double alpha, const double *A,
                      int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                      int64_t ldc);

static uint64_t state = 12345;
static double small_int(void) {   /* integers in [-4, 4]: every product and sum is exact */
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)((int)((state >> 33) % 9) - 4);
}

static double *matrix(int64_t rows, int64_t cols, int64_t ld) {
  double *x = (double *)malloc((size_t)(ld * (cols - 1) + rows) * sizeof(double));
  for (int64_t j = 0; j < cols; ++j)
    for (int64_t i = 0; i < rows; ++i) x[i + j * ld] = small_int();
  return x;
}

static int failures = 0;
static void expect(int ok, const char *what, int64_t m, int64_t n, int64_t k, int lv) {
  if (!ok) {
    fprintf(stderr, "FAIL %s m=%lld n=%lld k=%lld levels=%d\n", what, (long long)m,
            (long long)n, (long long)k, lv);
    ++failures;
  }
}

int main(void) {
  const int64_t sizes[] = {1, 2, 3, 5, 8, 9, 17};
  const int ns = (int)(sizeof sizes / sizeof sizes[0]);
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b)
      for (int c = 0; c < ns; ++c) {
        const int64_t m = sizes[a], n = sizes[b], k = sizes[c];
        const int64_t lda = m + (a & 1), ldb = k + (b & 1), ldc = m + (c & 1);
        double *A = matrix(m, k, lda), *B = matrix(k, n, ldb), *C0 = matrix(m, n, ldc);
        double *R = matrix(m, n, ldc), *S = matrix(m, n, ldc);
        for (int64_t i = 0; i < ldc * (n - 1) + m; ++i) R[i] = C0[i];
        expect(oracle_dgemm(m, n, k, 1.0, A, lda, B, ldb, 1.0, R, ldc) == 0, "dgemm", m, n, k, 0);
        for (int lv = 0; lv <= 3; ++lv)
          for (int w = 0; w < 3; ++w) {
            for (int64_t i = 0; i < ldc * (n - 1) + m; ++i) S[i] = C0[i];
            int rc;
            if (w == 0) rc = oracle_strassen(m, n, k, 1.0, A, lda, B, ldb, 1.0, S, ldc, lv);
            else if (w == 1) rc = oracle_winograd(m, n, k, 1.0, A, lda, B, ldb, 1.0, S, ldc, lv);
            else rc = oracle_dgemm_dot2(m, n, k, 1.0, A, lda, B, ldb, 1.0, S, ldc);
            expect(rc == 0, "rc", m, n, k, lv);
            for (int64_t j = 0; j < n; ++j)
              for (int64_t i = 0; i < m; ++i)
                if (S[i + j * ldc] != R[i + j * ldc]) {   /* integers: exact */
                  expect(0, w == 0 ? "strassen" : w == 1 ? "winograd" : "dot2", m, n, k, lv);
                  j = n;
                  break;
                }
          }
        free(A); free(B); free(C0); free(R); free(S);
      }
  /* LU of a diagonally dominant matrix: L U recovers it */
  for (int64_t n = 1; n <= 33; n += 8) {
    const int64_t ld = n + 1;
    double *A = matrix(n, n, ld), *F = matrix(n, n, ld);
    for (int64_t i = 0; i < n; ++i) A[i + i * ld] = 8.0 * (double)n;
    for (int64_t i = 0; i < ld * (n - 1) + n; ++i) F[i] = A[i];
    expect(oracle_lu_nopiv(n, F, ld) == 0, "lu rc", n, n, n, 0);
    double err = 0.0;
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = 0; p <= (i < j ? i : j); ++p)
          s += (p == i ? 1.0 : F[i + p * ld]) * F[p + j * ld];
        err = fmax(err, fabs(s - A[i + j * ld]));
      }
    expect(err < 1e-9 * n * n, "lu", n, n, n, 0);
    free(A); free(F);
  }
  if (failures) return 1;
  printf("oracle checks passed\n");
  return 0;
}
