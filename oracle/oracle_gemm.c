/*
 * CPU oracle for C := alpha*A*B + beta*C — TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this file's library.  The product path (the HIP library) never links,
 * calls or shares code with it.
 *
 * All matrices are column-major: element (i,j) of X is X[i + j*ldX].
 * Built with -O2 -fopenmp -ffp-contract=off so that every multiply and every
 * add is rounded separately, exactly as written below.
 *
 *   oracle_dgemm     — the definition of Sec. 2.1 ("Computing C = alpha A B + C"),
 *                      with the BLAS beta of Sec. 2.2: each c_ij is alpha times the
 *                      sum over p of a_ip*b_pj, summed in increasing p, plus beta*c_ij.
 *   oracle_winograd  — recursive Winograd variant (the Strassen-like scheme of the
 *                      paper's references and future work): seven products whose
 *                      operand sums and C sums reuse one another (15 additions per
 *                      level instead of 18), same padding and base case.
 *   oracle_lu_nopiv  — LU factorization without pivoting, plain elimination (the
 *                      rank-k-update algorithm of the paper's future work, Sec. 6).
 *   oracle_strassen  — classic recursive Strassen (Sec. 3.2), each level being the
 *                      seven operations of Fig. "All operations for one-level
 *                      Strassen" (Sec. 3.1) written out with explicit temporaries.
 *                      Odd dimensions are zero-padded to even at every level, the
 *                      traditional treatment of fringes that Sec. 3.3 mentions.
 *                      The base case is oracle_dgemm's summation.
 */
#include <stdint.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* S := X*Y (overwrite), the plain definition; loops ordered j, p, i so that the
 * sum for each (i,j) is still accumulated in increasing p. */
static void plain_product(int64_t m, int64_t n, int64_t k,
                          const double *X, int64_t ldx,
                          const double *Y, int64_t ldy,
                          double *S, int64_t lds)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        double *s = S + j * lds;
        for (int64_t i = 0; i < m; ++i) s[i] = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double y = Y[p + j * ldy];
            const double *x = X + p * ldx;
            for (int64_t i = 0; i < m; ++i) s[i] = s[i] + x[i] * y;
        }
    }
}

/* C := alpha*S + beta*C; beta == 0 means C is not read (BLAS convention). */
static void scale_add(int64_t m, int64_t n, double alpha, const double *S, int64_t lds,
                      double beta, double *C, int64_t ldc)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            const double t = alpha * S[i + j * lds];
            C[i + j * ldc] = (beta == 0.0) ? t : t + beta * C[i + j * ldc];
        }
}

int oracle_dgemm(int64_t m, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc)
{
    if (m <= 0 || n <= 0) return 0;
    double *S = (double *)calloc((size_t)m * (size_t)n, sizeof(double));
    if (!S) return 1;
    /* BLAS: with alpha == 0 or k == 0, A and B are not referenced. */
    if (k > 0 && alpha != 0.0) plain_product(m, n, k, A, lda, B, ldb, S, m);
    scale_add(m, n, alpha, S, m, beta, C, ldc);
    free(S);
    return 0;
}

/* ---- recursive Strassen ------------------------------------------------ */

/* Copy quadrant (bi,bj) of the rows x cols matrix X into the h x w buffer Q,
 * filling positions that fall outside X with zeros. */
static void get_quadrant(const double *X, int64_t ldx, int64_t rows, int64_t cols,
                         int bi, int bj, int64_t h, int64_t w, double *Q)
{
    for (int64_t j = 0; j < w; ++j)
        for (int64_t i = 0; i < h; ++i) {
            const int64_t r = bi * h + i, c = bj * w + j;
            Q[i + j * h] = (r < rows && c < cols) ? X[r + c * ldx] : 0.0;
        }
}

static void add_into(int64_t len, const double *X, double sx, const double *Y, double sy, double *Z)
{
    for (int64_t e = 0; e < len; ++e) Z[e] = sx * X[e] + sy * Y[e];
}

static void accumulate(int64_t len, double *Z, double s, const double *M)
{
    for (int64_t e = 0; e < len; ++e) Z[e] = Z[e] + s * M[e];
}

/* P := X*Y (overwrite) for X m x k, Y k x n, P m x n (ld = m), using `levels`
 * levels of Strassen and the plain product below them. */
static int strassen_product(int64_t m, int64_t n, int64_t k,
                            const double *X, int64_t ldx, const double *Y, int64_t ldy,
                            double *P, int levels)
{
    if (levels == 0) { plain_product(m, n, k, X, ldx, Y, ldy, P, m); return 0; }
    /* one level: h = ceil(m/2), w = ceil(n/2), d = ceil(k/2) */
    const int64_t h = (m + 1) / 2, w = (n + 1) / 2, d = (k + 1) / 2;
    const int64_t sa = h * d, sb = d * w, sc = h * w;
    double *buf = (double *)calloc((size_t)(4 * sa + 4 * sb + 2 * sa + 2 * sb + 5 * sc), sizeof(double));
    if (!buf) return 1;
    double *A00 = buf, *A01 = A00 + sa, *A10 = A01 + sa, *A11 = A10 + sa;
    double *B00 = A11 + sa, *B01 = B00 + sb, *B10 = B01 + sb, *B11 = B10 + sb;
    double *TA = B11 + sb, *TA2 = TA + sa, *TB = TA2 + sa, *TB2 = TB + sb;
    double *M = TB2 + sb, *C00 = M + sc, *C01 = C00 + sc, *C10 = C01 + sc, *C11 = C10 + sc;
    (void)TA2; (void)TB2;
    get_quadrant(X, ldx, m, k, 0, 0, h, d, A00);
    get_quadrant(X, ldx, m, k, 0, 1, h, d, A01);
    get_quadrant(X, ldx, m, k, 1, 0, h, d, A10);
    get_quadrant(X, ldx, m, k, 1, 1, h, d, A11);
    get_quadrant(Y, ldy, k, n, 0, 0, d, w, B00);
    get_quadrant(Y, ldy, k, n, 0, 1, d, w, B01);
    get_quadrant(Y, ldy, k, n, 1, 0, d, w, B10);
    get_quadrant(Y, ldy, k, n, 1, 1, d, w, B11);
    int rc = 0;
    /* M0 = (A00 + A11)(B00 + B11);  C00 += M0; C11 += M0 */
    add_into(sa, A00, 1, A11, 1, TA); add_into(sb, B00, 1, B11, 1, TB);
    rc |= strassen_product(h, w, d, TA, h, TB, d, M, levels - 1);
    accumulate(sc, C00, 1, M); accumulate(sc, C11, 1, M);
    /* M1 = (A10 + A11) B00;  C10 += M1; C11 -= M1 */
    add_into(sa, A10, 1, A11, 1, TA);
    rc |= strassen_product(h, w, d, TA, h, B00, d, M, levels - 1);
    accumulate(sc, C10, 1, M); accumulate(sc, C11, -1, M);
    /* M2 = A00 (B01 - B11);  C01 += M2; C11 += M2 */
    add_into(sb, B01, 1, B11, -1, TB);
    rc |= strassen_product(h, w, d, A00, h, TB, d, M, levels - 1);
    accumulate(sc, C01, 1, M); accumulate(sc, C11, 1, M);
    /* M3 = A11 (B10 - B00);  C00 += M3; C10 += M3 */
    add_into(sb, B10, 1, B00, -1, TB);
    rc |= strassen_product(h, w, d, A11, h, TB, d, M, levels - 1);
    accumulate(sc, C00, 1, M); accumulate(sc, C10, 1, M);
    /* M4 = (A00 + A01) B11;  C01 += M4; C00 -= M4 */
    add_into(sa, A00, 1, A01, 1, TA);
    rc |= strassen_product(h, w, d, TA, h, B11, d, M, levels - 1);
    accumulate(sc, C01, 1, M); accumulate(sc, C00, -1, M);
    /* M5 = (A10 - A00)(B00 + B01);  C11 += M5 */
    add_into(sa, A10, 1, A00, -1, TA); add_into(sb, B00, 1, B01, 1, TB);
    rc |= strassen_product(h, w, d, TA, h, TB, d, M, levels - 1);
    accumulate(sc, C11, 1, M);
    /* M6 = (A01 - A11)(B10 + B11);  C00 += M6 */
    add_into(sa, A01, 1, A11, -1, TA); add_into(sb, B10, 1, B11, 1, TB);
    rc |= strassen_product(h, w, d, TA, h, TB, d, M, levels - 1);
    accumulate(sc, C00, 1, M);
    /* P = [C00 C01; C10 C11], dropping the zero padding */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            const double *Q = (i < h) ? (j < w ? C00 : C01) : (j < w ? C10 : C11);
            P[i + j * m] = Q[(i % h) + (j % w) * h];
        }
    free(buf);
    return rc;
}

int oracle_strassen(int64_t m, int64_t n, int64_t k, double alpha,
                    const double *A, int64_t lda, const double *B, int64_t ldb,
                    double beta, double *C, int64_t ldc, int levels)
{
    if (m <= 0 || n <= 0) return 0;
    if (levels < 0) return -12;
    double *P = (double *)calloc((size_t)m * (size_t)n, sizeof(double));
    if (!P) return 1;
    int rc = 0;
    if (k > 0 && alpha != 0.0) rc = strassen_product(m, n, k, A, lda, B, ldb, P, levels);
    scale_add(m, n, alpha, P, m, beta, C, ldc);
    free(P);
    return rc;
}

/* ---- recursive Winograd variant ------------------------------------------ */

/* Z := X - Y (or X + Y), elementwise over len entries. */
static void sub_into(int64_t len, const double *X, const double *Y, double *Z)
{
    for (int64_t e = 0; e < len; ++e) Z[e] = X[e] - Y[e];
}

/* P := X*Y (overwrite) with `levels` levels of Winograd's variant of Strassen's
 * algorithm (seven products; the operand sums reuse each other, S2 = S1 - A00,
 * S4 = A01 - S2, T2 = B11 - T1, T4 = T2 - B10, and so do the sums that form C,
 * U2 = M1 + M6, U3 = U2 + M7, U4 = U2 + M5), the plain product below them.
 * Same zero padding of odd dimensions as strassen_product. */
static int winograd_product(int64_t m, int64_t n, int64_t k,
                            const double *X, int64_t ldx, const double *Y, int64_t ldy,
                            double *P, int levels)
{
    if (levels == 0) { plain_product(m, n, k, X, ldx, Y, ldy, P, m); return 0; }
    const int64_t h = (m + 1) / 2, w = (n + 1) / 2, d = (k + 1) / 2;
    const int64_t sa = h * d, sb = d * w, sc = h * w;
    double *buf = (double *)calloc((size_t)(8 * sa + 8 * sb + 11 * sc), sizeof(double));
    if (!buf) return 1;
    double *A00 = buf, *A01 = A00 + sa, *A10 = A01 + sa, *A11 = A10 + sa;
    double *S1 = A11 + sa, *S2 = S1 + sa, *S3 = S2 + sa, *S4 = S3 + sa;
    double *B00 = S4 + sa, *B01 = B00 + sb, *B10 = B01 + sb, *B11 = B10 + sb;
    double *T1 = B11 + sb, *T2 = T1 + sb, *T3 = T2 + sb, *T4 = T3 + sb;
    double *M[8];
    M[1] = T4 + sb;
    for (int i = 2; i <= 7; ++i) M[i] = M[i - 1] + sc;
    double *U2 = M[7] + sc, *U3 = U2 + sc, *Q = U3 + sc;
    get_quadrant(X, ldx, m, k, 0, 0, h, d, A00);
    get_quadrant(X, ldx, m, k, 0, 1, h, d, A01);
    get_quadrant(X, ldx, m, k, 1, 0, h, d, A10);
    get_quadrant(X, ldx, m, k, 1, 1, h, d, A11);
    get_quadrant(Y, ldy, k, n, 0, 0, d, w, B00);
    get_quadrant(Y, ldy, k, n, 0, 1, d, w, B01);
    get_quadrant(Y, ldy, k, n, 1, 0, d, w, B10);
    get_quadrant(Y, ldy, k, n, 1, 1, d, w, B11);
    add_into(sa, A10, 1, A11, 1, S1);          /* S1 = A10 + A11 */
    sub_into(sa, S1, A00, S2);                 /* S2 = S1 - A00  */
    sub_into(sa, A00, A10, S3);                /* S3 = A00 - A10 */
    sub_into(sa, A01, S2, S4);                 /* S4 = A01 - S2  */
    sub_into(sb, B01, B00, T1);                /* T1 = B01 - B00 */
    sub_into(sb, B11, T1, T2);                 /* T2 = B11 - T1  */
    sub_into(sb, B11, B01, T3);                /* T3 = B11 - B01 */
    sub_into(sb, T2, B10, T4);                 /* T4 = T2 - B10  */
    int rc = 0;
    rc |= winograd_product(h, w, d, A00, h, B00, d, M[1], levels - 1);   /* M1 = A00 B00 */
    rc |= winograd_product(h, w, d, A01, h, B10, d, M[2], levels - 1);   /* M2 = A01 B10 */
    rc |= winograd_product(h, w, d, S4, h, B11, d, M[3], levels - 1);    /* M3 = S4 B11  */
    rc |= winograd_product(h, w, d, A11, h, T4, d, M[4], levels - 1);    /* M4 = A11 T4  */
    rc |= winograd_product(h, w, d, S1, h, T1, d, M[5], levels - 1);     /* M5 = S1 T1   */
    rc |= winograd_product(h, w, d, S2, h, T2, d, M[6], levels - 1);     /* M6 = S2 T2   */
    rc |= winograd_product(h, w, d, S3, h, T3, d, M[7], levels - 1);     /* M7 = S3 T3   */
    add_into(sc, M[1], 1, M[6], 1, U2);        /* U2 = M1 + M6 */
    add_into(sc, U2, 1, M[7], 1, U3);          /* U3 = U2 + M7 */
    /* the four C blocks: C00 = M1 + M2, C01 = (U2 + M5) + M3, C10 = U3 - M4,
     * C11 = U3 + M5 */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            const int64_t e = (i % h) + (j % w) * h;
            double v;
            if (i < h && j < w) v = M[1][e] + M[2][e];
            else if (i < h) v = (U2[e] + M[5][e]) + M[3][e];
            else if (j < w) v = U3[e] - M[4][e];
            else v = U3[e] + M[5][e];
            P[i + j * m] = v;
        }
    (void)Q;
    free(buf);
    return rc;
}

int oracle_winograd(int64_t m, int64_t n, int64_t k, double alpha,
                    const double *A, int64_t lda, const double *B, int64_t ldb,
                    double beta, double *C, int64_t ldc, int levels)
{
    if (m <= 0 || n <= 0) return 0;
    if (levels < 0) return -12;
    double *P = (double *)calloc((size_t)m * (size_t)n, sizeof(double));
    if (!P) return 1;
    int rc = 0;
    if (k > 0 && alpha != 0.0) rc = winograd_product(m, n, k, A, lda, B, ldb, P, levels);
    scale_add(m, n, alpha, P, m, beta, C, ldc);
    free(P);
    return rc;
}

/* ---- LU factorization without pivoting ------------------------------------ */

/* A = L U in place for the n x n matrix A (column-major, lda): L unit lower
 * triangular below the diagonal, U upper triangular on and above it, by the
 * plain right-looking elimination: for each p, the multipliers
 * l_ip = a_ip / a_pp (i > p) replace column p below the diagonal, then
 * a_ij := a_ij - l_ip a_pj for i, j > p.  No pivoting: the leading principal
 * minors must be nonzero (as in a diagonally dominant matrix).  Returns p + 1
 * if the pivot a_pp is exactly zero (A is then partly factored), else 0. */
int oracle_lu_nopiv(int64_t n, double *A, int64_t lda)
{
    for (int64_t p = 0; p < n; ++p) {
        const double piv = A[p + p * lda];
        if (piv == 0.0) return (int)(p + 1);
        for (int64_t i = p + 1; i < n; ++i) A[i + p * lda] = A[i + p * lda] / piv;
#pragma omp parallel for schedule(static)
        for (int64_t j = p + 1; j < n; ++j) {
            const double u = A[p + j * lda];
            double *col = A + j * lda;
            const double *l = A + p * lda;
            for (int64_t i = p + 1; i < n; ++i) col[i] = col[i] - l[i] * u;
        }
    }
    return 0;
}

/* A = L L^T in place for the symmetric positive definite n x n matrix A
 * (column-major, lda; only the lower triangle is read and written): the plain
 * right-looking Cholesky factorization.  For each p: l_pp = sqrt(a_pp), the
 * column below is divided by it (l_ip = a_ip / l_pp, i > p), then the
 * trailing lower triangle is reduced, a_ij := a_ij - l_ip l_jp for i >= j > p.
 * Returns p + 1 if a_pp is not positive (the leading minor of order p + 1 is
 * not positive definite; A is then partly factored), else 0. */
int oracle_cholesky_lower(int64_t n, double *A, int64_t lda)
{
    for (int64_t p = 0; p < n; ++p) {
        const double d = A[p + p * lda];
        if (!(d > 0.0)) return (int)(p + 1);
        const double l = sqrt(d);
        A[p + p * lda] = l;
        for (int64_t i = p + 1; i < n; ++i) A[i + p * lda] = A[i + p * lda] / l;
#pragma omp parallel for schedule(static)
        for (int64_t j = p + 1; j < n; ++j) {
            const double ljp = A[j + p * lda];
            double *col = A + j * lda;
            const double *lp = A + p * lda;
            for (int64_t i = j; i < n; ++i) col[i] = col[i] - lp[i] * ljp;
        }
    }
    return 0;
}

/* Compensated dot products (Ogita, Rump and Oishi's Dot2: TwoProduct by
 * Dekker splitting, TwoSum by Knuth), used only to measure how far a result
 * lies from the exact product at small sizes.  C := alpha*A*B + beta*C with
 * the sum over p carried in twice the working precision. */
static void two_sum(double a, double b, double *s, double *e)
{
    const double x = a + b, z = x - a;
    *s = x;
    *e = (a - (x - z)) + (b - z);
}
static void split(double a, double *hi, double *lo)
{
    const double c = 134217729.0 * a; /* 2^27 + 1 */
    const double h = c - (c - a);
    *hi = h;
    *lo = a - h;
}
static void two_prod(double a, double b, double *p, double *e)
{
    double ah, al, bh, bl;
    const double x = a * b;
    split(a, &ah, &al);
    split(b, &bh, &bl);
    *p = x;
    *e = al * bl - (((x - ah * bh) - al * bh) - ah * bl);
}

int oracle_dgemm_dot2(int64_t m, int64_t n, int64_t k, double alpha,
                      const double *A, int64_t lda, const double *B, int64_t ldb,
                      double beta, double *C, int64_t ldc)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0, c = 0.0;
            for (int64_t p = 0; p < k; ++p) {
                double h, r, q;
                two_prod(A[i + p * lda], B[p + j * ldb], &h, &r);
                two_sum(s, h, &s, &q);
                c = c + (q + r);
            }
            const double t = alpha * (s + c);
            C[i + j * ldc] = (beta == 0.0) ? t : t + beta * C[i + j * ldc];
        }
    return 0;
}
