/*
 * strassen.h — one- and two-level Strassen matrix multiplication on AMD MI355X (gfx950).
 *
 * Implements the family of practical Strassen implementations of Huang, Smith, Henry and
 * van de Geijn, "Implementing Strassen's Algorithm with BLIS" (arXiv 1605.01078):
 *
 *   C := alpha * A * B + beta * C                                 (Sec. 2.1, Sec. 2.2)
 *
 * computed with `levels` levels of Strassen, each product being the general operation
 *
 *   M = (sum_s delta_s X_s)(sum_t eps_t V_t);   C_r += alpha * gamma_r * M    (eq. e:straprim4)
 *
 * over the sub-blocks of the 2^L x 2^L partition of A, B and C given by the one-level table
 * (Fig. "All operations for one-level Strassen") and the two-level table (Fig. "Computations
 * for two-level Strassen", built as the Kronecker composition of the one-level table, Sec. 3.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Column-major storage: element (i,j) of X is X[i + j*ldX].  A is m x k (lda >= max(1,m)),
 *    B is k x n (ldb >= max(1,k)), C is m x n (ldc >= max(1,m)).  strassen_gemm takes
 *    transposed operands (BLAS transa / transb); the other entry points take none.
 *  - A, B, C are DEVICE pointers owned by the caller.  The library never frees or retains
 *    them.  A and B are only read.  C must not overlap A or B.
 *  - Dimensions that are not multiples of 2^L are handled inside the kernels: every sub-block
 *    has ceil(m/2^L) x ceil(k/2^L) (etc.) elements, positions past the matrix read as zero
 *    and are never written (Sec. 3.3, "Practical considerations", fringes).
 *  - beta is applied once to every element of C, at the first update that touches it; with
 *    beta == 0 C is write-only (NaN/Inf already in C do not propagate), as in BLAS.
 *  - alpha == 0 or k == 0: A and B are not read; C := beta*C (nothing at all when beta == 1).
 *    m == 0 or n == 0: nothing is done.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue work and return;
 *    errors that can be detected on the host are reported on return, kernel faults surface
 *    at the next synchronisation.  Calls on one stream execute in order.
 *  - Return value: 0 on success; -i when the i-th argument (1-based) is invalid (nothing is
 *    enqueued and C is untouched); a positive STRASSEN_ERR_* code for runtime failures.
 *    strassen_last_error() gives a message for the calling thread's last failure.
 *  - Results are deterministic: the same call on the same data gives bitwise identical C.
 *    For a given number of levels the three variants give bitwise identical C.
 */
#ifndef STRASSEN_MI355X_H
#define STRASSEN_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Variants of Sec. 4.1 ("Variations on a theme"). */
enum strassen_variant {
    STRASSEN_ABC = 0,   /* sums formed in the operand load, products added to every C
                           destination in the kernel epilogue; runs without workspace
                           (staging its sums where workspace is available is faster)   */
    STRASSEN_AB = 1,    /* sums formed in the operand load, products stored to explicit
                           temporaries M_r, C assembled from them by a second kernel    */
    STRASSEN_NAIVE = 2  /* explicit operand-sum temporaries, plain GEMM on them, then
                           the same C assembly as AB                                    */
};

/* Runtime error codes (positive). */
enum strassen_error {
    STRASSEN_OK = 0,
    STRASSEN_ERR_HIP = 1,        /* a HIP runtime call failed (message has the HIP error)  */
    STRASSEN_ERR_ALLOC = 2,      /* workspace allocation failed / caller workspace too small */
    STRASSEN_ERR_UNSUPPORTED = 3,/* valid arguments the library cannot run (e.g. sizes past
                                    the 32-bit tile grid)                                    */
    STRASSEN_ERR_NO_DEVICE = 4   /* no gfx950 device is visible                            */
};

/* Precisions of the reduced-precision mode (strassen_gemm_ex). */
enum strassen_compute {
    STRASSEN_COMPUTE_F64 = 0,    /* FP64 products on FP64 MFMA (same as strassen_dgemm)     */
    STRASSEN_COMPUTE_BF16 = 1,   /* operand sums rounded to bf16, FP32-accumulated MFMA     */
    STRASSEN_COMPUTE_BF16X3 = 2  /* sums split x = hi + lo (hi = bf16(x), lo = bf16(x - hi)),
                                    product hi*hi + hi*lo + lo*hi, FP32 accumulation        */
};
enum strassen_precision { STRASSEN_PREC_F32 = 0, STRASSEN_PREC_F64 = 1 };

/*
 * strassen_dgemm — C := alpha*A*B + beta*C with `levels` levels of Strassen.
 *   levels : 0 (classical GEMM on FP64 MFMA, the effective-GFLOPS yardstick), 1, 2 or 3.
 *   variant: STRASSEN_ABC, STRASSEN_AB or STRASSEN_NAIVE (ignored when levels == 0; three
 *            levels run ABC only: -13 for the others).
 * Three levels (343 products, eq. e:straprim4 with L = 3) stage the operand sums of the two
 * upper levels in workspace (five m/2 x k/2 and five k/2 x n/2 slots, five m/4 x k/4 and five
 * k/4 x n/4 slots reused per top-level product) and run the one-level fused kernel for each of
 * the 49 upper products, adding its seven products into up to four destination blocks; every C
 * element receives its updates in increasing product index.  m and k must be multiples of 16
 * and n of 8 with aligned operands of even leading dimensions, else block-padded copies are
 * made (as below).  The workspace is required (STRASSEN_ERR_ALLOC when it cannot be had).
 * The general operation is eq. (e:straprim1) at one level and eq. (e:straprim3) at two.
 * AB runs its products on the fused kernel of ABC, stored to the temporaries instead of added to
 * C (one level; two levels over staged outer sums), on block-padded copies of A and B where
 * their layout does not fit that kernel (as ABC below; C is updated in place by the assembly)
 * and a launch has at least 192 tile positions of 64 x 64 (below that the general tile kernel
 * is faster than the copies), else on the general tile kernel (also where a tile configuration
 * 0..3 forces it, or a caller workspace is too small for the copies and staging); the results
 * are the same bits.
 * AB and NAIVE use a library-owned workspace (grown on demand, kept until
 * strassen_release_workspace or process exit) unless strassen_set_workspace gave one;
 * strassen_workspace_size reports its size.  ABC needs no workspace (Sec. 4.1): it can always
 * run without one, and only uses one where it is available, to stage its outer-level operand
 * sums at two levels (the ten two-term sums of the one-level
 * table over the 2 x 2 outer blocks, formed once by a streaming pass; the seven outer products
 * then run the one-level fused kernel on them and update C in place, bitwise as without
 * staging): by default where (m/2)(n/2) >= 2048^2 and k >= 2048 and a library-owned or large
 * enough caller workspace is available.  A workspace (the caller's, or the library's under
 * strassen_set_workspace_limit) too small for the ten sums but holding one m/2 x k/2 and one
 * k/2 x n/2 slot (a fifth of it) stages one outer product's sums at a time, just before its
 * launch (each sum still formed once; the same bits); smaller still, the sums are formed in
 * the load.  At one level ABC likewise stages its five sums per side (m/2 x k/2 and k/2 x n/2
 * slots, by the same streaming pass over the four quadrants) where m and k are multiples of 4,
 * n is even, the operands fit the classical kernel's layout, k/2 >= 2048, the 256 x 128 tiles
 * of a product fill whole rounds of the 256 CUs (at least 95% of the last one) and k/2 >= 4096
 * or there are at least 1024 tiles: the seven products then run on the classical kernel, one
 * launch each
 * in product order, adding the product to its one or two C quadrants in the epilogue (beta at a
 * quadrant's first update): bitwise the result of the all-products kernel.  A workspace that
 * holds one slot per side but not ten stages one product's sums just before its launch; with
 * less, the all-products kernel runs (no workspace).
 * ABC at levels >= 1 runs on block-padded copies of the operands that do not fit the fused
 * kernel's layout (m or k not a multiple of 2^(L+1), an operand not 16-byte aligned or with an
 * odd leading dimension; B and C also where staging needs n % 4 == 0): every sub-block of the
 * partition is stored with an even extent, the extra rows and columns zero, and C is copied
 * back.  The result is bitwise that of the unpadded computation; the copies take workspace
 * (reported by strassen_workspace_size for aligned operands with even leading dimensions) and
 * are skipped, with the same result, when a caller workspace is too small for them, when
 * they would exceed the limit of strassen_set_workspace_limit, or when the library-owned
 * allocation fails: ABC then runs its workspace-free path (the all-products kernel in place,
 * with the two-level outer sums formed in the load, or the general tile kernel).
 * The general tile kernel (classical levels = 0, AB and Naive where they do not run the fused
 * kernel, and ABC where neither fused form applies) addresses each tile with 32-bit byte
 * offsets: a leading dimension of 2^21 - 1 or more on such a path returns
 * STRASSEN_ERR_UNSUPPORTED before anything is enqueued (decided on the host, before any device
 * call); the fused paths accept leading dimensions up to their block-padded copies' limits.
 * Argument positions for -i: m=1 n=2 k=3 alpha=4 A=5 lda=6 B=7 ldb=8 beta=9 C=10 ldc=11
 * levels=12 variant=13.
 */
int strassen_dgemm(int64_t m, int64_t n, int64_t k, double alpha,
                   const double *A, int64_t lda, const double *B, int64_t ldb,
                   double beta, double *C, int64_t ldc,
                   int levels, int variant, void *stream);

/*
 * strassen_dgemm_winograd — C := alpha*A*B + beta*C with `levels` (1 or 2) levels of Winograd's
 * variant of Strassen's algorithm (a Strassen-like scheme among the paper's references and
 * future work), in the ABC form: seven products per level,
 *   M1 = A00 B00, M2 = A01 B10, M3 = S4 B11, M4 = A11 T4, M5 = S1 T1, M6 = S2 T2, M7 = S3 T3,
 * with the operand sums formed in the load by Winograd's chain (S1 = A10 + A11, S2 = S1 - A00,
 * S3 = A00 - A10, S4 = A01 - S2; T1 = B01 - B00, T2 = B11 - T1, T3 = B11 - B01, T4 = T2 - B10:
 * eight additions per level where Strassen's table needs ten), and every product added in the
 * epilogue to each C block it reaches (C00 = M1 + M2, C01 = M1 + M3 + M5 + M6,
 * C10 = M1 - M4 + M6 + M7, C11 = M1 + M5 + M6 + M7), in product order.  Two levels stage the
 * outer chain sums in workspace (four m/2 x k/2 and four k/2 x n/2 slots) and run one launch
 * per outer product.  One level, where one-level ABC runs its products on the classical kernel
 * (see strassen_dgemm) and the workspace holds the eight chain-sum slots, stages the chain sums
 * over the quadrants and runs the seven products on the classical kernel, each added to every
 * C quadrant it reaches (the same bits; without that workspace, the fused kernel as above).
 * Sizes, layouts and conventions as strassen_dgemm; block-padded copies
 * where m or k is not a multiple of 2^(L+1), n (two levels) not a multiple of 4, an operand is
 * not 16-byte aligned or a leading dimension odd.  Workspace (copies, staging:
 * strassen_workspace_size_winograd) is required: STRASSEN_ERR_ALLOC when it cannot be had.
 * Argument positions for -i as strassen_dgemm, levels = 12.
 */
int strassen_dgemm_winograd(int64_t m, int64_t n, int64_t k, double alpha,
                            const double *A, int64_t lda, const double *B, int64_t ldb,
                            double beta, double *C, int64_t ldc, int levels, void *stream);
/* Workspace bytes of strassen_dgemm_winograd for aligned operands with even leading dimensions.
 * Returns 0 or -i (m=1 n=2 k=3 levels=4 bytes=5). */
int strassen_workspace_size_winograd(int64_t m, int64_t n, int64_t k, int levels, size_t *bytes);

/*
 * strassen_dgetrf_nopiv — LU factorization without pivoting, A = L U in place (L unit lower
 * triangular, stored below the diagonal; U upper triangular, on and above it), with Strassen in
 * its rank-k updates: the blocked algorithms under LAPACK cast their work as rank-k updates,
 * and the paper's future work (Sec. 6) asks how ABC Strassen can accelerate them.  Right-looking
 * blocked LU with block width nb (a positive multiple of 64; nb >= n makes it fully
 * recursive): per block column the panel is factored (recursively, halving its width down to
 * 64 columns), the block row to its right is solved against the panel's unit lower triangle
 * (recursively), and the trailing matrix gets the rank-nb update A22 := A22 - L21 U12 through
 * strassen_dgemm.  Every update with min(m, n) >= 2048 and k >= 1024 runs with `levels` levels
 * (0..3; -1: strassen_select chooses per update), smaller ones classical.  A is an n x n
 * column-major device matrix (lda >= max(1, n)).  No pivoting: every leading principal minor
 * must be nonzero (e.g. a diagonally dominant matrix); a zero pivot is not detected and yields
 * infinities or NaNs.  Uses the workspace of the products it calls.  Asynchronous on `stream`.
 * Returns 0 or -i (n=1 A=2 lda=3 nb=4 levels=5), or a positive error of a product.
 */
int strassen_dgetrf_nopiv(int64_t n, double *A, int64_t lda, int64_t nb, int levels,
                          void *stream);

/*
 * strassen_dpotrf_lower — Cholesky factorization A = L L^T of the symmetric positive definite
 * n x n matrix A (column-major, device memory; only the lower triangle is read, and L overwrites
 * it; the strict upper triangle is not touched), with Strassen in its trailing updates (the
 * rank-k updates of LAPACK's blocked algorithms that the paper's future work, Sec. 6, points
 * at).  Right-looking, block columns of nb (a positive multiple of 64): the diagonal block is
 * factored recursively (64-column base kernel), L21 := A21 L11^{-T} by a recursive triangular
 * solve, and the trailing lower triangle receives A22 -= L21 L21^T in block columns of at most
 * 2048: below each diagonal block one GEMM through the library (levels: 0..3 for the updates
 * with min(m, n) >= 2048 and k >= 1024, -1 = strassen_select per update; smaller ones
 * classical), each diagonal block a product into a scratch block whose lower triangle is
 * subtracted.  *info (host, may be NULL) receives 0, or j + 1 when the leading minor of order
 * j + 1 is not positive definite (the first non-positive pivot; the factorization then
 * continues with NaN).  Enqueued on `stream`; returns after it completes (reading info
 * synchronises the stream).  Uses the library workspace (as strassen_gemm with a transposed
 * operand) and a scratch block of 2048^2 doubles per device, kept until process exit.
 * Returns 0, -1 n < 0, -2 A NULL, -3 lda < max(1, n), -4 nb not a positive multiple of 64,
 * -5 levels not in -1..3, or a positive error.
 */
int strassen_dpotrf_lower(int64_t n, double *A, int64_t lda, int64_t nb, int levels,
                          int64_t *info, void *stream);

/*
 * strassen_gemm — the full dgemm interface of Sec. 2.2 with transposes:
 *   C := alpha * op(A) * op(B) + beta * C,   op(X) = X (trans 'N'/'n') or X^T ('T'/'t'/'C'/'c')
 * op(A) is m x k (A is m x k with lda >= max(1,m), or k x m with lda >= max(1,k) when
 * transposed), op(B) is k x n (B is k x n with ldb >= max(1,k), or n x k with ldb >= max(1,n)).
 * levels 0..2 and variant as strassen_dgemm; levels = -1 lets the library choose the member
 * (strassen_select, FP64; variant is then ignored).  A transposed operand is packed, transposed,
 * into workspace first (a tiled copy, the counterpart of BLIS's packing of a transposed block;
 * round_up(m, 2) * k or round_up(k, 2) * n doubles, each rounded up to 32), and the member then
 * runs on the packed operands with the remaining workspace; untransposed calls are exactly
 * strassen_dgemm.  One exception packs nothing: A untransposed, B transposed, levels 0 and a
 * problem below the classical kernel's size (fewer than 256 of its 256 x 128 tiles) — the
 * general tile kernel then reads B^T in place (no workspace).  Otherwise the packed operands need
 * workspace even for ABC: STRASSEN_ERR_ALLOC when the caller workspace or the workspace limit
 * cannot hold them.  The result is bitwise that of strassen_dgemm on the explicitly transposed
 * matrices.
 * Argument positions for -i: transa=1 transb=2 m=3 n=4 k=5 alpha=6 A=7 lda=8 B=9 ldb=10
 * beta=11 C=12 ldc=13 levels=14 variant=15.
 */
int strassen_gemm(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                  const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                  double *C, int64_t ldc, int levels, int variant, void *stream);

/*
 * strassen_dgemm_noalloc — strassen_dgemm for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, semantics, error codes and bits as strassen_dgemm; it calls no hipMalloc, hipFree
 * or allocating routine.  Its workspace is a static device array of
 * STRASSEN_NOALLOC_SCRATCH_BYTES that every device the library runs on holds until the process
 * ends (its address is resolved on the first call on each device); the caller workspace of
 * strassen_set_workspace and the library-owned workspace are not used.  AB and NAIVE keep
 * their temporaries there: a call whose workspace (strassen_workspace_size) exceeds the
 * scratch returns STRASSEN_ERR_ALLOC before anything is enqueued.  ABC uses it for block-padded
 * copies and staged sums only where they fit, else runs its workspace-free path (same bits).
 * Every call on a device shares that device's scratch, which keeps the last call's contents
 * (nothing in it needs to start at zero): calls that overlap in time on one device (different
 * streams, or different host threads) race.  Calls on one stream are ordered and safe.
 */
#define STRASSEN_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int strassen_dgemm_noalloc(int64_t m, int64_t n, int64_t k, double alpha,
                           const double *A, int64_t lda, const double *B, int64_t ldb,
                           double beta, double *C, int64_t ldc,
                           int levels, int variant, void *stream);

/*
 * strassen_workspace_size — bytes of device workspace strassen_dgemm needs for these sizes
 * (0 for levels 0).  AB: one M_r temporary per product (7^L of ceil(m/2^L) x ceil(n/2^L)
 * doubles, leading dimension rounded up to 8, each slot to 32), plus, where AB runs the fused
 * kernel (see strassen_dgemm), the block-padded A and B copies described below for ABC (where
 * m or k is not a multiple of 2^(L+1)) and at two levels the staging buffers of the (padded)
 * problem; NAIVE adds the operand-sum temporaries.  ABC, for 16-byte aligned operands with
 * even leading dimensions: where m, k are multiples of 2^(L+1) (and, for two levels, n of 4 or
 * no staging), at one level the five m/2 x k/2 and five k/2 x n/2 sum slots where its
 * products run on the classical kernel (see strassen_dgemm; else 0), and at two the staging
 * buffers of its outer operand sums where staging is the default (five m/2 x k/2 and five
 * k/2 x n/2 slots; every slot rounded up to 32 doubles); otherwise the block-padded copies (A as mp x kp, B as kp x n', C as mp x n' where
 * it is copied; mp = 2^L * (ceil(m/2^L) rounded up to even), kp likewise, n' = n rounded up to
 * 4 where staging needs it; each rounded up to 32 doubles) plus the staging buffers of the
 * padded problem.  A smaller caller workspace stages one (outer) product at a time (see
 * above), or turns staging or the copies off.
 * Returns 0 or -i as strassen_dgemm does for the same argument (m=1 n=2 k=3 levels=4
 * variant=5 bytes=6).
 */
int strassen_workspace_size(int64_t m, int64_t n, int64_t k, int levels, int variant,
                            size_t *bytes);

/*
 * strassen_set_workspace — use caller-owned device memory [ptr, ptr+bytes) as workspace
 * instead of the library's own (ptr must stay valid while calls that use it are in
 * flight; 256-byte alignment required).  ptr == NULL returns to library-owned workspace.
 * A call needing more than `bytes` fails with STRASSEN_ERR_ALLOC without touching C (ABC only
 * drops its staging or padded copies instead).  The workspace, the caller's or the library's,
 * is shared by every call on the device: calls that use it (AB, NAIVE; ABC where it stages or
 * pads) must not run at the same time on different streams.
 * Returns 0, -1 (misaligned ptr) or -2 (ptr != NULL with bytes == 0).
 */
int strassen_set_workspace(void *ptr, size_t bytes);

/*
 * strassen_set_workspace_limit — cap the library-owned workspace at `bytes` (0 = no cap, the
 * default) for memory-constrained callers.  A call needing more behaves as if the allocation
 * failed: ABC drops its block-padded copies or staging (same result, workspace-free path),
 * AB, NAIVE and strassen_gemm_ex fail with STRASSEN_ERR_ALLOC without touching C.  A buffer
 * already allocated is kept (strassen_release_workspace frees it).  No effect on a caller
 * workspace set by strassen_set_workspace.  Returns 0.
 */
int strassen_set_workspace_limit(size_t bytes);

/* strassen_release_workspace — synchronise the device and free the library-owned workspace. */
int strassen_release_workspace(void);

/*
 * strassen_gemm_ex — the reduced-precision mode (an extension; the paper is FP64 only, and
 * Strassen's weaker error bound (Sec. 1) is why the sums and the C update keep FP32 or FP64).
 * C (FP64) := alpha*A*B + beta*C where each product M_r of the table runs on BF16 MFMA with FP32
 * accumulation (compute = STRASSEN_COMPUTE_BF16 or _BF16X3; _F64 forwards to strassen_dgemm).
 * A, B, C are FP64 as in strassen_dgemm; levels 0 is the classical product in the same mode.
 *   sum_prec: precision in which each operand sum sum_s delta_s X_s is formed (F32: every term
 *             is first rounded to FP32; F64: formed in FP64, then rounded once to FP32); the
 *             FP32 value x becomes hi = bf16(x) and, for bf16x3, lo = bf16(x - hi), rounding
 *             to nearest even; bf16x3 computes hi*hi + hi*lo + lo*hi.
 *   c_prec  : precision of the C update  c := c + alpha*gamma*M  (F32: c is rounded to FP32
 *             before the first update of the call and each update is one FP32 fused
 *             multiply-add; F64: FP64 fused multiply-add).  C is stored as FP64 either way.
 * The products add straight into every destination C sub-block (variant must be STRASSEN_ABC).
 * The operand sums are rounded to bf16 in a first pass into workspace (library-owned, or the
 * caller's: strassen_workspace_size_ex gives the size), since a bf16 operand needs its
 * full-precision sum first.  Argument positions as strassen_dgemm, then compute=14,
 * sum_prec=15, c_prec=16.
 */
int strassen_gemm_ex(int64_t m, int64_t n, int64_t k, double alpha,
                     const double *A, int64_t lda, const double *B, int64_t ldb,
                     double beta, double *C, int64_t ldc,
                     int levels, int variant, int compute, int sum_prec, int c_prec,
                     void *stream);

/*
 * strassen_workspace_size_ex — bytes of workspace strassen_gemm_ex needs: 7^levels products
 * times (ceil(m/2^L) rounded up to 128 + ceil(n/2^L) rounded up to 128) times ceil(k/2^L)
 * rounded up to 64, two bytes each, twice for bf16x3; 0 for STRASSEN_COMPUTE_F64.
 * Returns 0 or -i (m=1 n=2 k=3 levels=4 compute=5 bytes=6).
 */
int strassen_workspace_size_ex(int64_t m, int64_t n, int64_t k, int levels, int compute,
                               size_t *bytes);

/*
 * Batched mode — many independent FP64 GEMMs  C_p := alpha*A_p*B_p + beta*C_p  (p < count) in
 * one persistent kernel launch.  The paper chooses "the right member of the family" per problem
 * size (Sec. 5); here every problem gets its own Strassen level (0, 1, 2; the ABC variant) and
 * tile choice (0: 128 x 128, 1: 64 x 64 in the persistent kernel; 2: the problem runs as its own
 * all-products launch(es), one at one level, seven at two with the outer sums in the load,
 * after the persistent kernel, where that kernel's layout applies (strassen_dgemm's conditions),
 * else in the persistent kernel with the tiles a single call would use; 3: the problem runs as
 * a single call would (the classical, all-products or tile kernel) but with no workspace, on one
 * of four side streams forked from the caller's stream before the persistent kernel and joined
 * back after it, so that problems too small to fill the GPU share it; longest first, each to the
 * side stream with the least work).  A work item of the
 * persistent kernel is one tile position of one problem, on which one workgroup runs all the
 * problem's products; items are handed out longest first through a device counter.  Per problem
 * the result is bitwise that of strassen_dgemm with the same level (every FP64 kernel rounds the
 * same operations in the same order).
 *
 * strassen_batched_plan(count, m, n, k, levels, cfg, plan): problem sizes (host arrays of
 *   `count`).  levels / cfg (host, may be NULL = all -1): -1 lets the library choose by its rule
 *   (level from min(m, n, k) thresholds; problems above one size threshold on the side streams
 *   at level 0 or 1, one-level problems above another as their own all-products launch, else
 *   64 x 64 tiles when the 128 x 128 grid of a sub-block is small);
 *   the chosen values are written back.  *plan receives an opaque handle (host memory).
 *   Returns 0, -1 count < 0, -2 NULL or negative sizes, -5 / -6 a level / cfg out of range,
 *   -7 plan NULL.  Needs no device.
 * strassen_batched_autotune(plan, sample, seed, stream): times the batch (persistent kernel,
 *   side streams and all-products launches) on `sample` problems of the plan (seeded choice; 0 = all) under
 *   candidate rule thresholds, on zeroed
 *   library-owned buffers of the same shapes, and re-chooses every -1 entry with the fastest
 *   rule.  Synchronises `stream`.  Returns 0, -1, -2, or a positive error.
 * strassen_batched_choice(plan, i, level, cfg): the current choice for problem i.
 * strassen_batched_run(plan, A, lda, B, ldb, C, ldc, alpha, beta, stream): host arrays of
 *   `count` device pointers and leading dimensions (column-major, as strassen_dgemm); enqueues
 *   the launch on `stream` (after copying the work list to the device, which synchronises the
 *   stream).  alpha, beta are common to the batch; problems with alpha == 0 or k == 0 only
 *   scale C.  Returns 0, -1 plan NULL, -2 NULL arrays, -3 a bad problem (message names it), or
 *   a positive error.
 * strassen_batched_capture(...same arguments...): prepares the work list for these operands
 *   and records the launches (counter clear, persistent kernel, then the all-products launches
 *   in problem order; with side-stream problems, by stream capture, the side streams as parallel
 *   branches) as a HIP graph in the plan,
 *   without running it.  alpha == 0 / k == 0 problems are refused (STRASSEN_ERR_UNSUPPORTED).
 * strassen_batched_replay(plan, stream): launches the recorded graph on `stream`; every replay
 *   recomputes C from the operands recorded at capture.  A later run or capture on the plan
 *   discards the recording (replay then returns -1 until the next capture).
 * strassen_batched_destroy(plan): synchronises the device and frees the plan (NULL is a no-op).
 * A plan's device buffers are shared by its runs and replays: calls on one plan that overlap in
 * time (different streams) race.
 */
int strassen_batched_plan(int count, const int64_t *m, const int64_t *n, const int64_t *k,
                          int *levels, int *cfg, void **plan);
int strassen_batched_autotune(void *plan, int sample, uint64_t seed, void *stream);
int strassen_batched_choice(void *plan, int i, int *level, int *cfg);
int strassen_batched_run(void *plan, const double *const *A, const int64_t *lda,
                         const double *const *B, const int64_t *ldb, double *const *C,
                         const int64_t *ldc, double alpha, double beta, void *stream);
int strassen_batched_capture(void *plan, const double *const *A, const int64_t *lda,
                             const double *const *B, const int64_t *ldb, double *const *C,
                             const int64_t *ldc, double alpha, double beta, void *stream);
int strassen_batched_replay(void *plan, void *stream);
int strassen_batched_destroy(void *plan);

/*
 * Selector — picks the member of the family for a shape: member c in 0..6 is
 *   0 classical, 1 one-level ABC, 2 one-level AB, 3 one-level Naive,
 *   4 two-level ABC, 5 two-level AB, 6 two-level Naive
 * (the paper leaves this choice, as a function of problem size, to the user: Sec. 5).
 *
 * strassen_select(m, n, k, dtype, levels, variant): dtype 0 = FP64 (strassen_dgemm), 1 = BF16
 *   (strassen_gemm_ex, ABC members only).  With a network loaded: arg-max of its scores
 *   (computed by the library's inference kernel on the current device, blocking); otherwise:
 *   arg-min of strassen_cost_model.  Returns 0 or -i.
 * strassen_cost_model(m, n, k, dtype, seconds[7]): the analytical model of each member's time
 *   (the GPU counterpart of the paper's Fig. "tab:breakdown": MFMA time at this library's
 *   rates and efficiencies, launch latency, and HBM time of the extra passes); +inf for
 *   members not offered for dtype.  Host only.
 * strassen_selector_load(params): host array of 5383 floats (the network below) copied into
 *   the library; NULL unloads it (back to the model).  -1 if a value is not finite.
 * strassen_selector_features(m, n, k, dtype, x[11]): the network's input for a shape (host
 *   only): x[0..2] = (ln s - ln 256) / (ln 20000 - ln 256) for s = m, n, k; x[3] = dtype;
 *   x[4 + c] = min(ln(t_c / t_best), 1) with t_c = strassen_cost_model's time of member c and
 *   t_best the smallest of them (1 for members not offered for dtype).  The network scores the
 *   members from the shape and from where the model ranks them, so it learns where measured
 *   times depart from the model.  Returns 0 or -i.
 *
 * The network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), scores = W3 h2 + b3 with W1 64x11,
 * W2 64x64, W3 7x64 (row-major), FP32; parameters flat in the order W1, b1, W2, b2, W3, b3.
 * Training entry points (device pointers, enqueued on `stream`):
 * strassen_mlp_forward(params, X, n, logits, stream): X n x 11, logits n x 7 (row-major).
 * strassen_mlp_work_size(n, bytes): workspace bytes strassen_mlp_loss_grad needs for n samples.
 * strassen_mlp_loss_grad(params, X, labels, n, work, grad, loss, stream): mean softmax
 *   cross-entropy over the n samples into *loss and its gradient (flat, as params) into grad;
 *   every gradient is summed over the samples in order (deterministic).
 * strassen_mlp_adam(params, grad, m, v, t, lr, beta1, beta2, eps, stream): one Adam step
 *   (t counts from 1; m, v the moment buffers, zero before the first step).
 */
int strassen_select(int64_t m, int64_t n, int64_t k, int dtype, int *levels, int *variant);
int strassen_cost_model(int64_t m, int64_t n, int64_t k, int dtype, double *seconds);
int strassen_selector_load(const float *params);
int strassen_selector_features(int64_t m, int64_t n, int64_t k, int dtype, float *x);
int strassen_mlp_forward(const float *params, const float *X, int n, float *logits, void *stream);
int strassen_mlp_work_size(int n, size_t *bytes);
int strassen_mlp_loss_grad(const float *params, const float *X, const int *labels, int n,
                           float *work, float *grad, float *loss, void *stream);
int strassen_mlp_adam(float *params, const float *grad, float *m, float *v, int t, float lr,
                      float beta1, float beta2, float eps, void *stream);

/*
 * strassen_set_tile_config — tuning control.  cfg = -1 (default) lets the library choose the
 * kernel and tile configuration per call; 0..6 forces one for every later call in the process:
 *   0: 128 x 128 tile, k step 16, two workgroups per CU;   1: 64 x 64, k step 16;
 *   2: 128 x 128, k step 8, two workgroups per CU;        3: 128 x 128, k step 16, one per CU;
 *   4: ABC and AB with levels >= 1 run the all-products kernel (the seven products of a level
 *      side by side on 64 x 64 tiles of the four quadrants) on the operands as given where its
 *      layout applies (m and k multiples of 2^(levels+1), 16-byte aligned operands, even
 *      leading dimensions), else on block-padded copies as by default; ABC forms the two-level
 *      outer sums in the load (two-level AB, which needs them staged, runs the tile kernel);
 *   5: as 4, with the two-level outer operand sums staged wherever n % 4 == 0 (the workspace,
 *      library-owned or the caller's, must then hold them: STRASSEN_ERR_ALLOC otherwise);
 *   6: the default, except that one-level ABC on the classical kernel (see strassen_dgemm) is
 *      required where its layout and size conditions hold: STRASSEN_ERR_ALLOC when the
 *      workspace cannot hold one product's two sum slots.
 * The default (-1) uses the all-products kernel wherever it applies and stages as described
 * at strassen_dgemm.  For strassen_gemm_ex, 0 / 1 force the BF16 product kernel's 128 x 128 /
 * 128 x 64 workgroup tiles (default: 128 x 64 where 128 x 128 tiles would number fewer than 512).
 * Results do not depend on the configuration (bitwise).  The environment variable
 * STRASSEN_TILE_CFG sets the initial value.  Returns 0 or -1 (cfg out of range).
 */
int strassen_set_tile_config(int cfg);

/*
 * Kernel timing (measurement support).  strassen_timing_enable(1) makes every later call record
 * a pair of HIP events on its stream around each launch of the kernels below (events from an
 * internal pool; the extra work is two event records per launch); 0 stops recording.
 * strassen_timing_collect(kind, ms_total, launches) waits for the recorded launches of `kind`,
 * returns their summed duration in milliseconds and their number, and forgets them (the other
 * kinds stay recorded).  Returns 0, -2 (NULL output) or STRASSEN_ERR_HIP.
 */
enum strassen_kernel_kind {
    STRASSEN_KERNEL_ALL_PRODUCTS = 0,  /* the fused ABC kernel (one level; each two-level outer product) */
    STRASSEN_KERNEL_OUTER_SUMS = 1,    /* the staged outer-sum pass of two-level ABC            */
    STRASSEN_KERNEL_TILE = 2,          /* the general FP64 tile kernel (classical, AB, Naive, ABC fallback) */
    STRASSEN_KERNEL_BF16 = 3,          /* the reduced-precision product kernel (strassen_gemm_ex) */
    STRASSEN_KERNEL_CAST = 4,          /* its operand pass (sums rounded to bf16 hi / lo)       */
    STRASSEN_KERNEL_PAD = 5,           /* block-padded operand copies of ABC (and the copy back) */
    STRASSEN_KERNEL_CLASSICAL = 6      /* the classical FP64 kernel on the fused load path (levels 0) */
};
int strassen_timing_enable(int on);
int strassen_timing_collect(int kind, double *ms_total, int *launches);

/*
 * strassen_probe_rates(fp64_tflops, bf16_tflops, stream) — measurement support: the matrix
 * cores' issue rate on the current device, measured by a kernel in which every wave issues
 * eight independent chains of the instruction the library's kernels use (FP64
 * v_mfma_f64_16x16x4_f64; BF16 v_mfma_f32_16x16x32_bf16), eight waves per SIMD, about 20 ms
 * each; the roofline fractions are also quoted against these.  Allocates and frees a small
 * device buffer, synchronises `stream`.  Returns 0, -1 (NULL output) or a positive error.
 */
int strassen_probe_rates(double *fp64_tflops, double *bf16_tflops, void *stream);

/*
 * Table introspection (host only, no device needed): the operation table the kernels execute.
 * strassen_table_size returns the number of products for `levels` (1, 7, 49, 343) or -1.
 * strassen_table_get fills, for product r, the operand and destination terms as
 * codes  sign * (1 + row_block + 2^L * col_block)  (sign = -1 for a subtraction) in
 * a_terms[0..*na), b_terms[0..*nb), c_terms[0..*nc) (arrays of at least 8 entries).
 * Returns 0, or -1 for levels out of range, -2 for r out of range.
 */
int strassen_table_size(int levels);
int strassen_table_get(int levels, int r, int *na, int *a_terms, int *nb, int *b_terms,
                       int *nc, int *c_terms);

/* strassen_last_error — message describing the calling thread's most recent failure
 * ("" if none).  The pointer stays valid until the next library call on this thread. */
const char *strassen_last_error(void);

/* strassen_version — library version string. */
const char *strassen_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STRASSEN_MI355X_H */
