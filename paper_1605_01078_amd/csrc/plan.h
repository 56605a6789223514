// Internal structures shared by the host planner and the HIP kernels.
//
// A Strassen "table" lists, for every product M_r, the general operation of eq. (e:straprim4):
//   M_r = (sum_s delta_s X_s)(sum_t eps_t V_t);  C_d += alpha * gamma_d * M_r for each destination d,
// with X_s sub-blocks of A, V_t sub-blocks of B and C_d sub-blocks of C in the 2^L x 2^L partition.
#pragma once
#include <stdint.h>
#include <vector>

namespace smx {

constexpr int kMaxLevels = 2;      // device tables (tile kernel, AB, Naive, batched, BF16 mode)
constexpr int kMaxLevelsAbc = 3;   // strassen_dgemm's ABC (three levels: staged upper levels)
constexpr int kMaxProducts = 49;   // 7^kMaxLevels
constexpr int kMaxTerms = 4;       // 2^kMaxLevels operand terms / destinations per product

// Term code: bits 0-2 row block, bits 3-5 column block, bit 7 set for a minus sign.
inline constexpr uint8_t term_code(int row, int col, int sign) {
  return (uint8_t)((row & 7) | ((col & 7) << 3) | (sign < 0 ? 0x80 : 0));
}

struct ProdDesc {
  uint8_t na, nb, nc;   // number of A terms, B terms, C destinations
  uint8_t first;        // bit d: destination d is the first update of its C sub-block (apply beta)
  uint8_t flags;        // bit 0: A operand is Naive temporary slot `tslot_a`; bit 1: same for B
  uint8_t tslot_a, tslot_b, pad0;
  uint8_t a[kMaxTerms], b[kMaxTerms], c[kMaxTerms];
  uint8_t pad1[4];
};
static_assert(sizeof(ProdDesc) == 24, "ProdDesc layout");

enum : int32_t { kModeABC = 0, kModeStoreM = 1 };

// Everything the kernels need to know about one table, kept in __constant__ memory
// (uploaded once per device).  Table ids: see table_id().
struct TableDev {
  int32_t nprod;
  int32_t q;                                  // 2^levels
  int32_t nslot_a, nslot_b;                   // Naive operand-sum temporaries
  ProdDesc prod[kMaxProducts];
  uint8_t asm_cnt[16];                        // products feeding C sub-block s = ci*q + cj
  uint8_t asm_list[16][16];                   // their indices (| 0x80 for a minus sign), increasing
  uint8_t slot_prod_a[kMaxProducts];          // product whose A sum fills Naive slot s
  uint8_t slot_prod_b[kMaxProducts];
};
constexpr int kNumTables = 5;
// 0: classical; 1, 2: one / two levels (ABC, AB); 3, 4: one / two levels, Naive slots
inline int table_id(int levels, bool naive) { return levels == 0 ? 0 : (naive ? 2 + levels : levels); }

// Arguments of the FP64 tile kernel.
struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  double* M;            // StoreM mode: M_r at M + r * m_stride, leading dimension ldm
  const double* TA;     // Naive: A-sum slot s at TA + s * ta_stride (leading dimension mq)
  const double* TB;     // Naive: B-sum slot s at TB + s * tb_stride (leading dimension kq)
  int64_t lda, ldb, ldc, ldm, m_stride, ta_stride, tb_stride;
  int64_t m, n, k;      // full problem
  int64_t mq, nq, kq;   // sub-block extents ceil(m/q), ceil(n/q), ceil(k/q)
  double alpha, beta;
  int32_t tab;          // table id
  int32_t tiles_m, tiles_n;
  int32_t mode;         // kModeABC: a workgroup owns one tile position in every C sub-block and
                        //           runs every product; kModeStoreM: one (product, tile) each
  int32_t prod_begin;   // StoreM: first product of this launch
  int32_t tb;           // B given transposed: op(B)(p, j) at B[j + p * ldb] (ABC, one-term
                        // products only)
};

// Arguments of the all-products kernel: one launch computes the seven products of the one-level
// table on the 2 x 2 inner sub-blocks of one outer product's operands (at one level the outer
// product is the identity: one term of sign +1 covering the whole matrix; at three levels the
// outer product is a pair of products of the two upper levels, its operands staged sums and its
// destinations the Kronecker products of their destinations).
struct FusedArgs {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int64_t n;                    // columns of B and C
  int64_t mq, nq, kq;           // inner sub-block extents (mq and kq even and exact)
  double alpha, beta;
  int32_t tiles_m, tiles_n;     // 64 x 64 tiles of one inner sub-block
  int32_t nc;                   // outer destinations (1 or 2; up to 4 at three levels)
  int32_t c_first;              // bit d: outer destination d gets its first update in this launch
  int64_t a_off[2], b_off[2], c_off[4];   // element offsets of the outer blocks
  int32_t b_cb[2], c_cb[4];     // first column block (units of nq) of outer B terms / destinations
  double a_sg[2], b_sg[2], c_sg[4];
  // AB form (store_m = 1): product r of this launch goes to temporary prod_base + r at
  // M + (prod_base + r) * m_stride, leading dimension ldm (even); C is not touched
  double* M;
  int64_t ldm, m_stride;
  int32_t store_m, prod_base;
  int32_t scheme;               // 0: Strassen's table, 1: Winograd's variant (one term per side)
  int32_t pad_;
};

// Classical FP64 GEMM on the all-products kernel's load path (levels = 0).
struct ClassicalArgs {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int64_t m, n, k;
  double alpha, beta;
  int32_t tiles_m, tiles_n;     // 256 x 128 tiles of C
  // Further destinations (one-level ABC and Winograd's variant on this kernel): the product is
  // also added to Cx[0 .. extra-1] (same shape and ldc) with coefficients ax[], after C, in
  // that order.  Bit d of not_first: destination d (0 = C) is not receiving its first update
  // (beta is not applied, C is read).
  double* Cx[3];
  double ax[3];
  int32_t extra;
  int32_t not_first;
};

// C assembly for AB / Naive: C_s := beta*C_s at the first update, then C_s += alpha*gamma*M_r
// for the products r feeding sub-block s, in increasing r.
struct AssembleArgs {
  const double* M;
  double* C;
  int64_t ldm, m_stride, ldc;
  int64_t m, n, mq, nq;
  double alpha, beta;
  int32_t tab;
  int32_t chunks_m;     // ceil(mq / rows per workgroup)
};

// Staged outer-level operand sums of two-level ABC, one side (A or B) per launch: the four outer
// blocks of the operand (rows x cols each, leading dimension ld, at src + blk[q]) are read once
// and every two-term sum of that side of the one-level table (in product order) is written as a
// rows x cols slot (leading dimension rows) at dst + s * dst_stride.  rows even, ld even, src and
// dst 16-byte aligned.
struct OuterSumArgs {
  const double* src;
  double* dst;
  int64_t ld, rows, cols, dst_stride;
  int64_t blk[4];
  int32_t chunks_r;     // row chunks per column group (set by the launcher)
  int32_t single;       // 0: every two-term sum of the side, each into its slot; r + 1: only
                        // the sum of outer product r, into slot 0 (only its two blocks read)
};

// Winograd's variant, staged outer level: the four chain sums of one side (S1..S4 of A, T1..T4
// of B) over the four outer blocks of src (rows x cols each, leading dimension ld, at
// src + blk[q]) into slots of rows x cols (leading dimension rows) at dst + s * dst_stride.
// Same layout requirements as OuterSumArgs.
typedef OuterSumArgs ChainSumArgs;

// Block-padded copy.  Pad (unpad = 0): dst (dst_rows x dst_cols, leading dimension ld_d) gets
// src (rows x cols, ld_s) with source row block b (rows [b*rb, b*rb + rb)) placed at destination
// rows [b*rb_e, b*rb_e + rb) and likewise for column blocks (cb, cb_e); every other destination
// element is zero.  Unpad (unpad = 1): the reverse, writing only the rows x cols plain elements
// of dst from the padded src.
struct PadArgs {
  const double* src;
  double* dst;
  int64_t ld_s, ld_d;
  int64_t rows, cols;           // plain extents
  int64_t rb, rb_e, cb, cb_e;   // plain and padded block extents (rows, columns)
  int64_t dst_rows, dst_cols;   // padded extents (pad direction)
  int32_t unpad;
  int32_t pad;
};

// Naive operand sums: slot s := sum_t delta_t X_t over the zero-padded sub-block extent.
struct SumArgs {
  const double* src;
  double* dst;          // slot s at dst + s * dst_stride, leading dimension rows_q
  int64_t ld, rows, cols, rows_q, cols_q, dst_stride;
  int32_t tab;
  int32_t side;         // 0: A operand (rows = m, cols = k); 1: B operand (rows = k, cols = n)
  int32_t chunks_r;
};

// Reduced-precision mode, operand pass: slot r (product r) gets the bf16 operand(s) of the
// product's A-side (side 0) or B-side (side 1) sum, k-contiguous: element (outer o, k) at
// hi/lo + r * slot_stride + o * kpad + k, where outer is the row (A) or the column (B).
struct CastArgs {
  const double* src;
  uint16_t* hi;
  uint16_t* lo;                 // null: BF16 (no low part)
  int64_t ld, rows, cols;       // source matrix (A: m x k, B: k x n)
  int64_t rq, cq;               // sub-block extents (A: mq x kq, B: kq x nq)
  int64_t outer_pad, kpad;      // padded outer extent (multiple of 128) and k extent (of 64)
  int64_t slot_stride;          // elements per slot
  int32_t tab;
  int32_t side;
  int32_t sum_f64;              // 1: sums in FP64 then rounded to FP32; 0: FP32 throughout
};

// Reduced-precision mode, product kernel.
struct Bf16Args {
  const uint16_t* TAh;
  const uint16_t* TAl;
  const uint16_t* TBh;
  const uint16_t* TBl;
  int64_t stride_a, stride_b, kpad;   // slot strides (elements); padded k (multiple of 64)
  double* C;
  int64_t ldc, m, n, mq, nq;
  double alpha, beta;
  int32_t tab, tiles_m, tiles_n;
  int32_t x3;                   // 1: bf16x3 (hi*hi + hi*lo + lo*hi)
  int32_t c_f64;                // 1: C update in FP64, 0: in FP32
  int32_t shape;                // workgroup tile: 0 = 128 x 128, 1 = 128 x 64
  int32_t vec_c;                // 1: C 16-byte aligned, ldc and the sub-block rows even
};

// Batched mode: one problem (its tile-kernel arguments and tile shape) and one work item.
struct BatchProblem {
  GemmArgs g;
  int32_t cfg;                  // 0: 128 x 128 tiles, 1: 64 x 64
  int32_t pad;
};
struct BatchItem {
  int32_t problem;
  int32_t tile;                 // tile index, ti + tiles_m * tj
};

// Transposed copy: dst (rows x cols, leading dimension ld_d) := src^T, src cols x rows (ld_s).
struct TransposeArgs {
  const double* src;
  double* dst;
  int64_t ld_s, ld_d, rows, cols;
};

// C := beta*C (alpha == 0 or k == 0).
struct ScaleArgs {
  double* C;
  int64_t ldc, m, n;
  double beta;
};

// The one-level table of Fig. "All operations for one-level Strassen" (Sec. 3.1) with sub-blocks
// named by quadrant index q = 2*row + col: for product r its A terms, B terms and C destinations,
// each with a sign.  Both the host table builder and the all-products kernel read it.
struct QTerm { int8_t q, sign; };
struct QProduct { int8_t na, nb, nc; QTerm a[2], b[2], c[2]; };
constexpr QProduct kOneLevel[7] = {
    {2, 2, 2, {{0, 1}, {3, 1}}, {{0, 1}, {3, 1}}, {{0, 1}, {3, 1}}},     // (A00+A11)(B00+B11)
    {2, 1, 2, {{2, 1}, {3, 1}}, {{0, 1}, {0, 0}}, {{2, 1}, {3, -1}}},    // (A10+A11) B00
    {1, 2, 2, {{0, 1}, {0, 0}}, {{1, 1}, {3, -1}}, {{1, 1}, {3, 1}}},    // A00 (B01-B11)
    {1, 2, 2, {{3, 1}, {0, 0}}, {{2, 1}, {0, -1}}, {{0, 1}, {2, 1}}},    // A11 (B10-B00)
    {2, 1, 2, {{0, 1}, {1, 1}}, {{3, 1}, {0, 0}}, {{1, 1}, {0, -1}}},    // (A00+A01) B11
    {2, 2, 1, {{2, 1}, {0, -1}}, {{0, 1}, {1, 1}}, {{3, 1}, {0, 0}}},    // (A10-A00)(B00+B01)
    {2, 2, 1, {{1, 1}, {3, -1}}, {{2, 1}, {3, 1}}, {{0, 1}, {0, 0}}},    // (A01-A11)(B10+B11)
};

// Winograd's variant of the one-level table: operand 0..3 is quadrant q of A (B); 4..7 are the
// chain sums S1 = A10 + A11, S2 = S1 - A00, S3 = A00 - A10, S4 = A01 - S2 (for B:
// T1 = B01 - B00, T2 = B11 - T1, T3 = B11 - B01, T4 = T2 - B10); every C quadrant each product
// reaches, with its sign.  C00 = M1 + M2, C01 = M1 + M3 + M5 + M6, C10 = M1 - M4 + M6 + M7,
// C11 = M1 + M5 + M6 + M7.
struct WProduct { int8_t a, b, nc; QTerm c[4]; };
constexpr WProduct kWinograd[7] = {
    {0, 0, 4, {{0, 1}, {1, 1}, {2, 1}, {3, 1}}},   // M1 = A00 B00
    {1, 2, 1, {{0, 1}, {0, 0}, {0, 0}, {0, 0}}},   // M2 = A01 B10
    {7, 3, 1, {{1, 1}, {0, 0}, {0, 0}, {0, 0}}},   // M3 = S4 B11
    {3, 7, 1, {{2, -1}, {0, 0}, {0, 0}, {0, 0}}},  // M4 = A11 T4
    {4, 4, 2, {{1, 1}, {3, 1}, {0, 0}, {0, 0}}},   // M5 = S1 T1
    {5, 5, 3, {{1, 1}, {2, 1}, {3, 1}, {0, 0}}},   // M6 = S2 T2
    {6, 6, 2, {{2, 1}, {3, 1}, {0, 0}, {0, 0}}},   // M7 = S3 T3
};

struct Term { int row, col, sign; };
struct Product { std::vector<Term> a, b, c; };

// Product-side table construction (one-level figure + Kronecker composition, Sec. 3.5).
std::vector<Product> build_table(int levels);

}  // namespace smx
