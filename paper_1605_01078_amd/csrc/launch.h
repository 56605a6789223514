// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace smx {

// Tile configurations of the FP64 tile kernel: workgroup tile BM x BN, k step BK, 256 threads.
enum TileCfg : int {
  kCfg128 = 0,     // 128 x 128, BK 16, two workgroups per CU
  kCfg64 = 1,      // 64 x 64, BK 16
  kCfg128k8 = 2,   // 128 x 128, BK 8, two workgroups per CU
  kCfg128w1 = 3,   // 128 x 128, BK 16, one workgroup per CU (512 registers per lane)
  kCfgAll = 4,     // ABC with levels >= 1: the all-products kernel (where its layout applies)
  kCfgAllStaged = 5,   // as 4; at two levels the outer operand sums are staged in a workspace
  kCfgClassicalStaged = 6,   // ABC with one level: sums staged, products on the classical kernel
  kNumCfgs = 7
};
inline int cfg_bm(int cfg) { return cfg == kCfg64 ? 64 : 128; }
inline int cfg_bn(int cfg) { return cfg == kCfg64 ? 64 : 128; }

// Copies the kNumTables table descriptors into the current device's constant memory.
hipError_t upload_tables(const TableDev* tabs);

// FP64 tile kernel.  maxt: largest operand term count in the table (1, 2 or 4);
// vec: operands are 16-byte aligned with even leading dimensions and even extents, so
// pairs of doubles can be loaded together.  grid = number of workgroups.
hipError_t launch_fp64_tile(const GemmArgs& a, int cfg, int maxt, bool vec, int grid,
                            hipStream_t s);
// All-products kernel for one outer product with na A terms and nb B terms (1 or 2 each);
// grid = a.tiles_m * a.tiles_n workgroups of 512 threads.
hipError_t launch_all_products(const FusedArgs& a, int na, int nb, hipStream_t s);
const void* all_products_fn(const FusedArgs& a, int na, int nb);   // its kernel symbol (graph nodes)
// Classical FP64 GEMM (levels = 0) on the same load path; grid = tiles_m * tiles_n workgroups of
// 512 threads, 256 x 128 tiles.
hipError_t launch_classical(const ClassicalArgs& a, hipStream_t s);
// Reduced-precision mode: operand pass over nslots products; BF16 product kernel.
hipError_t upload_tables_bf16(const TableDev* tabs);
hipError_t launch_cast(const CastArgs& a, int nslots, hipStream_t s);
hipError_t launch_bf16_gemm(const Bf16Args& a, hipStream_t s);
// Batched mode: clear the item counter, then the persistent kernel over `grid` workgroups.
hipError_t upload_tables_batched(const TableDev* tabs);
hipError_t launch_batched(const BatchProblem* probs, const BatchItem* items, int n_items,
                          unsigned* counter, bool vec, int grid, hipStream_t s);
const void* batched_kernel_fn(bool vec);   // kernel symbols, for graph nodes
const void* clear_counter_fn();
// Selector network (kernels_mlp.hip): flat FP32 parameters W1, b1, W2, b2, W3, b3.
// Inputs: the shape's four size features and the analytical model's seven time ratios.
constexpr int kMlpIn = 11;
constexpr int kMlpParams = 64 * kMlpIn + 64 + 64 * 64 + 64 + 7 * 64 + 7;
hipError_t launch_mlp_forward(const float* params, const float* X, int n, float* logits,
                              float* A1, float* A2, hipStream_t s);
hipError_t launch_mlp_backward(const float* params, const float* X, const int* y, int n,
                               float* work, float* grad, float* loss, hipStream_t s);
hipError_t launch_mlp_adam(float* params, const float* grad, float* m, float* v, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_assemble(const AssembleArgs& a, int q2, hipStream_t s);
hipError_t launch_sums(const SumArgs& a, int nslots, hipStream_t s);
hipError_t launch_outer_sums(const OuterSumArgs& a, int side, hipStream_t s);   // side 0 A, 1 B
hipError_t launch_chain_sums(const ChainSumArgs& a, int side, hipStream_t s);   // Winograd's
hipError_t launch_scale(const ScaleArgs& a, hipStream_t s);
hipError_t launch_transpose(const TransposeArgs& a, hipStream_t s);
// LU base cases (kernels_lu.hip), w / k <= 64: in-place LU of a w x w block (one workgroup);
// B := B U^{-1} (upper, one thread per row); B := L^{-1} B (unit lower, one thread per column).
hipError_t launch_chol_base(double* P, int64_t ld, int w, int* info, int col0, hipStream_t s);
hipError_t launch_sub_lower(double* C, int64_t ldc, const double* W, int64_t ldw, int64_t n,
                            hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
hipError_t launch_trsm_rows_lower_t(const double* L, int64_t ldl, int w, double* B, int64_t ldb,
                                    int64_t rows, hipStream_t s);
hipError_t launch_lu_base(double* P, int64_t ld, int w, hipStream_t s);
hipError_t launch_trsm_rows_upper(const double* U, int64_t ldu, int w, double* B, int64_t ldb,
                                  int64_t rows, hipStream_t s);
hipError_t launch_trsm_cols_lower_unit(const double* L, int64_t ldl, int k, double* B,
                                       int64_t ldb, int64_t cols, hipStream_t s);
hipError_t launch_pad_copy(const PadArgs& a, hipStream_t s);
// Matrix-core rate probe (probe_rates.hip): kind 0 FP64, 1 BF16; `out` holds grid * 256 doubles.
int probe_grid(int cus);
hipError_t launch_rate_probe(int kind, double* out, int grid, int iters, hipStream_t s);
double probe_flops_per_wave_iter(int kind);

}  // namespace smx
