// FP64 kernels for one- and two-level Strassen on gfx950 (CDNA4).
//
// fp64_tile_kernel is the paper's modified GEMM (Sec. 4.1, "Building blocks"): the operand sums
// sum_s delta_s X_s and sum_t eps_t V_t are formed while the tiles travel from HBM to LDS (the
// GPU counterpart of packing A~_i and B~_p), the product runs on FP64 MFMA
// (v_mfma_f64_16x16x4_f64) with the accumulator in registers (the micro-kernel), and the
// epilogue either adds alpha*gamma_d*M to every destination sub-block of C (ABC) or stores M
// to a temporary (AB, Naive).  assemble_kernel is the separate C update of AB and Naive;
// sum_kernel forms Naive's explicit operand-sum temporaries.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "plan.h"
#include "tile_fp64.h"

namespace smx {

__constant__ TableDev g_tables[kNumTables];

// ---------------------------------------------------------------------------------------------
// FP64 tile kernel: ABC mode runs every product for one tile position (owner computes: no two
// workgroups ever update the same C element, so no atomics and a fixed update order); StoreM
// mode computes one (product, tile) pair per workgroup and writes M_r to its temporary.
// ---------------------------------------------------------------------------------------------
template <int BM, int BN, int BK, int MAXT, bool VEC, int WPE, int MODE, bool TB = false>
__global__ __launch_bounds__(256, WPE) void fp64_tile_kernel(const GemmArgs args) {
  using Tile = Fp64Tile<BM, BN, BK, MAXT, VEC, TB>;
  __shared__ double lds[Tile::LDS_DOUBLES];
  const TableDev& tab = g_tables[args.tab];
  const int T = args.tiles_m * args.tiles_n;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  int r_begin, r_end, tile;
  if (MODE == kModeABC) {
    r_begin = 0;
    r_end = tab.nprod;
    tile = logical;
  } else {
    r_begin = args.prod_begin + logical / T;
    r_end = r_begin + 1;
    tile = logical % T;
  }
  int ti, tj;
  tile_coords(tile, args.tiles_m, args.tiles_n, ti, tj);
  const int64_t row0 = (int64_t)ti * BM, col0 = (int64_t)tj * BN;
  for (int r = r_begin; r < r_end; ++r) {
    const ProdDesc& pd = tab.prod[r];
    typename Tile::Acc acc;
    Tile::product(args, pd, row0, col0, lds, acc);
    if (MODE == kModeABC)
      Tile::update_c(args, pd, row0, col0, acc);
    else
      Tile::store_m(args, r, row0, col0, acc);
  }
}

// ---------------------------------------------------------------------------------------------
// C assembly (AB, Naive): one thread per element (i, j) of one C sub-block s.  Workgroups are
// ordered sub-block fastest so the M_r chunks a row of workgroups reads stay in L2.
// ---------------------------------------------------------------------------------------------
constexpr int kAsmRows = 256;

__global__ __launch_bounds__(256) void assemble_kernel(const AssembleArgs args, int q2) {
  const TableDev& tab = g_tables[args.tab];
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int s = logical % q2;
  const int chunk = logical / q2;
  const int64_t j = chunk / args.chunks_m;
  const int64_t i = (int64_t)(chunk % args.chunks_m) * kAsmRows + threadIdx.x;
  if (i >= args.mq || j >= args.nq) return;
  const int q = tab.q;
  const int64_t ci = s / q, cj = s % q;
  const int64_t row = ci * args.mq + i, col = cj * args.nq + j;
  if (row >= args.m || col >= args.n) return;
  double* p = args.C + row + col * args.ldc;
  double c = args.beta == 0.0 ? 0.0 : *p;
  const int cnt = tab.asm_cnt[s];
  const double* mp = args.M + i + j * args.ldm;
  for (int e = 0; e < cnt; ++e) {
    const uint8_t code = tab.asm_list[s][e];
    const int r = code & 0x7f;
    const double ag = (code & 0x80) ? -args.alpha : args.alpha;
    c = c_update(c, mp[(int64_t)r * args.m_stride], ag, args.beta, e == 0);
  }
  *p = c;
}

// ---------------------------------------------------------------------------------------------
// Naive operand sums: one thread per element of one temporary slot (zero-padded extent).
// ---------------------------------------------------------------------------------------------
constexpr int kSumRows = 256;

__global__ __launch_bounds__(256) void sum_kernel(const SumArgs args) {
  const TableDev& tab = g_tables[args.tab];
  const int slot = blockIdx.y;
  const int64_t j = blockIdx.x / args.chunks_r;
  const int64_t i = (int64_t)(blockIdx.x % args.chunks_r) * kSumRows + threadIdx.x;
  if (i >= args.rows_q || j >= args.cols_q) return;
  const int r = args.side == 0 ? tab.slot_prod_a[slot] : tab.slot_prod_b[slot];
  const ProdDesc& pd = tab.prod[r];
  const int nt = args.side == 0 ? pd.na : pd.nb;
  const uint8_t* codes = args.side == 0 ? pd.a : pd.b;
  // Same arithmetic as signed_sum: each pair is c0 * (x0 + (c0*c1) x1), a four-term sum adds
  // the two pairs.
  double x[kMaxTerms], sg[kMaxTerms];
  for (int t = 0; t < nt; ++t) {
    const uint8_t code = codes[t];
    const int64_t row = code_row(code) * args.rows_q + i;
    const int64_t col = code_col(code) * args.cols_q + j;
    const bool ok = row < args.rows && col < args.cols;
    x[t] = ok ? args.src[row + col * args.ld] : 0.0;
    sg[t] = code_neg(code) ? -1.0 : 1.0;
  }
  double v;
  if (nt == 1) v = signed_sum<1>(sg, x);
  else if (nt == 2) v = signed_sum<2>(sg, x);
  else v = signed_sum<4>(sg, x);
  args.dst[(int64_t)slot * args.dst_stride + i + j * args.rows_q] = v;
}

// Staged outer sums: a workgroup covers kOuterSumRows rows of kOuterSumCols consecutive columns,
// each lane a row pair (16-byte accesses): it reads the four outer blocks once and writes every
// two-term sum of its side of the one-level table, x0 + s1 x1 rounded once (the pair rule of
// signed_sum with a first sign of +1, as the all-products kernel forms the same sum).
constexpr int kOuterSumRows = 512, kOuterSumCols = 4;

template <int SIDE>
__global__ __launch_bounds__(256) void outer_sum_kernel(const OuterSumArgs args) {
  const int64_t i = (int64_t)(blockIdx.x % args.chunks_r) * kOuterSumRows + 2 * threadIdx.x;
  const int64_t j0 = (int64_t)(blockIdx.x / args.chunks_r) * kOuterSumCols;
  if (i >= args.rows) return;
  // the blocks the requested sums read (all four, or the two terms of one product's sum)
  int need = 15;
  if (args.single > 0) {
    const QProduct& P = kOneLevel[args.single - 1];
    need = SIDE == 0 ? (1 << P.a[0].q) | (1 << P.a[1].q) : (1 << P.b[0].q) | (1 << P.b[1].q);
  }
  d2_t x[4][kOuterSumCols];
#pragma unroll
  for (int c = 0; c < kOuterSumCols; ++c) {
    if (j0 + c < args.cols) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((need >> q) & 1)
          x[q][c] = *reinterpret_cast<const d2_t*>(args.src + args.blk[q] + i + (j0 + c) * args.ld);
    }
  }
  int slot = 0;
#pragma unroll
  for (int r = 0; r < 7; ++r) {
    const QProduct& P = kOneLevel[r];
    if ((SIDE == 0 ? P.na : P.nb) != 2) continue;
    if (args.single > 0 && r != args.single - 1) continue;
    const QTerm t0 = SIDE == 0 ? P.a[0] : P.b[0], t1 = SIDE == 0 ? P.a[1] : P.b[1];
    const double s1 = t1.sign;
    double* d = args.dst + (args.single > 0 ? 0 : slot) * args.dst_stride + i;
#pragma unroll
    for (int c = 0; c < kOuterSumCols; ++c) {
      if (j0 + c < args.cols) {
        d2_t v;
        v.x = __builtin_fma(s1, x[t1.q][c].x, x[t0.q][c].x);
        v.y = __builtin_fma(s1, x[t1.q][c].y, x[t0.q][c].y);
        *reinterpret_cast<d2_t*>(d + (j0 + c) * args.rows) = v;
      }
    }
    ++slot;
  }
}

// Winograd's variant, staged outer level: the same walk as outer_sum_kernel, writing the four
// chain sums of the side (A: S1 = X10 + X11, S2 = S1 - X00, S3 = X00 - X10, S4 = X01 - S2;
// B: T1 = X01 - X00, T2 = X11 - T1, T3 = X11 - X01, T4 = T2 - X10), each rounded once from the
// rounded sums before it, as the recursive algorithm forms them.
template <int SIDE>
__global__ __launch_bounds__(256) void chain_sum_kernel(const ChainSumArgs args) {
  const int64_t i = (int64_t)(blockIdx.x % args.chunks_r) * kOuterSumRows + 2 * threadIdx.x;
  const int64_t j0 = (int64_t)(blockIdx.x / args.chunks_r) * kOuterSumCols;
  if (i >= args.rows) return;
#pragma unroll
  for (int c = 0; c < kOuterSumCols; ++c) {
    if (j0 + c >= args.cols) break;
    d2_t x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      x[q] = *reinterpret_cast<const d2_t*>(args.src + args.blk[q] + i + (j0 + c) * args.ld);
    d2_t v[4];
    if (SIDE == 0) {
      v[0] = x[2] + x[3];
      v[1] = v[0] - x[0];
      v[2] = x[0] - x[2];
      v[3] = x[1] - v[1];
    } else {
      v[0] = x[1] - x[0];
      v[1] = x[3] - v[0];
      v[2] = x[3] - x[1];
      v[3] = v[1] - x[2];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      *reinterpret_cast<d2_t*>(args.dst + t * args.dst_stride + i + (j0 + c) * args.rows) = v[t];
  }
}

__global__ __launch_bounds__(256) void scale_kernel(const ScaleArgs args, int chunks_m) {
  const int64_t j = blockIdx.x / chunks_m;
  const int64_t i = (int64_t)(blockIdx.x % chunks_m) * 256 + threadIdx.x;
  if (i >= args.m || j >= args.n) return;
  double* p = args.C + i + j * args.ldc;
  *p = args.beta == 0.0 ? 0.0 : args.beta * *p;
}

// ---------------------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------------------
hipError_t upload_tables(const TableDev* tabs) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tables), tabs, sizeof(TableDev) * kNumTables, 0,
                           hipMemcpyHostToDevice);
}

template <int BM, int BN, int BK, int WPE, int MODE>
static void launch_mode(const GemmArgs& a, int maxt, bool vec, dim3 g, hipStream_t s) {
  const dim3 b(256);
  if constexpr (MODE == kModeABC) {
    if (a.tb) {   // B given transposed: one-term products (host-checked)
      if (vec) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 1, true, WPE, MODE, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 1, false, WPE, MODE, true>), g, b, 0, s, a);
      return;
    }
  }
  if (vec) {
    if (maxt == 1) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 1, true, WPE, MODE>), g, b, 0, s, a);
    else if (maxt == 2) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 2, true, WPE, MODE>), g, b, 0, s, a);
    else hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 4, true, WPE, MODE>), g, b, 0, s, a);
  } else {
    if (maxt == 1) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 1, false, WPE, MODE>), g, b, 0, s, a);
    else if (maxt == 2) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 2, false, WPE, MODE>), g, b, 0, s, a);
    else hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 4, false, WPE, MODE>), g, b, 0, s, a);
  }
}

template <int BM, int BN, int BK, int WPE>
static hipError_t launch_cfg(const GemmArgs& a, int maxt, bool vec, int grid, hipStream_t s) {
  if (a.mode == kModeABC) launch_mode<BM, BN, BK, WPE, kModeABC>(a, maxt, vec, dim3(grid), s);
  else launch_mode<BM, BN, BK, WPE, kModeStoreM>(a, maxt, vec, dim3(grid), s);
  return hipGetLastError();
}

hipError_t launch_fp64_tile(const GemmArgs& a, int cfg, int maxt, bool vec, int grid,
                            hipStream_t s) {
  switch (cfg) {
    case kCfg128: return launch_cfg<128, 128, 16, 2>(a, maxt, vec, grid, s);
    case kCfg128k8: return launch_cfg<128, 128, 8, 2>(a, maxt, vec, grid, s);
    case kCfg128w1: return launch_cfg<128, 128, 16, 1>(a, maxt, vec, grid, s);
    default: return launch_cfg<64, 64, 16, 2>(a, maxt, vec, grid, s);
  }
}

hipError_t launch_assemble(const AssembleArgs& a, int q2, hipStream_t s) {
  const int64_t grid = (int64_t)a.chunks_m * a.nq * q2;
  hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)grid), dim3(256), 0, s, a, q2);
  return hipGetLastError();
}

hipError_t launch_sums(const SumArgs& a, int nslots, hipStream_t s) {
  const int64_t gx = (int64_t)a.chunks_r * a.cols_q;
  hipLaunchKernelGGL(sum_kernel, dim3((unsigned)gx, nslots), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_outer_sums(const OuterSumArgs& a, int side, hipStream_t s) {
  OuterSumArgs b = a;
  b.chunks_r = (int32_t)((a.rows + kOuterSumRows - 1) / kOuterSumRows);
  const int64_t gx = (int64_t)b.chunks_r * ((a.cols + kOuterSumCols - 1) / kOuterSumCols);
  if (gx >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  if (side == 0) hipLaunchKernelGGL(outer_sum_kernel<0>, dim3((unsigned)gx), dim3(256), 0, s, b);
  else hipLaunchKernelGGL(outer_sum_kernel<1>, dim3((unsigned)gx), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_chain_sums(const ChainSumArgs& a, int side, hipStream_t s) {
  ChainSumArgs b = a;
  b.chunks_r = (int32_t)((a.rows + kOuterSumRows - 1) / kOuterSumRows);
  const int64_t gx = (int64_t)b.chunks_r * ((a.cols + kOuterSumCols - 1) / kOuterSumCols);
  if (gx >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  if (side == 0) hipLaunchKernelGGL(chain_sum_kernel<0>, dim3((unsigned)gx), dim3(256), 0, s, b);
  else hipLaunchKernelGGL(chain_sum_kernel<1>, dim3((unsigned)gx), dim3(256), 0, s, b);
  return hipGetLastError();
}

// Block-padded copy (PadArgs): one workgroup per column of the iterated matrix (the padded
// destination when padding, the plain destination when unpadding) and kPadRows consecutive rows
// of it, four rows per lane at a stride of 256 so that every access instruction of a wave covers
// contiguous addresses.  Extents fit 32 bits (checked by the launcher).
constexpr int kPadRows = 1024;

__global__ __launch_bounds__(256) void pad_copy_kernel(const PadArgs a) {
  const uint32_t j = blockIdx.x;
  const uint32_t i0 = blockIdx.y * kPadRows + threadIdx.x;
  const uint32_t rb = (uint32_t)a.rb, rb_e = (uint32_t)a.rb_e;
  if (!a.unpad) {
    const uint32_t bj = j / (uint32_t)a.cb_e, lj = j - bj * (uint32_t)a.cb_e;
    const int64_t js = (int64_t)bj * a.cb + lj;
    const bool col_ok = lj < (uint32_t)a.cb && js < a.cols;
    double* dcol = a.dst + (int64_t)j * a.ld_d;
    const double* scol = a.src + js * a.ld_s;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = i0 + 256u * u;
      if (i >= (uint32_t)a.dst_rows) break;
      const uint32_t bi = i / rb_e, li = i - bi * rb_e;
      const int64_t is = (int64_t)bi * rb + li;
      dcol[i] = (col_ok && li < rb && is < a.rows) ? scol[is] : 0.0;
    }
  } else {
    const uint32_t bj = j / (uint32_t)a.cb, lj = j - bj * (uint32_t)a.cb;
    const double* scol = a.src + ((int64_t)bj * a.cb_e + lj) * a.ld_s;
    double* dcol = a.dst + (int64_t)j * a.ld_d;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = i0 + 256u * u;
      if (i >= (uint32_t)a.rows) break;
      const uint32_t bi = i / rb, li = i - bi * rb;
      dcol[i] = scol[(int64_t)bi * rb_e + li];
    }
  }
}

hipError_t launch_pad_copy(const PadArgs& a, hipStream_t s) {
  const int64_t cols = a.unpad ? a.cols : a.dst_cols;
  const int64_t rows = a.unpad ? a.rows : a.dst_rows;
  const int64_t lim = int64_t(1) << 31;
  if (cols <= 0 || rows <= 0) return hipSuccess;
  if (cols >= lim || a.dst_rows >= lim || a.dst_cols >= lim || a.rb <= 0 || a.cb <= 0 ||
      a.rb_e < a.rb || a.cb_e < a.cb || (rows + kPadRows - 1) / kPadRows > 65535)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)cols, (unsigned)((rows + kPadRows - 1) / kPadRows));
  hipLaunchKernelGGL(pad_copy_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// Transposed copy (the packing of a transposed operand, Sec. 2.2 / Sec. 4.1): dst (rows x cols,
// leading dimension ld_d) := src^T with src cols x rows (ld_s).  A workgroup moves a 64 x 64
// block through LDS: it reads 64 consecutive elements of each source column (coalesced) and
// writes 64 consecutive elements of each destination column (coalesced).
constexpr int kTrT = 64;

__global__ __launch_bounds__(256) void transpose_kernel(const TransposeArgs a) {
  __shared__ double tile[kTrT][kTrT + 1];
  const int64_t bi = (int64_t)blockIdx.x * kTrT;   // destination rows (source columns)
  const int64_t bj = (int64_t)blockIdx.y * kTrT;   // destination columns (source rows)
  const int t = threadIdx.x, lo = t & 63, hi = t >> 6;
#pragma unroll
  for (int p = 0; p < kTrT / 4; ++p) {
    const int c = hi + 4 * p;                        // source column bi + c, row bj + lo
    const bool ok = bi + c < a.rows && bj + lo < a.cols;
    tile[c][lo] = ok ? a.src[(bj + lo) + (bi + c) * a.ld_s] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < kTrT / 4; ++p) {
    const int c = hi + 4 * p;                        // destination column bj + c, row bi + lo
    if (bi + lo < a.rows && bj + c < a.cols) a.dst[(bi + lo) + (bj + c) * a.ld_d] = tile[lo][c];
  }
}

hipError_t launch_transpose(const TransposeArgs& a, hipStream_t s) {
  if (a.rows <= 0 || a.cols <= 0) return hipSuccess;
  const int64_t gx = (a.rows + kTrT - 1) / kTrT, gy = (a.cols + kTrT - 1) / kTrT;
  if (gx >= (int64_t(1) << 31) || gy > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scale(const ScaleArgs& a, hipStream_t s) {
  const int chunks_m = (int)((a.m + 255) / 256);
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)(chunks_m * a.n)), dim3(256), 0, s, a, chunks_m);
  return hipGetLastError();
}

}  // namespace smx
