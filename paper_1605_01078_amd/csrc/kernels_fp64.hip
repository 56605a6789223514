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

namespace smx {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

__constant__ TableDev g_tables[kNumTables];

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int code_row(uint8_t c) { return c & 7; }
__device__ __forceinline__ int code_col(uint8_t c) { return (c >> 3) & 7; }
__device__ __forceinline__ bool code_neg(uint8_t c) { return (c & 0x80) != 0; }

// One C update.  Every variant goes through this function in the same product order, so
// ABC, AB and Naive give bitwise identical results for the same table.
__device__ __forceinline__ double c_update(double c, double mv, double ag, double beta,
                                           bool first) {
  if (!first) return __builtin_fma(ag, mv, c);
  if (beta == 0.0) return ag * mv;
  return __builtin_fma(ag, mv, beta * c);
}

// Signed operand sum, term by term in table order: v = +-x0, then v = v +- x_s.
__device__ __forceinline__ double sum_first(double x, bool neg) { return neg ? -x : x; }
__device__ __forceinline__ double sum_next(double v, double x, bool neg) {
  return neg ? v - x : v + x;
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b % 8).
// Give each XCD a contiguous range of logical ids so neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_remap(int b, int nwg) {
  const int per = nwg >> 3, rem = nwg & 7, x = b & 7, idx = b >> 3;
  return x * per + min(x, rem) + idx;
}

// Logical tile id -> (ti, tj), walking groups of 8 tile rows column by column so that the
// workgroups resident at one time cover a compact block of C (operand panels reused in L2).
__device__ __forceinline__ void tile_coords(int t, int tiles_m, int tiles_n, int& ti, int& tj) {
  constexpr int G = 8;
  const int per_group = G * tiles_n;
  const int group = t / per_group;
  const int first = group * G;
  const int gsize = min(tiles_m - first, G);
  const int w = t - group * per_group;
  ti = first + w % gsize;
  tj = w / gsize;
}

// ---------------------------------------------------------------------------------------------
// FP64 tile kernel.
//   256 threads = 4 waves in a 2 x 2 arrangement; each wave owns a (BM/2) x (BN/2) block of the
//   tile as (BM/32) x (BN/32) MFMA 16x16 accumulators.  LDS holds two stages of
//   As[BK][BM] (k-major) and Bs[BK][BN + 1] (k-major, padded so the transposing store of the
//   column-major B tile is free of bank conflicts).
//   The MFMA is fed B as its first operand and A as its second, so it produces the transposed
//   16x16 block: lane l, element e holds C(row l % 16, column l / 16 + 4e), i.e. 16 lanes cover
//   16 consecutive rows of one column and the column-major C updates are coalesced.
// ---------------------------------------------------------------------------------------------
template <int BM, int BN, int BK, int MAXT, bool VEC>
__global__ __launch_bounds__(256, 2) void fp64_tile_kernel(const GemmArgs args) {
  constexpr int NT = 256;
  constexpr int A_TPC = BM / 2;          // threads per A tile column (2 rows each)
  constexpr int A_CPP = NT / A_TPC;      // A tile columns per load pass
  constexpr int A_PASSES = BK / A_CPP;
  constexpr int B_TPC = BK / 2;          // threads per B tile column (2 k each)
  constexpr int B_CPP = NT / B_TPC;
  constexpr int B_PASSES = BN / B_CPP;
  constexpr int LDA_S = BM;
  constexpr int LDB_S = BN + 1;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(A_PASSES >= 1 && B_PASSES >= 1 && BK % 4 == 0, "tile shape");

  __shared__ double As[2][BK * LDA_S];
  __shared__ double Bs[2][BK * LDB_S];

  const TableDev& tab = g_tables[args.tab];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int a_row = 2 * (tid % A_TPC), a_col = tid / A_TPC;
  const int b_k = 2 * (tid % B_TPC), b_col = tid / B_TPC;

  const int T = args.tiles_m * args.tiles_n;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  int r_begin, r_end, tile;
  if (args.mode == kModeABC) {
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
  const int nk = (int)((args.kq + BK - 1) / BK);

  for (int r = r_begin; r < r_end; ++r) {
    const ProdDesc& pd = tab.prod[r];
    const int na = pd.na, nb = pd.nb;

    // Operand terms: base pointer, leading dimension, valid extent inside the sub-block.
    const double* a_ptr[MAXT];
    const double* a_safe[MAXT];
    int64_t a_ld[MAXT], a_rlim[MAXT], a_klim[MAXT];
    bool a_neg[MAXT];
    const double* b_ptr[MAXT];
    const double* b_safe[MAXT];
    int64_t b_ld[MAXT], b_klim[MAXT], b_clim[MAXT];
    bool b_neg[MAXT];
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
      const uint8_t ca = s < na ? pd.a[s] : 0;
      if (pd.flags & 1) {  // Naive temporary (zero-padded to the full sub-block)
        a_ptr[s] = args.TA + (int64_t)pd.tslot_a * args.ta_stride;
        a_safe[s] = args.TA;
        a_ld[s] = args.mq;
        a_rlim[s] = args.mq;
        a_klim[s] = args.kq;
        a_neg[s] = false;
      } else {
        const int64_t bi = code_row(ca), bp = code_col(ca);
        a_ptr[s] = args.A + bi * args.mq + bp * args.kq * args.lda;
        a_safe[s] = args.A;
        a_ld[s] = args.lda;
        a_rlim[s] = min64(args.mq, args.m - bi * args.mq);
        a_klim[s] = min64(args.kq, args.k - bp * args.kq);
        a_neg[s] = code_neg(ca);
      }
      const uint8_t cb = s < nb ? pd.b[s] : 0;
      if (pd.flags & 2) {
        b_ptr[s] = args.TB + (int64_t)pd.tslot_b * args.tb_stride;
        b_safe[s] = args.TB;
        b_ld[s] = args.kq;
        b_klim[s] = args.kq;
        b_clim[s] = args.nq;
        b_neg[s] = false;
      } else {
        const int64_t bp = code_row(cb), bj = code_col(cb);
        b_ptr[s] = args.B + bp * args.kq + bj * args.nq * args.ldb;
        b_safe[s] = args.B;
        b_ld[s] = args.ldb;
        b_klim[s] = min64(args.kq, args.k - bp * args.kq);
        b_clim[s] = min64(args.nq, args.n - bj * args.nq);
        b_neg[s] = code_neg(cb);
      }
    }

    d2_t ra[MAXT][A_PASSES], rb[MAXT][B_PASSES];

    // Global loads of k step kt for every term (out-of-range positions read a safe address
    // and are replaced by zero, so no lane branches around a load).
    auto load_stage = [&](int kt) {
      const int64_t kb = (int64_t)kt * BK;
#pragma unroll
      for (int s = 0; s < MAXT; ++s) {
        if (s < na) {
          const int64_t rr = row0 + a_row;
#pragma unroll
          for (int p = 0; p < A_PASSES; ++p) {
            const int64_t kk = kb + a_col + p * A_CPP;
            const bool kok = kk < a_klim[s];
            const double* src = a_ptr[s] + rr + kk * a_ld[s];
            if (VEC) {
              const bool ok = kok && rr < a_rlim[s];
              const d2_t v = *reinterpret_cast<const d2_t*>(ok ? src : a_safe[s]);
              ra[s][p] = ok ? v : (d2_t){0.0, 0.0};
            } else {
              const bool ok0 = kok && rr < a_rlim[s];
              const bool ok1 = kok && rr + 1 < a_rlim[s];
              const double v0 = *(ok0 ? src : a_safe[s]);
              const double v1 = *(ok1 ? src + 1 : a_safe[s]);
              ra[s][p] = (d2_t){ok0 ? v0 : 0.0, ok1 ? v1 : 0.0};
            }
          }
        }
        if (s < nb) {
          const int64_t kk = kb + b_k;
#pragma unroll
          for (int p = 0; p < B_PASSES; ++p) {
            const int64_t cc = col0 + b_col + p * B_CPP;
            const bool cok = cc < b_clim[s];
            const double* src = b_ptr[s] + kk + cc * b_ld[s];
            if (VEC) {
              const bool ok = cok && kk < b_klim[s];
              const d2_t v = *reinterpret_cast<const d2_t*>(ok ? src : b_safe[s]);
              rb[s][p] = ok ? v : (d2_t){0.0, 0.0};
            } else {
              const bool ok0 = cok && kk < b_klim[s];
              const bool ok1 = cok && kk + 1 < b_klim[s];
              const double v0 = *(ok0 ? src : b_safe[s]);
              const double v1 = *(ok1 ? src + 1 : b_safe[s]);
              rb[s][p] = (d2_t){ok0 ? v0 : 0.0, ok1 ? v1 : 0.0};
            }
          }
        }
      }
    };

    // Signed sums in registers, then into LDS stage `buf`.
    auto store_stage = [&](int buf) {
#pragma unroll
      for (int p = 0; p < A_PASSES; ++p) {
        double v0 = sum_first(ra[0][p].x, a_neg[0]);
        double v1 = sum_first(ra[0][p].y, a_neg[0]);
#pragma unroll
        for (int s = 1; s < MAXT; ++s)
          if (s < na) {
            v0 = sum_next(v0, ra[s][p].x, a_neg[s]);
            v1 = sum_next(v1, ra[s][p].y, a_neg[s]);
          }
        *reinterpret_cast<d2_t*>(&As[buf][(a_col + p * A_CPP) * LDA_S + a_row]) =
            (d2_t){v0, v1};
      }
#pragma unroll
      for (int p = 0; p < B_PASSES; ++p) {
        double v0 = sum_first(rb[0][p].x, b_neg[0]);
        double v1 = sum_first(rb[0][p].y, b_neg[0]);
#pragma unroll
        for (int s = 1; s < MAXT; ++s)
          if (s < nb) {
            v0 = sum_next(v0, rb[s][p].x, b_neg[s]);
            v1 = sum_next(v1, rb[s][p].y, b_neg[s]);
          }
        const int j = b_col + p * B_CPP;
        Bs[buf][b_k * LDB_S + j] = v0;
        Bs[buf][(b_k + 1) * LDB_S + j] = v1;
      }
    };

    d4_t acc[FM][FN];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = (d4_t){0.0, 0.0, 0.0, 0.0};

    auto mfma_stage = [&](int buf) {
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        double af[FM], bf[FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
          af[fm] = As[buf][kr * LDA_S + wm * WM + fm * 16 + (lane & 15)];
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
          bf[fn] = Bs[buf][kr * LDB_S + wn * WN + fn * 16 + (lane & 15)];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < FN; ++fn)
            acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[fn], af[fm], acc[fm][fn], 0, 0, 0);
      }
    };

    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      if (kt + 1 < nk) load_stage(kt + 1);
      mfma_stage(cur);
      if (kt + 1 < nk) store_stage(cur ^ 1);
      __syncthreads();
    }

    // Epilogue.
    const int lrow = wm * WM + (lane & 15);
    const int lcol = wn * WN + (lane >> 4);
    if (args.mode == kModeABC) {
      for (int d = 0; d < pd.nc; ++d) {
        const uint8_t cc = pd.c[d];
        const int64_t ci = code_row(cc), cj = code_col(cc);
        const double ag = code_neg(cc) ? -args.alpha : args.alpha;
        const bool first = (pd.first >> d) & 1;
        const int64_t rlim = min64(args.mq, args.m - ci * args.mq) - row0;
        const int64_t clim = min64(args.nq, args.n - cj * args.nq) - col0;
        double* cbase = args.C + (ci * args.mq + row0) + (cj * args.nq + col0) * args.ldc;
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int rr = lrow + fm * 16, cc2 = lcol + fn * 16 + 4 * e;
              if (rr < rlim && cc2 < clim) {
                double* p = cbase + rr + (int64_t)cc2 * args.ldc;
                *p = c_update(*p, acc[fm][fn][e], ag, args.beta, first);
              }
            }
      }
    } else {
      const int64_t rlim = args.mq - row0, clim = args.nq - col0;
      double* mbase = args.M + (int64_t)r * args.m_stride + row0 + col0 * args.ldm;
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int rr = lrow + fm * 16, cc2 = lcol + fn * 16 + 4 * e;
            if (rr < rlim && cc2 < clim) mbase[rr + (int64_t)cc2 * args.ldm] = acc[fm][fn][e];
          }
    }
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
  double v = 0.0;
  for (int t = 0; t < nt; ++t) {
    const uint8_t code = codes[t];
    const int64_t row = code_row(code) * args.rows_q + i;
    const int64_t col = code_col(code) * args.cols_q + j;
    const bool ok = row < args.rows && col < args.cols;
    const double x = ok ? args.src[row + col * args.ld] : 0.0;
    v = t == 0 ? sum_first(x, code_neg(code)) : sum_next(v, x, code_neg(code));
  }
  args.dst[(int64_t)slot * args.dst_stride + i + j * args.rows_q] = v;
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

template <int BM, int BN, int BK>
static hipError_t launch_cfg(const GemmArgs& a, int maxt, bool vec, int grid, hipStream_t s) {
  const dim3 g(grid), b(256);
  if (vec) {
    if (maxt == 1) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 1, true>), g, b, 0, s, a);
    else if (maxt == 2) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 2, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 4, true>), g, b, 0, s, a);
  } else {
    if (maxt == 1) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 1, false>), g, b, 0, s, a);
    else if (maxt == 2) hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 2, false>), g, b, 0, s, a);
    else hipLaunchKernelGGL((fp64_tile_kernel<BM, BN, BK, 4, false>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fp64_tile(const GemmArgs& a, int cfg, int maxt, bool vec, int grid,
                            hipStream_t s) {
  if (cfg == kCfg128) return launch_cfg<128, 128, 16>(a, maxt, vec, grid, s);
  return launch_cfg<64, 64, 16>(a, maxt, vec, grid, s);
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

hipError_t launch_scale(const ScaleArgs& a, hipStream_t s) {
  const int chunks_m = (int)((a.m + 255) / 256);
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)(chunks_m * a.n)), dim3(256), 0, s, a, chunks_m);
  return hipGetLastError();
}

}  // namespace smx
