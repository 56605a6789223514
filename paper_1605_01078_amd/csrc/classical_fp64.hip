// Classical FP64 GEMM (levels = 0), the yardstick of the effective-GFLOPS ratio (Sec. 5):
// C := alpha*A*B + beta*C on FP64 MFMA, fed by the all-products kernel's load path.
//
// A workgroup of 512 threads (8 waves as 4 rows x 2 columns) owns a 256 x 128 tile of C; each
// wave computes a 64 x 64 block of it as 2 x 4 pairs of 16 x 16 MFMA accumulators (even and odd
// rows of 32-row blocks, as in the all-products kernel).
//
// Data movement: every k step of 16 brings the 256 x 16 A tile and the 16 x 128 B tile from HBM
// into LDS by buffer loads that write LDS directly (16 bytes per lane, no registers), two stages,
// one barrier per step.  A is stored as loaded, k-major (row pairs); B as k pairs per column,
// the pair index XOR-swizzled by column so that sixteen lanes reading sixteen columns hit
// distinct banks.  Each load instruction has a wave-uniform base (the k row of A, or the first
// of the eight B columns it covers) and per-lane offsets that do not grow with the leading
// dimension of A and only span eight columns of B.  Positions outside the matrix read as zero.
//
// Fragments and MFMA order are those of every other FP64 kernel of the library: within each
// group of eight k values, lane group g takes k = 2g in the first MFMA and 2g + 1 in the second;
// the MFMA takes B first and A second, so lane l, element e of accumulator (fb, fm, fn) holds
// row 64 wm + 32 fb + 2 (l % 16) + fm, column 64 wn + 16 fn + l / 16 + 4 e, and a C row pair is
// one 16-byte access.  Every C element therefore receives exactly the FP64 operations of the
// general tile kernel at levels = 0 (bitwise the same result), then one update
// c = fma(alpha, acc, beta*c) (alpha*acc when beta = 0: C is not read).  One-level ABC (and
// Winograd's variant) run their seven products on this kernel with further destinations: the
// product is then added to each of its C quadrants (up to two, four for Winograd's M1), with
// the quadrant's coefficient, the first update of a quadrant applying beta: the C update of
// the all-products kernel, one product per launch.
//
// Requirements (checked by the host): m and k even, A, B, C 16-byte aligned, even leading
// dimensions, 8 * 64 * ldc < 2^31 and 8 * 8 * ldb < 2^31.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.h"
#include "plan.h"
#include "tile_fp64.h"

namespace smx {

namespace {

typedef __attribute__((address_space(3))) void* lds_ptr_t;

__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, double* dst, uint32_t voff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)(dst), 16, voff, 0, 0, 0);
}

template <bool FULL>
struct Classical {
  static constexpr int BM = 256, BN = 128, BK = 16, NS = 2, NT = 512;
  static constexpr int NPAIR = BK / 8;            // groups of eight k values per step
  static constexpr int CPC = BK / 2;              // k pairs per B column
  static constexpr int A_TILE = BM * BK;          // doubles
  static constexpr int B_TILE = BN * BK;
  static constexpr int STAGE = A_TILE + B_TILE;
  static constexpr int APW = A_TILE / 128 / 8;    // A load instructions per wave and step (4)
  static constexpr int BPW = B_TILE / 128 / 8;    // B (2)
  static constexpr int IPW = APW + BPW;
  static constexpr int FMB = 2, FN = 4;           // wave tile: 2 blocks of 32 rows, 4 of 16 columns
  static constexpr int LDS_D = NS * STAGE;
  static_assert(LDS_D * 8 <= 160 * 1024, "LDS");

  __device__ static void run(const ClassicalArgs& args, double* lds) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 3, wn = wave >> 2;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int ti, tj;
    tile_coords(logical, args.tiles_m, args.tiles_n, ti, tj);
    const int64_t i0 = (int64_t)ti * BM, j0 = (int64_t)tj * BN;
    const int64_t m = args.m, n = args.n, K = args.k, lda = args.lda, ldb = args.ldb;

    // ---- loads ----
    // A instruction v = wave + 8 j (j < APW): k row v / 2 of the step, rows 128 (v % 2) + 2 lane.
    const int a_half = wave & 1;
    const bool a_row_ok = FULL || i0 + 128 * a_half + 2 * lane < m;
    const uint32_t a_voff = 16u * lane;
    // B instruction v = wave + 8 j (j < BPW): columns 8 v .. 8 v + 7; lane l takes column
    // 8 v + l / 8 and stored pair slot l % 8, i.e. source pair (l % 8) ^ swizzle(column).
    const int b_cl = lane >> 3;
    uint32_t b_voff[BPW];
    bool b_col_ok[BPW];
    int b_pair[BPW];
#pragma unroll
    for (int j = 0; j < BPW; ++j) {
      const int col = 8 * (wave + 8 * j) + b_cl;   // column inside the tile
      b_pair[j] = (lane & 7) ^ ((col >> 1) & (CPC - 1));
      b_voff[j] = (uint32_t)(8 * (2 * b_pair[j] + (int64_t)b_cl * ldb));
      b_col_ok[j] = FULL || j0 + col < n;
    }

    const int nk = (int)((K + BK - 1) / BK);
    auto issue_loads = [&](int stage, int kt) {
      const int64_t kb = (int64_t)kt * BK;
      double* sbase = lds + stage * STAGE;
#pragma unroll
      for (int j = 0; j < APW; ++j) {
        const int v = wave + 8 * j;
        const int kr = v >> 1;
        const bool ok = kt < nk && a_row_ok && (FULL || kb + kr < K);
        dma16(make_rsrc(args.A + (kb + kr) * lda + i0 + 128 * a_half), sbase + v * 128,
              ok ? a_voff : kOOB);
      }
#pragma unroll
      for (int j = 0; j < BPW; ++j) {
        const int v = wave + 8 * j;
        const bool ok = kt < nk && b_col_ok[j] && (FULL || kb + 2 * b_pair[j] < K);
        dma16(make_rsrc(args.B + kb + (j0 + 8 * v) * ldb), sbase + A_TILE + v * 128,
              ok ? b_voff[j] : kOOB);
      }
    };

    // ---- fragments (offsets in doubles inside a stage) ----
    const int g = lane >> 4;
    // A block fb, group h, MFMA e: rows 64 wm + 32 fb + 2 (lane % 16) (+1), k = 8 h + 2 g + e
    const int a_frag = (2 * g) * BM + 64 * wm + 2 * (lane & 15);
    // B block fn, group h: column 64 wn + 16 fn + lane % 16, pair 4 h + g (swizzled)
    int b_frag[NPAIR][FN];
#pragma unroll
    for (int h = 0; h < NPAIR; ++h)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) {
        const int col = 64 * wn + 16 * fn + (lane & 15);
        b_frag[h][fn] = A_TILE + 2 * (col * CPC + ((4 * h + g) ^ ((col >> 1) & (CPC - 1))));
      }

    struct Frag {
      d2_t a[FMB][2];
      d2_t b[FN];
    };
    auto load_frag = [&](int stage, int h, Frag& f) {
      const double* sb = lds + stage * STAGE;
#pragma unroll
      for (int fb = 0; fb < FMB; ++fb)
#pragma unroll
        for (int e = 0; e < 2; ++e)
          f.a[fb][e] = *reinterpret_cast<const d2_t*>(sb + a_frag + (8 * h + e) * BM + 32 * fb);
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) f.b[fn] = *reinterpret_cast<const d2_t*>(sb + b_frag[h][fn]);
    };

    d4_t acc[FMB][2][FN];
#pragma unroll
    for (int fb = 0; fb < FMB; ++fb)
#pragma unroll
      for (int fm = 0; fm < 2; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) acc[fb][fm][fn] = (d4_t){0.0, 0.0, 0.0, 0.0};

    // the 32 MFMAs of one group of eight k values, each accumulator taking e = 0 then e = 1
    auto mfma_frag = [&](const Frag& f) {
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int fb = 0; fb < FMB; ++fb)
#pragma unroll
          for (int fn = 0; fn < FN; ++fn) {
            const double bf = e == 0 ? f.b[fn].x : f.b[fn].y;
            acc[fb][0][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf, f.a[fb][e].x, acc[fb][0][fn], 0, 0, 0);
            acc[fb][1][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf, f.a[fb][e].y, acc[fb][1][fn], 0, 0, 0);
          }
    };

    constexpr int kReads = 2 * FMB + FN;    // 16-byte LDS reads per wave and group
    constexpr int kMfma = 2 * 2 * FMB * FN; // MFMAs per wave and group
    auto interleave = [&]() {
#pragma unroll
      for (int i = 0; i < kReads; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
      }
      __builtin_amdgcn_sched_group_barrier(0x008, kMfma - kReads, 0);
    };
    auto interleave_dma = [&]() {
#pragma unroll
      for (int i = 0; i < kMfma; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        if (i < kReads) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
        if (i >= 8 && (i - 8) % 3 == 0 && (i - 8) / 3 < IPW)
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // one DMA
      }
    };
    auto sync_stage = [&]() {
      asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(IPW * (NS - 2)) : "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    };

    // ---- main loop: two groups per step, two stages (the all-products kernel's schedule) ----
    Frag f0, f1;
    issue_loads(0, 0);
    issue_loads(1, 1);
    sync_stage();
    load_frag(0, 0, f0);
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      load_frag(cur, 1, f1);
      mfma_frag(f0);
      interleave();
      sync_stage();
      load_frag(cur ^ 1, 0, f0);
      issue_loads(cur, kt + 2);
      mfma_frag(f1);
      interleave_dma();
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

    // ---- epilogue: C row pairs of each destination, read once (unless its first update has
    // beta == 0), updated, written once.  The update's case is chosen once per destination and
    // each 32-row block's sixteen loads are issued before its first store: the vector memory
    // counter counts loads and stores in one queue, so a store between two loads would make
    // the wait for the second load cover the store too (one round trip per row pair). ----
    const int64_t ldc = args.ldc;
    const double beta = args.beta;
    for (int d = 0; d <= args.extra; ++d) {
      const double alpha = d == 0 ? args.alpha : (d == 1 ? args.ax[0] : (d == 2 ? args.ax[1] : args.ax[2]));
      double* const cd = d == 0 ? args.C : (d == 1 ? args.Cx[0] : (d == 2 ? args.Cx[1] : args.Cx[2]));
      const bool first = !((args.not_first >> d) & 1);
      const __amdgpu_buffer_rsrc_t rs = make_rsrc(cd + i0 + (j0 + 64 * wn) * ldc);
      auto update = [&](auto case_tag) {
        constexpr int CASE = decltype(case_tag)::value;
#pragma unroll
        for (int fb = 0; fb < FMB; ++fb) {
          const int er = 64 * wm + 32 * fb + 2 * (lane & 15);
          const bool row_ok = FULL || i0 + er < m;
          uint32_t off[FN][4];
          d2_t c[FN][4];
#pragma unroll
          for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int ec = 16 * fn + (lane >> 4) + 4 * e;   // column inside the wave's block
              const bool ok = row_ok && (FULL || j0 + 64 * wn + ec < n);
              off[fn][e] = ok ? (uint32_t)(8 * (er + (int64_t)ec * ldc)) : kOOB;
              if constexpr (CASE == 1)
                c[fn][e] = (d2_t){0.0, 0.0};
              else
                c[fn][e] = __builtin_bit_cast(
                    d2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off[fn][e], 0, 0));
            }
#pragma unroll
          for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              d2_t v;
              v.x = c_update_case<CASE>(c[fn][e].x, acc[fb][0][fn][e], alpha, beta);
              v.y = c_update_case<CASE>(c[fn][e].y, acc[fb][1][fn][e], alpha, beta);
              __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4_t, v), rs, off[fn][e],
                                                     0, 0);
            }
        }
      };
      if (!first) update(std::integral_constant<int, 0>{});
      else if (beta == 0.0) update(std::integral_constant<int, 1>{});
      else update(std::integral_constant<int, 2>{});
    }
  }
};

template <bool FULL>
__global__ __launch_bounds__(512, 1) void classical_kernel(const ClassicalArgs args) {
  using K = Classical<FULL>;
  __shared__ __attribute__((aligned(16))) double lds[K::LDS_D];
  K::run(args, lds);
}

}  // namespace

hipError_t launch_classical(const ClassicalArgs& a, hipStream_t s) {
  const bool full = a.m % 256 == 0 && a.n % 128 == 0 && a.k % 16 == 0;
  const dim3 grid((unsigned)((int64_t)a.tiles_m * a.tiles_n)), block(512);
  if (full) hipLaunchKernelGGL(classical_kernel<true>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(classical_kernel<false>, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace smx
