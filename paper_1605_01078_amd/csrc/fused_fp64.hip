// All-products FP64 Strassen kernel: the ABC variant (Sec. 4.1) with the seven products of one
// level computed side by side.
//
// A workgroup owns one 64 x 64 tile position in all four quadrants of C.  Each k step brings the
// matching 64 x BK tiles of the four A quadrants and BK x 64 tiles of the four B quadrants into
// LDS once; the operand sums of all seven products (Fig. "All operations for one-level
// Strassen") are then formed from those tiles at fragment-read time and fed to seven sets of
// FP64 MFMA accumulators, and at the end each C quadrant is read, updated with every product
// that feeds it (in increasing product order) and written once.  Per element of C this does
// what the one-level ABC algorithm does, with the tiles of A and B fetched once instead of once
// per product and C touched once instead of once per product.
//
// Two levels run as seven launches, one per outer product R of the one-level table (Sec. 3.5):
// launch R works on the virtual operands  sum_s delta_s A_s  and  sum_t eps_t B_t  of its outer
// terms (blocks of 2 x 2 inner sub-blocks), forming those outer sums from LDS as well, and adds
// its 7 inner products to the inner sub-blocks of its outer destinations.  Launches on one
// stream run in order, so every C element receives the 49 updates in increasing product index
// 7R + r, the order of the two-level table.
//
// Data movement
//   Tiles travel HBM -> LDS by buffer loads that write LDS directly (no registers), 16 bytes per
//   lane, double-buffered with one barrier per k step.  A tile columns are stored as loaded
//   (32 row pairs per k).  B tile columns hold BK/2 pairs of consecutive k; the pair index is
//   XOR-swizzled with the column so that sixteen lanes reading sixteen consecutive columns at
//   one pair index hit distinct banks.  Positions outside the matrix, its sub-blocks or the k
//   range get an offset past the buffer range and arrive as zeros (the zero padding of Sec. 3.3).
//
// Fragments
//   512 threads = 8 waves as 2 (rows) x 4 (columns); a wave owns rows [32 wm, 32 wm + 32) and
//   columns [16 wn, 16 wn + 16) of the tile in every product.  A 16-byte LDS read of A gives one
//   lane rows 2i and 2i + 1 (the even-row and odd-row accumulators), one of B gives k values
//   2g and 2g + 1; MFMA e of a group of eight k values takes k = 2g + e in lane group g.  The
//   MFMA takes B first and A second, so lane l, element e of accumulator (r, fm) holds product r
//   at tile row 32 wm + 2 (l % 16) + fm, column 16 wn + l / 16 + 4e; a C row pair is one 16-byte
//   access.
//
// Requirements (checked by the host, which otherwise uses the general tile kernel): m and k
// multiples of 2^(L+1) (all sub-blocks full, even extents), A, B, C 16-byte aligned, even
// leading dimensions.  n is arbitrary.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.h"
#include "plan.h"
#include "tile_fp64.h"

namespace smx {

namespace {

typedef __attribute__((address_space(3))) void* lds_ptr_t;

__device__ __forceinline__ lds_ptr_t to_lds(double* p) { return (lds_ptr_t)(p); }

// 16 bytes from global memory straight into LDS: lane i of the wave writes dst + 16 i bytes.
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, double* dst, uint32_t voff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, to_lds(dst), 16, voff, 0, 0, 0);
}

__device__ __forceinline__ d2_t fma2(double s, d2_t x, d2_t y) {
  return (d2_t){__builtin_fma(s, x.x, y.x), __builtin_fma(s, x.y, y.y)};
}

// FULL: every tile is whole (sub-block extents multiples of the tile, every B column present),
// so the loads need no per-lane range masks; the registers this frees keep the main loop free of
// spill reloads, whose wait on the vector-memory counter would also wait for the tile loads just
// issued and stall the pipeline.
// SCHEME 0: Strassen's one-level table; 1: Winograd's variant (one term per side only): the
// chain sums S1..S4 and T1..T4 are formed on the fragments in the chain's order (S2 from the
// rounded S1, and so on, as the recursive algorithm rounds them) and the C epilogue adds every
// product to each quadrant it reaches, in product order.
template <int NA, int NB, int BK, int NS, bool FULL, int SCHEME = 0>
struct AllProducts {
  static constexpr int T = 64;                    // tile edge inside one inner sub-block
  static constexpr int NT = 512;
  static constexpr int NPAIR = BK / 8;            // groups of eight k values per k step
  static constexpr int CPC = BK / 2;              // k pairs per B tile column
  static constexpr int TILE_D = T * BK;           // doubles per staged tile
  static constexpr int NTILES = 4 * (NA + NB);    // A tiles (term-major, quadrant minor), then B
  static constexpr int STAGE_D = NTILES * TILE_D;
  static constexpr int IPT = TILE_D / 128;        // 64-lane x 16-byte loads per tile
  static constexpr int IPW = NTILES * IPT / 8;    // per wave and k step
  static constexpr int LDS_D = NS * STAGE_D;      // NS stages in flight
  static constexpr int SWZ_SHIFT = CPC == 8 ? 1 : 2;   // 16 / CPC columns share a swizzle
  static_assert(BK == 8 || BK == 16, "k step");
  static_assert((NTILES * IPT) % 8 == 0 && (4 * NA * IPT) % 8 == 0, "load split");
  static_assert(NS == 2 || (NS == 3 && NPAIR == 1), "stages");
  static_assert(LDS_D * 8 <= 160 * 1024, "LDS");
  static_assert(SCHEME == 0 || (NA == 1 && NB == 1), "Winograd's variant: one term per side");

  typedef d4_t Acc[7][2];

  // STORE_M: the AB variant's form: every product M_r (unscaled) is stored to its temporary
  // (slot prod_base + r, leading dimension ldm) instead of being added to C.
  template <bool STORE_M>
  __device__ static void run(const FusedArgs& args, double* lds) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar addressing
    const int wm = wave & 1, wn = wave >> 1;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int ti, tj;
    tile_coords(logical, args.tiles_m, args.tiles_n, ti, tj);
    const int64_t i0 = (int64_t)ti * T, j0 = (int64_t)tj * T;
    const int64_t lda = args.lda, ldb = args.ldb, mq = args.mq, nq = args.nq, kq = args.kq;

    // ---- loads: which tile and which part of it this wave fills, and the lane's offsets ----
    // Load u = wave + 8 j (j < IPW) fills part v = u % IPT of tile u / IPT.  The lane's byte
    // offset inside a tile does not depend on the tile, only on v.
    const int v = wave % IPT;
    // A: position p = 64 v + lane -> k = p / 32, row pair p % 32
    const int a_k = (64 * v + lane) >> 5, a_r = 2 * (lane & 31);
    const uint32_t a_off = (uint32_t)(8 * (a_r + (int64_t)a_k * lda));
    const bool a_row_ok = i0 + a_r < mq;
    // B: position p = 64 v + lane -> column p / CPC, stored pair p % CPC = pair ^ swizzle(column)
    const int b_j = (64 * v + lane) / CPC;
    const int b_c = ((64 * v + lane) % CPC) ^ ((b_j >> SWZ_SHIFT) & (CPC - 1));
    const uint32_t b_off = (uint32_t)(8 * (2 * b_c + (int64_t)b_j * ldb));
    const bool b_col_in = j0 + b_j < nq;

    // Tile base of term s, inner quadrant q (uniform), and whether the lane's B column exists.
    auto a_tile = [&](int s, int q) {
      return args.A + args.a_off[s] + (q >> 1) * mq + (q & 1) * kq * lda + i0;
    };
    auto b_tile = [&](int s, int q) {
      return args.B + args.b_off[s] + (q >> 1) * kq + (q & 1) * nq * ldb + j0 * ldb;
    };
    // bit 4s + q: the lane's B column exists in term s, quadrant q
    uint32_t b_cols = 0;
#pragma unroll
    for (int s = 0; s < NB; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        b_cols |= (uint32_t)(b_col_in & ((args.b_cb[s] + (q & 1)) * nq + j0 + b_j < args.n))
                  << (4 * s + q);

    const int nk = (int)((kq + BK - 1) / BK);
    auto issue_loads = [&](int stage, int kt) {
      const int64_t kb = (int64_t)kt * BK;
      double* sbase = lds + stage * STAGE_D;
      const bool a_ok = a_row_ok & (kb + a_k < kq);
      const bool b_k_ok = kb + 2 * b_c < kq;
#pragma unroll
      for (int j = 0; j < IPW; ++j) {
        // Tile of load u = wave + 8 j.  With one term per side every tile's block offsets are
        // then compile-time indices into the arguments, loaded once instead of in every step
        // (with two terms the extra registers this takes cost more than the loads).
        const int t = (NA == 1 && NB == 1) ? (8 * j) / IPT + (wave & 7) / IPT : (wave + 8 * j) / IPT;
        double* dst = sbase + t * TILE_D + v * 128;
        if (8 * j < 4 * NA * IPT) {           // an A tile (compile-time split, see static_assert)
          dma16(make_rsrc(a_tile(t >> 2, t & 3) + kb * lda), dst,
                FULL ? (kt < nk ? a_off : kOOB) : (a_ok ? a_off : kOOB));
        } else {
          const int tb = t - 4 * NA;
          const bool ok = ((b_cols >> tb) & 1u) & b_k_ok;
          dma16(make_rsrc(b_tile(tb >> 2, tb & 3) + kb), dst,
                FULL ? (kt < nk ? b_off : kOOB) : (ok ? b_off : kOOB));
        }
      }
    };

    // ---- fragment reads (offsets in doubles inside a stage) ----
    // A (term s, quadrant q), group h, MFMA e: k = 8h + 2g + e, row pair 16 wm + lane % 16.
    const int g = lane >> 4;
    const int a_frag = (2 * g) * T + 2 * (16 * wm + (lane & 15));
    // B (term s, quadrant q), group h: column 16 wn + lane % 16, pair 4h + g (swizzled).
    const int fj = 16 * wn + (lane & 15);
    int b_frag[NPAIR];
#pragma unroll
    for (int h = 0; h < NPAIR; ++h)
      b_frag[h] = 4 * NA * TILE_D +
                  2 * (fj * CPC + ((4 * h + g) ^ ((fj >> SWZ_SHIFT) & (CPC - 1))));

    // Sign of the second outer term (the first one's is +1, host-checked).
    const double asg1 = args.a_sg[1], bsg1 = args.b_sg[1];

    // Outer sums of one group of eight k values: per inner quadrant q, the A row pairs for
    // MFMA e = 0, 1 and the B k pair.  x0 + s1 x1 in one FMA (the pair rule of signed_sum with a
    // first sign of +1).
    struct Frag {
      d2_t a[4][2];
      d2_t b[4];
    };
    auto load_frag = [&](int stage, int h, Frag& f) {
      const double* sb = lds + stage * STAGE_D;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int off = q * TILE_D + a_frag + (8 * h + e) * T;
          const d2_t x0 = *reinterpret_cast<const d2_t*>(sb + off);
          if (NA == 1) {
            f.a[q][e] = x0;
          } else {
            const d2_t x1 = *reinterpret_cast<const d2_t*>(sb + off + 4 * TILE_D);
            f.a[q][e] = fma2(asg1, x1, x0);
          }
        }
        const int offb = q * TILE_D + b_frag[h];
        const d2_t y0 = *reinterpret_cast<const d2_t*>(sb + offb);
        if (NB == 1) {
          f.b[q] = y0;
        } else {
          const d2_t y1 = *reinterpret_cast<const d2_t*>(sb + offb + 4 * TILE_D);
          f.b[q] = fma2(bsg1, y1, y0);
        }
      }
    };

    Acc acc;
#pragma unroll
    for (int r = 0; r < 7; ++r) {
      acc[r][0] = (d4_t){0.0, 0.0, 0.0, 0.0};
      acc[r][1] = (d4_t){0.0, 0.0, 0.0, 0.0};
    }

    // Winograd's variant: the chain sums (A: S1..S4 per MFMA e on row pairs; B: T1..T4 per e)
    // and the 28 MFMAs of one group of eight k values.
    auto mfma_frag_winograd = [&](const Frag& f) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        d2_t ao[8];
        double bo[8];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ao[q] = f.a[q][e];
          bo[q] = e == 0 ? f.b[q].x : f.b[q].y;
        }
        ao[4] = ao[2] + ao[3];   // S1 = A10 + A11
        ao[5] = ao[4] - ao[0];   // S2 = S1 - A00
        ao[6] = ao[0] - ao[2];   // S3 = A00 - A10
        ao[7] = ao[1] - ao[5];   // S4 = A01 - S2
        bo[4] = bo[1] - bo[0];   // T1 = B01 - B00
        bo[5] = bo[3] - bo[4];   // T2 = B11 - T1
        bo[6] = bo[3] - bo[1];   // T3 = B11 - B01
        bo[7] = bo[5] - bo[2];   // T4 = T2 - B10
#pragma unroll
        for (int r = 0; r < 7; ++r) {
          const WProduct& P = kWinograd[r];
          acc[r][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(bo[P.b], ao[P.a].x, acc[r][0], 0, 0, 0);
          acc[r][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(bo[P.b], ao[P.a].y, acc[r][1], 0, 0, 0);
        }
      }
    };

    // Inner sums (the one-level table; every first inner term has sign +1) and the 28 MFMAs of
    // one group of eight k values.
    auto mfma_frag = [&](const Frag& f) {
      if (SCHEME == 1) return mfma_frag_winograd(f);
#pragma unroll
      for (int r = 0; r < 7; ++r) {
        const QProduct& P = kOneLevel[r];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          d2_t af = f.a[P.a[0].q][e];
          if (P.na == 2) {
            if (P.a[1].sign > 0) af += f.a[P.a[1].q][e];
            else af -= f.a[P.a[1].q][e];
          }
          double bf = e == 0 ? f.b[P.b[0].q].x : f.b[P.b[0].q].y;
          if (P.nb == 2) {
            const double b1 = e == 0 ? f.b[P.b[1].q].x : f.b[P.b[1].q].y;
            if (P.b[1].sign > 0) bf += b1;
            else bf -= b1;
          }
          acc[r][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf, af.x, acc[r][0], 0, 0, 0);
          acc[r][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf, af.y, acc[r][1], 0, 0, 0);
        }
      }
    };

    // ---- main loop ----
    // The fragments of the next group of eight k values are read from LDS while the MFMAs of
    // the current group run (they do not depend on those reads); the instruction order is
    // pinned so the reads alternate with the first MFMAs.  Loads past the last step are out of
    // range (zeros, no memory access) and land in a stage nobody reads.
    constexpr int kReads = 8 * NA + 4 * NB;   // 16-byte LDS reads per wave and group
    auto interleave = [&]() {
#pragma unroll
      for (int i = 0; i < kReads; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 28 - kReads, 0);
    };
    // Second half of a k step: the LDS reads of the next group among the first MFMAs, the DMA
    // of the step after next spread over the later ones, so that waves leaving the barrier
    // together keep MFMAs queued while they issue it.
    auto interleave_dma = [&]() {
#pragma unroll
      for (int i = 0; i < 28; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        if (i < kReads) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
        if (i >= 6 && (i - 6) % 2 == 0 && (i - 6) / 2 < IPW)
          __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // one DMA
      }
    };
    // End of a stage: this wave's DMA of the step to be read next has landed (the NS - 2 newest
    // batches may still fly) and its LDS reads are done; then the barrier.  The waits are
    // explicit because a workgroup fence (as in __syncthreads) would also wait for every DMA in
    // flight, which serialises the deeper pipelines.
    auto sync_stage = [&]() {
      asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(IPW * (NS - 2)) : "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    };
    Frag f0, f1;
    if (NPAIR == 2) {
      // Two groups per stage, two stages.  Iteration kt: read group 1 of step kt during the
      // MFMAs of group 0; the barrier then has step kt + 1 landed and every read of step kt
      // done, so the DMA of step kt + 2 goes into its stage; read group 0 of step kt + 1
      // during the MFMAs of group 1.  Each DMA has one full step to land.  (The reads come
      // before the DMA in program order: the compiler cannot tell the stages apart and keeps
      // LDS reads after an earlier DMA into LDS.)
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
    } else {
      // One group per stage, NS stages; step kt lives in stage kt % NS.  Iteration kt issues
      // the DMA of step kt + NS into the stage of step kt (read during the previous
      // iteration), reads step kt + 1 and runs the MFMAs of step kt.  The barrier that ends
      // it has every read done and step kt + 2 landed (the NS - 2 newest DMA batches may
      // still fly).
#pragma unroll
      for (int st = 0; st < NS; ++st) issue_loads(st, st);
      sync_stage();
      load_frag(0, 0, f0);
      __syncthreads();   // stage 0 is refilled by the first iteration
      auto step = [&](int kt, int stage, Frag& now, Frag& next) {
        issue_loads(stage, kt + NS);
        load_frag(stage + 1 == NS ? 0 : stage + 1, 0, next);
        mfma_frag(now);
        interleave();
        sync_stage();
      };
      int kt = 0, stage = 0;
      for (; kt + 1 < nk; kt += 2) {
        step(kt, stage, f0, f1);
        stage = stage + 1 == NS ? 0 : stage + 1;
        step(kt + 1, stage, f1, f0);
        stage = stage + 1 == NS ? 0 : stage + 1;
      }
      if (kt < nk) step(kt, stage, f0, f1);
    }
    // no DMA may still be writing this workgroup's LDS when its waves end
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

    const int er = 32 * wm + 2 * (lane & 15);   // tile row of the lane's row pair
    const int ec = 16 * wn + (lane >> 4);       // tile column of element 0
    const bool e_row_ok = i0 + er < mq;
    if (STORE_M) {
      // ---- epilogue (AB): the seven products to their temporaries, a row pair per 16-byte
      // store with the whole offset in the lane offset (scalar offset 0: the compiler inserts
      // the wait state before the pair's registers are rewritten only for such stores) ----
      const int64_t ldm = args.ldm;
      const uint32_t m_off = (uint32_t)(8 * (er + (int64_t)ec * ldm));
#pragma unroll
      for (int r = 0; r < 7; ++r) {
        const __amdgpu_buffer_rsrc_t rs =
            make_rsrc(args.M + (int64_t)(args.prod_base + r) * args.m_stride + i0 + j0 * ldm);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = e_row_ok && j0 + ec + 4 * e < nq;
          d2_t v;
          v.x = acc[r][0][e];
          v.y = acc[r][1][e];
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4_t, v), rs,
                                                 ok ? m_off + (uint32_t)(8 * 4 * e * ldm) : kOOB,
                                                 0, 0);
        }
      }
      return;
    }

    // ---- epilogue: every C quadrant of every outer destination, read once, written once.
    // The case of each element's first update is chosen once per destination, and the sixteen
    // loads of a destination (four quadrants x four row pairs) are issued before its first
    // store: the vector memory counter counts loads and stores in one queue, so a store between
    // two loads would make the wait for the second load cover the store too.  Every access
    // carries its whole offset in the lane offset (scalar offset 0; below 2^31 bytes as
    // 8 * 64 * ldc < 2^31): the compiler inserts the wait state that a 16-byte store needs
    // before its data registers are rewritten only for stores without a scalar offset
    // register, and with the stores issued back to back the registers are rewritten at once. ----
    const int64_t ldc = args.ldc;
    const uint32_t e_off = (uint32_t)(8 * (er + (int64_t)ec * ldc));
    for (int d = 0; d < args.nc; ++d) {
      const double ag_outer = args.c_sg[d] * args.alpha;
      const bool first_outer = (args.c_first >> d) & 1;
      auto update = [&](auto case_tag) {
        constexpr int CASE = decltype(case_tag)::value;   // case of each element's first update
        __amdgpu_buffer_rsrc_t rs[4];
        uint32_t off[4][4];
        d2_t c[4][4];
#pragma unroll
        for (int cq = 0; cq < 4; ++cq) {
          const int64_t cb = args.c_cb[d] + (cq & 1);   // column block in units of nq
          rs[cq] = make_rsrc(args.C + args.c_off[d] + (cq >> 1) * mq + (cq & 1) * nq * ldc + i0 +
                             j0 * ldc);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t col = j0 + ec + 4 * e;
            const bool ok = e_row_ok && col < nq && cb * nq + col < args.n;
            off[cq][e] = ok ? e_off + (uint32_t)(8 * 4 * e * ldc) : kOOB;
            if constexpr (CASE == 1)
              c[cq][e] = (d2_t){0.0, 0.0};
            else
              c[cq][e] = __builtin_bit_cast(
                  d2_t, __builtin_amdgcn_raw_buffer_load_b128(rs[cq], off[cq][e], 0, 0));
          }
        }
#pragma unroll
        for (int cq = 0; cq < 4; ++cq)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            d2_t v = c[cq][e];
            bool first = true;
#pragma unroll
            for (int r = 0; r < 7; ++r) {
              const int nc = SCHEME == 1 ? kWinograd[r].nc : kOneLevel[r].nc;
#pragma unroll
              for (int dd = 0; dd < 4; ++dd) {
                const QTerm t = SCHEME == 1 ? kWinograd[r].c[dd] : kOneLevel[r].c[dd < 2 ? dd : 0];
                if (dd < nc && t.q == cq) {
                  const double ag = t.sign > 0 ? ag_outer : -ag_outer;
                  if (first) {
                    v.x = c_update_case<CASE>(v.x, acc[r][0][e], ag, args.beta);
                    v.y = c_update_case<CASE>(v.y, acc[r][1][e], ag, args.beta);
                  } else {
                    v.x = c_update_case<0>(v.x, acc[r][0][e], ag, args.beta);
                    v.y = c_update_case<0>(v.y, acc[r][1][e], ag, args.beta);
                  }
                  first = false;
                }
              }
            }
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4_t, v), rs[cq],
                                                   off[cq][e], 0, 0);
          }
      };
      if (!first_outer) update(std::integral_constant<int, 0>{});
      else if (args.beta == 0.0) update(std::integral_constant<int, 1>{});
      else update(std::integral_constant<int, 2>{});
    }
  }
};

template <int NA, int NB, int BK, int NS, bool FULL, int SCHEME = 0>
__global__ __launch_bounds__(512, 1) void all_products_kernel(const FusedArgs args) {
  using K = AllProducts<NA, NB, BK, NS, FULL, SCHEME>;
  __shared__ __attribute__((aligned(16))) double lds[K::LDS_D];
  K::template run<false>(args, lds);
}

// The AB variant on the same main loop: the products are stored, C is assembled afterwards.
template <int NA, int NB, int BK, int NS, bool FULL>
__global__ __launch_bounds__(512, 1) void all_products_store_kernel(const FusedArgs args) {
  using K = AllProducts<NA, NB, BK, NS, FULL>;
  __shared__ __attribute__((aligned(16))) double lds[K::LDS_D];
  K::template run<true>(args, lds);
}

}  // namespace

const void* all_products_fn(const FusedArgs& a, int na, int nb) {
  // whole tiles: sub-block extents multiples of 64 (m, n) and of the k step, and the B columns
  // of the highest column block used present
  int64_t cb_max = 0;
  for (int t = 0; t < nb; ++t) cb_max = cb_max > a.b_cb[t] ? cb_max : a.b_cb[t];
  const bool full = a.mq % 64 == 0 && a.nq % 64 == 0 && a.kq % 16 == 0 && (cb_max + 2) * a.nq <= a.n;
  if (a.store_m) {   // the AB form: one term per side (one level, or staged two-level sums)
    if (na != 1 || nb != 1 || a.scheme != 0) return nullptr;
    return full ? (const void*)all_products_store_kernel<1, 1, 16, 2, true>
                : (const void*)all_products_store_kernel<1, 1, 16, 2, false>;
  }
  if (a.scheme == 1) {   // Winograd's variant: ABC, one term per side
    if (na != 1 || nb != 1) return nullptr;
    return full ? (const void*)all_products_kernel<1, 1, 16, 2, true, 1>
                : (const void*)all_products_kernel<1, 1, 16, 2, false, 1>;
  }
  if (na == 1 && nb == 1 && full) return (const void*)all_products_kernel<1, 1, 16, 2, true>;
  if (na == 1 && nb == 1) return (const void*)all_products_kernel<1, 1, 16, 2, false>;
  // (the whole-tile form of the two-level kernels measured slower: they keep the masked loads)
  if (na == 2 && nb == 2) return (const void*)all_products_kernel<2, 2, 8, 2, false>;
  if (na == 2 && nb == 1) return (const void*)all_products_kernel<2, 1, 8, 3, false>;
  if (na == 1 && nb == 2) return (const void*)all_products_kernel<1, 2, 8, 3, false>;
  return nullptr;
}

hipError_t launch_all_products(const FusedArgs& a, int na, int nb, hipStream_t s) {
  const void* fn = all_products_fn(a, na, nb);
  if (!fn) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((int64_t)a.tiles_m * a.tiles_n)), block(512);
  void* args[] = {const_cast<FusedArgs*>(&a)};
  return hipLaunchKernel(fn, grid, block, args, 0, s);
}

}  // namespace smx
