// Reduced-precision mode: the Strassen products on BF16 MFMA (v_mfma_f32_16x16x32_bf16) with
// FP32 accumulation; the operand sums and the C update stay in FP32 or FP64.
//
// A bf16 operand can only be formed once its full-precision sum exists, so the mode runs in two
// passes:
//   cast_kernel     forms, for every product r, the A-side sum  sum_s delta_s X_s  and the B-side
//                   sum over the zero-padded sub-blocks (FP64, or FP32 with every term rounded to
//                   FP32 first; pairs as c0*(x0 + (c0*c1) x1), four terms as the sum of the two
//                   pairs, as in the FP64 kernels), rounds it to FP32, and writes hi = bf16(x)
//                   (and lo = bf16(x - hi) for bf16x3), rounding to nearest even.  Both sides are
//                   stored k-contiguous: A-side slot r holds row i at [i * kpad, +kpad), B-side
//                   slot r column j at [j * kpad, +kpad); padding is zero.  This pass is bound
//                   by HBM bandwidth.
//   bf16_gemm_kernel  owns one 128 x 128 tile position in every C sub-block and runs every
//                   product on it in table order (ABC epilogue: each product is added to each of
//                   its destination C sub-blocks, beta at the first update).  BF16 operands go
//                   HBM -> LDS by direct-to-LDS buffer loads in two stages (k step 64, 32 for
//                   bf16x3), streamed across the product boundary, two workgroups per CU; bf16x3
//                   runs hi*hi + hi*lo + lo*hi into the same FP32 accumulator.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "plan.h"
#include "tile_fp64.h"

namespace smx {

__constant__ TableDev g_tables_bf16[kNumTables];

hipError_t upload_tables_bf16(const TableDev* tabs) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tables_bf16), tabs, sizeof(TableDev) * kNumTables, 0,
                           hipMemcpyHostToDevice);
}

namespace {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

// float -> bf16 bits, round to nearest, ties to even (NaN -> quiet NaN).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  const uint32_t b = __builtin_bit_cast(uint32_t, x);
  if ((b & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  return (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// ---------------------------------------------------------------------------------------------
// Operand pass.  One workgroup: a 64 (outer index) x 64 (k) block of one product's operand.
// ---------------------------------------------------------------------------------------------
constexpr int kCastT = 64;

template <int NT, bool F64>
__device__ __forceinline__ float pair_rule_sum(const double* x, const double* sg) {
  if (F64) return (float)signed_sum<NT>(sg, x);
  float xf[NT], sf[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    xf[t] = (float)x[t];
    sf[t] = (float)sg[t];
  }
  if (NT == 1) return sf[0] * xf[0];
  const float p01 = sf[0] * (xf[0] + (sf[0] * sf[1]) * xf[1]);
  if (NT == 2) return p01;
  return p01 + sf[2] * (xf[2] + (sf[2] * sf[3]) * xf[3]);
}

// Each thread sums one source row of a 64 x 64 block across 16 consecutive columns: lane l of
// wave w takes row l and columns 16 w .. 16 w + 15, so every load instruction of a wave reads 64
// consecutive doubles of one column (coalesced).  The term pointers and their valid extents are
// set up once per thread; the element loop only loads and adds.
template <int NT, bool F64>
__device__ __forceinline__ void cast_row(const CastArgs& args, const ProdDesc& pd, int64_t o0,
                                         int64_t k0, int row_local, int col_base, float* v) {
  const uint8_t* codes = args.side == 0 ? pd.a : pd.b;
  // per term: a buffer over the workgroup's block of the term (uniform base), the lane's byte
  // offset in it and how many of its 16 columns exist; missing ones get an offset past the
  // buffer range and load as zero, without a branch
  __amdgpu_buffer_rsrc_t rs[NT];
  uint32_t off[NT];
  int ncol[NT];
  double sg[NT];
  const int64_t r_blk = args.side == 0 ? o0 : k0, c_blk = args.side == 0 ? k0 : o0;
#pragma unroll
  for (int s = 0; s < NT; ++s) {
    const uint8_t c = codes[s];
    const int64_t br = code_row(c), bc = code_col(c);
    const int64_t r_ext = min64(args.rq, args.rows - br * args.rq);   // valid rows of the block
    const int64_t c_ext = min64(args.cq, args.cols - bc * args.cq);
    rs[s] = make_rsrc(args.src + (br * args.rq + r_blk) + (bc * args.cq + c_blk) * args.ld);
    const bool row_ok = r_blk + row_local < r_ext;
    ncol[s] = row_ok ? (int)min64(16, max(int64_t(0), c_ext - c_blk - col_base)) : 0;
    off[s] = (uint32_t)(8 * (row_local + (int64_t)col_base * args.ld));
    sg[s] = code_neg(c) ? -1.0 : 1.0;
  }
  double xs[NT][16];
#pragma unroll
  for (int s = 0; s < NT; ++s)
#pragma unroll
    for (int e = 0; e < 16; ++e)
      xs[s][e] = __builtin_bit_cast(
          double, __builtin_amdgcn_raw_buffer_load_b64(
                      rs[s], e < ncol[s] ? off[s] + (uint32_t)(8 * e * args.ld) : kOOB, 0, 0));
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    double x[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) x[s] = xs[s][e];
    v[e] = pair_rule_sum<NT, F64>(x, sg);
  }
}

// Workgroup b takes slot b % nslots of block position b / nslots (outer block fastest, then k
// block): the slots of one block position run back to back, so the operand blocks they share
// are read from HBM about once and then from L2.
template <bool F64>
__global__ __launch_bounds__(256) void cast_kernel(const CastArgs args, int nslots, int blocks_o) {
  __shared__ float tile[kCastT][kCastT + 1];
  const TableDev& tab = g_tables_bf16[args.tab];
  const int slot = (int)(blockIdx.x % (unsigned)nslots);
  const int pos = (int)(blockIdx.x / (unsigned)nslots);
  const ProdDesc& pd = tab.prod[slot];
  const int nt = args.side == 0 ? pd.na : pd.nb;
  const int64_t o0 = (int64_t)(pos % blocks_o) * kCastT;   // outer index (A: row, B: column)
  const int64_t k0 = (int64_t)(pos / blocks_o) * kCastT;
  const int t = threadIdx.x;
  const size_t slot_off = (size_t)slot * args.slot_stride;
  auto store16 = [&](int64_t o, int64_t kc, const float* v) {
    // 16 consecutive k of outer index o: hi (and lo) as two 16-byte stores each
    uint32_t hw[8], lw[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint16_t h0 = bf16_bits(v[2 * e]), h1 = bf16_bits(v[2 * e + 1]);
      hw[e] = (uint32_t)h0 | ((uint32_t)h1 << 16);
      const uint16_t l0 = bf16_bits(v[2 * e] - bf16_value(h0));
      const uint16_t l1 = bf16_bits(v[2 * e + 1] - bf16_value(h1));
      lw[e] = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
    const size_t off = slot_off + (size_t)o * args.kpad + kc;
    u4_t* dh = reinterpret_cast<u4_t*>(args.hi + off);
    dh[0] = (u4_t){hw[0], hw[1], hw[2], hw[3]};
    dh[1] = (u4_t){hw[4], hw[5], hw[6], hw[7]};
    if (args.lo) {
      u4_t* dl = reinterpret_cast<u4_t*>(args.lo + off);
      dl[0] = (u4_t){lw[0], lw[1], lw[2], lw[3]};
      dl[1] = (u4_t){lw[4], lw[5], lw[6], lw[7]};
    }
  };
  const int rl = t & 63, cb = (t >> 6) * 16;   // row within the block, first of 16 columns
  float v[16];
  if (nt == 1) cast_row<1, F64>(args, pd, o0, k0, rl, cb, v);
  else if (nt == 2) cast_row<2, F64>(args, pd, o0, k0, rl, cb, v);
  else cast_row<4, F64>(args, pd, o0, k0, rl, cb, v);
  if (args.side == 0) {   // A: row rl is outer index o0 + rl, the columns are k values k0 + cb..
    store16(o0 + rl, k0 + cb, v);
    return;
  }
  // B: row rl is k value k0 + rl, the columns are outer indices o0 + cb..; transpose via LDS
#pragma unroll
  for (int e = 0; e < 16; ++e) tile[cb + e][rl] = v[e];
  __syncthreads();
  const int oo = t >> 2, kc = (t & 3) * 16;
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = tile[oo][kc + e];
  store16(o0 + oo, k0 + kc, v);
}

// ---------------------------------------------------------------------------------------------
// BF16 product kernel.
// ---------------------------------------------------------------------------------------------
// Tiles: BM x BN per workgroup, NWM x NWN waves, each wave a WTM x WTN block (WTM / 16 x WTN / 16
// blocks of 16 x 16 MFMA), k step BK (bf16 elements).  Stage s holds the tiles of stream
// position s: A hi, B hi (, A lo, B lo), A tiles BM rows and B tiles BN rows of BK values,
// 16-byte chunks XOR-swizzled by row (swz).  The 128 x 128 form runs four waves of 64 x 64; the
// 128 x 64 form (four waves of 64 x 32, half again the LDS reads per flop) doubles the
// workgroups where the product's sub-blocks are small.  (A 256 x 256 form of eight waves of
// 128 x 64, three quarters of the LDS reads per flop, measured no faster: at 8192 its LDS was
// active 18% of the time, free of bank conflicts, while its waves waited on memory counters
// for about half of theirs.)
template <bool X3, int BK, int NS, int BM, int BN, int NWM, int NWN>
struct Bf16Gemm {
  static constexpr int NW = NWM * NWN;                 // waves
  static constexpr int WTM = BM / NWM, WTN = BN / NWN; // wave block
  static constexpr int NFM = WTM / 16, NFN = WTN / 16; // 16 x 16 MFMA blocks per wave
  static constexpr int CPR = BK / 8;                  // 16-byte chunks per tile row
  static constexpr int TILE_A = BM * BK * 2;          // bytes of one A tile
  static constexpr int TILE_B = BN * BK * 2;          // bytes of one B tile
  static constexpr int PAIR = TILE_A + TILE_B;         // one A and one B tile
  static constexpr int STAGE_B = (X3 ? 2 : 1) * PAIR;
  static constexpr int ROUND = NW * 1024;             // bytes of one load by every wave
  static constexpr int LPA = TILE_A / ROUND;          // 64-lane x 16-byte loads per wave, A tile
  static constexpr int LPB = TILE_B / ROUND;          // B tile
  static constexpr int IPW = (X3 ? 2 : 1) * (LPA + LPB);   // loads per wave and step
  static constexpr int KK = BK / 32;                  // MFMA k sub-steps per step
  static constexpr int LDS_B = NS * STAGE_B;
  static_assert(LDS_B <= 160 * 1024, "LDS");
  static_assert(BK == 32 || BK == 64, "k step");
  static_assert(LPA >= 1 && LPB >= 1 && TILE_A % ROUND == 0 && TILE_B % ROUND == 0, "load split");
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave block");

  // 16-byte chunk swizzle of tile row r: the chunk index XOR-ed with the row pair.  A fragment
  // read (one chunk of 16 consecutive rows per quarter-wave) is then free of bank conflicts for
  // rows of 64 and 128 bytes (k steps 32 and 64), as the bank-conflict counter shows for both
  // on gfx950; XOR-ing with r / 4 instead conflicts 2-way at 64-byte rows.
  __device__ static int swz(int r) { return (r >> 1) & (CPR - 1); }

  __device__ __attribute__((always_inline)) static void run(const Bf16Args& args, char* lds) {
    const TableDev& tab = g_tables_bf16[args.tab];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % NWM, wn = wave / NWM;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int ti, tj;
    tile_coords(logical, args.tiles_m, args.tiles_n, ti, tj);
    const int64_t row0 = (int64_t)ti * BM, col0 = (int64_t)tj * BN;
    const int nk = (int)(args.kpad / BK);
    const int nprod = tab.nprod;

    // Lane byte offsets inside a product slot for load jj of a tile (part wave + NW jj):
    // position p = 64 part + lane is row p / CPR, stored chunk p % CPR = logical chunk ^ swizzle.
    auto lane_off = [&](int jj, int64_t rc0) {
      const int p = (wave + NW * jj) * 64 + lane;
      const int row = p / CPR, pc = p % CPR, c = pc ^ swz(row);
      return (uint32_t)(2 * ((rc0 + row) * args.kpad + c * 8));
    };
    uint32_t off_a[LPA], off_b[LPB];
#pragma unroll
    for (int jj = 0; jj < LPA; ++jj) off_a[jj] = lane_off(jj, row0);
#pragma unroll
    for (int jj = 0; jj < LPB; ++jj) off_b[jj] = lane_off(jj, col0);
    // the load stream: product ri, k step ki, and the slot bases of product ri (uniform)
    int ri = 0, ki = 0;
    const uint16_t* base[4];   // A hi, B hi, A lo, B lo of product ri
    auto set_bases = [&](int r) {
      base[0] = args.TAh + (int64_t)r * args.stride_a;
      base[1] = args.TBh + (int64_t)r * args.stride_b;
      if (X3) {
        base[2] = args.TAl + (int64_t)r * args.stride_a;
        base[3] = args.TBl + (int64_t)r * args.stride_b;
      }
    };
    set_bases(0);
    auto issue = [&](int stage) {
      const bool live = ri < nprod;
      const uint32_t kofs = (uint32_t)(2 * BK * ki);
      char* sb = lds + stage * STAGE_B;
      auto load = [&](int tl, char* dst, uint32_t o) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(base[tl]), (short)0, 0x7fffffff, 0x00020000);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)dst, 16, live ? o + kofs : kOOB, 0, 0, 0);
      };
#pragma unroll
      for (int h = 0; h < (X3 ? 2 : 1); ++h) {   // hi tiles, then lo tiles
#pragma unroll
        for (int jj = 0; jj < LPA; ++jj)
          load(2 * h, sb + h * PAIR + (wave + NW * jj) * 1024, off_a[jj]);
#pragma unroll
        for (int jj = 0; jj < LPB; ++jj)
          load(2 * h + 1, sb + h * PAIR + TILE_A + (wave + NW * jj) * 1024, off_b[jj]);
      }
      if (++ki == nk) {
        ki = 0;
        if (++ri < nprod) set_bases(ri);
      }
    };

    // fragment reads: rows (A) / columns (B) 16 f + lane % 16 of the wave's block, chunk 4 kk + g
    const int g = lane >> 4, li = lane & 15;
    auto frag = [&](const char* tile, int rr, int chunk) {
      const int pc = chunk ^ swz(rr);
      return *reinterpret_cast<const bf8_t*>(tile + rr * (2 * BK) + pc * 16);
    };

    f4_t acc[NFM][NFN];
    auto zero = [&]() {
#pragma unroll
      for (int a = 0; a < NFM; ++a)
#pragma unroll
        for (int b = 0; b < NFN; ++b) acc[a][b] = (f4_t){0.f, 0.f, 0.f, 0.f};
    };
    // one k sub-step at a time: its fragments, then its MFMAs (fragments of one sub-step live)
    auto compute = [&](int stage) {
      const char* sb = lds + stage * STAGE_B;
#pragma unroll
      for (int kk = 0; kk < KK; ++kk) {
        bf8_t ah[NFM], bh[NFN], al[NFM], bl[NFN];
#pragma unroll
        for (int f = 0; f < NFM; ++f) {
          ah[f] = frag(sb, wm * WTM + 16 * f + li, 4 * kk + g);
          if (X3) al[f] = frag(sb + PAIR, wm * WTM + 16 * f + li, 4 * kk + g);
        }
#pragma unroll
        for (int f = 0; f < NFN; ++f) {
          bh[f] = frag(sb + TILE_A, wn * WTN + 16 * f + li, 4 * kk + g);
          if (X3) bl[f] = frag(sb + PAIR + TILE_A, wn * WTN + 16 * f + li, 4 * kk + g);
        }
#pragma unroll
        for (int fm = 0; fm < NFM; ++fm)
#pragma unroll
          for (int fn = 0; fn < NFN; ++fn) {
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[fm], bh[fn], acc[fm][fn], 0, 0, 0);
            if (X3) {
              acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[fm], bl[fn], acc[fm][fn], 0, 0, 0);
              acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[fm], bh[fn], acc[fm][fn], 0, 0, 0);
            }
          }
      }
    };

    // The C update of one element: FP64, or FP32 (C rounded to FP32, the update in FP32).  The
    // empty asm keeps the product's conversion inside the destination loop: hoisted out of it,
    // the FP64 copies of every accumulator would need twice the accumulators' registers.
    auto update = [&](double c, float mv, double ag, bool first) {
      asm volatile("" : "+v"(mv));
      if (args.c_f64) return c_update(c, (double)mv, ag, args.beta, first);
      const float ag32 = (float)ag, b32 = (float)args.beta;
      float c32 = (float)c;
      if (first) c32 = args.beta == 0.0 ? ag32 * mv : __builtin_fmaf(ag32, mv, b32 * c32);
      else c32 = __builtin_fmaf(ag32, mv, c32);
      return (double)c32;
    };
    // Epilogue of product r: lane l, element e of block (fm, fn) is tile row
    // WTM wm + 16 fm + 4 (l / 16) + e, column WTN wn + 16 fn + l % 16.  Its byte offset is the
    // lane's base (row WTM wm + 4 (l / 16), column WTN wn + l % 16) plus 8 (16 fm + e) plus
    // 128 fn ldc, all in the lane offset (below 2^31 bytes as 8 * 128 * ldc < 2^31).  Where the
    // workgroup's block of this destination lies wholly inside C and its row pairs are 16-byte
    // aligned (vec_c), rows e = 0, 1 and 2, 3 move as 16-byte pairs; else element by element,
    // masked.  Each 16-row block's loads are issued before its first store: the vector memory
    // counter counts loads and stores in one queue, so a store between two loads would make
    // the wait for the second load cover the store too.  No access carries a scalar offset
    // register: the compiler inserts the wait state that a 16-byte store needs before its data
    // registers are rewritten only for stores without one.
    const uint32_t e_base = (uint32_t)(8 * (wm * WTM + 4 * g + (int64_t)(wn * WTN + li) * args.ldc));
    auto epilogue = [&](int r) {
      const ProdDesc& pd = tab.prod[r];
      const int64_t ldc = args.ldc;
      for (int d = 0; d < pd.nc; ++d) {
        const uint8_t cc = pd.c[d];
        const int64_t ci = code_row(cc), cj = code_col(cc);
        const double ag = code_neg(cc) ? -args.alpha : args.alpha;
        const bool first = (pd.first >> d) & 1;
        const bool read_c = !(first && args.beta == 0.0);
        const int64_t rlim = min64(args.mq, args.m - ci * args.mq) - row0;
        const int64_t clim = min64(args.nq, args.n - cj * args.nq) - col0;
        const __amdgpu_buffer_rsrc_t rs =
            make_rsrc(args.C + (ci * args.mq + row0) + (cj * args.nq + col0) * ldc);
        if (args.vec_c && rlim >= BM && clim >= BN) {
#pragma unroll
          for (int fm = 0; fm < NFM; ++fm) {
            uint32_t off[NFN][2];
            d2_t c[NFN][2];
#pragma unroll
            for (int fn = 0; fn < NFN; ++fn)
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                off[fn][h] = e_base + 8 * (16 * fm + 2 * h) + (uint32_t)(128 * fn * ldc);
                c[fn][h] = __builtin_bit_cast(
                    d2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, read_c ? off[fn][h] : kOOB, 0, 0));
              }
#pragma unroll
            for (int fn = 0; fn < NFN; ++fn)
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                d2_t v;
                v.x = update(c[fn][h].x, acc[fm][fn][2 * h], ag, first);
                v.y = update(c[fn][h].y, acc[fm][fn][2 * h + 1], ag, first);
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4_t, v), rs, off[fn][h], 0, 0);
              }
            __builtin_amdgcn_sched_barrier(0);   // keep the C traffic of one row block together
          }
          continue;
        }
#pragma unroll
        for (int fm = 0; fm < NFM; ++fm) {
          uint32_t off[NFN][4];
          double c[NFN][4];
#pragma unroll
          for (int fn = 0; fn < NFN; ++fn) {
            const bool col_ok = wn * WTN + 16 * fn + li < clim;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const bool ok = col_ok && wm * WTM + 16 * fm + 4 * g + e < rlim;
              off[fn][e] = ok ? e_base + 8 * (16 * fm + e) + (uint32_t)(128 * fn * ldc) : kOOB;
              c[fn][e] = __builtin_bit_cast(
                  double, __builtin_amdgcn_raw_buffer_load_b64(rs, read_c ? off[fn][e] : kOOB, 0, 0));
            }
          }
#pragma unroll
          for (int fn = 0; fn < NFN; ++fn)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const double out = update(c[fn][e], acc[fm][fn][e], ag, first);
              __builtin_amdgcn_raw_buffer_store_b64(as_u2(out), rs, off[fn][e], 0, 0);
            }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    };

    // Stream position s lives in stage s % NS.  At each step: with the step landed (the NS - 2
    // newest batches may still fly) the barrier publishes it and has every read of the previous
    // step done, so the next position's loads go into that step's stage.
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) issue(s);
    int stage = 0;
    for (int r = 0; r < nprod; ++r) {
      zero();
      for (int kt = 0; kt < nk; ++kt) {
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(IPW * (NS - 2)) : "memory");
        __syncthreads();
        issue(stage == 0 ? NS - 1 : stage - 1);
        compute(stage);
        stage = stage + 1 == NS ? 0 : stage + 1;
      }
      epilogue(r);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
};

template <bool X3, int BK, int NS, int WPC, int BM, int BN, int NWM, int NWN>
__global__ __launch_bounds__(64 * NWM * NWN, WPC) void bf16_gemm_kernel(const Bf16Args args) {
  using K = Bf16Gemm<X3, BK, NS, BM, BN, NWM, NWN>;
  __shared__ __attribute__((aligned(16))) char lds[K::LDS_B];
  K::run(args, lds);
}

}  // namespace

hipError_t launch_cast(const CastArgs& a, int nslots, hipStream_t s) {
  const int64_t blocks_o = a.outer_pad / kCastT, blocks_k = a.kpad / kCastT;
  const int64_t grid = blocks_o * blocks_k * nslots;
  if (nslots < 1 || grid >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  if (a.sum_f64)
    hipLaunchKernelGGL(cast_kernel<true>, dim3((unsigned)grid), dim3(256), 0, s, a, nslots, (int)blocks_o);
  else
    hipLaunchKernelGGL(cast_kernel<false>, dim3((unsigned)grid), dim3(256), 0, s, a, nslots, (int)blocks_o);
  return hipGetLastError();
}

hipError_t launch_bf16_gemm(const Bf16Args& a, hipStream_t s) {
  const dim3 grid((unsigned)((int64_t)a.tiles_m * a.tiles_n));
  // four waves, two workgroups per CU (at most 64 KB of LDS each), one hiding the other's LDS
  // latency and barriers
  if (a.shape == 1) {
    if (a.x3) hipLaunchKernelGGL((bf16_gemm_kernel<true, 32, 2, 2, 128, 64, 2, 2>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((bf16_gemm_kernel<false, 64, 2, 2, 128, 64, 2, 2>), grid, dim3(256), 0, s, a);
  } else {
    if (a.x3) hipLaunchKernelGGL((bf16_gemm_kernel<true, 32, 2, 2, 128, 128, 2, 2>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((bf16_gemm_kernel<false, 64, 2, 2, 128, 128, 2, 2>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace smx
