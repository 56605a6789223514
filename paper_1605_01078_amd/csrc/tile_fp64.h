// FP64 Strassen tile: the quadrant-summing operand load and the FP64 MFMA main loop for one
// product M_r on one BM x BN tile (the GPU form of the paper's modified packing routines and
// micro-kernel, Sec. 4.1).  Included by the translation units that launch it.
//
// Layout
//   256 threads = 4 waves in a 2 x 2 arrangement; each wave owns a (BM/2) x (BN/2) block as
//   (BM/32) x (BN/32) 16x16 MFMA accumulators (v_mfma_f64_16x16x4_f64).
//   LDS holds two stages of As[BK][BM] and Bs[BK][BN + 1] (both k-major; B is transposed on its
//   way in, the +1 padding keeps that store free of bank conflicts).
//   The MFMA takes B as its first operand and A as its second, so it produces the transposed
//   16x16 block: lane l, element e holds C(row l % 16, column l / 16 + 4e).  Sixteen lanes thus
//   cover 16 consecutive rows of one column, which keeps column-major C and M traffic coalesced.
//
// Operand load
//   Every term X_s of the product has a wave-uniform base pointer (scalar registers) and all
//   terms share the per-thread 32-bit offsets, so summing 2 or 4 quadrant tiles costs no extra
//   vector address registers.  Tiles strictly inside every term's valid extent take an
//   unmasked path; fringe tiles and the last partial k step take a masked path in which
//   out-of-range positions read a safe address and are replaced by zero (the paper's internal
//   zero padding, Sec. 3.3).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace smx {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int code_row(uint8_t c) { return c & 7; }
__device__ __forceinline__ int code_col(uint8_t c) { return (c >> 3) & 7; }
__device__ __forceinline__ bool code_neg(uint8_t c) { return (c & 0x80) != 0; }

// One C update, its case fixed at compile time: 0, a later update of the element
// (c + ag*mv); 1, its first update with beta == 0 (C is not read); 2, its first update with
// beta != 0.  Epilogues that know the case for a whole destination pick it once, outside their
// loops.
template <int CASE>
__device__ __forceinline__ double c_update_case(double c, double mv, double ag, double beta) {
  if constexpr (CASE == 0) return __builtin_fma(ag, mv, c);
  else if constexpr (CASE == 1) return ag * mv;
  else return __builtin_fma(ag, mv, beta * c);
}

// One C update.  Every variant goes through this function (or its cases above) in the same
// product order, so ABC, AB and Naive give bitwise identical results for the same table.
__device__ __forceinline__ double c_update(double c, double mv, double ag, double beta,
                                           bool first) {
  if (!first) return c_update_case<0>(c, mv, ag, beta);
  if (beta == 0.0) return c_update_case<1>(c, mv, ag, beta);
  return c_update_case<2>(c, mv, ag, beta);
}

// Signed operand sums.  A pair of terms c0*x0 + c1*x1 (c = +-1) is rounded once as
// c0 * (x0 + (c0*c1) x1): the first term's sign is factored out (exact), so the sum of the
// negated pair is the exact negation of the pair's sum.  A four-term sum of the two-level table
// (terms listed inner-term-major: (outer 0, inner 0), (outer 1, inner 0), (outer 0, inner 1),
// (outer 1, inner 1)) adds its two pair sums: each pair is the outer-level sum for one inner
// block, so the association is that of applying the one-level algorithm recursively.
// (fma(+-1, x, v) rounds exactly like v +- x.)
__device__ __forceinline__ double pair_sum(double c0, double x0, double c1, double x1) {
  return c0 * __builtin_fma(c0 * c1, x1, x0);
}
template <int N>
__device__ __forceinline__ double signed_sum(const double* sg, const double* x) {
  static_assert(N == 1 || N == 2 || N == 4, "term count");
  if (N == 1) return sg[0] * x[0];
  const double p01 = pair_sum(sg[0], x[0], sg[1], x[1]);
  if (N == 2) return p01;
  return p01 + pair_sum(sg[2], x[2], sg[3], x[3]);
}

// Raw buffer access (gfx9 buffer resource: stride 0, 2 GiB range).  A load whose offset lies
// past the range returns zero without touching memory; kOOB is such an offset.
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u2_t __attribute__((ext_vector_type(2)));
constexpr uint32_t kOOB = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const double* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, 0x7fffffff,
                                           0x00020000);
}
__device__ __forceinline__ d2_t load2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ double load1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// Store operand for the 64-bit buffer store.  Goes through uint64_t: a direct bit_cast of an
// element of a double vector to the 2 x u32 vector is lowered to the wrong register by this
// compiler (every element of the vector is stored as element 0).
__device__ __forceinline__ u2_t as_u2(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  return (u2_t){(unsigned)b, (unsigned)(b >> 32)};
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

// TB: B is given transposed (op(B) = B^T, element (p, j) of op(B) at B[j + p * ldb]); the tile
// of op(B) is then loaded along its columns (contiguous in memory) and written to the same LDS
// layout, so the product is bitwise that of a packed transposed copy.
template <int BM, int BN, int BK, int MAXT, bool VEC, bool TB = false>
struct Fp64Tile {
  static constexpr int NT = 256;
  static constexpr int A_TPC = BM / 2;       // threads per A tile column (2 rows each)
  static constexpr int A_CPP = NT / A_TPC;   // A tile columns per load pass
  static constexpr int A_PASSES = BK / A_CPP;
  static constexpr int B_TPC = BK / 2;       // threads per B tile column (2 k each)
  static constexpr int B_CPP = NT / B_TPC;
  static constexpr int B_PASSES = BN / B_CPP;
  static constexpr int BT_TPR = BN / 2;      // TB: threads per k row of the B tile (2 columns each)
  static constexpr int BT_RPP = NT / BT_TPR; // TB: k rows per load pass
  static constexpr int BT_PASSES = TB ? BK / BT_RPP : 1;
  static constexpr int LDA_S = BM;
  static constexpr int LDB_S = BN + 1;
  static constexpr int WM = BM / 2, WN = BN / 2;
  static constexpr int FM = WM / 16, FN = WN / 16;
  static constexpr int A_STAGE = BK * LDA_S, B_STAGE = BK * LDB_S;
  static constexpr int LDS_DOUBLES = 2 * (A_STAGE + B_STAGE);
  static_assert(A_PASSES >= 1 && B_PASSES >= 1 && BK % 8 == 0 && A_CPP * A_PASSES == BK &&
                    B_CPP * B_PASSES == BN,
                "tile shape");
  static_assert(!TB || (BT_RPP >= 1 && BK % BT_RPP == 0 && MAXT == 1), "tile shape (transposed B)");

  typedef d4_t Acc[FM][FN];

  // Computes M = (sum_s delta_s X_s)(sum_t eps_t V_t) for the tile at (row0, col0) of the
  // sub-block grid into acc.  lds: LDS_DOUBLES doubles.  Ends with a barrier, so the caller may
  // reuse the LDS right away.  The term counts select a loop specialised for them (a uniform
  // branch per product), so no k step carries work for absent terms.
  __device__ static void product(const GemmArgs& args, const ProdDesc& pd, int64_t row0,
                                 int64_t col0, double* lds, Acc& acc) {
    const int na = (pd.flags & 1) ? 1 : pd.na, nb = (pd.flags & 2) ? 1 : pd.nb;
    if (MAXT == 1 || (na == 1 && nb == 1)) return product_n<1, 1>(args, pd, row0, col0, lds, acc);
    if (MAXT >= 2) {
      if (na == 2 && nb == 2) return product_n<2, 2>(args, pd, row0, col0, lds, acc);
      if (na == 2 && nb == 1) return product_n<2, 1>(args, pd, row0, col0, lds, acc);
      if (na == 1 && nb == 2) return product_n<1, 2>(args, pd, row0, col0, lds, acc);
    }
    if (MAXT >= 4) {
      if (na == 4 && nb == 4) return product_n<4, 4>(args, pd, row0, col0, lds, acc);
      if (na == 4 && nb == 2) return product_n<4, 2>(args, pd, row0, col0, lds, acc);
      if (na == 2 && nb == 4) return product_n<2, 4>(args, pd, row0, col0, lds, acc);
      if (na == 4 && nb == 1) return product_n<4, 1>(args, pd, row0, col0, lds, acc);
      if (na == 1 && nb == 4) return product_n<1, 4>(args, pd, row0, col0, lds, acc);
    }
  }

  template <int NA, int NB>
  __device__ static void product_n(const GemmArgs& args, const ProdDesc& pd, int64_t row0,
                                   int64_t col0, double* lds, Acc& acc) {
    double* As = lds;
    double* Bs = lds + 2 * A_STAGE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int a_row = 2 * (tid % A_TPC), a_col = tid / A_TPC;
    const int b_k = 2 * (tid % B_TPC), b_col = tid / B_TPC;
    const int bt_j = 2 * (tid % BT_TPR), bt_k = tid / BT_TPR;   // TB

    // ---- per-term (wave-uniform) setup: base pointer of the tile, valid extents, sign ----
    const double* a_base[NA];
    const double* b_base[NB];
    int64_t a_klim[NA], b_klim[NB];
    int a_rv[NA], b_cv[NB];             // valid rows / columns of the term inside this tile
    double a_sg[NA], b_sg[NB];
    const int64_t lda_e = (pd.flags & 1) ? args.mq : args.lda;
    const int64_t ldb_e = (pd.flags & 2) ? args.kq : args.ldb;
#pragma unroll
    for (int s = 0; s < NA; ++s) {
      if (pd.flags & 1) {  // Naive temporary: zero-padded to the full sub-block
        a_base[s] = args.TA + (int64_t)pd.tslot_a * args.ta_stride;
        a_rv[s] = (int)min64(BM, args.mq - row0);
        a_klim[s] = args.kq;
        a_sg[s] = 1.0;
      } else {
        const uint8_t c = pd.a[s];
        const int64_t bi = code_row(c), bp = code_col(c);
        a_base[s] = args.A + bi * args.mq + bp * args.kq * args.lda;
        a_rv[s] = (int)min64(BM, min64(args.mq, args.m - bi * args.mq) - row0);
        a_klim[s] = min64(args.kq, args.k - bp * args.kq);
        a_sg[s] = code_neg(c) ? -1.0 : 1.0;
      }
      a_base[s] += row0;
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      if (pd.flags & 2) {
        b_base[s] = args.TB + (int64_t)pd.tslot_b * args.tb_stride;
        b_cv[s] = (int)min64(BN, args.nq - col0);
        b_klim[s] = args.kq;
        b_sg[s] = 1.0;
      } else {
        const uint8_t c = pd.b[s];
        const int64_t bp = code_row(c), bj = code_col(c);
        b_base[s] = TB ? args.B + bj * args.nq + bp * args.kq * args.ldb
                       : args.B + bp * args.kq + bj * args.nq * args.ldb;
        b_cv[s] = (int)min64(BN, min64(args.nq, args.n - bj * args.nq) - col0);
        b_klim[s] = min64(args.kq, args.k - bp * args.kq);
        b_sg[s] = code_neg(c) ? -1.0 : 1.0;
      }
      b_base[s] += TB ? col0 : col0 * ldb_e;
    }
    const int nk = (int)((args.kq + BK - 1) / BK);

    // per-thread byte offsets inside a tile, shared by all terms
    uint32_t oa[A_PASSES], ob[B_PASSES];
#pragma unroll
    for (int p = 0; p < A_PASSES; ++p)
      oa[p] = (uint32_t)(8 * (a_row + (int64_t)(a_col + p * A_CPP) * lda_e));
#pragma unroll
    for (int p = 0; p < B_PASSES; ++p)
      ob[p] = (uint32_t)(8 * (b_k + (int64_t)(b_col + p * B_CPP) * ldb_e));
    uint32_t obt[BT_PASSES];
#pragma unroll
    for (int p = 0; p < BT_PASSES; ++p)
      obt[p] = (uint32_t)(8 * (bt_j + (int64_t)(bt_k + p * BT_RPP) * args.ldb));

    d2_t ra[NA][A_PASSES], rb[NB][TB ? BT_PASSES : B_PASSES];

    // Global loads of k step kt for every term.  Buffer loads: an out-of-range position (fringe
    // of the matrix or of its sub-block, or a k step past the end) gets an offset past the
    // buffer's range and the hardware returns zero without touching memory, so the loads need
    // no branch and all stay in flight across the MFMA work.
    auto load_a = [&](int kt) {
      const int64_t kb = (int64_t)kt * BK;
#pragma unroll
      for (int s = 0; s < NA; ++s) {
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(a_base[s] + kb * lda_e);
        const int kv = (int)min64(BK, a_klim[s] - kb);
        const bool r0 = a_row < a_rv[s], r1 = a_row + 1 < a_rv[s];
#pragma unroll
        for (int p = 0; p < A_PASSES; ++p) {
          const bool kok = a_col + p * A_CPP < kv;
          if (VEC) {
            ra[s][p] = load2(rs, (kok && r0) ? oa[p] : kOOB);
          } else {
            ra[s][p] = (d2_t){load1(rs, (kok && r0) ? oa[p] : kOOB),
                              load1(rs, (kok && r1) ? oa[p] + 8 : kOOB)};
          }
        }
      }
    };
    auto load_b = [&](int kt) {
      const int64_t kb = (int64_t)kt * BK;
      if constexpr (TB) {   // column pairs (j, j + 1) of one k row: contiguous in memory
#pragma unroll
        for (int s = 0; s < NB; ++s) {
          const __amdgpu_buffer_rsrc_t rs = make_rsrc(b_base[s] + kb * args.ldb);
          const int kv = (int)min64(BK, b_klim[s] - kb);
          const bool c0 = bt_j < b_cv[s], c1 = bt_j + 1 < b_cv[s];
#pragma unroll
          for (int p = 0; p < BT_PASSES; ++p) {
            const bool kok = bt_k + p * BT_RPP < kv;
            if (VEC) {
              rb[s][p] = load2(rs, (kok && c0) ? obt[p] : kOOB);
            } else {
              rb[s][p] = (d2_t){load1(rs, (kok && c0) ? obt[p] : kOOB),
                                load1(rs, (kok && c1) ? obt[p] + 8 : kOOB)};
            }
          }
        }
        return;
      }
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(b_base[s] + kb);
        const int kv = (int)min64(BK, b_klim[s] - kb);
        const bool k0 = b_k < kv, k1 = b_k + 1 < kv;
#pragma unroll
        for (int p = 0; p < B_PASSES; ++p) {
          const bool cok = b_col + p * B_CPP < b_cv[s];
          if (VEC) {
            rb[s][p] = load2(rs, (cok && k0) ? ob[p] : kOOB);
          } else {
            rb[s][p] = (d2_t){load1(rs, (cok && k0) ? ob[p] : kOOB),
                              load1(rs, (cok && k1) ? ob[p] + 8 : kOOB)};
          }
        }
      }
    };
    auto load_stage = [&](int kt) {
      load_a(kt);
      load_b(kt);
    };

    // Signed sums in registers (signed_sum: the association every kernel uses), then into LDS
    // stage `buf`.
    auto store_a = [&](int buf) {
#pragma unroll
      for (int p = 0; p < A_PASSES; ++p) {
        double xs[NA], ys[NA];
#pragma unroll
        for (int s = 0; s < NA; ++s) {
          xs[s] = ra[s][p].x;
          ys[s] = ra[s][p].y;
        }
        const double v0 = signed_sum<NA>(a_sg, xs), v1 = signed_sum<NA>(a_sg, ys);
        *reinterpret_cast<d2_t*>(&As[buf * A_STAGE + (a_col + p * A_CPP) * LDA_S + a_row]) =
            (d2_t){v0, v1};
      }
    };
    auto store_b = [&](int buf) {
      if constexpr (TB) {
#pragma unroll
        for (int p = 0; p < BT_PASSES; ++p) {
          double xs[NB], ys[NB];
#pragma unroll
          for (int s = 0; s < NB; ++s) {
            xs[s] = rb[s][p].x;
            ys[s] = rb[s][p].y;
          }
          const double v0 = signed_sum<NB>(b_sg, xs), v1 = signed_sum<NB>(b_sg, ys);
          double* row = &Bs[buf * B_STAGE + (bt_k + p * BT_RPP) * LDB_S + bt_j];
          row[0] = v0;
          row[1] = v1;
        }
        return;
      }
#pragma unroll
      for (int p = 0; p < B_PASSES; ++p) {
        double xs[NB], ys[NB];
#pragma unroll
        for (int s = 0; s < NB; ++s) {
          xs[s] = rb[s][p].x;
          ys[s] = rb[s][p].y;
        }
        const double v0 = signed_sum<NB>(b_sg, xs), v1 = signed_sum<NB>(b_sg, ys);
        const int j = b_col + p * B_CPP;
        Bs[buf * B_STAGE + b_k * LDB_S + j] = v0;
        Bs[buf * B_STAGE + (b_k + 1) * LDB_S + j] = v1;
      }
    };

    // One k sub-step (four k values): FM x FN MFMAs on fragments read from LDS stage `buf`.
    // Within each group of eight k values, lane group g = lane / 16 takes k = 2g in the first
    // sub-step and k = 2g + 1 in the second (the pairing that 16-byte operand reads give the
    // all-products kernel); every FP64 kernel feeds the MFMA this way, so the products agree
    // bit for bit across kernels.
    auto mfma_substep = [&](int buf, int ks) {
      const double* as = As + buf * A_STAGE + wm * WM + (lane & 15);
      const double* bs = Bs + buf * B_STAGE + wn * WN + (lane & 15);
      const int kr = (ks >> 1) * 8 + 2 * (lane >> 4) + (ks & 1);
      double af[FM], bf[FN];
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) af[fm] = as[kr * LDA_S + fm * 16];
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) bf[fn] = bs[kr * LDB_S + fn * 16];
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
          acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[fn], af[fm], acc[fm][fn], 0, 0, 0);
    };

#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = (d4_t){0.0, 0.0, 0.0, 0.0};

    constexpr int KS = BK / 4;
    // Products with many terms keep only one operand's raw tiles in registers at a time: the
    // A and B staging share the same registers (their live ranges do not overlap), which lets
    // a four-term product run beside the 128 x 128 accumulator at two workgroups per CU.
    constexpr bool SPLIT = (NA + NB >= 5) && KS >= 4;
    if (!SPLIT) {
      // At the top of iteration kt the registers hold the raw terms of step kt+1, loaded during
      // iteration kt-1.  Their sums go to the other LDS stage between the first sub-steps of
      // step kt (no wait: the data is already there), then the loads of step kt+2 are issued
      // into the freed registers and the remaining sub-steps run.
      load_stage(0);
      store_a(0);
      store_b(0);
      load_stage(1);   // past the end of k every position is out of range: no memory access
      __syncthreads();
      for (int kt = 0; kt + 1 < nk; ++kt) {
        const int cur = kt & 1;
        mfma_substep(cur, 0);
        store_a(cur ^ 1);
        if (KS > 1) mfma_substep(cur, 1);
        store_b(cur ^ 1);
        // keep the next loads after the sums: hoisting them would keep two stages of raw
        // terms live at once
        asm volatile("" ::: "memory");
        load_stage(kt + 2);
#pragma unroll
        for (int ks = 2; ks < KS; ++ks) mfma_substep(cur, ks);
        __syncthreads();
      }
    } else {
      // Top of iteration kt: registers hold the raw A terms of step kt+1.  Sum them during
      // sub-step 0, load B of step kt+1 into the same registers, sum B two sub-steps later,
      // then load A of step kt+2 for the next iteration.
      load_a(0);
      store_a(0);
      asm volatile("" ::: "memory");
      load_b(0);
      store_b(0);
      asm volatile("" ::: "memory");
      load_a(1);
      __syncthreads();
      for (int kt = 0; kt + 1 < nk; ++kt) {
        const int cur = kt & 1;
        mfma_substep(cur, 0);
        store_a(cur ^ 1);
        asm volatile("" ::: "memory");
        load_b(kt + 1);
        mfma_substep(cur, 1);
        mfma_substep(cur, 2);
        store_b(cur ^ 1);
        asm volatile("" ::: "memory");
        load_a(kt + 2);
#pragma unroll
        for (int ks = 3; ks < KS; ++ks) mfma_substep(cur, ks);
        __syncthreads();
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) mfma_substep((nk - 1) & 1, ks);
    __syncthreads();
  }

  // Accumulator element (fm, fn, e) of this lane sits at tile row  wm*WM + fm*16 + lane%16  and
  // tile column  wn*WN + fn*16 + lane/16 + 4e.  The epilogues address it as a per-lane byte
  // offset (voffset, range-checked: kOOB drops the access) plus a wave-uniform byte offset
  // (soffset) of fm*16 + (fn*16 + 4e)*ld elements.

  // ABC epilogue: C_d[tile] := c_update(C_d[tile], M, alpha*gamma_d) for every destination.
  __device__ static void update_c(const GemmArgs& args, const ProdDesc& pd, int64_t row0,
                                  int64_t col0, const Acc& acc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = (wave & 1) * WM + (lane & 15);        // tile row of fm = 0
    const int lc = (wave >> 1) * WN + (lane >> 4);       // tile column of fn = 0, e = 0
    const int64_t ldc = args.ldc;
    const uint32_t voff = (uint32_t)(8 * (lr + (int64_t)lc * ldc));
    for (int d = 0; d < pd.nc; ++d) {
      const uint8_t cc = pd.c[d];
      const int64_t ci = code_row(cc), cj = code_col(cc);
      const double ag = code_neg(cc) ? -args.alpha : args.alpha;
      const bool first = (pd.first >> d) & 1;
      const bool read_c = !(first && args.beta == 0.0);
      const int rlim = (int)min64(BM, min64(args.mq, args.m - ci * args.mq) - row0);
      const int clim = (int)min64(BN, min64(args.nq, args.n - cj * args.nq) - col0);
      const __amdgpu_buffer_rsrc_t rs =
          make_rsrc(args.C + (ci * args.mq + row0) + (cj * args.nq + col0) * ldc);
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
        const bool rok = lr + fm * 16 < rlim;
        double cv[FN][4];
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool ok = rok && lc + fn * 16 + 4 * e < clim && read_c;
            const uint32_t so = (uint32_t)(8 * (fm * 16 + (int64_t)(fn * 16 + 4 * e) * ldc));
            cv[fn][e] = __builtin_bit_cast(
                double, __builtin_amdgcn_raw_buffer_load_b64(rs, ok ? voff : kOOB, so, 0));
          }
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool ok = rok && lc + fn * 16 + 4 * e < clim;
            const uint32_t so = (uint32_t)(8 * (fm * 16 + (int64_t)(fn * 16 + 4 * e) * ldc));
            const double v = c_update(cv[fn][e], acc[fm][fn][e], ag, args.beta, first);
            __builtin_amdgcn_raw_buffer_store_b64(as_u2(v), rs, ok ? voff : kOOB, so, 0);
          }
      }
    }
  }

  // AB / Naive epilogue: store M_r (unscaled) to its temporary.
  __device__ static void store_m(const GemmArgs& args, int r, int64_t row0, int64_t col0,
                                 const Acc& acc) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = (wave & 1) * WM + (lane & 15);
    const int lc = (wave >> 1) * WN + (lane >> 4);
    const int64_t ldm = args.ldm;
    const uint32_t voff = (uint32_t)(8 * (lr + (int64_t)lc * ldm));
    const int rlim = (int)min64(BM, args.mq - row0), clim = (int)min64(BN, args.nq - col0);
    const __amdgpu_buffer_rsrc_t rs =
        make_rsrc(args.M + (int64_t)r * args.m_stride + row0 + col0 * ldm);
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = lr + fm * 16 < rlim && lc + fn * 16 + 4 * e < clim;
          const uint32_t so = (uint32_t)(8 * (fm * 16 + (int64_t)(fn * 16 + 4 * e) * ldm));
          __builtin_amdgcn_raw_buffer_store_b64(as_u2(acc[fm][fn][e]), rs, ok ? voff : kOOB,
                                                so, 0);
        }
  }
};

}  // namespace smx
