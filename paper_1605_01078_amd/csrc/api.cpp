// C-ABI of the Strassen library: argument checking, planning, workspace, launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/strassen.h"
#include "internal.h"
#include "launch.h"
#include "plan.h"

namespace smx {

// ---------------------------------------------------------------------------------------------
// Errors.
// ---------------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(STRASSEN_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

// ---------------------------------------------------------------------------------------------
// Tables.
// ---------------------------------------------------------------------------------------------
static TableDev make_table_dev(int levels, bool naive) {
  TableDev td;
  std::memset(&td, 0, sizeof td);
  const std::vector<Product> tab = build_table(levels);
  const int q = 1 << levels;
  td.nprod = (int32_t)tab.size();
  td.q = q;
  bool touched[16] = {false};
  for (size_t r = 0; r < tab.size(); ++r) {
    const Product& p = tab[r];
    ProdDesc& d = td.prod[r];
    d.na = (uint8_t)p.a.size();
    d.nb = (uint8_t)p.b.size();
    d.nc = (uint8_t)p.c.size();
    for (size_t s = 0; s < p.a.size(); ++s) d.a[s] = term_code(p.a[s].row, p.a[s].col, p.a[s].sign);
    for (size_t s = 0; s < p.b.size(); ++s) d.b[s] = term_code(p.b[s].row, p.b[s].col, p.b[s].sign);
    for (size_t s = 0; s < p.c.size(); ++s) {
      d.c[s] = term_code(p.c[s].row, p.c[s].col, p.c[s].sign);
      const int blk = p.c[s].row * q + p.c[s].col;
      if (!touched[blk]) {
        d.first |= (uint8_t)(1u << s);
        touched[blk] = true;
      }
      uint8_t& cnt = td.asm_cnt[blk];
      td.asm_list[blk][cnt++] = (uint8_t)(r | (p.c[s].sign < 0 ? 0x80 : 0));
    }
    if (naive) {
      if (p.a.size() > 1 || p.a[0].sign < 0) {
        d.flags |= 1;
        d.tslot_a = (uint8_t)td.nslot_a;
        td.slot_prod_a[td.nslot_a++] = (uint8_t)r;
      }
      if (p.b.size() > 1 || p.b[0].sign < 0) {
        d.flags |= 2;
        d.tslot_b = (uint8_t)td.nslot_b;
        td.slot_prod_b[td.nslot_b++] = (uint8_t)r;
      }
    }
  }
  return td;
}

const TableDev* host_tables() {
  static TableDev tabs[kNumTables];
  static std::once_flag once;
  std::call_once(once, [] {
    tabs[0] = make_table_dev(0, false);
    tabs[1] = make_table_dev(1, false);
    tabs[2] = make_table_dev(2, false);
    tabs[3] = make_table_dev(1, true);
    tabs[4] = make_table_dev(2, true);
  });
  return tabs;
}

// The product-side table for `levels` (0..kMaxLevelsAbc), built once.
const std::vector<Product>& host_table(int levels) {
  static std::vector<Product> tabs[kMaxLevelsAbc + 1];
  static std::once_flag once;
  std::call_once(once, [] {
    for (int l = 0; l <= kMaxLevelsAbc; ++l) tabs[l] = build_table(l);
  });
  return tabs[levels];
}

static int table_maxt(const TableDev& td) {
  int mx = 1;
  for (int r = 0; r < td.nprod; ++r) {
    const ProdDesc& d = td.prod[r];
    const int na = (d.flags & 1) ? 1 : d.na, nb = (d.flags & 2) ? 1 : d.nb;
    mx = std::max(mx, std::max(na, nb));
  }
  return mx <= 1 ? 1 : (mx <= 2 ? 2 : 4);
}

// ---------------------------------------------------------------------------------------------
// Per-device state: architecture check, constant tables, library-owned workspace.
// ---------------------------------------------------------------------------------------------
struct DeviceState {
  bool ready = false;
  void* ws = nullptr;
  size_t ws_bytes = 0;
};
static std::mutex g_mu;
static std::vector<DeviceState> g_dev;
static void* g_user_ws = nullptr;
static size_t g_user_ws_bytes = 0;

int device_ready(int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(STRASSEN_ERR_NO_DEVICE, "no HIP device: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  if (!g_dev[dev].ready) {
    hipDeviceProp_t prop;
    SMX_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(STRASSEN_ERR_NO_DEVICE, "device %d is %s, the library is built for gfx950", dev,
                  prop.gcnArchName);
    SMX_HIP(upload_tables(host_tables()));
    SMX_HIP(upload_tables_bf16(host_tables()));
    SMX_HIP(upload_tables_batched(host_tables()));
    SMX_HIP(hipDeviceSynchronize());
    g_dev[dev].ready = true;
  }
  *dev_out = dev;
  return 0;
}

// Library-owned workspace of at least `bytes` on device `dev` (grown on demand, capped by
// strassen_set_workspace_limit).
static size_t g_ws_limit = SIZE_MAX;

static int library_workspace(int dev, size_t bytes, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (bytes > g_ws_limit)
    return fail(STRASSEN_ERR_ALLOC, "workspace of %zu bytes exceeds the limit of %zu bytes", bytes,
                g_ws_limit);
  DeviceState& d = g_dev[dev];
  if (d.ws_bytes < bytes) {
    if (d.ws) {
      SMX_HIP(hipDeviceSynchronize());  // earlier calls may still use the old buffer
      SMX_HIP(hipFree(d.ws));
      d.ws = nullptr;
      d.ws_bytes = 0;
    }
    hipError_t e = hipMalloc(&d.ws, bytes);
    if (e != hipSuccess) {
      d.ws = nullptr;
      (void)hipGetLastError();   // an allocation failure is not sticky; clear it
      return fail(STRASSEN_ERR_ALLOC, "workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    d.ws_bytes = bytes;
  }
  *out = d.ws;
  return 0;
}

WsSource default_workspace() {
  std::lock_guard<std::mutex> lk(g_mu);
  WsSource w;
  if (g_user_ws) {
    w.fixed = true;
    w.ptr = g_user_ws;
    w.bytes = g_user_ws_bytes;
  } else {
    w.bytes = g_ws_limit;
  }
  return w;
}

// Device workspace of at least `bytes` from `src`: a fixed buffer (the caller's or the static
// scratch) if it is large enough, else the library's own.
static int get_workspace(const WsSource& src, int dev, size_t bytes, void** out) {
  if (src.fixed) {
    if (bytes > src.bytes)
      return fail(STRASSEN_ERR_ALLOC, "%s has %zu bytes, %zu needed",
                  src.what ? src.what : "caller workspace", src.bytes, bytes);
    void* ptr = src.ptr;
    if (!ptr && src.resolve)
      if (int rc = src.resolve(dev, &ptr)) return rc;
    *out = ptr;
    return 0;
  }
  return library_workspace(dev, bytes, out);
}

// ---------------------------------------------------------------------------------------------
// Optional kernel timing (strassen_timing_enable): a pair of events recorded on the launch's
// stream around every launch of the main kernels; events come from a pool that collect refills.
// ---------------------------------------------------------------------------------------------
struct TimedLaunch {
  int kind;
  hipEvent_t e0, e1;
};
static std::mutex g_tm_mu;
static std::atomic<bool> g_timing{false};
static std::vector<TimedLaunch> g_tm_log;
static std::vector<hipEvent_t> g_tm_pool;

static int pooled_event(hipEvent_t* e) {
  {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    if (!g_tm_pool.empty()) {
      *e = g_tm_pool.back();
      g_tm_pool.pop_back();
      return 0;
    }
  }
  SMX_HIP(hipEventCreate(e));
  return 0;
}

static thread_local bool t_timing_suspended = false;
void suspend_timing(bool on) { t_timing_suspended = on; }

// Runs launch() (returning hipError_t), bracketed by events when timing is on.
template <class F>
static int timed_launch(int kind, hipStream_t s, F&& launch, const char* what) {
  if (t_timing_suspended || !g_timing.load(std::memory_order_relaxed)) {
    hipError_t e = launch();
    return e == hipSuccess ? 0 : hip_fail(e, what);
  }
  TimedLaunch t;
  t.kind = kind;
  if (int rc = pooled_event(&t.e0)) return rc;
  if (int rc = pooled_event(&t.e1)) return rc;
  SMX_HIP(hipEventRecord(t.e0, s));
  hipError_t e = launch();
  if (e != hipSuccess) return hip_fail(e, what);
  SMX_HIP(hipEventRecord(t.e1, s));
  std::lock_guard<std::mutex> lk(g_tm_mu);
  g_tm_log.push_back(t);
  return 0;
}

#define SMX_LAUNCH(kind, stream, call)                                                 \
  do {                                                                                 \
    if (int rc_ = timed_launch((kind), (stream), [&] { return (call); }, #call)) return rc_; \
  } while (0)

// ---------------------------------------------------------------------------------------------
// Planning.
// ---------------------------------------------------------------------------------------------

struct Plan {
  int levels, variant, q;
  int64_t mq, nq, kq;
  const TableDev* td;
  int tab;
  // workspace layout (doubles)
  int64_t ldm, m_stride, ta_stride, tb_stride;
  int64_t off_m, off_ta, off_tb, total;
};

static Plan make_plan(int64_t m, int64_t n, int64_t k, int levels, int variant) {
  Plan p;
  p.levels = levels;
  p.variant = levels == 0 ? STRASSEN_ABC : variant;
  p.q = 1 << levels;
  p.mq = cdiv(m, p.q);
  p.nq = cdiv(n, p.q);
  p.kq = cdiv(k, p.q);
  p.tab = table_id(levels, p.variant == STRASSEN_NAIVE);
  p.td = &host_tables()[p.tab];
  p.ldm = round_up(p.mq, 8);
  p.m_stride = round_up(p.ldm * p.nq, 32);
  p.ta_stride = round_up(p.mq * p.kq, 32);
  p.tb_stride = round_up(p.kq * p.nq, 32);
  p.off_m = p.off_ta = p.off_tb = p.total = 0;
  if (p.variant != STRASSEN_ABC) {
    p.off_m = 0;
    p.total = p.m_stride * p.td->nprod;
    if (p.variant == STRASSEN_NAIVE) {
      p.off_ta = p.total;
      p.total += p.ta_stride * p.td->nslot_a;
      p.off_tb = p.total;
      p.total += p.tb_stride * p.td->nslot_b;
    }
  }
  return p;
}

// Tile configuration: 128 x 128 (k step 16, two workgroups per CU) when there are enough tiles
// to fill the 256 CUs twice over, else 64 x 64.
// STRASSEN_TILE_CFG=<0..3> forces one configuration (used by the tuning sweeps).
static std::atomic<int> g_forced_cfg{[] {
  const char* e = std::getenv("STRASSEN_TILE_CFG");
  return e ? std::atoi(e) : -1;
}()};

static int pick_cfg(const Plan& p, int64_t products_per_launch, int maxt) {
  const int forced = g_forced_cfg.load(std::memory_order_relaxed);
  if (forced >= 0 && forced < kCfgAll) return forced;
  const int64_t t128 = cdiv(p.mq, 128) * cdiv(p.nq, 128) * products_per_launch;
  if (t128 < 512) return kCfg64;
  (void)maxt;
  return kCfg128;
}

static bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15) == 0; }

// The all-products kernel needs every sub-block full with even extents in m and k, 16-byte
// aligned operands with even leading dimensions (16-byte loads of element pairs), and per-tile
// byte offsets that fit its 32-bit lane offsets.
static bool all_products_applies(int64_t m, int64_t k, const double* A, int64_t lda,
                                 const double* B, int64_t ldb, const double* C, int64_t ldc,
                                 int levels) {
  if (levels < 1) return false;
  const int64_t unit = int64_t(2) << levels;
  if (m % unit != 0 || k % unit != 0) return false;
  if (!aligned16(A) || !aligned16(B) || !aligned16(C)) return false;
  if (lda % 2 != 0 || ldb % 2 != 0 || ldc % 2 != 0) return false;
  const int64_t lim = int64_t(1) << 31;
  return 8 * 16 * lda < lim && 8 * 64 * ldb < lim && 8 * 64 * ldc < lim;
}

// Two-level ABC with staged outer sums: the outer level's two-term operand sums (five on each
// side in the one-level table) are formed once by a streaming pass into workspace slots, and
// each outer product then runs the one-level all-products kernel on its staged (or single-term)
// operands.  Every sum is rounded as in the unstaged kernel, so results are bitwise the same.
// Per outer product (one_at_a_time): where the workspace cannot hold all ten sums, one slot per
// side is refilled before each outer product that needs it (each sum formed once as before;
// the pass reads the sum's two blocks instead of all four once per side: 15 block passes per
// side instead of 9, for a fifth of the workspace).
struct StagePlan {
  int na_slots = 0, nb_slots = 0;
  int slot_a[7], slot_b[7];
  int64_t ta_stride = 0, tb_stride = 0, total = 0;   // doubles
  bool one_at_a_time = false;
};

// blocks: sub-blocks per staged block along each side's extent product (4 for the outer
// blocks of two levels, 2 x 2 inner sub-blocks; 1 for the quadrants of one level).
static StagePlan make_stage_plan(const Plan& p, bool one_at_a_time = false, int64_t blocks = 4) {
  StagePlan sp;
  sp.one_at_a_time = one_at_a_time;
  for (int R = 0; R < 7; ++R) {
    sp.slot_a[R] = kOneLevel[R].na == 2 ? (one_at_a_time ? 0 : sp.na_slots++) : -1;
    sp.slot_b[R] = kOneLevel[R].nb == 2 ? (one_at_a_time ? 0 : sp.nb_slots++) : -1;
  }
  if (one_at_a_time) {
    sp.na_slots = 1;
    sp.nb_slots = 1;
  }
  sp.ta_stride = round_up(blocks * p.mq * p.kq, 32);
  sp.tb_stride = round_up(blocks * p.kq * p.nq, 32);
  sp.total = sp.na_slots * sp.ta_stride + sp.nb_slots * sp.tb_stride;
  return sp;
}

// Staging needs every outer column block of B and C full (n a multiple of 4) besides the
// all-products layout.  Measured on MI355X it is faster than forming the outer sums in the load
// from 2048 x 2048 outer blocks of C and k = 2048 on (1.10x at m = n = k = 4096, 1.17x at
// 16384 with k = 8192); below that the default stays unstaged.
static bool staging_applies(int64_t m, int64_t n, int64_t k, int levels) {
  return levels == 2 && n % 4 == 0 && (m / 2) * (n / 2) >= int64_t(2048) * 2048 && k >= 2048;
}

// The all-products launches of ABC: one at one level; at two, one per outer product of the
// one-level table, in order.  `stage` (two levels only, may be null) holds the staged outer
// sums as laid out by make_stage_plan(p, one_at_a_time).
static int build_all_products(const Plan& p, const double* A, int64_t lda, const double* B,
                              int64_t ldb, double* C, int64_t ldc, int64_t n, double alpha,
                              double beta, const double* stage, std::vector<ApLaunch>* out,
                              bool one_at_a_time = false) {
  out->clear();
  FusedArgs f;
  std::memset(&f, 0, sizeof f);
  f.A = A;
  f.B = B;
  f.C = C;
  f.lda = lda;
  f.ldb = ldb;
  f.ldc = ldc;
  f.n = n;
  f.mq = p.mq;
  f.nq = p.nq;
  f.kq = p.kq;
  f.alpha = alpha;
  f.beta = beta;
  f.tiles_m = (int32_t)cdiv(p.mq, 64);
  f.tiles_n = (int32_t)cdiv(p.nq, 64);
  if ((int64_t)f.tiles_m * f.tiles_n >= (int64_t(1) << 30))
    return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
  if (p.levels == 1) {
    f.nc = 1;
    f.c_first = 1;
    f.a_sg[0] = f.b_sg[0] = f.c_sg[0] = 1.0;
    out->push_back({f, 1, 1});
    return 0;
  }
  // two levels: outer blocks are 2 x 2 inner sub-blocks
  const int64_t om = 2 * p.mq, on = 2 * p.nq, ok = 2 * p.kq;
  auto a_block = [&](int q) { return (q >> 1) * om + (q & 1) * ok * lda; };
  auto b_block = [&](int q) { return (q >> 1) * ok + (q & 1) * on * ldb; };
  for (int R = 0; R < 7; ++R)   // the kernels take the first term's sign as +1
    if (kOneLevel[R].a[0].sign != 1 || kOneLevel[R].b[0].sign != 1)
      return fail(STRASSEN_ERR_UNSUPPORTED, "outer product %d: first term negative", R);
  StagePlan sp;
  if (stage) sp = make_stage_plan(p, one_at_a_time);
  bool touched[4] = {false, false, false, false};
  for (int R = 0; R < 7; ++R) {
    const QProduct& P = kOneLevel[R];
    int na = P.na, nb = P.nb;
    f.A = A;
    f.lda = lda;
    if (stage && sp.slot_a[R] >= 0) {   // the staged sum, an om x ok matrix
      f.A = stage + sp.slot_a[R] * sp.ta_stride;
      f.lda = om;
      f.a_off[0] = 0;
      f.a_sg[0] = 1.0;
      na = 1;
    } else {
      for (int s = 0; s < P.na; ++s) {
        f.a_off[s] = a_block(P.a[s].q);
        f.a_sg[s] = P.a[s].sign;
      }
    }
    f.B = B;
    f.ldb = ldb;
    if (stage && sp.slot_b[R] >= 0) {   // an ok x on matrix whose columns all exist (n % 4 == 0)
      f.B = stage + sp.na_slots * sp.ta_stride + sp.slot_b[R] * sp.tb_stride;
      f.ldb = ok;
      f.b_off[0] = 0;
      f.b_cb[0] = 0;
      f.b_sg[0] = 1.0;
      nb = 1;
    } else {
      for (int s = 0; s < P.nb; ++s) {
        const int q = P.b[s].q;
        f.b_off[s] = b_block(q);
        f.b_cb[s] = 2 * (q & 1);
        f.b_sg[s] = P.b[s].sign;
      }
    }
    f.nc = P.nc;
    f.c_first = 0;
    for (int d = 0; d < P.nc; ++d) {
      const int q = P.c[d].q;
      f.c_off[d] = (q >> 1) * om + (q & 1) * on * ldc;
      f.c_cb[d] = 2 * (q & 1);
      f.c_sg[d] = P.c[d].sign;
      if (!touched[q]) f.c_first |= 1 << d;
      touched[q] = true;
    }
    out->push_back({f, na, nb});
  }
  return 0;
}

// ABC through the all-products kernel; at two levels with `stage` (may be null) the outer
// operand sums are first formed into it by two streaming launches, or (one_at_a_time) each
// outer product's sums just before its launch.
static int run_all_products(const Plan& p, const double* A, int64_t lda, const double* B,
                            int64_t ldb, double* C, int64_t ldc, int64_t n, double alpha,
                            double beta, double* stage, hipStream_t stream,
                            double* M = nullptr, int64_t ldm = 0, int64_t m_stride = 0,
                            bool one_at_a_time = false) {
  std::vector<ApLaunch> launches;
  const bool staged = p.levels == 2 && stage;
  if (int rc = build_all_products(p, A, lda, B, ldb, C, ldc, n, alpha, beta,
                                  staged ? stage : nullptr, &launches, one_at_a_time))
    return rc;
  const StagePlan sp = make_stage_plan(p, one_at_a_time);
  OuterSumArgs oa, ob;
  if (staged) {
    const int64_t om = 2 * p.mq, on = 2 * p.nq, ok = 2 * p.kq;
    std::memset(&oa, 0, sizeof oa);
    std::memset(&ob, 0, sizeof ob);
    oa.src = A;
    oa.dst = stage;
    oa.ld = lda;
    oa.rows = om;
    oa.cols = ok;
    oa.dst_stride = sp.ta_stride;
    ob.src = B;
    ob.dst = stage + sp.na_slots * sp.ta_stride;
    ob.ld = ldb;
    ob.rows = ok;
    ob.cols = on;
    ob.dst_stride = sp.tb_stride;
    for (int q = 0; q < 4; ++q) {
      oa.blk[q] = (q >> 1) * om + (q & 1) * ok * lda;
      ob.blk[q] = (q >> 1) * ok + (q & 1) * on * ldb;
    }
    if (!one_at_a_time) {
      SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(oa, 0, stream));
      SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(ob, 1, stream));
    }
  }
  for (size_t i = 0; i < launches.size(); ++i) {
    if (staged && one_at_a_time) {   // this outer product's sums into the two slots
      oa.single = ob.single = (int32_t)i + 1;
      if (sp.slot_a[i] >= 0)
        SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(oa, 0, stream));
      if (sp.slot_b[i] >= 0)
        SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(ob, 1, stream));
    }
    ApLaunch l = launches[i];
    if (M) {   // the AB form: launch i holds products 7i .. 7i + 6 of the table
      l.f.store_m = 1;
      l.f.M = M;
      l.f.ldm = ldm;
      l.f.m_stride = m_stride;
      l.f.prod_base = 7 * (int32_t)i;
    }
    SMX_LAUNCH(STRASSEN_KERNEL_ALL_PRODUCTS, stream, launch_all_products(l.f, l.na, l.nb, stream));
  }
  return 0;
}

// Classical GEMM on the all-products kernel's load path: its layout needs m and k even (16-byte
// row pairs of A and k pairs of B), 16-byte aligned operands with even leading dimensions, and
// per-lane offsets spanning eight columns of B and 64 of C below 2^31 bytes.
static bool classical_layout(int64_t m, int64_t k, const double* A, int64_t lda,
                             const double* B, int64_t ldb, const double* C, int64_t ldc) {
  const int64_t lim = int64_t(1) << 31;
  return m % 2 == 0 && k % 2 == 0 && aligned16(A) && aligned16(B) && aligned16(C) &&
         lda % 2 == 0 && ldb % 2 == 0 && ldc % 2 == 0 && 8 * 64 * (ldc + 1) < lim &&
         8 * 8 * (ldb + 1) < lim;
}

// Its 256 x 128 tiles fill MI355X's 256 CUs at least once; smaller problems keep the general
// tile kernel, whose 128 x 128 or 64 x 64 tiles spread them over more CUs.
static bool classical_size(int64_t m, int64_t n) { return cdiv(m, 256) * cdiv(n, 128) >= 256; }

static int run_classical(int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                         int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                         int64_t ldc, hipStream_t stream) {
  ClassicalArgs c;
  std::memset(&c, 0, sizeof c);
  c.A = A;
  c.B = B;
  c.C = C;
  c.lda = lda;
  c.ldb = ldb;
  c.ldc = ldc;
  c.m = m;
  c.n = n;
  c.k = k;
  c.alpha = alpha;
  c.beta = beta;
  c.tiles_m = (int32_t)cdiv(m, 256);
  c.tiles_n = (int32_t)cdiv(n, 128);
  if ((int64_t)c.tiles_m * c.tiles_n >= (int64_t(1) << 30))
    return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
  SMX_LAUNCH(STRASSEN_KERNEL_CLASSICAL, stream, launch_classical(c, stream));
  return 0;
}

// One-level ABC on the classical kernel: the operand sums of the one-level table staged in
// workspace (the outer-sum kernel over the four quadrants), then one classical launch per
// product in product order, each adding its product to its one or two C quadrants (beta at a
// quadrant's first update).  Every C element receives the operations of the all-products
// kernel (same sums, same MFMA k order, the same updates in product order): the same bits.
// The shapes where it is faster (measured on MI355X): quadrants that are exact halves (m and
// k multiples of 4, n even), k/2 >= 2048 (below, the staged sums and the second C quadrant of
// five products cost more than the classical kernel's efficiency gains: at k = 2048 the
// all-products kernel is 1.03x classical, this form 0.98x), each product's 256 x 128 tiles
// filling whole rounds of the 256 CUs (at least 95% of the last round busy: 12288^3, with
// 4.5 rounds, runs at 0.98x against 1.03x), and either k/2 >= 4096 or four rounds of tiles.
bool one_level_staged_shape(int64_t m, int64_t n, int64_t k) {
  if (m % 4 != 0 || k % 4 != 0 || n % 2 != 0) return false;
  const int64_t kq = k / 2, tiles = cdiv(m / 2, 256) * cdiv(n / 2, 128);
  const int64_t rounds = cdiv(tiles, 256);
  return tiles >= 256 && kq >= 2048 && 20 * tiles >= 19 * 256 * rounds &&
         (kq >= 4096 || tiles >= 1024);
}

static bool staged_classical_applies(int64_t m, int64_t n, int64_t k, const double* A,
                                     int64_t lda, const double* B, int64_t ldb, const double* C,
                                     int64_t ldc) {
  return one_level_staged_shape(m, n, k) && classical_layout(m / 2, k / 2, A, lda, B, ldb, C, ldc);
}

static int run_staged_classical(const Plan& p, const double* A, int64_t lda, const double* B,
                                int64_t ldb, double* C, int64_t ldc, double alpha, double beta,
                                double* stage, bool one_at_a_time, hipStream_t stream) {
  const int64_t om = p.mq, on = p.nq, okk = p.kq;   // the quadrants
  if (cdiv(om, 256) * cdiv(on, 128) >= (int64_t(1) << 30))
    return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
  const StagePlan sp = make_stage_plan(p, one_at_a_time, 1);
  OuterSumArgs oa, ob;
  std::memset(&oa, 0, sizeof oa);
  std::memset(&ob, 0, sizeof ob);
  oa.src = A;
  oa.dst = stage;
  oa.ld = lda;
  oa.rows = om;
  oa.cols = okk;
  oa.dst_stride = sp.ta_stride;
  ob.src = B;
  ob.dst = stage + sp.na_slots * sp.ta_stride;
  ob.ld = ldb;
  ob.rows = okk;
  ob.cols = on;
  ob.dst_stride = sp.tb_stride;
  for (int q = 0; q < 4; ++q) {
    oa.blk[q] = (q >> 1) * om + (q & 1) * okk * lda;
    ob.blk[q] = (q >> 1) * okk + (q & 1) * on * ldb;
  }
  if (!one_at_a_time) {
    SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(oa, 0, stream));
    SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(ob, 1, stream));
  }
  bool touched[4] = {false, false, false, false};
  for (int r = 0; r < 7; ++r) {
    const QProduct& P = kOneLevel[r];
    if (one_at_a_time) {   // this product's sums into the two slots
      oa.single = ob.single = r + 1;
      if (P.na == 2) SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(oa, 0, stream));
      if (P.nb == 2) SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(ob, 1, stream));
    }
    ClassicalArgs c;
    std::memset(&c, 0, sizeof c);
    // a one-term side is its quadrant (first terms have sign +1)
    c.A = P.na == 2 ? oa.dst + (int64_t)sp.slot_a[r] * sp.ta_stride : A + oa.blk[P.a[0].q];
    c.lda = P.na == 2 ? om : lda;
    c.B = P.nb == 2 ? ob.dst + (int64_t)sp.slot_b[r] * sp.tb_stride : B + ob.blk[P.b[0].q];
    c.ldb = P.nb == 2 ? okk : ldb;
    double* dst[2] = {nullptr, nullptr};
    double ag[2] = {0.0, 0.0};
    for (int d = 0; d < P.nc; ++d) {
      const int q = P.c[d].q;
      dst[d] = C + (q >> 1) * om + (q & 1) * on * ldc;
      ag[d] = P.c[d].sign > 0 ? alpha : -alpha;
      if (touched[q]) c.not_first |= 1 << d;
      touched[q] = true;
    }
    c.C = dst[0];
    c.alpha = ag[0];
    c.Cx[0] = dst[1];
    c.ax[0] = ag[1];
    c.extra = P.nc - 1;
    c.beta = beta;
    c.ldc = ldc;
    c.m = om;
    c.n = on;
    c.k = okk;
    c.tiles_m = (int32_t)cdiv(om, 256);
    c.tiles_n = (int32_t)cdiv(on, 128);
    SMX_LAUNCH(STRASSEN_KERNEL_CLASSICAL, stream, launch_classical(c, stream));
  }
  return 0;
}

// Naive on the classical kernel: every product is a plain GEMM of its two operands (a
// temporary of the padded sub-block extent, or one quadrant of A or B); where the partition is
// exact (m, n, k multiples of 2^L, so every quadrant is a full sub-block), the quadrants keep
// the classical kernel's layout (even sub-block extents, aligned operands, even leading
// dimensions) and each product fills the CUs, the products run there.
static inline int64_t code_row_h(uint8_t c) { return c & 7; }
static inline int64_t code_col_h(uint8_t c) { return (c >> 3) & 7; }

static bool naive_on_classical(const Plan& p, int64_t m, int64_t n, int64_t k, const double* A,
                               int64_t lda, const double* B, int64_t ldb, int forced) {
  if (p.variant != STRASSEN_NAIVE || forced != -1) return false;
  if (m % p.q != 0 || n % p.q != 0 || k % p.q != 0) return false;
  if (!classical_size(p.mq, p.nq)) return false;
  return classical_layout(p.mq, p.kq, A, lda, B, ldb, nullptr, p.ldm) &&
         8 * 64 * (p.ldm + 1) < (int64_t(1) << 31);
}

// Block padding (the zero padding of Sec. 3.3 made physical).// Block padding (the zero padding of Sec. 3.3 made physical).  Where the all-products layout
// does not apply to the operands as given (m or k not a multiple of 2^(L+1), operands not
// 16-byte aligned, odd leading dimensions) or two-level staging needs n % 4 == 0, ABC runs on
// copies in which every row (column) block of the 2^L x 2^L partition is stored with an even
// extent, the extra rows and columns zero.  Every real element keeps its sub-block, its
// position in it and the k positions it meets in the MFMA; the padding only feeds exact zeros
// to the positions the unpadded kernels mask to zero, so the result is bitwise that of the
// unpadded path.  Operands that already fit are used in place.
struct PadPlan {
  int64_t mq, kq, nq, mq_e, kq_e;   // sub-block extents, plain and padded (even)
  int64_t mp, kp, np;               // padded problem
  bool pa, pb, pc;                  // which operands are copied
  bool stage;                       // two-level staged outer sums on the padded problem
  bool ok;                          // the padded layout fits the kernel's 32-bit lane offsets
  int64_t a_off, b_off, c_off, s_off, total;   // workspace layout (doubles)
  int64_t total_one;                // the same with one outer product's sums staged at a time
};

static PadPlan make_pad_plan(int64_t m, int64_t n, int64_t k, int levels, const double* A,
                             int64_t lda, const double* B, int64_t ldb, const double* C,
                             int64_t ldc, int forced) {
  PadPlan pp;
  const int64_t q = int64_t(1) << levels, unit = 2 * q;
  pp.mq = cdiv(m, q);
  pp.kq = cdiv(k, q);
  pp.nq = cdiv(n, q);
  pp.mq_e = round_up(pp.mq, 2);
  pp.kq_e = round_up(pp.kq, 2);
  pp.mp = q * pp.mq_e;
  pp.kp = q * pp.kq_e;
  const int64_t n4 = round_up(n, 4);
  pp.stage = levels == 2 && (forced == kCfgAllStaged ||
                             (forced == -1 && staging_applies(pp.mp, n4, pp.kp, levels)));
  const bool need_n = pp.stage && n % 4 != 0;
  pp.np = need_n ? 4 * pp.nq : n;
  const bool need_m = m % unit != 0, need_k = k % unit != 0;
  const int64_t lim = int64_t(1) << 31;
  pp.pa = need_m || need_k || !aligned16(A) || lda % 2 != 0 || 8 * 16 * lda >= lim;
  pp.pb = need_k || need_n || !aligned16(B) || ldb % 2 != 0 || 8 * 64 * ldb >= lim;
  pp.pc = need_m || need_n || !aligned16(C) || ldc % 2 != 0 || 8 * 64 * ldc >= lim;
  pp.ok = 8 * 16 * (pp.pa ? pp.mp : lda) < lim && 8 * 64 * (pp.pb ? pp.kp : ldb) < lim &&
          8 * 64 * (pp.pc ? pp.mp : ldc) < lim;
  int64_t off = 0;
  auto take = [&](bool used, int64_t elems) {
    const int64_t at = off;
    if (used) off += round_up(elems, 32);
    return at;
  };
  pp.a_off = take(pp.pa, pp.mp * pp.kp);
  pp.b_off = take(pp.pb, pp.kp * pp.np);
  pp.c_off = take(pp.pc, pp.mp * pp.np);
  pp.s_off = off;
  pp.total = pp.total_one = off;
  if (pp.stage) {
    const Plan sp = make_plan(pp.mp, pp.np, pp.kp, levels, STRASSEN_ABC);
    pp.total = off + make_stage_plan(sp).total;
    pp.total_one = off + make_stage_plan(sp, true).total;
  }
  return pp;
}

static int run_padded(const PadPlan& pp, int levels, int64_t m, int64_t n, int64_t k,
                      double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                      double beta, double* C, int64_t ldc, double* ws, hipStream_t stream,
                      bool one_at_a_time = false) {
  auto copy = [&](const double* src, int64_t ld_s, int64_t rows, int64_t cols, int64_t rb,
                  int64_t rb_e, int64_t cb, int64_t cb_e, double* dst, int64_t ld_d,
                  int64_t dst_rows, int64_t dst_cols, int unpad) {
    PadArgs a;
    std::memset(&a, 0, sizeof a);
    a.src = src;
    a.dst = dst;
    a.ld_s = ld_s;
    a.ld_d = ld_d;
    a.rows = rows;
    a.cols = cols;
    a.rb = rb;
    a.rb_e = rb_e;
    a.cb = cb;
    a.cb_e = cb_e;
    a.dst_rows = dst_rows;
    a.dst_cols = dst_cols;
    a.unpad = unpad;
    return launch_pad_copy(a, stream);
  };
  const double* Ap = A;
  const double* Bp = B;
  double* Cp = C;
  int64_t lda_p = lda, ldb_p = ldb, ldc_p = ldc;
  const int64_t whole_n = pp.np;   // columns are not blocked: one block spanning them all
  if (pp.pa) {
    double* d = ws + pp.a_off;
    SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream,
               copy(A, lda, m, k, pp.mq, pp.mq_e, pp.kq, pp.kq_e, d, pp.mp, pp.mp, pp.kp, 0));
    Ap = d;
    lda_p = pp.mp;
  }
  if (pp.pb) {
    double* d = ws + pp.b_off;
    SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream,
               copy(B, ldb, k, n, pp.kq, pp.kq_e, whole_n, whole_n, d, pp.kp, pp.kp, pp.np, 0));
    Bp = d;
    ldb_p = pp.kp;
  }
  if (pp.pc) {
    Cp = ws + pp.c_off;
    ldc_p = pp.mp;
    if (beta != 0.0)   // with beta = 0 no update reads C
      SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream,
                 copy(C, ldc, m, n, pp.mq, pp.mq_e, whole_n, whole_n, Cp, pp.mp, pp.mp, pp.np, 0));
  }
  if (levels == 0) {
    if (int rc = run_classical(pp.mp, pp.np, pp.kp, alpha, Ap, lda_p, Bp, ldb_p, beta, Cp, ldc_p,
                               stream))
      return rc;
  } else {
    const Plan p = make_plan(pp.mp, pp.np, pp.kp, levels, STRASSEN_ABC);
    if (int rc = run_all_products(p, Ap, lda_p, Bp, ldb_p, Cp, ldc_p, pp.np, alpha, beta,
                                  pp.stage ? ws + pp.s_off : nullptr, stream, nullptr, 0, 0,
                                  one_at_a_time))
      return rc;
  }
  if (pp.pc)
    SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream,
               copy(Cp, pp.mp, m, n, pp.mq, pp.mq_e, whole_n, whole_n, C, ldc, pp.mp, pp.np, 1));
  return 0;
}

// AB on the all-products kernel: the store form writes each product to its temporary and the
// assembly of the tile path follows.  A and B are block-padded where they do not fit the
// kernel's layout (C is no operand of the fused loop); the temporaries keep the real problem's
// leading dimension, which is at least the padded sub-block extent, so the padded rows land
// outside the part the assembly reads.  Two levels need the staged outer sums (one term per
// side).  By default the copies are made only where a launch has at least kAbPadMinTiles
// 64 x 64 tile positions (three quarters of MI355X's 256 CUs at one 512-thread workgroup each):
// on 500 ragged shapes (m, n, k log-uniform in 256..20000) the copies plus the fused kernel
// were up to 3x slower than the tile kernel below that and up to 1.25x faster above it.
// Offsets are in doubles, behind the temporaries of `p`.
constexpr int64_t kAbPadMinTiles = 192;

struct AbLayout {
  PadPlan pp;
  bool fused = false;
  int64_t a_off = 0, b_off = 0, s_off = 0, total = 0;
};

static AbLayout make_ab_layout(const Plan& p, int64_t m, int64_t n, int64_t k, int levels,
                               const double* A, int64_t lda, const double* B, int64_t ldb,
                               int forced) {
  AbLayout l;
  l.total = p.total;
  const bool fused_cfg = forced == -1 || forced == kCfgAll || forced == kCfgAllStaged;
  if (p.variant != STRASSEN_AB || levels < 1 || !fused_cfg) return l;
  l.pp = make_pad_plan(m, n, k, levels, A, lda, B, ldb, nullptr, 2 * cdiv(m, 2), forced);
  if (!l.pp.ok || (levels == 2 && !l.pp.stage) || 8 * 64 * p.ldm >= (int64_t(1) << 31))
    return l;
  const int64_t positions = cdiv(l.pp.mq_e, 64) * cdiv(l.pp.nq, 64);   // per launch
  if (forced == -1 && (l.pp.pa || l.pp.pb) && positions < kAbPadMinTiles) return l;
  int64_t off = p.total;
  l.a_off = off;
  if (l.pp.pa) off += round_up(l.pp.mp * l.pp.kp, 32);
  l.b_off = off;
  if (l.pp.pb) off += round_up(l.pp.kp * l.pp.np, 32);
  l.s_off = off;
  if (l.pp.stage)
    off += make_stage_plan(make_plan(l.pp.mp, l.pp.np, l.pp.kp, levels, STRASSEN_ABC)).total;
  l.fused = true;
  l.total = off;
  return l;
}

bool all_products_ok(int64_t m, int64_t k, const double* A, int64_t lda, const double* B,
                     int64_t ldb, const double* C, int64_t ldc, int levels) {
  return all_products_applies(m, k, A, lda, B, ldb, C, ldc, levels);
}

int all_products_plan(int64_t m, int64_t n, int64_t k, int levels, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double* C, int64_t ldc, double alpha,
                      double beta, std::vector<ApLaunch>* out) {
  if (!all_products_applies(m, k, A, lda, B, ldb, C, ldc, levels))
    return fail(STRASSEN_ERR_UNSUPPORTED, "all-products layout does not apply");
  return build_all_products(make_plan(m, n, k, levels, STRASSEN_ABC), A, lda, B, ldb, C, ldc, n,
                            alpha, beta, nullptr, out);
}

// ---------------------------------------------------------------------------------------------
// Three levels (Sec. 3.5, eq. e:straprim4 with L = 3): product 49 R + 7 S + r applies outer row R
// of the one-level table to the 2 x 2 blocks of A, B and C, row S to the 2 x 2 blocks of those,
// and row r inside them.  The two upper levels' operand sums are staged: the five two-term sums
// of each side over the four top blocks once (slots of m/2 x k/2 and k/2 x n/2), then, for each
// R, the five sums over the four blocks of R's operand (slots of m/4 x k/4 and k/4 x n/4, reused
// from R to R); each pair (R, S) is one launch of the one-level all-products kernel on its
// staged (or single-term) operands, adding its seven products into the 2 x 2 sub-blocks of
// every destination block (2 row_R + row_S, 2 col_R + col_S) with sign gamma_R gamma_S.  Launches
// run in (R, S) order, so every C element receives its 343 updates in increasing product index.
// Each staged sum is x0 + s1 x1 rounded once, formed from the previous level's sums: the
// association of applying the one-level algorithm recursively.
// ---------------------------------------------------------------------------------------------
struct L3Plan {
  int64_t mq, kq, nq, mq_e, kq_e;   // level-3 sub-block extents, plain and padded (even)
  int64_t mp, kp, np;               // padded problem: 8 mq_e x 8 kq_e x 8 nq
  bool pa, pb, pc;                  // operands copied to block-padded buffers
  bool ok;                          // the layout fits the kernel's 32-bit lane offsets
  int64_t a_off, b_off, c_off, s1a, s1b, s2a, s2b, total;   // workspace layout (doubles)
};

static L3Plan make_l3_plan(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                           const double* B, int64_t ldb, const double* C, int64_t ldc) {
  L3Plan p;
  p.mq = cdiv(m, 8);
  p.kq = cdiv(k, 8);
  p.nq = cdiv(n, 8);
  p.mq_e = round_up(p.mq, 2);
  p.kq_e = round_up(p.kq, 2);
  p.mp = 8 * p.mq_e;
  p.kp = 8 * p.kq_e;
  p.np = 8 * p.nq;
  const int64_t lim = int64_t(1) << 31;
  p.pa = p.mp != m || p.kp != k || !aligned16(A) || lda % 2 != 0 || 8 * 16 * lda >= lim;
  p.pb = p.kp != k || p.np != n || !aligned16(B) || ldb % 2 != 0 || 8 * 64 * ldb >= lim;
  p.pc = p.mp != m || p.np != n || !aligned16(C) || ldc % 2 != 0 || 8 * 64 * ldc >= lim;
  p.ok = 8 * 16 * (p.pa ? p.mp : lda) < lim && 8 * 64 * (p.pb ? p.kp : ldb) < lim &&
         8 * 64 * (p.pc ? p.mp : ldc) < lim;
  int64_t off = 0;
  auto take = [&](bool used, int64_t elems) {
    const int64_t at = off;
    if (used) off += round_up(elems, 32);
    return at;
  };
  p.a_off = take(p.pa, p.mp * p.kp);
  p.b_off = take(p.pb, p.kp * p.np);
  p.c_off = take(p.pc, p.mp * p.np);
  p.s1a = take(true, 5 * round_up((p.mp / 2) * (p.kp / 2), 32));
  p.s1b = take(true, 5 * round_up((p.kp / 2) * (p.np / 2), 32));
  p.s2a = take(true, 5 * round_up((p.mp / 4) * (p.kp / 4), 32));
  p.s2b = take(true, 5 * round_up((p.kp / 4) * (p.np / 4), 32));
  p.total = off;
  return p;
}

// The five two-term sums of one side of the one-level table over the 2 x 2 blocks (rows x cols
// each) of src, into slots of rows x cols (leading dimension rows) at dst + s * stride.
static int stage_sums(const double* src, int64_t ld, int64_t rows, int64_t cols, double* dst,
                      int64_t stride, int side, hipStream_t stream) {
  OuterSumArgs o;
  std::memset(&o, 0, sizeof o);
  o.src = src;
  o.dst = dst;
  o.ld = ld;
  o.rows = rows;
  o.cols = cols;
  o.dst_stride = stride;
  for (int q = 0; q < 4; ++q) o.blk[q] = (q >> 1) * rows + (q & 1) * cols * ld;
  SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_outer_sums(o, side, stream));
  return 0;
}

// One side's operand of a one-level product P over the 2 x 2 blocks (rows x cols) of src: its
// staged sum (slot `slot` of dst, leading dimension rows) or its single block of src.
struct Operand {
  const double* p;
  int64_t ld;
};
static Operand level_operand(const QTerm* terms, int nt, int slot, const double* src, int64_t ld,
                             int64_t rows, int64_t cols, const double* slots, int64_t stride) {
  if (nt == 2) return {slots + slot * stride, rows};
  const int q = terms[0].q;
  return {src + (q >> 1) * rows + (q & 1) * cols * ld, ld};
}

static int run_l3(const L3Plan& lp, double alpha, const double* A, int64_t lda, const double* B,
                  int64_t ldb, double beta, double* C, int64_t ldc, double* ws,
                  hipStream_t stream) {
  const int64_t mq = lp.mq_e, kq = lp.kq_e, nq = lp.nq;   // level-3 extents (padded problem)
  const int64_t m1 = 4 * mq, k1 = 4 * kq, n1 = 4 * nq;    // level-1 blocks
  const int64_t m2 = 2 * mq, k2 = 2 * kq, n2 = 2 * nq;    // level-2 blocks
  const int64_t s1a = round_up(m1 * k1, 32), s1b = round_up(k1 * n1, 32);
  const int64_t s2a = round_up(m2 * k2, 32), s2b = round_up(k2 * n2, 32);
  double* S1A = ws + lp.s1a;
  double* S1B = ws + lp.s1b;
  double* S2A = ws + lp.s2a;
  double* S2B = ws + lp.s2b;
  if (int rc = stage_sums(A, lda, m1, k1, S1A, s1a, 0, stream)) return rc;
  if (int rc = stage_sums(B, ldb, k1, n1, S1B, s1b, 1, stream)) return rc;
  int slot_a[7], slot_b[7];
  for (int r = 0, sa = 0, sb = 0; r < 7; ++r) {
    slot_a[r] = kOneLevel[r].na == 2 ? sa++ : -1;
    slot_b[r] = kOneLevel[r].nb == 2 ? sb++ : -1;
  }
  bool touched[4][4] = {};
  FusedArgs f;
  std::memset(&f, 0, sizeof f);
  f.C = C;
  f.ldc = ldc;
  f.n = 8 * nq;
  f.mq = mq;
  f.nq = nq;
  f.kq = kq;
  f.alpha = alpha;
  f.beta = beta;
  f.tiles_m = (int32_t)cdiv(mq, 64);
  f.tiles_n = (int32_t)cdiv(nq, 64);
  f.a_sg[0] = f.b_sg[0] = 1.0;
  for (int R = 0; R < 7; ++R) {
    const QProduct& PR = kOneLevel[R];
    const Operand aR = level_operand(PR.a, PR.na, slot_a[R], A, lda, m1, k1, S1A, s1a);
    const Operand bR = level_operand(PR.b, PR.nb, slot_b[R], B, ldb, k1, n1, S1B, s1b);
    if (int rc = stage_sums(aR.p, aR.ld, m2, k2, S2A, s2a, 0, stream)) return rc;
    if (int rc = stage_sums(bR.p, bR.ld, k2, n2, S2B, s2b, 1, stream)) return rc;
    for (int S = 0; S < 7; ++S) {
      const QProduct& PS = kOneLevel[S];
      const Operand a = level_operand(PS.a, PS.na, slot_a[S], aR.p, aR.ld, m2, k2, S2A, s2a);
      const Operand b = level_operand(PS.b, PS.nb, slot_b[S], bR.p, bR.ld, k2, n2, S2B, s2b);
      f.A = a.p;
      f.lda = a.ld;
      f.B = b.p;
      f.ldb = b.ld;
      f.nc = PR.nc * PS.nc;
      f.c_first = 0;
      int d = 0;
      for (int dr = 0; dr < PR.nc; ++dr)
        for (int ds = 0; ds < PS.nc; ++ds, ++d) {
          const int row = 2 * (PR.c[dr].q >> 1) + (PS.c[ds].q >> 1);
          const int col = 2 * (PR.c[dr].q & 1) + (PS.c[ds].q & 1);
          f.c_off[d] = row * m2 + col * n2 * ldc;
          f.c_cb[d] = 2 * col;
          f.c_sg[d] = (double)(PR.c[dr].sign * PS.c[ds].sign);
          if (!touched[row][col]) f.c_first |= 1 << d;
          touched[row][col] = true;
        }
      SMX_LAUNCH(STRASSEN_KERNEL_ALL_PRODUCTS, stream, launch_all_products(f, 1, 1, stream));
    }
  }
  return 0;
}

static int pad_copy(const double* src, int64_t ld_s, int64_t rows, int64_t cols, int64_t rb,
                    int64_t rb_e, int64_t cb, int64_t cb_e, double* dst, int64_t ld_d,
                    int64_t dst_rows, int64_t dst_cols, int unpad, hipStream_t stream) {
  PadArgs a;
  std::memset(&a, 0, sizeof a);
  a.src = src;
  a.dst = dst;
  a.ld_s = ld_s;
  a.ld_d = ld_d;
  a.rows = rows;
  a.cols = cols;
  a.rb = rb;
  a.rb_e = rb_e;
  a.cb = cb;
  a.cb_e = cb_e;
  a.dst_rows = dst_rows;
  a.dst_cols = dst_cols;
  a.unpad = unpad;
  SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream, launch_pad_copy(a, stream));
  return 0;
}

static int dgemm_l3(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                    const WsSource& wsrc, hipStream_t stream) {
  const L3Plan lp = make_l3_plan(m, n, k, A, lda, B, ldb, C, ldc);
  if (!lp.ok)
    return fail(STRASSEN_ERR_UNSUPPORTED, "three levels: sizes past the 32-bit tile offsets");
  if ((int64_t)cdiv(lp.mq_e, 64) * cdiv(lp.nq, 64) >= (int64_t(1) << 30))
    return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
  const size_t bytes = (size_t)lp.total * sizeof(double);
  if (!wsrc.fits(bytes))
    return fail(STRASSEN_ERR_ALLOC, "three levels stage their upper operand sums: %zu bytes of "
                "workspace needed, %zu available", bytes, wsrc.bytes);
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  void* w = nullptr;
  if (int rc = get_workspace(wsrc, dev, bytes, &w)) return rc;
  double* ws = static_cast<double*>(w);
  const double* Ap = A;
  const double* Bp = B;
  double* Cp = C;
  int64_t la = lda, lb = ldb, lc = ldc;
  if (lp.pa) {
    if (int rc = pad_copy(A, lda, m, k, lp.mq, lp.mq_e, lp.kq, lp.kq_e, ws + lp.a_off, lp.mp,
                          lp.mp, lp.kp, 0, stream))
      return rc;
    Ap = ws + lp.a_off;
    la = lp.mp;
  }
  if (lp.pb) {
    if (int rc = pad_copy(B, ldb, k, n, lp.kq, lp.kq_e, lp.np, lp.np, ws + lp.b_off, lp.kp, lp.kp,
                          lp.np, 0, stream))
      return rc;
    Bp = ws + lp.b_off;
    lb = lp.kp;
  }
  if (lp.pc) {
    Cp = ws + lp.c_off;
    lc = lp.mp;
    if (beta != 0.0)   // with beta = 0 no update reads C
      if (int rc = pad_copy(C, ldc, m, n, lp.mq, lp.mq_e, lp.np, lp.np, Cp, lp.mp, lp.mp, lp.np,
                            0, stream))
        return rc;
  }
  if (int rc = run_l3(lp, alpha, Ap, la, Bp, lb, beta, Cp, lc, ws, stream)) return rc;
  if (lp.pc)
    if (int rc = pad_copy(Cp, lp.mp, m, n, lp.mq, lp.mq_e, lp.np, lp.np, C, ldc, lp.mp, lp.np, 1,
                          stream))
      return rc;
  return 0;
}

static int validate(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                    const double* B, int64_t ldb, double* C, int64_t ldc, int levels,
                    int variant) {
  if (m < 0) return fail(-1, "m = %lld < 0", (long long)m);
  if (n < 0) return fail(-2, "n = %lld < 0", (long long)n);
  if (k < 0) return fail(-3, "k = %lld < 0", (long long)k);
  const bool reads_ab = m > 0 && n > 0 && k > 0 && alpha != 0.0;
  if (reads_ab && A == nullptr) return fail(-5, "A is NULL");
  if (lda < std::max<int64_t>(1, m)) return fail(-6, "lda = %lld < max(1, m)", (long long)lda);
  if (reads_ab && B == nullptr) return fail(-7, "B is NULL");
  if (ldb < std::max<int64_t>(1, k)) return fail(-8, "ldb = %lld < max(1, k)", (long long)ldb);
  if (m > 0 && n > 0 && C == nullptr) return fail(-10, "C is NULL");
  if (ldc < std::max<int64_t>(1, m)) return fail(-11, "ldc = %lld < max(1, m)", (long long)ldc);
  if (levels < 0 || levels > kMaxLevelsAbc)
    return fail(-12, "levels = %d not in 0..%d", levels, kMaxLevelsAbc);
  if (variant < 0 || variant > 2) return fail(-13, "variant = %d not in 0..2", variant);
  if (levels > kMaxLevels && variant != STRASSEN_ABC)
    return fail(-13, "levels = %d runs the ABC variant only (variant = %d)", levels, variant);
  return 0;
}

static int run_scale(double* C, int64_t ldc, int64_t m, int64_t n, double beta, hipStream_t s) {
  ScaleArgs a;
  a.C = C;
  a.ldc = ldc;
  a.m = m;
  a.n = n;
  a.beta = beta;
  SMX_HIP(launch_scale(a, s));
  return 0;
}

// ---------------------------------------------------------------------------------------------
// Winograd's variant (a Strassen-like scheme of the paper's references and future work), ABC:
// one level is one launch of the all-products kernel with Winograd's table (the chain sums
// formed on the fragments); two levels stage the outer chain sums (four slots per side) and run
// one launch per outer product, each adding its seven inner products into the inner sub-blocks
// of every outer block that product reaches (up to four), in product order.
// ---------------------------------------------------------------------------------------------
struct WPlan {
  int levels;
  int64_t mq, kq, nq, mq_e, kq_e;   // innermost sub-block extents, plain and padded (even)
  int64_t mp, kp, np;               // padded problem
  bool pa, pb, pc, ok;
  int64_t a_off, b_off, c_off, sa, sb, sa_stride, sb_stride, total;   // doubles
};

static WPlan make_w_plan(int64_t m, int64_t n, int64_t k, int levels, const double* A,
                         int64_t lda, const double* B, int64_t ldb, const double* C, int64_t ldc) {
  WPlan p;
  p.levels = levels;
  const int64_t q = int64_t(1) << levels;
  p.mq = cdiv(m, q);
  p.kq = cdiv(k, q);
  p.nq = cdiv(n, q);
  p.mq_e = round_up(p.mq, 2);
  p.kq_e = round_up(p.kq, 2);
  p.mp = q * p.mq_e;
  p.kp = q * p.kq_e;
  p.np = levels == 2 ? q * p.nq : n;   // staged B sums need every outer column block full
  const int64_t lim = int64_t(1) << 31;
  p.pa = p.mp != m || p.kp != k || !aligned16(A) || lda % 2 != 0 || 8 * 16 * lda >= lim;
  p.pb = p.kp != k || p.np != n || !aligned16(B) || ldb % 2 != 0 || 8 * 64 * ldb >= lim;
  p.pc = p.mp != m || p.np != n || !aligned16(C) || ldc % 2 != 0 || 8 * 64 * ldc >= lim;
  p.ok = 8 * 16 * (p.pa ? p.mp : lda) < lim && 8 * 64 * (p.pb ? p.kp : ldb) < lim &&
         8 * 64 * (p.pc ? p.mp : ldc) < lim;
  int64_t off = 0;
  auto take = [&](bool used, int64_t elems) {
    const int64_t at = off;
    if (used) off += round_up(elems, 32);
    return at;
  };
  p.a_off = take(p.pa, p.mp * p.kp);
  p.b_off = take(p.pb, p.kp * p.np);
  p.c_off = take(p.pc, p.mp * p.np);
  p.sa_stride = round_up((p.mp / 2) * (p.kp / 2), 32);
  p.sb_stride = round_up((p.kp / 2) * (p.np / 2), 32);
  p.sa = take(levels == 2, 4 * p.sa_stride);
  p.sb = take(levels == 2, 4 * p.sb_stride);
  p.total = off;
  return p;
}

static int run_winograd(const WPlan& wp, double alpha, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                        double* ws, hipStream_t stream) {
  FusedArgs f;
  std::memset(&f, 0, sizeof f);
  f.scheme = 1;
  f.C = C;
  f.ldc = ldc;
  f.n = wp.np;
  f.mq = wp.mq_e;
  f.nq = wp.nq;
  f.kq = wp.kq_e;
  f.alpha = alpha;
  f.beta = beta;
  f.tiles_m = (int32_t)cdiv(f.mq, 64);
  f.tiles_n = (int32_t)cdiv(f.nq, 64);
  f.a_sg[0] = f.b_sg[0] = 1.0;
  if (wp.levels == 1) {
    f.A = A;
    f.lda = lda;
    f.B = B;
    f.ldb = ldb;
    f.nc = 1;
    f.c_first = 1;
    f.c_sg[0] = 1.0;
    SMX_LAUNCH(STRASSEN_KERNEL_ALL_PRODUCTS, stream, launch_all_products(f, 1, 1, stream));
    return 0;
  }
  // two levels: outer blocks of m1 x k1 (A), k1 x n1 (B), m1 x n1 (C)
  const int64_t m1 = 2 * wp.mq_e, k1 = 2 * wp.kq_e, n1 = 2 * wp.nq;
  double* SA = ws + wp.sa;
  double* SB = ws + wp.sb;
  ChainSumArgs ca;
  std::memset(&ca, 0, sizeof ca);
  ca.src = A;
  ca.dst = SA;
  ca.ld = lda;
  ca.rows = m1;
  ca.cols = k1;
  ca.dst_stride = wp.sa_stride;
  ChainSumArgs cb = ca;
  cb.src = B;
  cb.dst = SB;
  cb.ld = ldb;
  cb.rows = k1;
  cb.cols = n1;
  cb.dst_stride = wp.sb_stride;
  for (int q = 0; q < 4; ++q) {
    ca.blk[q] = (q >> 1) * m1 + (q & 1) * k1 * lda;
    cb.blk[q] = (q >> 1) * k1 + (q & 1) * n1 * ldb;
  }
  SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_chain_sums(ca, 0, stream));
  SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_chain_sums(cb, 1, stream));
  bool touched[4] = {false, false, false, false};
  for (int R = 0; R < 7; ++R) {
    const WProduct& P = kWinograd[R];
    if (P.a < 4) {
      f.A = A + ca.blk[P.a];
      f.lda = lda;
    } else {
      f.A = SA + (P.a - 4) * wp.sa_stride;
      f.lda = m1;
    }
    if (P.b < 4) {
      f.B = B + cb.blk[P.b];
      f.ldb = ldb;
    } else {
      f.B = SB + (P.b - 4) * wp.sb_stride;
      f.ldb = k1;
    }
    f.nc = P.nc;
    f.c_first = 0;
    for (int d = 0; d < P.nc; ++d) {
      const int q = P.c[d].q;
      f.c_off[d] = (q >> 1) * m1 + (q & 1) * n1 * ldc;
      f.c_cb[d] = 2 * (q & 1);
      f.c_sg[d] = P.c[d].sign;
      if (!touched[q]) f.c_first |= 1 << d;
      touched[q] = true;
    }
    SMX_LAUNCH(STRASSEN_KERNEL_ALL_PRODUCTS, stream, launch_all_products(f, 1, 1, stream));
  }
  return 0;
}

// Winograd's variant at one level on the classical kernel (where one-level ABC takes that
// route): the chain sums S1..S4 and T1..T4 over the four quadrants staged in workspace (four
// m/2 x k/2 and four k/2 x n/2 slots), then one classical launch per product in product order,
// each adding its product to every C quadrant it reaches (M1 all four): the all-products
// kernel's C update, one product at a time, so the same bits.
static size_t winograd_staged_bytes(int64_t m, int64_t n, int64_t k) {
  const int64_t mq = m / 2, nq = n / 2, kq = k / 2;
  return (size_t)(4 * round_up(mq * kq, 32) + 4 * round_up(kq * nq, 32)) * sizeof(double);
}

static int run_winograd_classical(int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                                  int64_t lda, const double* B, int64_t ldb, double beta,
                                  double* C, int64_t ldc, double* ws, hipStream_t stream) {
  const int64_t mq = m / 2, nq = n / 2, kq = k / 2;
  if (cdiv(mq, 256) * cdiv(nq, 128) >= (int64_t(1) << 30))
    return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
  const int64_t sa_stride = round_up(mq * kq, 32), sb_stride = round_up(kq * nq, 32);
  double* SA = ws;
  double* SB = ws + 4 * sa_stride;
  ChainSumArgs ca;
  std::memset(&ca, 0, sizeof ca);
  ca.src = A;
  ca.dst = SA;
  ca.ld = lda;
  ca.rows = mq;
  ca.cols = kq;
  ca.dst_stride = sa_stride;
  ChainSumArgs cb = ca;
  cb.src = B;
  cb.dst = SB;
  cb.ld = ldb;
  cb.rows = kq;
  cb.cols = nq;
  cb.dst_stride = sb_stride;
  for (int q = 0; q < 4; ++q) {
    ca.blk[q] = (q >> 1) * mq + (q & 1) * kq * lda;
    cb.blk[q] = (q >> 1) * kq + (q & 1) * nq * ldb;
  }
  SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_chain_sums(ca, 0, stream));
  SMX_LAUNCH(STRASSEN_KERNEL_OUTER_SUMS, stream, launch_chain_sums(cb, 1, stream));
  bool touched[4] = {false, false, false, false};
  for (int r = 0; r < 7; ++r) {
    const WProduct& P = kWinograd[r];
    ClassicalArgs c;
    std::memset(&c, 0, sizeof c);
    c.A = P.a < 4 ? A + ca.blk[P.a] : SA + (P.a - 4) * sa_stride;
    c.lda = P.a < 4 ? lda : mq;
    c.B = P.b < 4 ? B + cb.blk[P.b] : SB + (P.b - 4) * sb_stride;
    c.ldb = P.b < 4 ? ldb : kq;
    for (int d = 0; d < P.nc; ++d) {
      const int q = P.c[d].q;
      double* dst = C + (q >> 1) * mq + (q & 1) * nq * ldc;
      const double ag = P.c[d].sign > 0 ? alpha : -alpha;
      if (d == 0) {
        c.C = dst;
        c.alpha = ag;
      } else {
        c.Cx[d - 1] = dst;
        c.ax[d - 1] = ag;
      }
      if (touched[q]) c.not_first |= 1 << d;
      touched[q] = true;
    }
    c.extra = P.nc - 1;
    c.beta = beta;
    c.ldc = ldc;
    c.m = mq;
    c.n = nq;
    c.k = kq;
    c.tiles_m = (int32_t)cdiv(mq, 256);
    c.tiles_n = (int32_t)cdiv(nq, 128);
    SMX_LAUNCH(STRASSEN_KERNEL_CLASSICAL, stream, launch_classical(c, stream));
  }
  return 0;
}

int dgemm_winograd(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int levels,
                   const WsSource& wsrc, hipStream_t stream) {
  g_last_error.clear();
  if (levels < 1 || levels > 2) return fail(-12, "levels = %d not in 1..2", levels);
  if (int rc = validate(m, n, k, alpha, A, lda, B, ldb, C, ldc, levels, STRASSEN_ABC)) return rc;
  if (m == 0 || n == 0) return 0;
  if (alpha == 0.0 || k == 0) {
    if (beta == 1.0) return 0;
    int dev = 0;
    if (int rc = device_ready(&dev)) return rc;
    return run_scale(C, ldc, m, n, beta, stream);
  }
  if (levels == 1 && one_level_staged_shape(m, n, k) &&
      classical_layout(m / 2, k / 2, A, lda, B, ldb, C, ldc) &&
      wsrc.fits(winograd_staged_bytes(m, n, k))) {
    int dev = 0;
    if (int rc = device_ready(&dev)) return rc;
    void* w = nullptr;
    const int rc = get_workspace(wsrc, dev, winograd_staged_bytes(m, n, k), &w);
    if (rc == 0)
      return run_winograd_classical(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                                    static_cast<double*>(w), stream);
    if (wsrc.fixed) return rc;
    g_last_error.clear();   // the library-owned allocation failed: the all-products kernel
  }
  const WPlan wp = make_w_plan(m, n, k, levels, A, lda, B, ldb, C, ldc);
  if (!wp.ok) return fail(STRASSEN_ERR_UNSUPPORTED, "sizes past the 32-bit tile offsets");
  if ((int64_t)cdiv(wp.mq_e, 64) * cdiv(wp.nq, 64) >= (int64_t(1) << 30))
    return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
  const size_t bytes = (size_t)wp.total * sizeof(double);
  if (bytes > 0 && !wsrc.fits(bytes))
    return fail(STRASSEN_ERR_ALLOC, "Winograd's variant needs %zu bytes of workspace here (%s), "
                "%zu available", bytes, levels == 2 ? "staged outer sums" : "block-padded copies",
                wsrc.bytes);
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  double* ws = nullptr;
  if (bytes > 0) {
    void* w = nullptr;
    if (int rc = get_workspace(wsrc, dev, bytes, &w)) return rc;
    ws = static_cast<double*>(w);
  }
  const double* Ap = A;
  const double* Bp = B;
  double* Cp = C;
  int64_t la = lda, lb = ldb, lc = ldc;
  if (wp.pa) {
    if (int rc = pad_copy(A, lda, m, k, wp.mq, wp.mq_e, wp.kq, wp.kq_e, ws + wp.a_off, wp.mp,
                          wp.mp, wp.kp, 0, stream))
      return rc;
    Ap = ws + wp.a_off;
    la = wp.mp;
  }
  if (wp.pb) {
    if (int rc = pad_copy(B, ldb, k, n, wp.kq, wp.kq_e, wp.np, wp.np, ws + wp.b_off, wp.kp, wp.kp,
                          wp.np, 0, stream))
      return rc;
    Bp = ws + wp.b_off;
    lb = wp.kp;
  }
  if (wp.pc) {
    Cp = ws + wp.c_off;
    lc = wp.mp;
    if (beta != 0.0)
      if (int rc = pad_copy(C, ldc, m, n, wp.mq, wp.mq_e, wp.np, wp.np, Cp, wp.mp, wp.mp, wp.np,
                            0, stream))
        return rc;
  }
  if (int rc = run_winograd(wp, alpha, Ap, la, Bp, lb, beta, Cp, lc, ws, stream)) return rc;
  if (wp.pc)
    if (int rc = pad_copy(Cp, wp.mp, m, n, wp.mq, wp.mq_e, wp.np, wp.np, C, ldc, wp.mp, wp.np, 1,
                          stream))
      return rc;
  return 0;
}

// Whether the general tile kernel's 32-bit lane offsets reach every element of its tiles: a
// tile spans at most 128 columns of B, C and the temporaries and 16 of A (8 bytes each), and
// each access is one wave-uniform base plus a per-lane offset below 2^31 bytes.
static bool tile_offsets_fit(int64_t lda, int64_t ldb, int64_t ldc, int64_t ldm) {
  const int64_t ld = std::max(std::max(lda, ldb), std::max(ldc, ldm));
  return 8 * 128 * (ld + 1) < (int64_t(1) << 31);
}

static int tile_offsets_error() {
  return fail(STRASSEN_ERR_UNSUPPORTED,
              "a leading dimension of 2^21 - 1 or more on a path that runs the general tile kernel "
              "(128 columns would span 2 GiB past its 32-bit lane offsets)");
}

int dgemm(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
          const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int levels,
          int variant, const WsSource& wsrc, hipStream_t stream) {
  g_last_error.clear();
  if (int rc = validate(m, n, k, alpha, A, lda, B, ldb, C, ldc, levels, variant)) return rc;
  if (m == 0 || n == 0) return 0;
  if (alpha == 0.0 || k == 0) {
    if (beta == 1.0) return 0;
    int dev = 0;
    if (int rc = device_ready(&dev)) return rc;
    return run_scale(C, ldc, m, n, beta, stream);
  }
  if (levels == 3) return dgemm_l3(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, wsrc, stream);
  const Plan p = make_plan(m, n, k, levels, variant);
  const int64_t tiles_limit = 1ll << 30;
  // configuration 6 forces the staged one-level route and is the default otherwise
  const int forced_cfg = g_forced_cfg.load(std::memory_order_relaxed);
  const bool force_staged_classical = forced_cfg == kCfgClassicalStaged;
  const int forced = force_staged_classical ? -1 : forced_cfg;

  GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.A = A;
  g.B = B;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.m = m;
  g.n = n;
  g.k = k;
  g.mq = p.mq;
  g.nq = p.nq;
  g.kq = p.kq;
  g.alpha = alpha;
  g.beta = beta;
  g.tab = p.tab;
  const int maxt = table_maxt(*p.td);
  bool vec = aligned16(A) && aligned16(B) && lda % 2 == 0 && ldb % 2 == 0 && m % 2 == 0 &&
             k % 2 == 0 && p.mq % 2 == 0 && p.kq % 2 == 0;

  if (p.variant == STRASSEN_ABC) {
    // Route (decided on the host): block-padded copies for the all-products kernel where its
    // layout does not fit the operands as given and the workspace allows them, else the
    // all-products kernel in place, else the general tile kernel.  ABC needs no workspace: a
    // workspace that is too small or cannot be allocated only drops the copies or the staging.
    const bool all_products = forced == -1 || forced == kCfgAll || forced == kCfgAllStaged;
    if (levels == 0 && all_products && classical_size(m, n)) {
      // classical: the fused load path in place, else on block-padded copies (m or k odd,
      // misaligned operands or odd leading dimensions), else the general tile kernel below
      const bool in_place = classical_layout(m, k, A, lda, B, ldb, C, ldc);
      PadPlan pp;
      bool padded = false;
      if (!in_place) {
        pp = make_pad_plan(m, n, k, 0, A, lda, B, ldb, C, ldc, forced);
        padded = pp.ok && wsrc.fits((size_t)pp.total * sizeof(double));
      }
      if (in_place || padded) {
        int dev = 0;
        if (int rc = device_ready(&dev)) return rc;
        if (in_place) return run_classical(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream);
        void* ws = nullptr;
        const int rc = get_workspace(wsrc, dev, (size_t)pp.total * sizeof(double), &ws);
        if (rc == 0)
          return run_padded(pp, 0, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                            static_cast<double*>(ws), stream);
        if (wsrc.fixed) return rc;
        g_last_error.clear();   // the library-owned allocation failed: the tile kernel
      }
    }
    // one level: the sums staged and the products on the classical kernel where that applies
    // and the workspace holds the ten sums (else one product's two at a time); without the
    // workspace, the all-products kernel below (the same bits)
    if (levels == 1 && forced == -1 && staged_classical_applies(m, n, k, A, lda, B, ldb, C, ldc)) {
      const size_t all = (size_t)make_stage_plan(p, false, 1).total * sizeof(double);
      const size_t one = (size_t)make_stage_plan(p, true, 1).total * sizeof(double);
      const bool use_one = !wsrc.fits(all);
      if (wsrc.fits(use_one ? one : all)) {
        int dev = 0;
        if (int rc = device_ready(&dev)) return rc;
        void* ws = nullptr;
        const int rc = get_workspace(wsrc, dev, use_one ? one : all, &ws);
        if (rc == 0)
          return run_staged_classical(p, A, lda, B, ldb, C, ldc, alpha, beta,
                                      static_cast<double*>(ws), use_one, stream);
        if (force_staged_classical || wsrc.fixed) return rc;
        g_last_error.clear();   // the library-owned allocation failed: the all-products kernel
      } else if (force_staged_classical) {
        return fail(STRASSEN_ERR_ALLOC, "one-level staged sums need %zu bytes of workspace", one);
      }
    }
    PadPlan pp;
    bool padded = false, pad_one = false;   // pad_one: staging one outer product at a time
    if (all_products && levels >= 1) {
      pp = make_pad_plan(m, n, k, levels, A, lda, B, ldb, C, ldc, forced);
      const bool copies = (pp.pa || pp.pb || pp.pc) && pp.ok;
      padded = copies && wsrc.fits((size_t)pp.total * sizeof(double));
      if (copies && !padded && pp.stage && forced == -1 &&
          wsrc.fits((size_t)pp.total_one * sizeof(double)))
        padded = pad_one = true;
    }
    const bool in_place = all_products && all_products_applies(m, k, A, lda, B, ldb, C, ldc, levels);
    const bool tile_ok = tile_offsets_fit(lda, ldb, ldc, 0);
    if (!padded && !in_place && !tile_ok) return tile_offsets_error();
    int dev = 0;
    if (int rc = device_ready(&dev)) return rc;
    if (padded) {
      void* ws = nullptr;
      const int rc = get_workspace(wsrc, dev,
                                   (size_t)(pad_one ? pp.total_one : pp.total) * sizeof(double), &ws);
      if (rc == 0)
        return run_padded(pp, levels, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                          static_cast<double*>(ws), stream, pad_one);
      // the library-owned allocation failed: the workspace-free path below (same result)
      if (wsrc.fixed) return rc;
      if (!in_place && !tile_ok) return tile_offsets_error();
      g_last_error.clear();
    }
    if (in_place) {
      double* stage = nullptr;
      const bool want = levels == 2 && n % 4 == 0 &&
                        (forced == kCfgAllStaged ||
                         (forced == -1 && staging_applies(m, n, k, levels)));
      bool one = false;
      if (want) {
        size_t bytes = (size_t)make_stage_plan(p).total * sizeof(double);
        // a workspace too small for all ten sums: one outer product's at a time; too small for
        // those too: form the sums in the load
        if (forced != kCfgAllStaged && !wsrc.fits(bytes)) {
          one = true;
          bytes = (size_t)make_stage_plan(p, true).total * sizeof(double);
        }
        if (forced == kCfgAllStaged || wsrc.fits(bytes)) {
          void* ws = nullptr;
          if (int rc = get_workspace(wsrc, dev, bytes, &ws)) {
            if (forced == kCfgAllStaged || wsrc.fixed) return rc;
            g_last_error.clear();
          } else {
            stage = static_cast<double*>(ws);
          }
        }
      }
      return run_all_products(p, A, lda, B, ldb, C, ldc, n, alpha, beta, stage, stream, nullptr,
                              0, 0, one);
    }
    const int cfg = pick_cfg(p, 1, maxt);
    g.tiles_m = (int32_t)cdiv(p.mq, cfg_bm(cfg));
    g.tiles_n = (int32_t)cdiv(p.nq, cfg_bn(cfg));
    const int64_t grid = (int64_t)g.tiles_m * g.tiles_n;
    if (grid >= tiles_limit) return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
    g.mode = kModeABC;
    SMX_LAUNCH(STRASSEN_KERNEL_TILE, stream, launch_fp64_tile(g, cfg, maxt, vec, (int)grid, stream));
    return 0;
  }

  // AB on the all-products kernel where it applies (block-padded A and B where needed), else
  // AB and Naive on the tile kernel (StoreM) over the operands or Naive's temporaries
  AbLayout abl;
  if (p.variant == STRASSEN_AB) abl = make_ab_layout(p, m, n, k, levels, A, lda, B, ldb, forced);
  bool ab_fused = abl.fused && wsrc.fits((size_t)abl.total * sizeof(double));
  const bool tile_ok = tile_offsets_fit(lda, ldb, 0, std::max(p.ldm, std::max(p.mq, p.kq)));
  if (!ab_fused && !tile_ok) return tile_offsets_error();
  if (!wsrc.fits((size_t)p.total * sizeof(double)))
    return fail(STRASSEN_ERR_ALLOC, "%s has %zu bytes, %zu needed",
                wsrc.fixed ? (wsrc.what ? wsrc.what : "caller workspace") : "the workspace limit",
                wsrc.bytes, (size_t)p.total * sizeof(double));
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  const PadPlan& abp = abl.pp;
  void* ws = nullptr;
  if (ab_fused) {
    if (int rc = get_workspace(wsrc, dev, (size_t)abl.total * sizeof(double), &ws)) {
      // the library-owned allocation failed: the tile kernel needs only the temporaries
      if (wsrc.fixed) return rc;
      if (!tile_ok) return tile_offsets_error();
      ab_fused = false;
      g_last_error.clear();
    }
  }
  if (!ab_fused)
    if (int rc = get_workspace(wsrc, dev, (size_t)p.total * sizeof(double), &ws)) return rc;
  double* wsd = static_cast<double*>(ws);
  g.M = wsd + p.off_m;
  g.ldm = p.ldm;
  g.m_stride = p.m_stride;

  if (p.variant == STRASSEN_NAIVE) {
    double* TA = wsd + p.off_ta;
    double* TB = wsd + p.off_tb;
    if (p.td->nslot_a > 0) {
      SumArgs sa;
      std::memset(&sa, 0, sizeof sa);
      sa.src = A;
      sa.dst = TA;
      sa.ld = lda;
      sa.rows = m;
      sa.cols = k;
      sa.rows_q = p.mq;
      sa.cols_q = p.kq;
      sa.dst_stride = p.ta_stride;
      sa.tab = p.tab;
      sa.side = 0;
      sa.chunks_r = (int32_t)cdiv(p.mq, 256);
      SMX_HIP(launch_sums(sa, p.td->nslot_a, stream));
    }
    if (p.td->nslot_b > 0) {
      SumArgs sb;
      std::memset(&sb, 0, sizeof sb);
      sb.src = B;
      sb.dst = TB;
      sb.ld = ldb;
      sb.rows = k;
      sb.cols = n;
      sb.rows_q = p.kq;
      sb.cols_q = p.nq;
      sb.dst_stride = p.tb_stride;
      sb.tab = p.tab;
      sb.side = 1;
      sb.chunks_r = (int32_t)cdiv(p.kq, 256);
      SMX_HIP(launch_sums(sb, p.td->nslot_b, stream));
    }
    g.TA = TA;
    g.TB = TB;
    g.ta_stride = p.ta_stride;
    g.tb_stride = p.tb_stride;
  }

  if (ab_fused) {
    const double* Af = A;
    const double* Bf = B;
    int64_t lda_f = lda, ldb_f = ldb;
    const int64_t whole_n = abp.np;
    if (abp.pa) {
      PadArgs a;
      std::memset(&a, 0, sizeof a);
      a.src = A;
      a.dst = wsd + abl.a_off;
      a.ld_s = lda;
      a.ld_d = abp.mp;
      a.rows = m;
      a.cols = k;
      a.rb = abp.mq;
      a.rb_e = abp.mq_e;
      a.cb = abp.kq;
      a.cb_e = abp.kq_e;
      a.dst_rows = abp.mp;
      a.dst_cols = abp.kp;
      SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream, launch_pad_copy(a, stream));
      Af = a.dst;
      lda_f = abp.mp;
    }
    if (abp.pb) {
      PadArgs b;
      std::memset(&b, 0, sizeof b);
      b.src = B;
      b.dst = wsd + abl.b_off;
      b.ld_s = ldb;
      b.ld_d = abp.kp;
      b.rows = k;
      b.cols = n;
      b.rb = abp.kq;
      b.rb_e = abp.kq_e;
      b.cb = whole_n;
      b.cb_e = whole_n;
      b.dst_rows = abp.kp;
      b.dst_cols = abp.np;
      SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream, launch_pad_copy(b, stream));
      Bf = b.dst;
      ldb_f = abp.kp;
    }
    // C is not read or written by the store form; its pointer only fills the arguments
    const Plan pf = make_plan(abp.mp, abp.np, abp.kp, levels, STRASSEN_ABC);
    if (int rc = run_all_products(pf, Af, lda_f, Bf, ldb_f, C, ldc, abp.np, alpha, beta,
                                  abp.stage ? wsd + abl.s_off : nullptr, stream, g.M, p.ldm,
                                  p.m_stride))
      return rc;
  } else if (naive_on_classical(p, m, n, k, A, lda, B, ldb, forced)) {
    // Naive's products are plain GEMMs on its temporaries (or single quadrants): each runs on the
    // classical kernel with beta = 0, writing M_r (the same MFMA order as the tile kernel: the
    // same bits)
    for (int r = 0; r < p.td->nprod; ++r) {
      const ProdDesc& d = p.td->prod[r];
      const double* Ar = (d.flags & 1) ? g.TA + (int64_t)d.tslot_a * p.ta_stride
                                       : A + code_row_h(d.a[0]) * p.mq + code_col_h(d.a[0]) * p.kq * lda;
      const double* Br = (d.flags & 2) ? g.TB + (int64_t)d.tslot_b * p.tb_stride
                                       : B + code_row_h(d.b[0]) * p.kq + code_col_h(d.b[0]) * p.nq * ldb;
      if (int rc = run_classical(p.mq, p.nq, p.kq, 1.0, Ar, (d.flags & 1) ? p.mq : lda, Br,
                                 (d.flags & 2) ? p.kq : ldb, 0.0, g.M + (int64_t)r * p.m_stride,
                                 p.ldm, stream))
        return rc;
    }
  } else {
    const int cfg = pick_cfg(p, p.td->nprod, maxt);
    g.tiles_m = (int32_t)cdiv(p.mq, cfg_bm(cfg));
    g.tiles_n = (int32_t)cdiv(p.nq, cfg_bn(cfg));
    g.mode = kModeStoreM;
    g.prod_begin = 0;
    const int64_t grid = (int64_t)g.tiles_m * g.tiles_n * p.td->nprod;
    if (grid >= tiles_limit) return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
    SMX_LAUNCH(STRASSEN_KERNEL_TILE, stream, launch_fp64_tile(g, cfg, maxt, vec, (int)grid, stream));
  }

  AssembleArgs asmb;
  std::memset(&asmb, 0, sizeof asmb);
  asmb.M = g.M;
  asmb.C = C;
  asmb.ldm = p.ldm;
  asmb.m_stride = p.m_stride;
  asmb.ldc = ldc;
  asmb.m = m;
  asmb.n = n;
  asmb.mq = p.mq;
  asmb.nq = p.nq;
  asmb.alpha = alpha;
  asmb.beta = beta;
  asmb.tab = p.tab;
  asmb.chunks_m = (int32_t)cdiv(p.mq, 256);
  if ((int64_t)asmb.chunks_m * p.nq * p.q * p.q >= tiles_limit)
    return fail(STRASSEN_ERR_UNSUPPORTED, "too many assembly workgroups");
  SMX_HIP(launch_assemble(asmb, p.q * p.q, stream));
  return 0;
}

// ---------------------------------------------------------------------------------------------
// Reduced-precision mode (BF16 / bf16x3 products).
// ---------------------------------------------------------------------------------------------
struct LowPlan {
  int64_t mq, nq, kq, mp, np, kp, slot_a, slot_b, nslots;
  bool x3;
  size_t bytes;
};

static LowPlan make_low_plan(int64_t m, int64_t n, int64_t k, int levels, int compute) {
  LowPlan p;
  const int64_t q = int64_t(1) << levels;
  p.mq = cdiv(m, q);
  p.nq = cdiv(n, q);
  p.kq = cdiv(k, q);
  p.mp = round_up(p.mq, 128);
  p.np = round_up(p.nq, 128);
  p.kp = round_up(p.kq, 64);
  p.slot_a = p.mp * p.kp;
  p.slot_b = p.np * p.kp;
  p.nslots = host_tables()[table_id(levels, false)].nprod;
  p.x3 = compute == STRASSEN_COMPUTE_BF16X3;
  p.bytes = (size_t)(p.slot_a + p.slot_b) * p.nslots * 2 * (p.x3 ? 2 : 1);
  return p;
}

int gemm_ex(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
            const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int levels,
            int variant, int compute, int sum_prec, int c_prec, hipStream_t stream) {
  g_last_error.clear();
  if (int rc = validate(m, n, k, alpha, A, lda, B, ldb, C, ldc, levels, variant)) return rc;
  if (compute < 0 || compute > 2) return fail(-14, "compute = %d not in 0..2", compute);
  if (sum_prec < 0 || sum_prec > 1) return fail(-15, "sum_prec = %d not in 0..1", sum_prec);
  if (c_prec < 0 || c_prec > 1) return fail(-16, "c_prec = %d not in 0..1", c_prec);
  if (compute == STRASSEN_COMPUTE_F64)
    return dgemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, levels, variant,
                 default_workspace(), stream);
  if (levels > kMaxLevels)
    return fail(-12, "the reduced-precision mode runs levels 0..%d (levels = %d)", kMaxLevels, levels);
  if (variant != STRASSEN_ABC)
    return fail(-13, "the reduced-precision mode runs the ABC variant only (variant = %d)", variant);
  if (m == 0 || n == 0) return 0;
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  if (alpha == 0.0 || k == 0) {
    if (beta == 1.0) return 0;
    return run_scale(C, ldc, m, n, beta, stream);
  }
  const LowPlan p = make_low_plan(m, n, k, levels, compute);
  const int64_t lim = int64_t(1) << 31;
  if (2 * p.slot_a >= lim || 2 * p.slot_b >= lim || 8 * 128 * ldc >= lim)
    return fail(STRASSEN_ERR_UNSUPPORTED, "reduced-precision operands past the 32-bit offset range");
  void* ws = nullptr;
  if (int rc = get_workspace(default_workspace(), dev, p.bytes, &ws)) return rc;
  uint16_t* w = static_cast<uint16_t*>(ws);
  uint16_t* TAh = w;
  uint16_t* TBh = TAh + p.slot_a * p.nslots;
  uint16_t* TAl = p.x3 ? TBh + p.slot_b * p.nslots : nullptr;
  uint16_t* TBl = p.x3 ? TAl + p.slot_a * p.nslots : nullptr;
  const int tab = table_id(levels, false);

  CastArgs ca;
  std::memset(&ca, 0, sizeof ca);
  ca.src = A;
  ca.hi = TAh;
  ca.lo = TAl;
  ca.ld = lda;
  ca.rows = m;
  ca.cols = k;
  ca.rq = p.mq;
  ca.cq = p.kq;
  ca.outer_pad = p.mp;
  ca.kpad = p.kp;
  ca.slot_stride = p.slot_a;
  ca.tab = tab;
  ca.side = 0;
  ca.sum_f64 = sum_prec == STRASSEN_PREC_F64;
  SMX_LAUNCH(STRASSEN_KERNEL_CAST, stream, launch_cast(ca, (int)p.nslots, stream));
  CastArgs cb = ca;
  cb.src = B;
  cb.hi = TBh;
  cb.lo = TBl;
  cb.ld = ldb;
  cb.rows = k;
  cb.cols = n;
  cb.rq = p.kq;
  cb.cq = p.nq;
  cb.outer_pad = p.np;
  cb.slot_stride = p.slot_b;
  cb.side = 1;
  SMX_LAUNCH(STRASSEN_KERNEL_CAST, stream, launch_cast(cb, (int)p.nslots, stream));

  Bf16Args g;
  std::memset(&g, 0, sizeof g);
  g.TAh = TAh;
  g.TAl = TAl;
  g.TBh = TBh;
  g.TBl = TBl;
  g.stride_a = p.slot_a;
  g.stride_b = p.slot_b;
  g.kpad = p.kp;
  g.C = C;
  g.ldc = ldc;
  g.m = m;
  g.n = n;
  g.mq = p.mq;
  g.nq = p.nq;
  g.alpha = alpha;
  g.beta = beta;
  g.tab = tab;
  g.x3 = p.x3;
  g.c_f64 = c_prec == STRASSEN_PREC_F64;
  g.vec_c = aligned16(C) && ldc % 2 == 0 && p.mq % 2 == 0;
  // 128 x 64 workgroup tiles where 128 x 128 ones would not give every CU two workgroups
  // (tile configuration 0 / 1 force 128 x 128 / 128 x 64)
  {
    const int forced = g_forced_cfg.load(std::memory_order_relaxed);
    const int64_t t128 = (p.mp / 128) * (p.np / 128);
    g.shape = forced == kCfg64 || (forced != kCfg128 && t128 < 512) ? 1 : 0;
    g.tiles_m = (int32_t)(p.mp / 128);
    g.tiles_n = (int32_t)(p.np / (g.shape == 1 ? 64 : 128));
  }
  SMX_LAUNCH(STRASSEN_KERNEL_BF16, stream, launch_bf16_gemm(g, stream));
  return 0;
}

// Workspace strassen_dgemm uses for these sizes with 16-byte aligned operands of even leading
// dimensions (strassen_workspace_size).
size_t workspace_bytes(int64_t m, int64_t n, int64_t k, int levels, int variant) {
  if (m == 0 || n == 0 || k == 0) return 0;
  if (levels == 3)
    return (size_t)make_l3_plan(m, n, k, nullptr, 2 * cdiv(m, 2), nullptr, 2 * cdiv(k, 2),
                                nullptr, 2 * cdiv(m, 2)).total * sizeof(double);
  const Plan p = make_plan(m, n, k, levels, variant);
  size_t bytes = (size_t)p.total * sizeof(double);
  if (levels == 0 && classical_size(m, n) && (m % 2 != 0 || k % 2 != 0)) {
    // the classical kernel on block-padded copies (m or k rounded up to even)
    const PadPlan pp = make_pad_plan(m, n, k, 0, nullptr, 2 * cdiv(m, 2), nullptr,
                                     2 * cdiv(k, 2), nullptr, 2 * cdiv(m, 2), -1);
    if (pp.ok) bytes = (size_t)pp.total * sizeof(double);
  }
  if (variant == STRASSEN_AB)
    // the all-products form of AB: padded A and B copies and staged outer sums behind the
    // temporaries (operands taken as 16-byte aligned with even leading dimensions)
    bytes = (size_t)make_ab_layout(p, m, n, k, levels, nullptr, 2 * cdiv(m, 2), nullptr,
                                   2 * cdiv(k, 2), -1).total *
            sizeof(double);
  if (variant == STRASSEN_ABC && levels >= 1) {
    // operands taken as 16-byte aligned with even leading dimensions
    const PadPlan pp = make_pad_plan(m, n, k, levels, nullptr, 2 * cdiv(m, 2), nullptr,
                                     2 * cdiv(k, 2), nullptr, 2 * cdiv(m, 2), -1);
    if ((pp.pa || pp.pb || pp.pc) && pp.ok)
      bytes = (size_t)pp.total * sizeof(double);
    else if (staging_applies(m, n, k, levels))
      bytes = (size_t)make_stage_plan(p).total * sizeof(double);
    else if (levels == 1 && one_level_staged_shape(m, n, k))
      bytes = (size_t)make_stage_plan(p, false, 1).total * sizeof(double);   // staged sums
  }
  return bytes;
}

// C := alpha*op(A)*op(B) + beta*C with op(X) = X or X^T (Sec. 2.2).  A transposed operand is
// packed, transposed, into workspace (a tiled copy through LDS, the counterpart of BLIS packing
// a transposed block) with an even leading dimension and 16-byte alignment; the call then runs
// strassen_dgemm on the packed operands with the rest of the same workspace.  levels < 0: the
// member is chosen by strassen_select.
static bool trans_code(char t, bool* out) {
  if (t == 'N' || t == 'n') *out = false;
  else if (t == 'T' || t == 't' || t == 'C' || t == 'c') *out = true;
  else return false;
  return true;
}

// C := alpha*A*B^T + beta*C (levels 0) on the general tile kernel reading B^T in place: where
// the classical product runs on that kernel anyway (problems too small for the classical
// kernel's 256 x 128 tiles), this saves the packing launch and gives the same bits.
static int run_tile_tb(int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                       int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, hipStream_t stream) {
  if (!tile_offsets_fit(lda, ldb, ldc, 0)) return tile_offsets_error();
  const Plan p = make_plan(m, n, k, 0, STRASSEN_ABC);
  GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.A = A;
  g.B = B;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.m = m;
  g.n = n;
  g.k = k;
  g.mq = p.mq;
  g.nq = p.nq;
  g.kq = p.kq;
  g.alpha = alpha;
  g.beta = beta;
  g.tab = p.tab;
  g.tb = 1;
  const int maxt = table_maxt(*p.td);
  // 16-byte loads: A row pairs (m even), B^T column pairs (n even)
  const bool vec = aligned16(A) && aligned16(B) && lda % 2 == 0 && ldb % 2 == 0 && m % 2 == 0 &&
                   n % 2 == 0;
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  const int cfg = pick_cfg(p, 1, maxt);
  g.tiles_m = (int32_t)cdiv(p.mq, cfg_bm(cfg));
  g.tiles_n = (int32_t)cdiv(p.nq, cfg_bn(cfg));
  const int64_t grid = (int64_t)g.tiles_m * g.tiles_n;
  if (grid >= (int64_t(1) << 30)) return fail(STRASSEN_ERR_UNSUPPORTED, "too many tiles");
  g.mode = kModeABC;
  SMX_LAUNCH(STRASSEN_KERNEL_TILE, stream, launch_fp64_tile(g, cfg, maxt, vec, (int)grid, stream));
  return 0;
}

int gemm_t(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
           const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
           int64_t ldc, int levels, int variant, const WsSource& wsrc, hipStream_t stream) {
  g_last_error.clear();
  bool ta = false, tb = false;
  if (!trans_code(transa, &ta)) return fail(-1, "transa = '%c' is not N, T or C", transa);
  if (!trans_code(transb, &tb)) return fail(-2, "transb = '%c' is not N, T or C", transb);
  if (m < 0) return fail(-3, "m = %lld < 0", (long long)m);
  if (n < 0) return fail(-4, "n = %lld < 0", (long long)n);
  if (k < 0) return fail(-5, "k = %lld < 0", (long long)k);
  const bool reads_ab = m > 0 && n > 0 && k > 0 && alpha != 0.0;
  if (reads_ab && A == nullptr) return fail(-7, "A is NULL");
  if (lda < std::max<int64_t>(1, ta ? k : m)) return fail(-8, "lda = %lld too small", (long long)lda);
  if (reads_ab && B == nullptr) return fail(-9, "B is NULL");
  if (ldb < std::max<int64_t>(1, tb ? n : k)) return fail(-10, "ldb = %lld too small", (long long)ldb);
  if (m > 0 && n > 0 && C == nullptr) return fail(-12, "C is NULL");
  if (ldc < std::max<int64_t>(1, m)) return fail(-13, "ldc = %lld < max(1, m)", (long long)ldc);
  if (levels < -1 || levels > kMaxLevelsAbc)
    return fail(-14, "levels = %d not in -1..%d", levels, kMaxLevelsAbc);
  if (levels >= 0 && (variant < 0 || variant > 2)) return fail(-15, "variant = %d not in 0..2", variant);
  if (levels > kMaxLevels && variant != STRASSEN_ABC)
    return fail(-15, "levels = %d runs the ABC variant only (variant = %d)", levels, variant);
  if (m == 0 || n == 0) return 0;
  if (levels < 0) {
    if (int rc = strassen_select(m, n, k, 0, &levels, &variant)) return rc;
    g_last_error.clear();
  }
  if (!reads_ab || (!ta && !tb)) {   // nothing to pack (A and B unread when !reads_ab)
    const int64_t la = ta ? std::max<int64_t>(1, m) : lda, lb = tb ? std::max<int64_t>(1, k) : ldb;
    return dgemm(m, n, k, alpha, ta ? nullptr : A, la, tb ? nullptr : B, lb, beta, C, ldc,
                 levels, variant, wsrc, stream);
  }
  const int fcfg = g_forced_cfg.load();
  if (!ta && levels == 0 && !classical_size(m, n) && (fcfg < kCfgAll || fcfg == kCfgClassicalStaged))
    return run_tile_tb(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream);
  // packed operands: op(A) as m x k with ld round_up(m, 2), op(B) as k x n with ld round_up(k, 2)
  const int64_t lda_p = round_up(m, 2), ldb_p = round_up(k, 2);
  const int64_t a_elems = ta ? round_up(lda_p * k, 32) : 0;
  const int64_t b_elems = tb ? round_up(ldb_p * n, 32) : 0;
  const size_t pack = (size_t)(a_elems + b_elems) * sizeof(double);
  const size_t rest = workspace_bytes(m, n, k, levels, variant);
  if (!wsrc.fits(pack + rest)) {
    // the packed operands are required; the rest only as far as the member needs it
    if (!wsrc.fits(pack))
      return fail(STRASSEN_ERR_ALLOC, "packing the transposed operands needs %zu bytes of workspace",
                  pack);
  }
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  const size_t want = wsrc.fits(pack + rest) ? pack + rest : pack;
  void* ws = nullptr;
  if (int rc = get_workspace(wsrc, dev, want, &ws)) return rc;
  double* wsd = static_cast<double*>(ws);
  const double* Ap = A;
  const double* Bp = B;
  int64_t la = lda, lb = ldb;
  if (ta) {
    TransposeArgs t{A, wsd, lda, lda_p, m, k};
    SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream, launch_transpose(t, stream));
    Ap = wsd;
    la = lda_p;
  }
  if (tb) {
    TransposeArgs t{B, wsd + a_elems, ldb, ldb_p, k, n};
    SMX_LAUNCH(STRASSEN_KERNEL_PAD, stream, launch_transpose(t, stream));
    Bp = wsd + a_elems;
    lb = ldb_p;
  }
  // the member's own workspace: the rest of the same buffer (nothing is reallocated under the
  // packed operands)
  WsSource tail;
  tail.fixed = true;
  tail.ptr = static_cast<char*>(ws) + pack;
  tail.bytes = want - pack;
  tail.what = wsrc.fixed ? wsrc.what : "the workspace left after packing";
  return dgemm(m, n, k, alpha, Ap, la, Bp, lb, beta, C, ldc, levels, variant, tail, stream);
}

}  // namespace smx

// ---------------------------------------------------------------------------------------------
// extern "C" entry points.
// ---------------------------------------------------------------------------------------------
extern "C" {

int strassen_dgemm(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int levels,
                   int variant, void* stream) {
  return smx::dgemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, levels, variant,
                    smx::default_workspace(), static_cast<hipStream_t>(stream));
}

int strassen_gemm(char transa, char transb, int64_t m, int64_t n, int64_t k, double alpha,
                  const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                  double* C, int64_t ldc, int levels, int variant, void* stream) {
  return smx::gemm_t(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, levels,
                     variant, smx::default_workspace(), static_cast<hipStream_t>(stream));
}

int strassen_dgemm_winograd(int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                            int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                            int64_t ldc, int levels, void* stream) {
  return smx::dgemm_winograd(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, levels,
                             smx::default_workspace(), static_cast<hipStream_t>(stream));
}

int strassen_workspace_size_winograd(int64_t m, int64_t n, int64_t k, int levels, size_t* bytes) {
  smx::g_last_error.clear();
  if (m < 0) return smx::fail(-1, "m < 0");
  if (n < 0) return smx::fail(-2, "n < 0");
  if (k < 0) return smx::fail(-3, "k < 0");
  if (levels < 1 || levels > 2) return smx::fail(-4, "levels out of range");
  if (!bytes) return smx::fail(-5, "bytes is NULL");
  *bytes = (m == 0 || n == 0 || k == 0)
               ? 0
               : (size_t)smx::make_w_plan(m, n, k, levels, nullptr, 2 * smx::cdiv(m, 2), nullptr,
                                          2 * smx::cdiv(k, 2), nullptr, 2 * smx::cdiv(m, 2))
                         .total * sizeof(double);
  if (levels == 1 && m > 0 && n > 0 && k > 0 && smx::one_level_staged_shape(m, n, k))
    *bytes = smx::winograd_staged_bytes(m, n, k);   // the staged chain sums
  return 0;
}

int strassen_workspace_size(int64_t m, int64_t n, int64_t k, int levels, int variant,
                            size_t* bytes) {
  smx::g_last_error.clear();
  if (m < 0) return smx::fail(-1, "m < 0");
  if (n < 0) return smx::fail(-2, "n < 0");
  if (k < 0) return smx::fail(-3, "k < 0");
  if (levels < 0 || levels > smx::kMaxLevelsAbc) return smx::fail(-4, "levels out of range");
  if (variant < 0 || variant > 2) return smx::fail(-5, "variant out of range");
  if (levels > smx::kMaxLevels && variant != STRASSEN_ABC)
    return smx::fail(-5, "levels %d runs the ABC variant only", levels);
  if (!bytes) return smx::fail(-6, "bytes is NULL");
  *bytes = smx::workspace_bytes(m, n, k, levels, variant);
  return 0;
}

int strassen_set_workspace(void* ptr, size_t bytes) {
  smx::g_last_error.clear();
  if (ptr && ((uintptr_t)ptr & 255) != 0) return smx::fail(-1, "workspace not 256-byte aligned");
  if (ptr && bytes == 0) return smx::fail(-2, "workspace of 0 bytes");
  std::lock_guard<std::mutex> lk(smx::g_mu);
  smx::g_user_ws = ptr;
  smx::g_user_ws_bytes = ptr ? bytes : 0;
  return 0;
}

int strassen_set_workspace_limit(size_t bytes) {
  smx::g_last_error.clear();
  std::lock_guard<std::mutex> lk(smx::g_mu);
  smx::g_ws_limit = bytes == 0 ? SIZE_MAX : bytes;
  return 0;
}

int strassen_release_workspace(void) {
  smx::g_last_error.clear();
  std::lock_guard<std::mutex> lk(smx::g_mu);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return 0;
  for (size_t d = 0; d < smx::g_dev.size(); ++d) {
    if (!smx::g_dev[d].ws) continue;
    SMX_HIP(hipSetDevice((int)d));
    SMX_HIP(hipDeviceSynchronize());
    SMX_HIP(hipFree(smx::g_dev[d].ws));
    smx::g_dev[d].ws = nullptr;
    smx::g_dev[d].ws_bytes = 0;
  }
  SMX_HIP(hipSetDevice(cur));
  return 0;
}

int strassen_gemm_ex(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                     const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int levels,
                     int variant, int compute, int sum_prec, int c_prec, void* stream) {
  return smx::gemm_ex(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, levels, variant, compute,
                      sum_prec, c_prec, static_cast<hipStream_t>(stream));
}

int strassen_workspace_size_ex(int64_t m, int64_t n, int64_t k, int levels, int compute,
                               size_t* bytes) {
  smx::g_last_error.clear();
  if (m < 0) return smx::fail(-1, "m < 0");
  if (n < 0) return smx::fail(-2, "n < 0");
  if (k < 0) return smx::fail(-3, "k < 0");
  if (levels < 0 || levels > smx::kMaxLevels) return smx::fail(-4, "levels out of range");
  if (compute < 0 || compute > 2) return smx::fail(-5, "compute out of range");
  if (!bytes) return smx::fail(-6, "bytes is NULL");
  if (compute == STRASSEN_COMPUTE_F64 || m == 0 || n == 0 || k == 0) {
    *bytes = 0;
    return 0;
  }
  *bytes = smx::make_low_plan(m, n, k, levels, compute).bytes;
  return 0;
}

int strassen_timing_enable(int on) {
  smx::g_last_error.clear();
  smx::g_timing.store(on != 0);
  return 0;
}

int strassen_probe_rates(double* fp64_tflops, double* bf16_tflops, void* stream) {
  smx::g_last_error.clear();
  if (!fp64_tflops || !bf16_tflops) return smx::fail(-1, "NULL output");
  int dev = 0;
  if (int rc = smx::device_ready(&dev)) return rc;
  hipDeviceProp_t prop;
  SMX_HIP(hipGetDeviceProperties(&prop, dev));
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int grid = smx::probe_grid(prop.multiProcessorCount);
  double* out = nullptr;
  SMX_HIP(hipMalloc(&out, (size_t)grid * 256 * sizeof(double)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // about 20 ms per timed launch at the datasheet rates
  const int iters[2] = {10000, 40000};
  double* res[2] = {fp64_tflops, bf16_tflops};
  for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) {
    e = smx::launch_rate_probe(kind, out, grid, iters[kind] / 10, s);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = smx::launch_rate_probe(kind, out, grid, iters[kind], s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) {
      const double flops = (double)grid * 4.0 * iters[kind] * smx::probe_flops_per_wave_iter(kind);
      *res[kind] = flops / (ms * 1e-3) * 1e-12;
    }
  }
  const hipError_t es = hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (e != hipSuccess) return smx::hip_fail(e, "rate probe");
  if (es != hipSuccess) return smx::hip_fail(es, "rate probe");
  return 0;
}

int strassen_timing_collect(int kind, double* ms_total, int* launches) {
  smx::g_last_error.clear();
  if (!ms_total || !launches) return smx::fail(-2, "NULL output");
  std::vector<smx::TimedLaunch> mine;
  {
    std::lock_guard<std::mutex> lk(smx::g_tm_mu);
    std::vector<smx::TimedLaunch> rest;
    for (const auto& t : smx::g_tm_log) (t.kind == kind ? mine : rest).push_back(t);
    smx::g_tm_log.swap(rest);
  }
  double total = 0.0;
  int rc = 0;
  for (const auto& t : mine) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(t.e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.e0, t.e1);
    if (e != hipSuccess && rc == 0) rc = smx::hip_fail(e, "timing events");
    total += ms;
  }
  {
    std::lock_guard<std::mutex> lk(smx::g_tm_mu);
    for (const auto& t : mine) {
      smx::g_tm_pool.push_back(t.e0);
      smx::g_tm_pool.push_back(t.e1);
    }
  }
  *ms_total = total;
  *launches = (int)mine.size();
  return rc;
}

int strassen_set_tile_config(int cfg) {
  smx::g_last_error.clear();
  if (cfg < -1 || cfg >= smx::kNumCfgs) return smx::fail(-1, "tile configuration %d out of range", cfg);
  smx::g_forced_cfg.store(cfg);
  return 0;
}

int strassen_table_size(int levels) {
  if (levels < 0 || levels > smx::kMaxLevelsAbc) return -1;
  return (int)smx::host_table(levels).size();
}

int strassen_table_get(int levels, int r, int* na, int* a_terms, int* nb, int* b_terms, int* nc,
                       int* c_terms) {
  if (levels < 0 || levels > smx::kMaxLevelsAbc) return -1;
  const std::vector<smx::Product>& tab = smx::host_table(levels);
  if (r < 0 || r >= (int)tab.size()) return -2;
  const smx::Product& p = tab[r];
  const int q = 1 << levels;
  auto dec = [q](const smx::Term& t) {
    const int v = 1 + t.row + q * t.col;
    return t.sign < 0 ? -v : v;
  };
  *na = (int)p.a.size();
  *nb = (int)p.b.size();
  *nc = (int)p.c.size();
  for (int s = 0; s < *na; ++s) a_terms[s] = dec(p.a[s]);
  for (int s = 0; s < *nb; ++s) b_terms[s] = dec(p.b[s]);
  for (int s = 0; s < *nc; ++s) c_terms[s] = dec(p.c[s]);
  return 0;
}

const char* strassen_last_error(void) { return smx::g_last_error.c_str(); }

const char* strassen_version(void) { return "strassen-mi355x 0.1 (gfx950, FP64 MFMA)"; }

}  // extern "C"
