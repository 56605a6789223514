// Selector: which member of the family (classical; one- or two-level ABC, AB, Naive) to run
// for a shape (the paper leaves the choice as a function of problem size to the user, Sec. 5).
//
// With a network loaded (strassen_selector_load) the choice is the arg-max of its scores, run
// by the library's inference kernel.  Without one it is the arg-min of an analytical time model:
// the GPU counterpart of the paper's breakdown (Sec. 4.2, Fig. "tab:breakdown"): MFMA time of
// each launch at this library's rates (the FP64 rate of the kernel a member runs, times the
// member's efficiency e relative to it), rounded to whole rounds of resident workgroups, plus launch
// latency, plus the HBM time of the extra passes (the AB / Naive temporaries: M_r written and
// read back by the C assembly, operand sums written and read; for BF16 the operand pass).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>

#include "../../include/strassen.h"
#include "internal.h"
#include "launch.h"
#include "plan.h"

namespace smx {

namespace {

// member index -> (levels, variant)
const int kMemberLevels[7] = {0, 1, 1, 1, 2, 2, 2};
const int kMemberVariant[7] = {STRASSEN_ABC, STRASSEN_ABC, STRASSEN_AB, STRASSEN_NAIVE,
                               STRASSEN_ABC, STRASSEN_AB, STRASSEN_NAIVE};

struct SelectorState {
  bool loaded = false;
  std::vector<float> host;
  int dev = -1;
  float* d_params = nullptr;
  float* d_io = nullptr;   // kMlpIn inputs then 7 logits
  hipStream_t stream = nullptr;
};
std::mutex g_sel_mu;
SelectorState g_sel;

bool member_available(int dtype, int c) {
  return dtype == 0 || kMemberVariant[c] == STRASSEN_ABC;
}

}  // namespace

// Analytical time model (seconds) of member c for C := A*B + C.  Each launch is `items` work
// items of `fi` MFMA flops spread over `slots` resident workgroups (two 256-thread workgroups
// per CU for the tile kernel, one 512-thread workgroup per CU for the all-products kernel, the
// classical kernel and the BF16 kernel); a workgroup runs at its share of the rate, and the launch takes
// ceil(items / slots) rounds.
static double launch_seconds(double items, double fi, double slots, double rate) {
  if (items <= 0.0) return 0.0;
  const double resident = std::min(items, slots);
  // with fewer items than CUs a workgroup has a CU to itself
  const double share = rate / std::max(resident, std::min(slots, 256.0));
  return std::ceil(items / slots) * fi / share;
}

// The kernel each member runs for these sizes follows the library's own dispatch.  Classical:
// where its 256 x 128 tiles fill the CUs, the classical kernel (on block-padded copies when m or
// k is odd), else the tile kernel.  ABC: the all-products kernel (whole tiles or masked) on the
// operands as given where m and k are multiples of 2^(L+1), else on block-padded copies (every
// sub-block extent rounded up to even; the copies cost their HBM traffic), at two levels with
// the staged outer sums where they apply (n rounded up to 4 by the copies).  AB: the
// all-products kernel storing M_r (block-padded A and B where needed, staged at two levels)
// where that applies, else the tile kernel; then the assembly of C from the M_r.  Naive: the
// operand sums, then each product a GEMM on the classical kernel where the partition is exact
// and its tiles fill the CUs, else the tile kernel; then the assembly.  Rates and efficiencies
// were fitted to this library's timings of the selector's 20000 training shapes (coordinate
// search on the regret of the model's choice; efficiencies capped at 1, rates at the MFMA peak,
// the bandwidth at the HBM peak, and every member's time at m = n = k = 16384 within 5% of the
// measured one).  The tile-kernel AB / Naive terms are fitted for the choice, not for their
// absolute times.
namespace {
struct ModelCoef {
  double R = 59.7e12;          // FP64 MFMA rate of the tile kernel
  double R_cl = 78.6e12;       // classical kernel, inside a round (the MFMA peak) ...
  double t_round = 188.0e-6;   // ... plus its fill and epilogue per round of resident tiles
  double e_full = 0.875;       // all-products kernel, whole tiles (relative to R_cl)
  double e_masked = 0.869;     // all-products kernel, masked loads
  double e_unstaged = 0.75;    // two levels, outer sums in the load
  double e_store = 0.99;       // all-products kernel storing M_r (AB), relative to the above
  double e_ab1 = 1.0, e_ab2 = 0.528, e_naive1 = 0.963, e_naive2 = 0.483;   // tile kernel
  double bw = 6.69e12;         // HBM bytes/s of the element-wise passes (fitted, capped at 8e12)
  double t_launch = 8.2e-6;    // per launch (latency and tail)
  double R_bf16 = 900.0e12;    // BF16 product kernel
  double bw_cast = 4.0e12;     // its operand pass
};
const ModelCoef kCoef;
}  // namespace

double model_seconds(int64_t m, int64_t n, int64_t k, int dtype, int c) {
  if (!member_available(dtype, c)) return std::numeric_limits<double>::infinity();
  const ModelCoef& K = kCoef;
  const int L = kMemberLevels[c], var = kMemberVariant[c];
  const int64_t q = int64_t(1) << L;
  const int64_t mqi = cdiv(m, q), nqi = cdiv(n, q), kqi = cdiv(k, q);
  const double mq = (double)mqi, nq = (double)nqi, kq = (double)kqi;
  const double dm = (double)m, dn = (double)n, dk = (double)k;
  const double p7 = L == 0 ? 1.0 : (L == 1 ? 7.0 : 49.0);
  // operand terms and C updates of the tables (Sec. 3.1, Sec. 3.5): 12^L each
  const double terms = L == 0 ? 1.0 : (L == 1 ? 12.0 : 144.0);
  auto tiles = [](double a, double b, double ta, double tb) {
    return std::ceil(a / ta) * std::ceil(b / tb);
  };
  // one classical-kernel launch of a x b x kk (256 x 128 tiles, one workgroup per CU)
  auto classical = [&](double a, double b, double kk) {
    const double items = tiles(a, b, 256.0, 128.0);
    return launch_seconds(items, 2.0 * 256 * 128 * kk, 256.0, K.R_cl) +
           std::ceil(items / 256.0) * K.t_round + K.t_launch;
  };
  // one tile-kernel launch of `prods` products of a x b x kk at efficiency e
  auto tile = [&](double prods, double a, double b, double kk, double e) {
    const double t128 = tiles(a, b, 128.0, 128.0);
    if (prods * t128 < 512.0)
      return launch_seconds(prods * tiles(a, b, 64.0, 64.0), 2.0 * 64 * 64 * kk, 1024.0,
                            K.R * 0.85 * e) + K.t_launch;
    return launch_seconds(prods * t128, 2.0 * 128 * 128 * kk, 512.0, K.R * e) + K.t_launch;
  };
  if (dtype != 0) {
    // BF16: all 7^L products per 128 x 128 item (two workgroups per CU); the operand pass
    // reads every term once in FP64 and writes the padded bf16 slots
    double t = launch_seconds(tiles(mq, nq, 128.0, 128.0), p7 * 2.0 * 128 * 128 * kq, 512.0,
                              K.R_bf16) + 3.0 * K.t_launch;
    const double mp = std::ceil(mq / 128.0) * 128.0, np_ = std::ceil(nq / 128.0) * 128.0,
                 kp = std::ceil(kq / 64.0) * 64.0;
    t += (8.0 * terms * (mq * kq + kq * nq) + 2.0 * p7 * (mp * kp + kp * np_)) / K.bw_cast;
    return t;
  }
  if (L == 0) {
    if (cdiv(m, 256) * cdiv(n, 128) < 256) return tile(1.0, dm, dn, dk, 1.0);
    double copies = 0.0;   // m or k odd: A copied, B when k is odd, C in and out when m is odd
    if (m % 2 != 0 || k % 2 != 0)
      copies = 8.0 * (2.0 * dm * dk + (k % 2 ? 2.0 * dk * dn : 0.0) + (m % 2 ? 4.0 * dm * dn : 0.0)) /
                   K.bw + (1.0 + (k % 2) + 2.0 * (m % 2)) * K.t_launch;
    return copies + classical(dm, dn, dk);
  }
  // the all-products kernel's block padding and staging (ABC; AB without the C copies)
  const int64_t unit = int64_t(2) << L;
  const int64_t mqe = round_up(mqi, 2), kqe = round_up(kqi, 2);
  const int64_t mp = q * mqe, kp = q * kqe, n4 = round_up(n, 4);
  const bool staged = L == 2 && (mp / 2) * (n4 / 2) >= int64_t(2048) * 2048 && kp >= 2048;
  const bool pad_mk = m % unit != 0 || k % unit != 0;
  const bool pad_n = staged && n % 4 != 0;
  const double mqp = (double)mqe, kqp = (double)kqe;
  const bool whole_p = mqe % 64 == 0 && nqi % 64 == 0 && kqe % 16 == 0 &&
                       q * nqi <= (pad_n ? n4 : n);
  auto ap = [&](double e) {   // one all-products launch: 7 products per 64 x 64 item
    return launch_seconds(tiles(mqp, nq, 64.0, 64.0), 7.0 * 2.0 * 64 * 64 * kqp, 256.0,
                          K.R_cl * e) + K.t_launch;
  };
  // all-products launches: one at one level, seven (after the staged outer sums) at two
  auto products = [&](double e) {
    if (L == 1) return ap(e);
    if (!staged) return 7.0 * ap(K.e_unstaged);
    // the outer sums: per side four blocks read, five sums written
    return 7.0 * ap(e) + 8.0 * 9.0 * (4.0 * mqp * kqp + 4.0 * kqp * nq) / K.bw + 2.0 * K.t_launch;
  };
  const double e_ap = whole_p ? K.e_full : K.e_masked;
  if (var == STRASSEN_ABC) {
    if (L == 1 && one_level_staged_shape(m, n, k)) {
      // the sums staged (per side four quadrants read, five sums written), the seven products
      // on the classical kernel, five of them updating a second C quadrant
      return 8.0 * 9.0 * (mq * kq + kq * nq) / K.bw + 2.0 * K.t_launch +
             7.0 * classical(mq, nq, kq) + 5.0 * 16.0 * mq * nq / K.bw;
    }
    double copies = 0.0;   // block-padded copies: A and B (or B only), C in and out
    if (pad_mk) copies = 8.0 * (2.0 * dm * dk + 2.0 * dk * dn + 4.0 * dm * dn) / K.bw + 4.0 * K.t_launch;
    else if (pad_n) copies = 8.0 * (2.0 * dk * dn + 4.0 * dm * dn) / K.bw + 3.0 * K.t_launch;
    return copies + products(e_ap);
  }
  // M_r written once and read by the assembly once per destination; C read and written
  const double assembly = (8.0 * mq * nq * (p7 + terms) + 16.0 * dm * dn) / K.bw + K.t_launch;
  if (var == STRASSEN_AB) {
    const bool fused = (L == 1 || staged) &&
                       (!(pad_mk || pad_n) || cdiv(mqe, 64) * cdiv(nqi, 64) >= 192);
    if (fused) {
      double copies = 0.0;   // block-padded A and B
      if (pad_mk) copies = 8.0 * (2.0 * dm * dk + 2.0 * dk * dn) / K.bw + 2.0 * K.t_launch;
      else if (pad_n) copies = 8.0 * 2.0 * dk * dn / K.bw + K.t_launch;
      return copies + products(e_ap * K.e_store) + assembly;
    }
    return tile(p7, mq, nq, kq, L == 1 ? K.e_ab1 : K.e_ab2) + assembly;
  }
  // Naive: operand sums (terms read, one temporary per product written), products, assembly
  const double sums = 8.0 * (terms + p7) * (mq * kq + kq * nq) / K.bw + 2.0 * K.t_launch;
  const bool on_classical = m % q == 0 && n % q == 0 && k % q == 0 &&
                            cdiv(mqi, 256) * cdiv(nqi, 128) >= 256 && mqi % 2 == 0 && kqi % 2 == 0;
  if (on_classical) return sums + p7 * classical(mq, nq, kq) + assembly;
  return sums + tile(p7, mq, nq, kq, L == 1 ? K.e_naive1 : K.e_naive2) + assembly;
}

// The network's input for a shape: the sizes on a log scale (256 -> 0, 20000 -> 1), the dtype
// flag, and for each member the analytical model's time over the model's best, as
// min(ln(t_c / t_best), 1) (members not offered for the dtype: 1).  The network learns where
// the measured order departs from the model's.
static void feature_vec(int64_t m, int64_t n, int64_t k, int dtype, float* x) {
  const double lo = std::log(256.0), hi = std::log(20000.0);
  auto f = [&](int64_t s) { return (float)((std::log((double)std::max<int64_t>(s, 1)) - lo) / (hi - lo)); };
  x[0] = f(m);
  x[1] = f(n);
  x[2] = f(k);
  x[3] = dtype == 0 ? 0.f : 1.f;
  double t[7], best = std::numeric_limits<double>::infinity();
  for (int c = 0; c < 7; ++c) {
    t[c] = model_seconds(m, n, k, dtype, c);
    best = std::min(best, t[c]);
  }
  for (int c = 0; c < 7; ++c)
    x[4 + c] = std::isfinite(t[c]) && best > 0.0 ? (float)std::min(std::log(t[c] / best), 1.0) : 1.f;
}

static int ensure_device_copy() {
  int dev = 0;
  SMX_HIP(hipGetDevice(&dev));
  if (g_sel.dev == dev && g_sel.d_params) return 0;
  if (g_sel.d_params) {
    (void)hipFree(g_sel.d_params);
    (void)hipFree(g_sel.d_io);
    if (g_sel.stream) (void)hipStreamDestroy(g_sel.stream);
  }
  g_sel.d_params = nullptr;
  g_sel.d_io = nullptr;
  g_sel.stream = nullptr;
  SMX_HIP(hipMalloc(&g_sel.d_params, kMlpParams * sizeof(float)));
  SMX_HIP(hipMalloc(&g_sel.d_io, 32 * sizeof(float)));
  SMX_HIP(hipStreamCreate(&g_sel.stream));   // default priority
  SMX_HIP(hipMemcpy(g_sel.d_params, g_sel.host.data(), kMlpParams * sizeof(float),
                    hipMemcpyHostToDevice));
  g_sel.dev = dev;
  return 0;
}

}  // namespace smx

extern "C" {

int strassen_mlp_forward(const float* params, const float* X, int n, float* logits,
                         void* stream) {
  smx::clear_error();
  if (!params) return smx::fail(-1, "params is NULL");
  if (n < 0) return smx::fail(-3, "n < 0");
  if (n > 0 && !X) return smx::fail(-2, "X is NULL");
  if (n > 0 && !logits) return smx::fail(-4, "logits is NULL");
  if (n == 0) return 0;
  SMX_HIP(smx::launch_mlp_forward(params, X, n, logits, nullptr, nullptr,
                                  static_cast<hipStream_t>(stream)));
  return 0;
}

int strassen_mlp_work_size(int n, size_t* bytes) {
  smx::clear_error();
  if (n < 0) return smx::fail(-1, "n < 0");
  if (!bytes) return smx::fail(-2, "bytes is NULL");
  *bytes = (size_t)n * (7 + 64 + 64 + 7 + 64 + 64 + 1) * sizeof(float);
  return 0;
}

int strassen_mlp_loss_grad(const float* params, const float* X, const int* labels, int n,
                           float* work, float* grad, float* loss, void* stream) {
  smx::clear_error();
  if (!params) return smx::fail(-1, "params is NULL");
  if (!X) return smx::fail(-2, "X is NULL");
  if (!labels) return smx::fail(-3, "labels is NULL");
  if (n <= 0) return smx::fail(-4, "n <= 0");
  if (!work) return smx::fail(-5, "work is NULL");
  if (!grad) return smx::fail(-6, "grad is NULL");
  if (!loss) return smx::fail(-7, "loss is NULL");
  SMX_HIP(smx::launch_mlp_backward(params, X, labels, n, work, grad, loss,
                                   static_cast<hipStream_t>(stream)));
  return 0;
}

int strassen_mlp_adam(float* params, const float* grad, float* m, float* v, int t, float lr,
                      float beta1, float beta2, float eps, void* stream) {
  smx::clear_error();
  if (!params || !grad || !m || !v) return smx::fail(-1, "NULL buffer");
  if (t < 1) return smx::fail(-5, "t < 1");
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, t)));
  SMX_HIP(smx::launch_mlp_adam(params, grad, m, v, lr, beta1, beta2, eps, c1, c2,
                               static_cast<hipStream_t>(stream)));
  return 0;
}

int strassen_selector_load(const float* params) {
  smx::clear_error();
  std::lock_guard<std::mutex> lk(smx::g_sel_mu);
  if (!params) {
    smx::g_sel.loaded = false;
    return 0;
  }
  for (int i = 0; i < smx::kMlpParams; ++i)
    if (!std::isfinite(params[i])) return smx::fail(-1, "parameter %d is not finite", i);
  smx::g_sel.host.assign(params, params + smx::kMlpParams);
  smx::g_sel.dev = -1;   // copied to the current device at the next selection
  smx::g_sel.loaded = true;
  return 0;
}

int strassen_cost_model(int64_t m, int64_t n, int64_t k, int dtype, double* seconds) {
  smx::clear_error();
  if (m < 0 || n < 0 || k < 0) return smx::fail(-1, "negative size");
  if (dtype < 0 || dtype > 1) return smx::fail(-4, "dtype not 0 (FP64) or 1 (BF16)");
  if (!seconds) return smx::fail(-5, "seconds is NULL");
  for (int c = 0; c < 7; ++c) seconds[c] = smx::model_seconds(m, n, k, dtype, c);
  return 0;
}

int strassen_selector_features(int64_t m, int64_t n, int64_t k, int dtype, float* x) {
  smx::clear_error();
  if (m < 0 || n < 0 || k < 0) return smx::fail(-1, "negative size");
  if (dtype < 0 || dtype > 1) return smx::fail(-4, "dtype not 0 (FP64) or 1 (BF16)");
  if (!x) return smx::fail(-5, "x is NULL");
  smx::feature_vec(m, n, k, dtype, x);
  return 0;
}

int strassen_select(int64_t m, int64_t n, int64_t k, int dtype, int* levels, int* variant) {
  smx::clear_error();
  if (m < 0) return smx::fail(-1, "m < 0");
  if (n < 0) return smx::fail(-2, "n < 0");
  if (k < 0) return smx::fail(-3, "k < 0");
  if (dtype < 0 || dtype > 1) return smx::fail(-4, "dtype not 0 (FP64) or 1 (BF16)");
  if (!levels || !variant) return smx::fail(-5, "NULL output");
  float score[7];
  bool use_net;
  {
    std::lock_guard<std::mutex> lk(smx::g_sel_mu);
    use_net = smx::g_sel.loaded;
    if (use_net) {
      int dev = 0;
      if (int rc = smx::device_ready(&dev)) return rc;
      if (int rc = smx::ensure_device_copy()) return rc;
      constexpr int kIn = smx::kMlpIn;
      float io[kIn + 7];
      smx::feature_vec(m, n, k, dtype, io);
      SMX_HIP(hipMemcpyAsync(smx::g_sel.d_io, io, kIn * sizeof(float), hipMemcpyHostToDevice,
                             smx::g_sel.stream));
      SMX_HIP(smx::launch_mlp_forward(smx::g_sel.d_params, smx::g_sel.d_io, 1, smx::g_sel.d_io + kIn,
                                      nullptr, nullptr, smx::g_sel.stream));
      SMX_HIP(hipMemcpyAsync(io + kIn, smx::g_sel.d_io + kIn, 7 * sizeof(float),
                             hipMemcpyDeviceToHost, smx::g_sel.stream));
      SMX_HIP(hipStreamSynchronize(smx::g_sel.stream));
      std::memcpy(score, io + kIn, sizeof score);
    }
  }
  if (!use_net)
    for (int c = 0; c < 7; ++c) score[c] = (float)-smx::model_seconds(m, n, k, dtype, c);
  int best = 0;
  for (int c = 1; c < 7; ++c)
    if (smx::member_available(dtype, c) && score[c] > score[best]) best = c;
  *levels = smx::kMemberLevels[best];
  *variant = smx::kMemberVariant[best];
  return 0;
}

}  // extern "C"
