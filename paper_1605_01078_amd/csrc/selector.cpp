// Selector: which member of the family (classical; one- or two-level ABC, AB, Naive) to run
// for a shape (the paper leaves the choice as a function of problem size to the user, Sec. 5).
//
// With a network loaded (strassen_selector_load) the choice is the arg-max of its scores, run
// by the library's inference kernel.  Without one it is the arg-min of an analytical time model:
// the GPU counterpart of the paper's breakdown (Sec. 4.2, Fig. "tab:breakdown"): MFMA time of
// each launch at this library's rates (classical FP64 rate R, times the member's kernel
// efficiency e relative to it), rounded to whole rounds of resident workgroups, plus launch
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
  float* d_io = nullptr;   // 4 inputs then 7 logits
  hipStream_t stream = nullptr;
};
std::mutex g_sel_mu;
SelectorState g_sel;

void feature_vec(int64_t m, int64_t n, int64_t k, int dtype, float* x) {
  const double lo = std::log(256.0), hi = std::log(20000.0);
  auto f = [&](int64_t s) { return (float)((std::log((double)std::max<int64_t>(s, 1)) - lo) / (hi - lo)); };
  x[0] = f(m);
  x[1] = f(n);
  x[2] = f(k);
  x[3] = dtype == 0 ? 0.f : 1.f;
}

bool member_available(int dtype, int c) {
  return dtype == 0 || kMemberVariant[c] == STRASSEN_ABC;
}

}  // namespace

// Analytical time model (seconds) of member c for C := A*B + C.  Each launch is `items` work
// items of `fi` MFMA flops spread over `slots` resident workgroups (two 256-thread workgroups
// per CU for the tile kernel, one 512-thread workgroup per CU for the all-products kernel and
// the BF16 kernel); a workgroup runs at its share of the rate, and the launch takes
// ceil(items / slots) rounds.
static double launch_seconds(double items, double fi, double slots, double rate) {
  if (items <= 0.0) return 0.0;
  const double resident = std::min(items, slots);
  // with fewer items than CUs a workgroup has a CU to itself
  const double share = rate / std::max(resident, std::min(slots, 256.0));
  return std::ceil(items / slots) * fi / share;
}

// The kernel each member runs for these sizes follows the library's own dispatch: ABC runs the
// all-products kernel (whole tiles or masked) on the operands as given where m and k are
// multiples of 2^(L+1), else on block-padded copies (every sub-block extent rounded up to even;
// the copies cost their HBM traffic), at two levels with the staged outer sums where they apply
// (n rounded up to 4 by the copies).  Rates and
// efficiencies were fitted to this library's timings of the selector's 20000 training shapes
// (coordinate search on the regret of the model's choice, efficiencies capped at 1 and the
// bandwidth at the HBM peak, keeping the measured order at m = n = k = 16384: two-level ABC,
// one-level ABC, classical, and those three within 5% of their measured times there).  The
// AB / Naive terms are fitted for the choice, not for their absolute times.
namespace {
struct ModelCoef {
  double R = 66.0e12;        // classical FP64 MFMA rate of the tile kernel
  double e_full = 0.99;      // all-products kernel, whole tiles (relative to R)
  double e_masked = 0.985;   // all-products kernel, masked loads
  double e_unstaged = 0.80;  // two levels, outer sums in the load
  double e_ab1 = 0.744, e_ab2 = 0.562, e_naive1 = 0.598, e_naive2 = 0.483;
  double bw = 7.97e12;       // HBM bytes/s of the element-wise passes (fitted, capped at 8e12)
  double t_launch = 9.6e-6;  // per launch (latency and tail)
  double R_bf16 = 900.0e12;  // BF16 product kernel
  double bw_cast = 4.0e12;   // its operand pass
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
  const double p7 = L == 0 ? 1.0 : (L == 1 ? 7.0 : 49.0);
  // operand terms and C updates of the tables (Sec. 3.1, Sec. 3.5): 12^L each
  const double terms = L == 0 ? 1.0 : (L == 1 ? 12.0 : 144.0);
  auto tiles = [](double a, double b, double t) { return std::ceil(a / t) * std::ceil(b / t); };
  double t = 0.0;
  if (dtype == 0) {
    if (L == 0) {
      const double t128 = tiles(mq, nq, 128.0);
      if (t128 < 512.0)
        return launch_seconds(tiles(mq, nq, 64.0), 2.0 * 64 * 64 * kq, 1024.0, K.R * 0.85) + K.t_launch;
      return launch_seconds(t128, 2.0 * 128 * 128 * kq, 512.0, K.R) + K.t_launch;
    }
    if (var == STRASSEN_ABC) {
      const int64_t unit = int64_t(2) << L;
      const int64_t mqe = round_up(mqi, 2), kqe = round_up(kqi, 2);
      const int64_t mp = q * mqe, kp = q * kqe, n4 = round_up(n, 4);
      const bool staged = L == 2 && (mp / 2) * (n4 / 2) >= int64_t(2048) * 2048 && kp >= 2048;
      const bool pad_mk = m % unit != 0 || k % unit != 0;
      const bool pad_n = staged && n % 4 != 0;
      double copies = 0.0;   // block-padded copies: A and B (or B only), C in and out
      const double dm = (double)m, dn = (double)n, dk = (double)k;
      if (pad_mk) copies = 8.0 * (2.0 * dm * dk + 2.0 * dk * dn + 4.0 * dm * dn) / K.bw + 4.0 * K.t_launch;
      else if (pad_n) copies = 8.0 * (2.0 * dk * dn + 4.0 * dm * dn) / K.bw + 3.0 * K.t_launch;
      const double mqp = (double)mqe, kqp = (double)kqe;
      const bool whole_p = mqe % 64 == 0 && nqi % 64 == 0 && kqe % 16 == 0 &&
                           q * nqi <= (pad_n ? n4 : n);
      auto ap = [&](double e) {   // one all-products launch: 7 products per 64 x 64 item
        return launch_seconds(tiles(mqp, nq, 64.0), 7.0 * 2.0 * 64 * 64 * kqp, 256.0, K.R * e) +
               K.t_launch;
      };
      if (L == 1) return copies + ap(whole_p ? K.e_full : K.e_masked);
      if (!staged) return copies + 7.0 * ap(K.e_unstaged);
      // the outer sums (per side four blocks read, five sums written), then seven one-level
      // launches
      return copies + 7.0 * ap(whole_p ? K.e_full : K.e_masked) +
             8.0 * 9.0 * (4.0 * mqp * kqp + 4.0 * kqp * nq) / K.bw + 2.0 * K.t_launch;
    }
    const double e = var == STRASSEN_AB ? (L == 1 ? K.e_ab1 : K.e_ab2) : (L == 1 ? K.e_naive1 : K.e_naive2);
    t = launch_seconds(p7 * tiles(mq, nq, 128.0), 2.0 * 128 * 128 * kq, 512.0, K.R * e) +
        (var == STRASSEN_AB ? 2.0 : 4.0) * K.t_launch;
    // M_r written once and read by the assembly once per destination; C read and written
    t += (8.0 * mq * nq * (p7 + terms) + 16.0 * (double)m * (double)n) / K.bw;
    if (var == STRASSEN_NAIVE)   // operand sums: terms read, one temporary per product written
      t += 8.0 * (terms + p7) * (mq * kq + kq * nq) / K.bw;
    return t;
  }
  // BF16: all 7^L products per 128 x 128 item (two workgroups per CU); the operand pass reads
  // every term once in FP64 and writes the padded bf16 slots
  t = launch_seconds(tiles(mq, nq, 128.0), p7 * 2.0 * 128 * 128 * kq, 512.0, K.R_bf16) + 3.0 * K.t_launch;
  const double mp = std::ceil(mq / 128.0) * 128.0, np_ = std::ceil(nq / 128.0) * 128.0,
               kp = std::ceil(kq / 64.0) * 64.0;
  t += (8.0 * terms * (mq * kq + kq * nq) + 2.0 * p7 * (mp * kp + kp * np_)) / K.bw_cast;
  return t;
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
  SMX_HIP(hipMalloc(&g_sel.d_io, 16 * sizeof(float)));
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
      float io[16];
      smx::feature_vec(m, n, k, dtype, io);
      SMX_HIP(hipMemcpyAsync(smx::g_sel.d_io, io, 4 * sizeof(float), hipMemcpyHostToDevice,
                             smx::g_sel.stream));
      SMX_HIP(smx::launch_mlp_forward(smx::g_sel.d_params, smx::g_sel.d_io, 1, smx::g_sel.d_io + 4,
                                      nullptr, nullptr, smx::g_sel.stream));
      SMX_HIP(hipMemcpyAsync(io + 4, smx::g_sel.d_io + 4, 7 * sizeof(float),
                             hipMemcpyDeviceToHost, smx::g_sel.stream));
      SMX_HIP(hipStreamSynchronize(smx::g_sel.stream));
      std::memcpy(score, io + 4, sizeof score);
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
