// Batched mode host side: plans, the per-problem choice rule and its autotuner, the work list,
// eager launches and graph capture / replay.
//
// Every problem gets a Strassen level and a tile shape.  Entries given as -1 follow a rule,
//   level = 2 if min(m, n, k) >= t2, else 1 if min(m, n, k) >= t1, else 0;
//   tile  = its own launches on a side stream (min(m, n, k) >= t_own; level at most 1), else
//           its own all-products launch (one level, min(m, n, k) >= t_ap), else
//           64 x 64 if the 128 x 128 grid of one sub-block has fewer than `small` tiles,
//           else 128 x 128;
// whose thresholds the autotuner picks by timing the batch itself (persistent kernel, side
// streams and all-products launches) on a sample of its problems: the quantity that matters is
// the batch's time, not one problem's latency.
//
// Side streams: problems of tile choice kBatchOwn run as ordinary single calls (the classical
// kernel, the all-products kernel or the tile kernel, as strassen_dgemm would choose them, with
// no workspace) spread over kBranches streams forked from the caller's stream and joined back
// into it, concurrently with the persistent kernel: several problems that each fill part of the
// GPU then share it.  A captured graph keeps the fork and join as parallel branches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <limits>
#include <numeric>
#include <random>
#include <vector>

#include "../../include/strassen.h"
#include "internal.h"
#include "launch.h"
#include "plan.h"

namespace smx {

struct Rule {
  int64_t t1 = std::numeric_limits<int64_t>::max();   // min dimension for one level
  int64_t t2 = std::numeric_limits<int64_t>::max();   // for two levels
  int64_t small = 0;                                  // 128-tile count below which tiles are 64
  int64_t t_ap = std::numeric_limits<int64_t>::max(); // min dimension for an all-products launch
  int64_t t_own = std::numeric_limits<int64_t>::max(); // min dimension for side-stream launches
};

constexpr int kBatchAllProducts = 2;   // problem tile choice: its own all-products launch(es)
constexpr int kBatchOwn = 3;           // its own single-call launches on a side stream
constexpr int kBranches = 4;           // side streams (the GPU's hardware queues per process)

// A problem run on a side stream.
struct OwnLaunch {
  int64_t m, n, k, lda, ldb, ldc;
  const double* A;
  const double* B;
  double* C;
  int level;
  double cost;
};

struct BatchedPlan {
  int count = 0;
  std::vector<int64_t> m, n, k;
  std::vector<int> level, cfg;
  std::vector<char> auto_level, auto_cfg;   // chosen by the rule (re-chosen by the autotuner)
  Rule rule;
  // device state of the last run / capture
  int dev = -1;
  BatchProblem* d_probs = nullptr;
  BatchItem* d_items = nullptr;
  unsigned* d_counter = nullptr;
  size_t cap_probs = 0, cap_items = 0;
  int n_items = 0;
  std::vector<ApLaunch> ap;   // all-products launches of the problems that have them, in order
  std::vector<OwnLaunch> own; // side-stream problems, longest first
  hipStream_t branch[kBranches] = {};
  hipStream_t cap = nullptr;   // the stream graph capture records on (the caller's may be the null stream)
  hipEvent_t fork = nullptr, join[kBranches] = {};
  double alpha = 1.0, beta = 1.0;
  bool vec = true;
  int grid = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void apply_rule(const Rule& r, int64_t m, int64_t n, int64_t k, int* level, int* cfg,
                       bool set_level, bool set_cfg) {
  const int64_t mn = std::min(m, std::min(n, k));
  if (set_level) *level = mn >= r.t2 ? 2 : (mn >= r.t1 ? 1 : 0);
  if (set_cfg) {
    if (mn >= r.t_own) {
      *cfg = kBatchOwn;
      if (set_level && *level > 1) *level = 1;   // side streams share no workspace: no staging
      return;
    }
    const int64_t q = int64_t(1) << *level;
    const int64_t tiles128 = cdiv(cdiv(m, q), 128) * cdiv(cdiv(n, q), 128);
    *cfg = *level == 1 && mn >= r.t_ap ? kBatchAllProducts : (tiles128 < r.small ? 1 : 0);
  }
}

static void drop_graph(BatchedPlan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

static void free_device(BatchedPlan* p) {
  drop_graph(p);
  for (int b = 0; b < kBranches; ++b) {
    if (p->branch[b]) (void)hipStreamDestroy(p->branch[b]);
    if (p->join[b]) (void)hipEventDestroy(p->join[b]);
    p->branch[b] = nullptr;
    p->join[b] = nullptr;
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  p->fork = nullptr;
  p->cap = nullptr;
  if (p->d_probs) (void)hipFree(p->d_probs);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_counter) (void)hipFree(p->d_counter);
  p->d_probs = nullptr;
  p->d_items = nullptr;
  p->d_counter = nullptr;
  p->cap_probs = p->cap_items = 0;
}

// Problems (GemmArgs per problem) and the cost-ordered work list of the persistent kernel for
// the given operands, and the all-products launches of the problems that run on their own.
static int build_work(const BatchedPlan& p, const double* const* A, const int64_t* lda,
                      const double* const* B, const int64_t* ldb, double* const* C,
                      const int64_t* ldc, double alpha, double beta,
                      std::vector<BatchProblem>* probs, std::vector<BatchItem>* items,
                      std::vector<ApLaunch>* ap, std::vector<OwnLaunch>* own, bool* vec) {
  const TableDev* tabs = host_tables();
  probs->clear();
  items->clear();
  ap->clear();
  own->clear();
  *vec = true;
  std::vector<double> cost;
  for (int i = 0; i < p.count; ++i) {
    const int64_t m = p.m[i], n = p.n[i], k = p.k[i];
    if (m == 0 || n == 0 || k == 0 || alpha == 0.0) continue;   // handled by the caller
    const int L = p.level[i];
    const int64_t q = int64_t(1) << L;
    int cfg = p.cfg[i];
    if (cfg == kBatchOwn) {
      const double c = (double)tabs[table_id(L, false)].nprod * (double)cdiv(m, q) *
                       (double)cdiv(n, q) * (double)cdiv(k, q);
      own->push_back({m, n, k, lda[i], ldb[i], ldc[i], A[i], B[i], C[i], L, c});
      continue;
    }
    if (cfg == kBatchAllProducts) {
      if (all_products_ok(m, k, A[i], lda[i], B[i], ldb[i], C[i], ldc[i], L)) {
        std::vector<ApLaunch> mine;
        if (int rc = all_products_plan(m, n, k, L, A[i], lda[i], B[i], ldb[i], C[i], ldc[i],
                                       alpha, beta, &mine))
          return rc;
        ap->insert(ap->end(), mine.begin(), mine.end());
        continue;
      }
      // layout does not apply: the persistent kernel, tiles as a single call would pick them
      cfg = cdiv(cdiv(m, q), 128) * cdiv(cdiv(n, q), 128) < 512 ? 1 : 0;
    }
    BatchProblem bp;
    std::memset(&bp, 0, sizeof bp);
    GemmArgs& g = bp.g;
    g.A = A[i];
    g.B = B[i];
    g.C = C[i];
    g.lda = lda[i];
    g.ldb = ldb[i];
    g.ldc = ldc[i];
    g.m = m;
    g.n = n;
    g.k = k;
    g.mq = cdiv(m, q);
    g.nq = cdiv(n, q);
    g.kq = cdiv(k, q);
    g.alpha = alpha;
    g.beta = beta;
    g.tab = table_id(L, false);
    g.mode = kModeABC;
    bp.cfg = cfg;
    const int64_t bm = bp.cfg == 0 ? 128 : 64;
    g.tiles_m = (int32_t)cdiv(g.mq, bm);
    g.tiles_n = (int32_t)cdiv(g.nq, bm);
    const bool v = ((uintptr_t)A[i] & 15) == 0 && ((uintptr_t)B[i] & 15) == 0 && lda[i] % 2 == 0 &&
                   ldb[i] % 2 == 0 && m % 2 == 0 && k % 2 == 0 && g.mq % 2 == 0 && g.kq % 2 == 0;
    *vec = *vec && v;
    const int pid = (int)probs->size();
    probs->push_back(bp);
    const double c = (double)tabs[g.tab].nprod * bm * bm * (double)g.kq;
    for (int t = 0; t < g.tiles_m * g.tiles_n; ++t) {
      items->push_back({pid, t});
      cost.push_back(c);
    }
  }
  // longest items first (stable: ties keep problem order)
  std::vector<int> order(items->size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<BatchItem> sorted(items->size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = (*items)[order[i]];
  items->swap(sorted);
  std::stable_sort(own->begin(), own->end(),
                   [](const OwnLaunch& a, const OwnLaunch& b) { return a.cost > b.cost; });
  if (items->size() >= (size_t)std::numeric_limits<int32_t>::max())
    return fail(STRASSEN_ERR_UNSUPPORTED, "batched: too many work items");
  return 0;
}

static int validate_operands(const BatchedPlan& p, const double* const* A, const int64_t* lda,
                             const double* const* B, const int64_t* ldb, double* const* C,
                             const int64_t* ldc) {
  if (!A || !lda || !B || !ldb || !C || !ldc) return fail(-2, "batched: NULL operand array");
  for (int i = 0; i < p.count; ++i) {
    const int64_t m = p.m[i], n = p.n[i], k = p.k[i];
    if (lda[i] < std::max<int64_t>(1, m) || ldb[i] < std::max<int64_t>(1, k) ||
        ldc[i] < std::max<int64_t>(1, m))
      return fail(-3, "batched: problem %d: leading dimension too small", i);
    if (m > 0 && n > 0 && !C[i]) return fail(-3, "batched: problem %d: C is NULL", i);
    if (m > 0 && n > 0 && k > 0 && (!A[i] || !B[i]))
      return fail(-3, "batched: problem %d: A or B is NULL", i);
    if (8 * 128 * std::max(lda[i], std::max(ldb[i], ldc[i])) >= (int64_t(1) << 31))
      return fail(STRASSEN_ERR_UNSUPPORTED, "batched: problem %d: leading dimension too large", i);
  }
  return 0;
}

// Device copies of the problems and the work list (grown on demand).
static int upload(BatchedPlan* p, const std::vector<BatchProblem>& probs,
                  const std::vector<BatchItem>& items, hipStream_t s) {
  int dev = 0;
  SMX_HIP(hipGetDevice(&dev));
  if (p->dev != dev) {
    free_device(p);
    p->dev = dev;
  }
  if (!p->d_counter) SMX_HIP(hipMalloc(&p->d_counter, 256));
  if (!p->fork) {
    SMX_HIP(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    SMX_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));   // default priority
    for (int b = 0; b < kBranches; ++b) {
      SMX_HIP(hipStreamCreateWithFlags(&p->branch[b], hipStreamNonBlocking));   // default priority
      SMX_HIP(hipEventCreateWithFlags(&p->join[b], hipEventDisableTiming));
    }
  }
  if (p->cap_probs < probs.size()) {
    if (p->d_probs) SMX_HIP(hipFree(p->d_probs));
    p->d_probs = nullptr;
    SMX_HIP(hipMalloc(&p->d_probs, std::max<size_t>(1, probs.size()) * sizeof(BatchProblem)));
    p->cap_probs = probs.size();
  }
  if (p->cap_items < items.size()) {
    if (p->d_items) SMX_HIP(hipFree(p->d_items));
    p->d_items = nullptr;
    SMX_HIP(hipMalloc(&p->d_items, std::max<size_t>(1, items.size()) * sizeof(BatchItem)));
    p->cap_items = items.size();
  }
  if (!probs.empty())
    SMX_HIP(hipMemcpyAsync(p->d_probs, probs.data(), probs.size() * sizeof(BatchProblem),
                           hipMemcpyHostToDevice, s));
  if (!items.empty())
    SMX_HIP(hipMemcpyAsync(p->d_items, items.data(), items.size() * sizeof(BatchItem),
                           hipMemcpyHostToDevice, s));
  // the host vectors go out of scope after this call: finish the copies first
  SMX_HIP(hipStreamSynchronize(s));
  p->n_items = (int)items.size();
  hipDeviceProp_t prop;
  SMX_HIP(hipGetDeviceProperties(&prop, dev));
  p->grid = 2 * prop.multiProcessorCount;   // two 256-thread workgroups per CU
  return 0;
}

// Problems with alpha == 0 or k == 0 only scale C (outside the persistent kernel).
static int scale_only(const BatchedPlan& p, double* const* C, const int64_t* ldc, double alpha,
                      double beta, hipStream_t s) {
  for (int i = 0; i < p.count; ++i) {
    if (p.m[i] == 0 || p.n[i] == 0) continue;
    if (!(alpha == 0.0 || p.k[i] == 0) || beta == 1.0) continue;
    ScaleArgs a;
    a.C = C[i];
    a.ldc = ldc[i];
    a.m = p.m[i];
    a.n = p.n[i];
    a.beta = beta;
    SMX_HIP(launch_scale(a, s));
  }
  return 0;
}

// The batch's launches for the uploaded work: the side streams forked from s, the persistent
// kernel over the items (after its counter clear) and the all-products launches in problem
// order on s, then the side streams joined back into s.  Side-stream problems go, longest
// first, to the stream with the least work so far.
static int launch_work(const BatchedPlan& p, hipStream_t s) {
  double load[kBranches] = {};
  if (!p.own.empty()) {
    SMX_HIP(hipEventRecord(p.fork, s));
    for (int b = 0; b < kBranches; ++b) SMX_HIP(hipStreamWaitEvent(p.branch[b], p.fork, 0));
    const WsSource none{true, nullptr, 0, "no workspace (batched side streams)", nullptr};
    for (const OwnLaunch& o : p.own) {
      const int b = (int)(std::min_element(load, load + kBranches) - load);
      load[b] += o.cost;
      if (int rc = dgemm(o.m, o.n, o.k, p.alpha, o.A, o.lda, o.B, o.ldb, p.beta, o.C, o.ldc,
                         o.level, STRASSEN_ABC, none, p.branch[b]))
        return rc;
    }
  }
  if (p.n_items > 0)
    SMX_HIP(launch_batched(p.d_probs, p.d_items, p.n_items, p.d_counter, p.vec, p.grid, s));
  for (const ApLaunch& l : p.ap) SMX_HIP(launch_all_products(l.f, l.na, l.nb, s));
  if (!p.own.empty())
    for (int b = 0; b < kBranches; ++b) {
      SMX_HIP(hipEventRecord(p.join[b], p.branch[b]));
      SMX_HIP(hipStreamWaitEvent(s, p.join[b], 0));
    }
  return 0;
}

static int run_plan(BatchedPlan* p, const double* const* A, const int64_t* lda,
                    const double* const* B, const int64_t* ldb, double* const* C,
                    const int64_t* ldc, double alpha, double beta, hipStream_t s) {
  if (int rc = validate_operands(*p, A, lda, B, ldb, C, ldc)) return rc;
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  std::vector<BatchProblem> probs;
  std::vector<BatchItem> items;
  std::vector<ApLaunch> ap;
  std::vector<OwnLaunch> own;
  bool vec = true;
  if (int rc = build_work(*p, A, lda, B, ldb, C, ldc, alpha, beta, &probs, &items, &ap, &own, &vec))
    return rc;
  if (int rc = scale_only(*p, C, ldc, alpha, beta, s)) return rc;
  drop_graph(p);   // the buffers a recorded graph reads are about to change
  if (int rc = upload(p, probs, items, s)) return rc;
  p->vec = vec;
  p->ap = std::move(ap);
  p->own = std::move(own);
  p->alpha = alpha;
  p->beta = beta;
  return launch_work(*p, s);
}

// ---------------------------------------------------------------------------------------------
// Autotuner.
// ---------------------------------------------------------------------------------------------
static int autotune(BatchedPlan* p, int sample, uint64_t seed, hipStream_t s) {
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  // the sample: up to `sample` problems, chosen by the seeded generator
  std::vector<int> idx(p->count);
  std::iota(idx.begin(), idx.end(), 0);
  std::mt19937_64 gen(seed);
  std::shuffle(idx.begin(), idx.end(), gen);
  if (sample > 0 && sample < p->count) idx.resize(sample);
  BatchedPlan sp;
  sp.count = (int)idx.size();
  size_t bytes = 0;
  std::vector<size_t> offa, offb, offc;
  for (int i : idx) {
    sp.m.push_back(p->m[i]);
    sp.n.push_back(p->n[i]);
    sp.k.push_back(p->k[i]);
    auto push = [&](std::vector<size_t>& v, int64_t elems) {
      v.push_back(bytes);
      bytes += (size_t)round_up(std::max<int64_t>(1, elems), 32) * 8;
    };
    push(offa, p->m[i] * p->k[i]);
    push(offb, p->k[i] * p->n[i]);
    push(offc, p->m[i] * p->n[i]);
  }
  sp.level.assign(sp.count, 0);
  sp.cfg.assign(sp.count, 0);
  char* buf = nullptr;
  SMX_HIP(hipMalloc(&buf, std::max<size_t>(bytes, 256)));
  // timing does not depend on the values: zero operands
  hipError_t e = hipMemsetAsync(buf, 0, bytes, s);
  std::vector<const double*> A(sp.count), B(sp.count);
  std::vector<double*> C(sp.count);
  std::vector<int64_t> lda(sp.count), ldb(sp.count), ldc(sp.count);
  for (int i = 0; i < sp.count; ++i) {
    A[i] = reinterpret_cast<const double*>(buf + offa[i]);
    B[i] = reinterpret_cast<const double*>(buf + offb[i]);
    C[i] = reinterpret_cast<double*>(buf + offc[i]);
    lda[i] = std::max<int64_t>(1, sp.m[i]);
    ldb[i] = std::max<int64_t>(1, sp.k[i]);
    ldc[i] = std::max<int64_t>(1, sp.m[i]);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int64_t inf = std::numeric_limits<int64_t>::max();
  const int64_t t1s[] = {inf, 3072, 2048, 1536, 1024};
  const int64_t t2s[] = {inf, 4096, 3072, 2048};
  const int64_t smalls[] = {0, 4, 16};
  const int64_t t_aps[] = {3072, 2048, 1536, 1024};
  const int64_t t_owns[] = {0, 512, 1024, 2048};
  Rule best = p->rule;
  float best_ms = std::numeric_limits<float>::max();
  int rc = 0;
  auto try_rule = [&](const Rule& r) {
    if (e != hipSuccess || rc != 0) return;
    for (int i = 0; i < sp.count; ++i)
      apply_rule(r, sp.m[i], sp.n[i], sp.k[i], &sp.level[i], &sp.cfg[i], true, true);
    // one warm call, then the median of three timed calls
    float ts[3];
    rc = run_plan(&sp, A.data(), lda.data(), B.data(), ldb.data(), C.data(), ldc.data(), 1.0, 0.0,
                  s);
    for (int rep = 0; rep < 3 && rc == 0 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, s);
      if (e == hipSuccess) rc = launch_work(sp, s);
      if (e == hipSuccess && rc == 0) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ts[rep], e0, e1);
    }
    if (rc != 0 || e != hipSuccess) return;
    std::sort(ts, ts + 3);
    if (ts[1] < best_ms) {
      best_ms = ts[1];
      best = r;
    }
  };
  // the persistent kernel alone: level thresholds and tile shapes
  for (int64_t t1 : t1s)
    for (int64_t t2 : t2s) {
      if (t2 != inf && t2 <= t1 && t1 != inf) continue;
      if (t1 == inf && t2 != inf) continue;
      for (int64_t sm : smalls) {
        Rule r;
        r.t1 = t1;
        r.t2 = t2;
        r.small = sm;
        try_rule(r);
      }
    }
  // then one-level problems from t_ap up as their own all-products launches, with the best
  // two-level threshold and tile rule kept
  const Rule base = best;
  for (int64_t t1 : t1s)
    for (int64_t ta : t_aps) {
      if (t1 == inf || ta < t1) continue;
      if (base.t2 != inf && base.t2 <= t1) continue;
      Rule r = base;
      r.t1 = t1;
      r.t_ap = ta;
      try_rule(r);
    }
  // then problems from t_own up on the side streams (levels 0 / 1 by t1), the rest as before
  const Rule base2 = best;
  for (int64_t t1 : t1s)
    for (int64_t to : t_owns) {
      Rule r = base2;
      r.t1 = t1;
      r.t_own = to;
      try_rule(r);
    }
  free_device(&sp);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  hipError_t ef = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (rc != 0) return rc;
  if (e != hipSuccess) return hip_fail(e, "batched autotune");
  if (ef != hipSuccess) return hip_fail(ef, "batched autotune");
  p->rule = best;
  for (int i = 0; i < p->count; ++i)
    apply_rule(best, p->m[i], p->n[i], p->k[i], &p->level[i], &p->cfg[i], p->auto_level[i],
               p->auto_cfg[i]);
  return 0;
}

// ---------------------------------------------------------------------------------------------
// Graph capture: the two launches as explicit kernel nodes (no stream capture needed).
// ---------------------------------------------------------------------------------------------
static int capture(BatchedPlan* p, const double* const* A, const int64_t* lda,
                   const double* const* B, const int64_t* ldb, double* const* C,
                   const int64_t* ldc, double alpha, double beta, hipStream_t s) {
  if (int rc = validate_operands(*p, A, lda, B, ldb, C, ldc)) return rc;
  int dev = 0;
  if (int rc = device_ready(&dev)) return rc;
  for (int i = 0; i < p->count; ++i)
    if ((alpha == 0.0 || p->k[i] == 0) && p->m[i] > 0 && p->n[i] > 0 && beta != 1.0)
      return fail(STRASSEN_ERR_UNSUPPORTED,
                  "batched capture: alpha == 0 or k == 0 (problem %d) is only run eagerly", i);
  std::vector<BatchProblem> probs;
  std::vector<BatchItem> items;
  std::vector<ApLaunch> ap;
  std::vector<OwnLaunch> own;
  bool vec = true;
  if (int rc = build_work(*p, A, lda, B, ldb, C, ldc, alpha, beta, &probs, &items, &ap, &own, &vec))
    return rc;
  drop_graph(p);
  if (int rc = upload(p, probs, items, s)) return rc;
  p->vec = vec;
  p->ap = std::move(ap);
  p->own = std::move(own);
  p->alpha = alpha;
  p->beta = beta;
  if (!p->own.empty()) {
    // side streams: the launches are recorded by stream capture on the plan's own stream (the
    // fork and join events make the side streams branches of the graph); the library's kernel
    // timing is suspended meanwhile
    SMX_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    suspend_timing(true);
    const int rc = launch_work(*p, p->cap);
    suspend_timing(false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (rc != 0) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "batched capture");
    p->graph = g;
    SMX_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return 0;
  }
  SMX_HIP(hipGraphCreate(&p->graph, 0));
  hipGraphNode_t clear_node = nullptr, run_node = nullptr;
  void* clear_args[] = {&p->d_counter};
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof kp);
  kp.func = const_cast<void*>(clear_counter_fn());
  kp.gridDim = dim3(1);
  kp.blockDim = dim3(64);
  kp.kernelParams = clear_args;
  SMX_HIP(hipGraphAddKernelNode(&clear_node, p->graph, nullptr, 0, &kp));
  if (p->n_items > 0) {
    void* run_args[] = {&p->d_probs, &p->d_items, &p->n_items, &p->d_counter};
    hipKernelNodeParams rp;
    std::memset(&rp, 0, sizeof rp);
    rp.func = const_cast<void*>(batched_kernel_fn(vec));
    rp.gridDim = dim3(p->grid);
    rp.blockDim = dim3(256);
    rp.kernelParams = run_args;
    SMX_HIP(hipGraphAddKernelNode(&run_node, p->graph, &clear_node, 1, &rp));
  }
  // the all-products launches, chained after the persistent kernel (the eager order)
  hipGraphNode_t prev = p->n_items > 0 ? run_node : clear_node;
  for (ApLaunch& l : p->ap) {
    void* ap_args[] = {&l.f};
    hipKernelNodeParams ak;
    std::memset(&ak, 0, sizeof ak);
    ak.func = const_cast<void*>(all_products_fn(l.f, l.na, l.nb));
    if (!ak.func) return fail(STRASSEN_ERR_UNSUPPORTED, "batched capture: no all-products kernel");
    ak.gridDim = dim3((unsigned)((int64_t)l.f.tiles_m * l.f.tiles_n));
    ak.blockDim = dim3(512);
    ak.kernelParams = ap_args;
    hipGraphNode_t node;
    SMX_HIP(hipGraphAddKernelNode(&node, p->graph, &prev, 1, &ak));
    prev = node;
  }
  SMX_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  return 0;
}

}  // namespace smx

// ---------------------------------------------------------------------------------------------
// extern "C"
// ---------------------------------------------------------------------------------------------
extern "C" {

int strassen_batched_plan(int count, const int64_t* m, const int64_t* n, const int64_t* k,
                          int* levels, int* cfg, void** plan) {
  smx::clear_error();
  if (count < 0) return smx::fail(-1, "count < 0");
  if (count > 0 && (!m || !n || !k)) return smx::fail(-2, "NULL shape array");
  if (!plan) return smx::fail(-7, "plan is NULL");
  for (int i = 0; i < count; ++i)
    if (m[i] < 0 || n[i] < 0 || k[i] < 0) return smx::fail(-2, "problem %d: negative size", i);
  for (int i = 0; levels && i < count; ++i)
    if (levels[i] < -1 || levels[i] > smx::kMaxLevels)
      return smx::fail(-5, "problem %d: level %d not in -1..%d", i, levels[i], smx::kMaxLevels);
  for (int i = 0; cfg && i < count; ++i)
    if (cfg[i] < -1 || cfg[i] > smx::kBatchOwn)
      return smx::fail(-6, "problem %d: tile %d not in -1..%d", i, cfg[i], smx::kBatchOwn);
  auto* p = new smx::BatchedPlan;
  p->count = count;
  p->m.assign(m, m + count);
  p->n.assign(n, n + count);
  p->k.assign(k, k + count);
  p->level.resize(count);
  p->cfg.resize(count);
  p->auto_level.resize(count);
  p->auto_cfg.resize(count);
  for (int i = 0; i < count; ++i) {
    p->auto_level[i] = !levels || levels[i] < 0;
    p->auto_cfg[i] = !cfg || cfg[i] < 0;
    p->level[i] = p->auto_level[i] ? 0 : levels[i];
    p->cfg[i] = p->auto_cfg[i] ? 0 : cfg[i];
    smx::apply_rule(p->rule, m[i], n[i], k[i], &p->level[i], &p->cfg[i], p->auto_level[i],
                    p->auto_cfg[i]);
    if (levels) levels[i] = p->level[i];
    if (cfg) cfg[i] = p->cfg[i];
  }
  *plan = p;
  return 0;
}

int strassen_batched_autotune(void* plan, int sample, uint64_t seed, void* stream) {
  smx::clear_error();
  if (!plan) return smx::fail(-1, "plan is NULL");
  if (sample < 0) return smx::fail(-2, "sample < 0");
  return smx::autotune(static_cast<smx::BatchedPlan*>(plan), sample, seed,
                       static_cast<hipStream_t>(stream));
}

int strassen_batched_choice(void* plan, int i, int* level, int* cfg) {
  smx::clear_error();
  auto* p = static_cast<smx::BatchedPlan*>(plan);
  if (!p) return smx::fail(-1, "plan is NULL");
  if (i < 0 || i >= p->count) return smx::fail(-2, "problem %d out of range", i);
  if (level) *level = p->level[i];
  if (cfg) *cfg = p->cfg[i];
  return 0;
}

int strassen_batched_run(void* plan, const double* const* A, const int64_t* lda,
                         const double* const* B, const int64_t* ldb, double* const* C,
                         const int64_t* ldc, double alpha, double beta, void* stream) {
  smx::clear_error();
  if (!plan) return smx::fail(-1, "plan is NULL");
  return smx::run_plan(static_cast<smx::BatchedPlan*>(plan), A, lda, B, ldb, C, ldc, alpha, beta,
                       static_cast<hipStream_t>(stream));
}

int strassen_batched_capture(void* plan, const double* const* A, const int64_t* lda,
                             const double* const* B, const int64_t* ldb, double* const* C,
                             const int64_t* ldc, double alpha, double beta, void* stream) {
  smx::clear_error();
  if (!plan) return smx::fail(-1, "plan is NULL");
  return smx::capture(static_cast<smx::BatchedPlan*>(plan), A, lda, B, ldb, C, ldc, alpha, beta,
                      static_cast<hipStream_t>(stream));
}

int strassen_batched_replay(void* plan, void* stream) {
  smx::clear_error();
  auto* p = static_cast<smx::BatchedPlan*>(plan);
  if (!p) return smx::fail(-1, "plan is NULL");
  if (!p->exec) return smx::fail(-1, "plan has no captured graph");
  SMX_HIP(hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream)));
  return 0;
}

int strassen_batched_destroy(void* plan) {
  smx::clear_error();
  auto* p = static_cast<smx::BatchedPlan*>(plan);
  if (!p) return 0;
  if (p->dev >= 0) (void)hipDeviceSynchronize();
  smx::free_device(p);
  delete p;
  return 0;
}

}  // extern "C"
