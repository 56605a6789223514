"""Benchmark: Strassen DGEMM on one MI355X (gfx950), effective TFLOPS = 2mnk / time.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 16384] [--levels 2] [--variant abc]

One step is one call C := A*B + C of the library at m = n = k = n (default 16384, FP64, entries
uniform on [-1, 1], inputs resident in HBM) with `levels` levels of Strassen in the given variant
(default: two-level ABC, which runs as seven back-to-back launches of the all-products kernel,
one per outer product).  Printed as ONE JSON line:
the headline value plus, measured in the same run,
  * the library's own classical FP64 MFMA GEMM (levels = 0) and every (levels, variant) pair,
    timed with HIP events, with the speedup over classical; classical, the headline member
    and AB at n - 1 (`ragged`: sub-block extents odd, ABC and AB on block-padded copies);
  * the relative Frobenius error of the headline result against the CPU oracle on sampled
    columns (and of the classical result), checked against 1e-12 (one level) / 1e-11 (two);
  * roofline of the dominant kernel (the all-products kernel for ABC, the FP64 tile kernel
    otherwise): executed MFMA flops per launch over its average duration, against the 78.6
    TFLOP/s FP64 matrix peak; `traffic` comes from the committed rocprofv3 counter summary when
    it was taken on the current kernel source;
  * cpu_baseline: the oracle's plain triple-loop GEMM timed on the host cores over a bounded
    column sample of the same problem.
Diagnostics go to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective TFLOPS (2mnk/t), Strassen vs own classical GEMM, at stated rel error"
PEAK_F64_MFMA = 78.6   # TFLOP/s, MI355X datasheet, dense FP64 matrix
TOL = {0: None, 1: 1e-12, 2: 1e-11}
KERNEL_SOURCES = ["paper_1605_01078_amd/csrc/tile_fp64.h", "paper_1605_01078_amd/csrc/kernels_fp64.hip",
                  "paper_1605_01078_amd/csrc/fused_fp64.hip", "paper_1605_01078_amd/csrc/classical_fp64.hip"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=16384)
    p.add_argument("--levels", type=int, default=2)
    p.add_argument("--variant", default="abc")
    p.add_argument("--no-compare", action="store_true", help="skip the per-variant table")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    p.add_argument("--no-parity", action="store_true", help="skip the sampled oracle check")
    p.add_argument("--cpu-seconds", type=float, default=20.0)
    p.add_argument("--reps", type=int, default=5,
                   help="rounds of the round-robin member timing (median per member)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a plain copy kernel of known size first (for HBM counter scaling)")
    p.add_argument("--factor-runs", default=None,
                   help="lu / cholesky suites: comma-separated runs to time (e.g. nb2048_L1) "
                        "instead of all of them; the LU suite then skips its separate timing "
                        "of the rank-nb updates")
    p.add_argument("--suite", default="headline", choices=["headline", "precision", "batched", "selector", "sweep", "levels", "lu", "cholesky"],
                   help="headline: the FP64 step above; precision: the reduced-precision mode "
                        "table (m=n=k=--n, default 8192 for this suite); batched: 512 GEMMs in "
                        "one persistent graph launch; selector: the committed network's choice "
                        "against exhaustive timing on held-out shapes; sweep: every member on the "
                        "square sizes 2048..16384 and the rank-k shapes; levels: three levels "
                        "against two and classical at 32768; lu: LU without pivoting with "
                        "Strassen rank-k updates; each prints one JSON line")
    p.add_argument("--shapes", type=int, default=200,
                   help="selector suite: held-out shapes timed exhaustively")
    p.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                   help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this script "
                        "with --copy-calibration into the traffic summary under profiles/, then exit")
    return p.parse_args()


COPY_BYTES = 1 << 30   # the calibration copy reads and writes this many bytes


def copy_calibration():
    """Plain copy kernel of known size: y := -x over COPY_BYTES of doubles (reads COPY_BYTES,
    writes COPY_BYTES)."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y


def one_level_staged(m, n, k):
    """The library's rule for one-level ABC on the classical kernel (staged sums, one launch
    per product): exact quadrants, k/2 >= 2048, whole rounds of 256 x 128 tiles (95% of the
    last one) and k/2 >= 4096 or at least 1024 tiles."""
    if m % 4 or k % 4 or n % 2:
        return False
    tiles = -(-(m // 2) // 256) * -(-(n // 2) // 128)
    rounds = -(-tiles // 256)
    return tiles >= 256 and k // 2 >= 2048 and 20 * tiles >= 19 * 256 * rounds and \
        (k // 2 >= 4096 or tiles >= 1024)


def dominant_kernel(L, variant, n=None):
    if L == 0:
        return "classical_kernel"
    if L == 1 and variant == "abc" and n is not None and one_level_staged(n, n, n):
        return "classical_kernel"
    return "all_products_kernel" if variant in ("abc", "ab") else "fp64_tile_kernel"


def kernel_kind(L, variant, n=None):
    return {"classical_kernel": "classical", "all_products_kernel": "all_products"}.get(
        dominant_kernel(L, variant, n), "tile")


def headline_key(L, variant, staged):
    """Member name of the headline call in the per-member table: two-level ABC with its outer
    operand sums staged in workspace is `L2_abc_staged`; `L2_abc` is the workspace-free form."""
    if L == 2 and variant == "abc" and staged:
        return "L2_abc_staged"
    return f"L{L}_{variant}"


def traffic_path(L, variant, n):
    return os.path.join(ROOT, "profiles", f"traffic_{dominant_kernel(L, variant, n)}_L{L}_{variant}_{n}.json")


def traffic_summary(args):
    """Per-launch HBM bytes of the dominant kernel from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch, averaged over its dispatches), each scaled by known/measured bytes of the
    calibration copy in the same run."""
    import csv
    import glob
    kname = dominant_kernel(args.levels, args.variant, args.n)

    def read(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        tile, copy = [], []
        for row in csv.DictReader(open(f)):
            if row["Counter_Name"] != counter:
                continue
            v = float(row["Counter_Value"])
            name = row["Kernel_Name"]
            if kname in name:
                tile.append(v)
            elif "neg" in name:
                copy.append(v)
        return tile, copy
    ft, fc = read(args.traffic_from[0], "FETCH_SIZE")
    wt, wc = read(args.traffic_from[1], "WRITE_SIZE")
    f_fetch = COPY_BYTES / (fc[-1] * 1024.0)
    f_write = COPY_BYTES / (wc[-1] * 1024.0)
    fetch = float(np.mean(ft)) * 1024.0 * f_fetch
    write = float(np.mean(wt)) * 1024.0 * f_write
    L, variant, n = args.levels, args.variant, args.n
    out = {"kernel": kname, "workload": f"L={L} {variant} m=n=k={n}",
           "kernel_source_hash": kernel_source_hash(),
           "fetch_kib_per_launch": float(np.mean(ft)), "write_kib_per_launch": float(np.mean(wt)),
           "copy_fetch_kib": fc[-1], "copy_write_kib": wc[-1], "copy_bytes": COPY_BYTES,
           "fetch_scale": f_fetch, "write_scale": f_write,
           "hbm_bytes_per_launch": fetch + write, "fetch_bytes": fetch, "write_bytes": write}
    path = traffic_path(L, variant, n)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log(json.dumps(out, indent=1))


def cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo) and its logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical CPUs, {len(os.sched_getaffinity(0))} available)"


def timed(fn, reps, stream):
    """Median milliseconds of `reps` calls, each bracketed by events on `stream`."""
    import torch
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), ts


def precision_suite(args):
    """Reduced-precision mode at m=n=k (default 8192): for each level, product type, sum and
    update precision and input class, the time of one call and the relative Frobenius error
    against the FP64 oracle on sampled columns; beside them the FP64 classical GEMM and the
    same-mode classical (levels 0) product, and the roofline of the BF16 product kernel."""
    import torch
    import paper_1605_01078_amd as sx
    import workloads as W
    from oracle import oracle_dgemm, rel_fro

    n = args.n if args.n != 16384 else 8192
    stream = torch.cuda.current_stream()
    flops = 2.0 * n ** 3
    g = np.random.default_rng(0)
    cols = np.sort(g.choice(n, size=16, replace=False))
    tcols = torch.as_tensor(cols, device="cuda")
    kinds = ["uniform", "wide_a", "wide_b", "wide_both"]
    modes = [(c, s_, u) for c in ("bf16", "bf16x3") for s_ in ("f32", "f64") for u in ("f32", "f64")]
    rows, kernel_ms = [], {}
    for kind in kinds:
        A_h, B_h, C_h = W.problem(7, n, n, n, kind)
        ref = oracle_dgemm(A_h, np.asfortranarray(B_h[:, cols]), np.asfortranarray(C_h[:, cols]),
                           1.0, 1.0)
        A, B, C0 = sx.to_device(A_h), sx.to_device(B_h), sx.to_device(C_h)
        del A_h, B_h, C_h
        sel = modes if kind == "uniform" else [("bf16", "f32", "f32"), ("bf16x3", "f64", "f64")]
        if kind == "uniform":
            C = C0.clone()
            f = lambda: sx.dgemm(A, B, C, 1.0, 1.0, 0, "abc", stream)
            f()
            ms64, _ = timed(f, 3, stream)
            rows.append({"input": kind, "levels": 0, "mode": "f64", "ms": round(ms64, 3),
                         "tflops": round(flops / (ms64 * 1e-3) * 1e-12, 2)})
        for L in (0, 1, 2):
            for mode in sel:
                C = C0.clone()
                f = lambda: sx.gemm_ex(A, B, C, 1.0, 1.0, L, *mode, stream=stream)
                f()
                torch.cuda.synchronize()
                err = float(rel_fro(C[:, tcols].cpu().numpy(), ref))
                for k_ in sx.KERNEL_KINDS:
                    sx.timing_collect(k_)
                sx.timing_enable(True)
                ms, _ = timed(f, 3, stream)
                sx.timing_enable(False)
                kms, kcnt = sx.timing_collect("bf16")
                cms, ccnt = sx.timing_collect("cast")
                rows.append({"input": kind, "levels": L, "mode": "/".join(mode), "ms": round(ms, 3),
                             "tflops": round(flops / (ms * 1e-3) * 1e-12, 2),
                             "rel_err_vs_fp64": float(f"{err:.3e}"),
                             "product_kernel_ms": round(kms / max(kcnt, 1), 3),
                             "operand_pass_ms": round(cms / 3, 3)})
                log(f"  {kind:9s} L={L} {'/'.join(mode):18s} {ms:8.3f} ms  err {err:.3e}")
        del A, B, C0, C
        sx.release_workspace()
        torch.cuda.empty_cache()
    # headline of the suite: two-level bf16x3 (FP64 sums and update) on uniform inputs
    base = {(r["mode"], r["levels"]): r for r in rows if r["input"] == "uniform"}
    head = base[("bf16x3/f64/f64", 2)]
    for r in rows:
        if r["input"] == "uniform" and r["levels"] > 0:
            r["speedup_vs_same_mode_classical"] = round(base[(r["mode"], 0)]["ms"] / r["ms"], 4)
    q = 4
    exec_flops = 49 * 2.0 * (n // q) ** 3 * 3
    _, bf16_rate = sx.probe_rates(stream)   # measured BF16 matrix-core issue rate
    out = {"metric": "effective TFLOPS (2mnk/t) of the reduced-precision mode, with rel error vs FP64",
           "value": head["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": 3, "warmup": 1,
           "ms_per_step": head["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16x3 products, FP32 accumulation, FP64 sums/update",
           "data": "synthetic",
           "config": {"workload": f"strassen_gemm_ex L=2 bf16x3 m=n=k={n}, inputs uniform[-1,1] "
                                  "and wide-range rows 2^U[-8,8]", "m": n, "n": n, "k": n},
           "roofline": {"bound": "mfma", "peak": 2500.0, "unit": "TFLOP/s",
                        "peak_measured": round(bf16_rate, 1),
                        "kernel": "bf16_gemm_kernel (bf16x3)",
                        "achieved_note": "executed bf16 MFMA flops of the two-level bf16x3 call "
                                         "(49 products x 3 MFMA passes) over the product kernel's "
                                         "time (library event pair around its launch)",
                        "achieved": round(exec_flops / (head["product_kernel_ms"] * 1e-3) * 1e-12, 2),
                        "frac": round(exec_flops / (head["product_kernel_ms"] * 1e-3) * 1e-12 / 2500.0, 4),
                        "avg_launch_ms": head["product_kernel_ms"],
                        "operand_pass_ms": head["operand_pass_ms"],
                        "classical_bf16_kernel": {
                            "achieved": round(flops / (base[("bf16/f64/f64", 0)]["product_kernel_ms"] * 1e-3) * 1e-12, 2),
                            "frac": round(flops / (base[("bf16/f64/f64", 0)]["product_kernel_ms"] * 1e-3) * 1e-12 / 2500.0, 4)}},
           "table": rows}
    print(json.dumps(out), flush=True)


def batched_suite(args):
    """512 independent FP64 GEMMs, m, n, k uniform over the multiples of 64 in [256, 4096],
    entries uniform[-1, 1]: the autotuned batch as one graph replay (the timed step), beside the
    same batch run eagerly, the all-classical batch and the problems one call at a time."""
    import torch
    import paper_1605_01078_amd as sx
    import workloads as W
    from oracle import oracle_dgemm, rel_fro

    shapes = W.batched_shapes(0)
    stream = torch.cuda.current_stream()
    flops = sum(2.0 * m * n * k for m, n, k in shapes)
    As = [W.device_uniform(10_000 + 3 * i, m, k) for i, (m, n, k) in enumerate(shapes)]
    Bs = [W.device_uniform(10_001 + 3 * i, k, n) for i, (m, n, k) in enumerate(shapes)]
    C0 = [W.device_uniform(10_002 + 3 * i, m, n) for i, (m, n, k) in enumerate(shapes)]
    Cs = [c.clone() for c in C0]
    torch.cuda.synchronize()

    def reset():
        for c, c0 in zip(Cs, C0):
            c.copy_(c0)

    def ev_time(fn, reps):
        ts = []
        for _ in range(reps):
            reset()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), ts

    t0 = time.perf_counter()
    tuned = sx.Batched(shapes)
    tuned.autotune(sample=0, seed=0, stream=stream)   # the whole batch: a sample packs differently
    tune_s = time.perf_counter() - t0
    choices = tuned.choices()
    hist = {}
    for lv, cf in choices:
        key = f"L{lv}_{['tile128', 'tile64', 'all_products', 'side_stream'][cf]}"
        hist[key] = hist.get(key, 0) + 1
    log(f"autotune: {tune_s:.1f} s, choices {hist}")
    # timed step: the captured graph
    tuned.capture(As, Bs, Cs, 1.0, 1.0, stream)
    for _ in range(args.warmup):
        reset()
        tuned.replay(stream)
    torch.cuda.synchronize()
    ms_graph, ts_graph = ev_time(lambda: tuned.replay(stream), max(3, args.steps))
    # parity: four problems, eight sampled columns each, against the oracle
    reset()
    tuned.replay(stream)
    torch.cuda.synchronize()
    g = np.random.default_rng(0)
    errs = []
    for i in g.choice(len(shapes), size=4, replace=False):
        m, n, k = shapes[i]
        cols = np.sort(g.choice(n, size=8, replace=False))
        A_h = sx.to_host(As[i])
        Bc = np.asfortranarray(sx.to_host(Bs[i])[:, cols])
        Cc = np.asfortranarray(sx.to_host(C0[i])[:, cols])
        ref = oracle_dgemm(A_h, Bc, Cc, 1.0, 1.0)
        got = Cs[i][:, torch.as_tensor(cols, device="cuda")].cpu().numpy()
        errs.append({"problem": int(i), "level": choices[i][0], "rel_err": float(rel_fro(got, ref))})
    tol = {0: 1e-13, 1: 1e-12, 2: 1e-11}
    parity_pass = all(e["rel_err"] <= tol[e["level"]] for e in errs)
    # the same batch run eagerly (work list upload included)
    ms_eager, _ = ev_time(lambda: tuned.run(As, Bs, Cs, 1.0, 1.0, stream), 3)
    # all-classical batch
    classical = sx.Batched(shapes, levels=[0] * len(shapes))
    classical.capture(As, Bs, Cs, 1.0, 1.0, stream)
    ms_classical, _ = ev_time(lambda: classical.replay(stream), 3)
    # one call per problem (the library's default single-call path, classical and autotuned level)
    def one_by_one(levels):
        for (A, B, C), lv in zip(zip(As, Bs, Cs), levels):
            sx.dgemm(A, B, C, 1.0, 1.0, lv, "abc", stream)
    ms_single0, _ = ev_time(lambda: one_by_one([0] * len(shapes)), 3)
    ms_single_t, _ = ev_time(lambda: one_by_one([lv for lv, _ in choices]), 3)
    tuned.close()
    classical.close()
    tf = lambda ms: round(flops / (ms * 1e-3) * 1e-12, 2)
    out = {"metric": "effective TFLOPS (sum of 2mnk / t) of 512 FP64 GEMMs in one persistent graph launch",
           "value": tf(ms_graph), "unit": "TFLOP/s", "n_gpus": 1, "steps": len(ts_graph),
           "warmup": args.warmup, "ms_per_step": round(ms_graph, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batched: 512 GEMMs, m, n, k uniform over multiples of 64 in "
                                  "[256, 4096], entries uniform[-1,1], autotuned level and tile "
                                  "per problem, one hipGraph replay", "problems": len(shapes),
                      "total_flops": flops},
           "roofline": {"bound": "mfma", "achieved": tf(ms_graph), "peak": PEAK_F64_MFMA,
                        "unit": "TFLOP/s", "frac": round(tf(ms_graph) / PEAK_F64_MFMA, 4),
                        "traffic": None, "kernel": "batched_kernel (persistent) + all_products_kernel",
                        "achieved_note": "all 512 problems' effective 2mnk flops over the graph "
                                         "replay (Strassen choices execute 7/8 of them per level)"},
           "choices": hist, "autotune_seconds": round(tune_s, 2),
           "compare": {"graph_replay_ms": round(ms_graph, 3), "eager_run_ms": round(ms_eager, 3),
                       "batched_all_classical_ms": round(ms_classical, 3),
                       "one_call_per_problem_classical_ms": round(ms_single0, 3),
                       "one_call_per_problem_tuned_levels_ms": round(ms_single_t, 3),
                       "tflops": {"graph": tf(ms_graph), "eager": tf(ms_eager),
                                  "batched_classical": tf(ms_classical),
                                  "single_classical": tf(ms_single0),
                                  "single_tuned": tf(ms_single_t)}},
           "parity": {"sampled": errs, "pass": parity_pass}}
    print(json.dumps(out), flush=True)


def selector_suite(args):
    """The learned selector against exhaustive timing, measured live: a seeded sample of the
    held-out shapes (m, n, k log-uniform in [256, 20000], FP64 or BF16), every member timed
    (best of two calls), the choice of the committed network (through the library's selection
    call and its inference kernel), of the analytical cost model and of each fixed member;
    regret = total time of the chosen members / total time of the best ones - 1."""
    import torch
    import paper_1605_01078_amd as sx
    from paper_1605_01078_amd import selector as S

    shapes, dtypes = S.dataset()
    g = np.random.default_rng(7)
    idx = np.sort(g.choice(np.arange(20000, len(shapes)), size=min(args.shapes, 2000), replace=False))
    sh = [shapes[i] for i in idx]
    dt = [dtypes[i] for i in idx]
    log(f"selector: {len(sh)} held-out shapes, every member timed twice")
    t0 = time.perf_counter()
    times = np.minimum(S.collect(sh, dt), S.collect(sh, dt))
    log(f"  timed in {time.perf_counter() - t0:.0f} s")
    if not S.install_committed():
        raise SystemExit("no committed selector network (selector_data/weights.json)")
    member = {mv: c for c, mv in enumerate(S.MEMBERS)}
    t1 = time.perf_counter()
    net = np.array([member[S.select(m, n, k, d)] for (m, n, k), d in zip(sh, dt)])
    sel_us = (time.perf_counter() - t1) / len(sh) * 1e6
    model = S.model_choice(sh, dt)
    reg = {"network": S.regret(times, net), "cost_model": S.regret(times, model)}
    for c, (lv, v) in enumerate(S.MEMBERS):
        ch = np.array([c if S.available(int(d))[c] else 0 for d in dt])
        reg[f"always_L{lv}_{v}"] = S.regret(times, ch)
    reg["best_fixed"] = min(v for k_, v in reg.items() if k_.startswith("always_"))
    hits = float(np.mean(net == times.argmin(axis=1)))
    out = {"metric": "regret of the learned selector against exhaustive timing (held-out shapes)",
           "value": round(100.0 * reg["network"], 3), "unit": "%", "n_gpus": 1,
           "steps": len(sh), "warmup": 0, "ms_per_step": round(float(times.min(axis=1).mean()), 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "selector: held-out GEMM shapes, m, n, k log-uniform in "
                                  "[256, 20000], FP64 or BF16, every member timed", "shapes": len(sh),
                      "members": [f"L{lv}_{v}" for lv, v in S.MEMBERS]},
           "regret": {k_: round(v, 5) for k_, v in reg.items()},
           "network_picks_best": round(hits, 4), "select_call_us": round(sel_us, 1),
           "total_best_ms": round(float(times.min(axis=1).sum()), 2),
           "total_network_ms": round(float(times[np.arange(len(sh)), net].sum()), 2)}
    print(json.dumps(out), flush=True)


def sweep_suite(args):
    """Every member (classical; one- and two-level ABC, AB, Naive) on the square sizes
    m = n = k = 2048, 4096, ..., 16384 and the rank-k shapes m = n = 16384, k = 256 ... 8192,
    entries uniform[-1, 1]: median of three event-timed calls each, effective TFLOPS and the
    ratio to classical at the same shape; the fastest member's result on four sampled columns
    against the oracle (relative Frobenius error within 1e-13 / 1e-12 / 1e-11 by level)."""
    import torch
    import paper_1605_01078_amd as sx
    import workloads as W
    from oracle import oracle_dgemm, rel_fro

    stream = torch.cuda.current_stream()
    shapes = [(s_, s_, s_) for s_ in range(2048, 16384 + 1, 2048)]
    shapes += [(16384, 16384, k) for k in (256, 512, 1024, 2048, 4096, 8192)]
    members = [(0, "abc")] + [(lv, v) for lv in (1, 2) for v in ("abc", "ab", "naive")]
    rows = []
    for m, n, k in shapes:
        A = W.device_uniform(1, m, k)
        B = W.device_uniform(2, k, n)
        C = W.device_uniform(3, m, n)
        row = {"m": m, "n": n, "k": k}
        for lv, v in members:
            f = lambda: sx.dgemm(A, B, C, 1.0, 1.0, lv, v, stream)
            f()
            ms, _ = timed(f, 3, stream)
            row[f"L{lv}_{v}"] = round(ms, 3)
        base = row["L0_abc"]
        row["speedup"] = {key: round(base / t, 4) for key, t in row.items()
                          if key.startswith("L") and key != "L0_abc"}
        best = min((key for key in row if key.startswith("L")), key=lambda key: row[key])
        row["best"] = best
        # sampled parity of the fastest member: four columns of C against the oracle
        lv, v = int(best[1]), best.split("_", 1)[1]
        cols = np.sort(np.random.default_rng(m + 3 * k).choice(n, size=4, replace=False))
        idx = torch.as_tensor(cols, device="cuda")
        C0 = W.device_uniform(3, m, n)
        Cc = C0[:, idx].cpu().numpy()
        sx.dgemm(A, B, C0, 1.0, 1.0, lv, v, stream)
        torch.cuda.synchronize()
        ref = oracle_dgemm(sx.to_host(A), np.asfortranarray(B[:, idx].cpu().numpy()),
                           np.asfortranarray(Cc), 1.0, 1.0)
        err = float(rel_fro(C0[:, idx].cpu().numpy(), ref))
        tol = {0: 1e-13, 1: 1e-12, 2: 1e-11}[lv]
        row["parity"] = {"member": best, "rel_err": err, "tolerance": tol, "pass": err <= tol}
        if err > tol:
            raise SystemExit(f"sweep parity failed at {m}x{n}x{k} ({best}): {err:.3e} > {tol:.0e}")
        log(f"  {m}x{n}x{k}: classical {base:.3f} ms, best {best} {row[best]:.3f} ms, "
            f"sampled rel err {err:.2e}")
        rows.append(row)
        del A, B, C, C0
        sx.release_workspace()
        torch.cuda.empty_cache()
    sq = [r for r in rows if r["m"] == r["k"]]
    top = max(sq, key=lambda r: r["m"])
    out = {"metric": "effective TFLOPS (2mnk/t) of the fastest member at m=n=k=16384 over the sweep",
           "value": round(2.0 * top["m"] ** 3 / (top[top["best"]] * 1e-3) * 1e-12, 3),
           "unit": "TFLOP/s", "n_gpus": 1, "steps": 3, "warmup": 1,
           "ms_per_step": top[top["best"]], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "FP64 Strassen sweep: square 2048..16384 step 2048 and rank-k "
                                  "m=n=16384, k=256..8192; all members; entries uniform[-1,1]"},
           "table_ms": rows}
    print(json.dumps(out), flush=True)


def levels_suite(args):
    """Three levels of Strassen (343 products) against two levels and classical at m = n = k =
    --n (default 32768, where three levels are meant to pay; FP64, uniform[-1, 1] entries):
    round-robin event timing, median of --reps rounds each, relative error of three levels on
    sampled columns against the oracle, and the roofline of its all-products launches."""
    import torch
    import paper_1605_01078_amd as sx
    import workloads as W
    from oracle import oracle_dgemm, rel_fro
    n = args.n if args.n != 16384 else 32768
    stream = torch.cuda.current_stream()
    A = W.device_uniform(1, n, n)
    B = W.device_uniform(2, n, n)
    C0 = W.device_uniform(3, n, n)
    C = C0.clone()
    flops = 2.0 * n * n * n
    members = {"L0_abc": 0, "L2_abc_staged": 2, "L3_abc": 3}
    times = {key: [] for key in members}

    def one(lev):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sx.dgemm(A, B, C, 1.0, 1.0, lev, "abc", stream)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1)
    for lev in members.values():
        one(lev)
    reps = max(3, args.reps)
    for k_ in sx.KERNEL_KINDS:
        sx.timing_collect(k_)
    for _ in range(reps):
        for key, lev in members.items():
            if lev == 3:
                sx.timing_enable(True)
            times[key].append(one(lev))
            sx.timing_enable(False)
    ap_ms, ap_n = sx.timing_collect("all_products")
    os_ms, os_n = sx.timing_collect("outer_sums")
    for k_ in sx.KERNEL_KINDS:
        sx.timing_collect(k_)
    base = float(np.median(times["L0_abc"]))
    variants = {}
    for key in members:
        ms = float(np.median(times[key]))
        variants[key] = {"ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) * 1e-12, 2),
                         "speedup_vs_classical": round(base / ms, 4),
                         "spread_ms": [round(min(times[key]), 3), round(max(times[key]), 3)]}
        log(f"  {n}^3 {key}: {ms:9.3f} ms  {variants[key]['tflops']:6.2f} TF")
    # parity of three levels on sampled columns
    C = C0.clone()
    sx.dgemm(A, B, C, 1.0, 1.0, 3, "abc", stream)
    torch.cuda.synchronize()
    cols = np.sort(np.random.default_rng(0).choice(n, size=4, replace=False))
    idx = torch.as_tensor(cols, device=C.device)
    got = C[:, idx].cpu().numpy()
    del C
    ref = oracle_dgemm(sx.to_host(A), np.asfortranarray(B[:, idx].cpu().numpy()),
                       np.asfortranarray(C0[:, idx].cpu().numpy()), 1.0, 1.0)
    err = float(rel_fro(got, ref))
    nq = n // 8
    exec_launch = 7 * 2.0 * nq ** 3
    avg = ap_ms / ap_n
    achieved = exec_launch / (avg * 1e-3) * 1e-12
    out = {"metric": METRIC, "value": variants["L3_abc"]["tflops"], "unit": "TFLOP/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"strassen_dgemm L=3 ABC m=n=k={n} FP64 C:=A*B+C, entries "
                                  f"uniform[-1,1] (343 products; upper two levels staged)",
                      "m": n, "n": n, "k": n, "levels": 3, "reps": reps},
           "variants": variants,
           "speedup_vs_classical": variants["L3_abc"]["speedup_vs_classical"],
           "parity": {"L3_abc": err, "tolerance": 1e-10, "columns": [int(c) for c in cols],
                      "pass": err <= 1e-10},
           "roofline": {"bound": "mfma", "kernel": "all_products_kernel",
                        "launches_per_step": ap_n // reps, "avg_launch_ms": round(avg, 4),
                        "exec_flops_per_launch": exec_launch, "achieved": round(achieved, 3),
                        "peak": PEAK_F64_MFMA, "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_F64_MFMA, 4),
                        "staged_sum_passes": {"launches_per_step": os_n // reps,
                                              "ms_per_step": round(os_ms / reps, 3)}}}
    print(json.dumps(out), flush=True)


def pick_runs(args, runs):
    """The factorization runs --factor-runs names (all of them without the option)."""
    if not args.factor_runs:
        return runs
    want = [key.strip() for key in args.factor_runs.split(",") if key.strip()]
    bad = [key for key in want if key not in runs]
    if bad or not want:
        raise SystemExit(f"--factor-runs: unknown run(s) {bad}; known: {sorted(runs)}")
    return {key: runs[key] for key in want}


def cholesky_suite(args):
    """Cholesky factorization (strassen_dpotrf_lower) of a symmetric positive definite n x n
    matrix (default 16384; X X^T / n + I with X uniform[-1, 1]), block columns of 2048, trailing
    updates with 0 (classical), 1, 2 and 3 levels of Strassen: round-robin event timing (median
    of --reps), rate = n^3 / 3 / t, and the backward error ||A - L L^T|| / ||A|| on sampled
    columns."""
    import torch
    import paper_1605_01078_amd as sx
    from oracle import rel_fro
    n, nb = args.n, 2048
    stream = torch.cuda.current_stream()
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    X = torch.empty((n, n), dtype=torch.float64, device="cuda").uniform_(-1, 1, generator=g)
    A0 = torch.matmul(X, X.t()).div_(float(n))
    A0.diagonal().add_(1.0)
    del X
    A = torch.empty_like(A0).t()   # column-major work matrix (A0 is symmetric: same values)
    flops = n ** 3 / 3.0
    runs = pick_runs(args, {f"nb{nb}_L{lev}": lev for lev in (0, 1, 2, 3)})
    times = {key: [] for key in runs}

    def one(lev):
        A.t().copy_(A0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info = sx.potrf_lower(A, nb, lev, stream)
        e1.record(stream)
        e1.synchronize()
        if info != 0:
            raise SystemExit(f"Cholesky reported info {info}")
        return e0.elapsed_time(e1)
    for lev in runs.values():
        one(lev)
    for _ in range(args.reps):
        for key, lev in runs.items():
            times[key].append(one(lev))
    out_runs = {}
    for key in runs:
        ms = float(np.median(times[key]))
        out_runs[key] = {"ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) * 1e-12, 2)}
        log(f"  Cholesky n={n} {key}: {ms:8.3f} ms  {out_runs[key]['tflops']:6.2f} TF")
    if f"nb{nb}_L0" in out_runs:
        base = out_runs[f"nb{nb}_L0"]["ms"]
        for lev in (1, 2, 3):
            if f"nb{nb}_L{lev}" in out_runs:
                out_runs[f"nb{nb}_L{lev}"]["speedup_vs_classical_updates"] = round(base / out_runs[f"nb{nb}_L{lev}"]["ms"], 4)
    best = min(out_runs, key=lambda key: out_runs[key]["ms"])
    one(runs[best])
    torch.cuda.synchronize()
    cols = np.sort(np.random.default_rng(0).choice(n, size=4, replace=False))
    L = np.tril(sx.to_host(A))
    err = float(rel_fro(L @ L[cols, :].T, A0[:, torch.as_tensor(cols, device="cuda")].cpu().numpy()))
    del L
    out = {"metric": "Cholesky factorization rate (n^3 / 3 / t) with Strassen trailing updates",
           "value": out_runs[best]["tflops"], "unit": "TFLOP/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"strassen_dpotrf_lower n={n}, X X^T / n + I with X "
                                  f"uniform[-1,1], block columns {nb}, best {best}", "n": n},
           "runs": out_runs,
           "backward_error": {"value": err, "columns": cols.tolist(), "run": best}}
    print(json.dumps(out), flush=True)


def lu_suite(args):
    """LU factorization without pivoting (strassen_dgetrf_nopiv) of a diagonally dominant n x n
    matrix (default 16384; entries uniform[-1, 1] plus n on the diagonal), rank-nb updates with
    0 (classical), 1, 2 and 3 levels of Strassen, and two block widths: round-robin event timing
    (median of --reps), rate = (2/3) n^3 / t, the rank-nb update products of the blocked loop
    timed on their own, and the backward error ||A - L U|| / ||A|| on sampled columns."""
    import torch
    import paper_1605_01078_amd as sx
    from oracle import rel_fro
    n = args.n
    stream = torch.cuda.current_stream()
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").uniform_(-1, 1, generator=g)
    A0.diagonal().add_(float(n))
    A0 = A0.t()
    A = torch.empty_like(A0.t()).t()   # column-major work copy
    flops = 2.0 / 3.0 * n ** 3
    runs = pick_runs(args, {f"nb{nb}_L{lev}": (nb, lev) for nb in (2048, 4096) for lev in (0, 1, 2, 3)})
    times = {key: [] for key in runs}

    def one(nb, lev):
        A.copy_(A0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sx.getrf_nopiv(A, nb, lev, stream)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1)
    for nb, lev in runs.values():
        one(nb, lev)
    for _ in range(args.reps):
        for key, (nb, lev) in runs.items():
            times[key].append(one(nb, lev))
    out_runs = {}
    for key in runs:
        ms = float(np.median(times[key]))
        out_runs[key] = {"ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) * 1e-12, 2)}
        log(f"  LU n={n} {key}: {ms:8.3f} ms  {out_runs[key]['tflops']:6.2f} TF")
    for nb in (2048, 4096):
        if f"nb{nb}_L0" not in out_runs:
            continue
        base = out_runs[f"nb{nb}_L0"]["ms"]
        for lev in (1, 2, 3):
            if f"nb{nb}_L{lev}" in out_runs:
                out_runs[f"nb{nb}_L{lev}"]["speedup_vs_classical_updates"] = round(base / out_runs[f"nb{nb}_L{lev}"]["ms"], 4)
    # the rank-nb updates of the blocked loop on their own: C (r x r) -= A (r x nb) B (nb x r)
    # for r = n - nb, n - 2 nb, ..., timed one by one (event pairs) and summed
    updates = {}
    for nb in (() if args.factor_runs else (2048, 4096)):
        shapes = [n - j - nb for j in range(0, n - nb, nb)]
        for lev in (0, 1, 2, 3):
            tot = []
            for _ in range(args.reps):
                t = 0.0
                for r in shapes:
                    Au, Bu, Cu = A[:r, :nb], A0[:nb, :r], A[r - r:r, n - r:]
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    sx.dgemm(Au, Bu, Cu, -1.0, 1.0, lev, "abc", stream)
                    e1.record(stream)
                    e1.synchronize()
                    t += e0.elapsed_time(e1)
                tot.append(t)
            ms = float(np.median(tot))
            uflops = sum(2.0 * r * r * nb for r in shapes)
            updates[f"nb{nb}_L{lev}"] = {"ms": round(ms, 3),
                                         "tflops": round(uflops / (ms * 1e-3) * 1e-12, 2)}
            log(f"  rank-{nb} updates L={lev}: {ms:8.3f} ms")
        for lev in (1, 2, 3):
            updates[f"nb{nb}_L{lev}"]["speedup_vs_classical"] = round(
                updates[f"nb{nb}_L0"]["ms"] / updates[f"nb{nb}_L{lev}"]["ms"], 4)
    best = min(out_runs, key=lambda key: out_runs[key]["ms"])
    # backward error of the best run on sampled columns
    nb, lev = runs[best]
    cols = np.sort(np.random.default_rng(0).choice(n, size=4, replace=False))
    idx = torch.as_tensor(cols, device="cuda")
    A.copy_(A0)
    sx.getrf_nopiv(A, nb, lev, stream)
    torch.cuda.synchronize()
    F = sx.to_host(A)
    L = np.tril(F, -1) + np.eye(n)
    err = float(rel_fro(L @ np.triu(F)[:, cols], A0[:, idx].cpu().numpy()))
    del F, L
    out = {"metric": "LU factorization rate (2/3 n^3 / t) with Strassen rank-k updates",
           "value": out_runs[best]["tflops"], "unit": "TFLOP/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"strassen_dgetrf_nopiv n={n}, diagonally dominant "
                                  f"(uniform[-1,1] + n I), best {best}", "n": n},
           "runs": out_runs,
           "rank_nb_updates": updates,
           "parity": {"backward_error": err, "tolerance": n * 2.0 ** -53, "run": best,
                      "columns": [int(c) for c in cols], "pass": err <= n * 2.0 ** -53}}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.traffic_from:
        traffic_summary(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this library has no multi-GPU path); got --gpus "
              f"{args.gpus}", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1605_01078_amd as sx
    import workloads as W

    sx.lib()  # fails loudly if the HIP library is not built
    if args.suite == "precision":
        precision_suite(args)
        return
    if args.suite == "batched":
        batched_suite(args)
        return
    if args.suite == "cholesky":
        cholesky_suite(args)
        return
    if args.suite == "selector":
        selector_suite(args)
        return
    if args.suite == "sweep":
        sweep_suite(args)
        return
    if args.suite == "levels":
        levels_suite(args)
        return
    if args.suite == "lu":
        lu_suite(args)
        return
    if args.copy_calibration:
        copy_calibration()
    dev = torch.cuda.current_device()
    props = torch.cuda.get_device_properties(dev)
    log(f"device: {props.name} {getattr(props, 'gcnArchName', '')} CUs={props.multi_processor_count}")
    n, L, variant = args.n, args.levels, args.variant
    stream = torch.cuda.current_stream()
    A = W.device_uniform(1, n, n)
    B = W.device_uniform(2, n, n)
    C0 = W.device_uniform(3, n, n)
    C = C0.clone()
    flops = 2.0 * n * n * n
    q = 2 ** L
    nq = -(-n // q)
    exec_flops = (7 ** L) * 2.0 * nq * nq * nq

    def call(levels, var, Cm):
        return lambda: sx.dgemm(A, B, Cm, 1.0, 1.0, levels, var, stream)

    # ---- parity on sampled columns against the CPU oracle --------------------------------------
    parity = {}
    A_h = None
    if not args.no_parity:
        from oracle import oracle_dgemm, rel_fro
        g = np.random.default_rng(0)
        cols = np.sort(g.choice(n, size=4, replace=False))
        A_h = sx.to_host(A)
        Bc = np.asfortranarray(sx.to_host(B)[:, cols])
        Cc = np.asfortranarray(sx.to_host(C0)[:, cols])
        ref = oracle_dgemm(A_h, Bc, Cc.copy(order="F"), 1.0, 1.0)
        for lev, var in ((0, "abc"), (L, variant)):
            Ct = C0.clone()
            sx.dgemm(A, B, Ct, 1.0, 1.0, lev, var, stream)
            torch.cuda.synchronize()
            got = Ct[:, torch.as_tensor(cols, device=Ct.device)].cpu().numpy()
            err = float(rel_fro(got, ref))
            parity[f"L{lev}_{var}"] = err
            del Ct
        tol = TOL[L]
        parity["tolerance"] = tol
        parity["columns"] = [int(c) for c in cols]
        parity["pass"] = bool(tol is None or parity[f"L{L}_{variant}"] <= tol)
        log(f"parity (rel Frobenius on sampled columns vs oracle): {parity}")

    # ---- headline: warmup, then exactly K timed steps -------------------------------------------
    step = call(L, variant, C)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    start_all = torch.cuda.Event(enable_timing=True)
    end_all = torch.cuda.Event(enable_timing=True)
    kind = kernel_kind(L, variant, n)
    for k_ in sx.KERNEL_KINDS:   # drop what the warmup recorded
        sx.timing_collect(k_)
    sx.timing_enable(True)       # library-side event pairs around each kernel launch
    start_all.record(stream)
    for e0, e1 in ev:
        e0.record(stream)
        step()
        e1.record(stream)
    end_all.record(stream)
    torch.cuda.synchronize()
    sx.timing_enable(False)
    kern_ms, kern_launches = sx.timing_collect(kind)
    sums_ms, sums_launches = sx.timing_collect("outer_sums")
    for k_ in sx.KERNEL_KINDS:
        sx.timing_collect(k_)
    wall = time.perf_counter() - t0
    total_ms = start_all.elapsed_time(end_all)
    per_launch = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms_per_step = total_ms / args.steps
    value = flops / (ms_per_step * 1e-3) * 1e-12
    log(f"headline L={L} {variant}: {ms_per_step:.3f} ms/step, {value:.2f} effective TFLOP/s "
        f"(wall {wall:.2f} s)")

    # ---- classical and every member (same inputs, outside the timed steps) --------------------
    # Round-robin: every round times each member once (HIP events around one call), so clock and
    # thermal drift reach all members alike; each member's figure is the median of its rounds,
    # and every ratio below divides medians.
    variants, vendor, ragged = {}, None, None
    if not args.no_compare:
        Cw = C0.clone()
        Ac, Bc = A.contiguous(), B.contiguous()   # plain row-major operands (same values)
        Cv = torch.empty(n, n, dtype=torch.float64, device=A.device)
        # (levels, variant, tile configuration); two-level ABC as the paper defines it, without
        # workspace (outer sums formed in the load: configuration 4), beside the default form
        # that stages the outer operand sums in workspace
        # (the staged form once more under a workspace cap that holds one outer product's two
        # sum slots, m/2 x k/2 and k/2 x n/2 doubles, but not all ten: one product at a time)
        one_slots = 8 * 2 * (n // 2) * (n // 2)
        # one level: the default stages the five sums per side and runs the products on the
        # classical kernel; configuration 4 forces the workspace-free all-products form
        members = {"L0_abc": (0, "abc", -1), "L1_abc": (1, "abc", -1),
                   "L1_abc_all_products": (1, "abc", 4), "L1_ab": (1, "ab", -1),
                   "L1_naive": (1, "naive", -1), "L2_abc": (2, "abc", 4),
                   "L2_abc_staged": (2, "abc", -1),
                   "L2_abc_staged_one_at_a_time": (2, "abc", -1, one_slots + (1 << 20)),
                   "L2_ab": (2, "ab", -1), "L2_naive": (2, "naive", -1),
                   # Winograd's variant (ABC; two levels with staged outer chain sums)
                   "L1_winograd": (1, "winograd", -1), "L2_winograd": (2, "winograd", -1)}

        def one(key):
            if key == "vendor":
                f = lambda: torch.matmul(Ac, Bc, out=Cv)
                cfg = -1
            else:
                lev, var, cfg = members[key][:3]
                if len(members[key]) > 3:
                    sx.set_workspace_limit(members[key][3])
                if var == "winograd":
                    f = lambda: sx.dgemm_winograd(A, B, Cw, 1.0, 1.0, lev, stream)
                else:
                    f = lambda: sx.dgemm(A, B, Cw, 1.0, 1.0, lev, var, stream)
            if cfg >= 0:
                sx.set_tile_config(cfg)
            try:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                f()
                e1.record(stream)
                e1.synchronize()
            finally:
                if cfg >= 0:
                    sx.set_tile_config(-1)
                if key != "vendor" and len(members[key]) > 3:
                    sx.set_workspace_limit(0)
            return e0.elapsed_time(e1)

        keys = list(members) + ["vendor"]
        for key in keys:   # one untimed call each (workspace, code objects)
            one(key)
        times = {key: [] for key in keys}
        for _ in range(args.reps):
            for key in keys:
                times[key].append(one(key))
        base_ms = float(np.median(times["L0_abc"]))
        for key in keys:
            ms = float(np.median(times[key]))
            entry = {"ms": round(ms, 3), "tflops": round(flops / (ms * 1e-3) * 1e-12, 2),
                     "speedup_vs_classical": round(base_ms / ms, 4),
                     "spread_ms": [round(min(times[key]), 3), round(max(times[key]), 3)]}
            if key == "vendor":
                vendor = entry
            else:
                variants[key] = entry
                if key.startswith("L2_abc") or key.startswith("L1_abc"):   # workspace each ABC form used
                    entry["workspace_bytes"] = {"L1_abc": sx.workspace_size(n, n, n, 1, "abc"),
                                                "L1_abc_all_products": 0, "L2_abc": 0,
                                                "L2_abc_staged": sx.workspace_size(n, n, n, 2, "abc"),
                                                "L2_abc_staged_one_at_a_time": one_slots}[key]
            log(f"  {key:16s}: {ms:8.3f} ms  {entry['tflops']:6.2f} TF  x{entry['speedup_vs_classical']:.3f}")
        del Cv, Ac, Bc
        # a size that does not split evenly (n - 1: every sub-block extent odd), classical, the
        # headline member and AB at its level, round-robin as above; every member runs on
        # block-padded copies there (copy time included)
        r = n - 1
        rflops = 2.0 * r * r * r
        Ar, Br, Cr = A[:r, :r], B[:r, :r], Cw[:r, :r]
        ragged = {"m": r, "n": r, "k": r}
        ragged_runs = [(0, "abc"), (L, variant)] + ([(L, "ab")] if L and variant != "ab" else [])
        fr = {f"L{lev}_{var}": (lambda lev=lev, var=var: sx.dgemm(Ar, Br, Cr, 1.0, 1.0, lev, var, stream))
              for lev, var in ragged_runs}
        rt = {key: [] for key in fr}
        for key, f in fr.items():
            f()
        torch.cuda.synchronize()
        for _ in range(args.reps):
            for key, f in fr.items():
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                f()
                e1.record(stream)
                e1.synchronize()
                rt[key].append(e0.elapsed_time(e1))
        for key in fr:
            ms = float(np.median(rt[key]))
            ragged[key] = {"ms": round(ms, 3), "tflops": round(rflops / (ms * 1e-3) * 1e-12, 2)}
            log(f"  {r}^3 {key}: {ms:8.3f} ms")
        ragged["speedup_vs_classical"] = round(float(np.median(rt["L0_abc"])) /
                                               float(np.median(rt[f"L{L}_{variant}"])), 4)
        del Cw
        sx.release_workspace()

    # ---- roofline of the dominant kernel --------------------------------------------------------
    # ABC at one level is one launch of the all-products kernel (7 products); at two levels it is
    # seven launches, one per outer product, each computing 7 inner products, so one launch
    # executes 7 * 2*mq*nq*kq MFMA flops.  AB / Naive: one tile-kernel launch holds all 7^L
    # products.  The average launch duration comes from the library's event pairs around each
    # launch of that kernel during the timed steps (the staged outer-sum passes of two-level ABC
    # and the assembly / sum passes are timed apart from it).
    launches = 7 ** (L - 1) if (variant in ("abc", "ab") and L >= 1) else 1
    if L == 1 and variant == "abc" and one_level_staged(n, n, n):
        launches = 7   # one classical launch per product
    if kern_launches != launches * args.steps:
        raise SystemExit(f"expected {launches * args.steps} launches of the {kind} kernel in the "
                         f"timed steps, recorded {kern_launches}")
    avg_launch_ms = kern_ms / kern_launches
    exec_flops_launch = exec_flops / launches
    achieved = exec_flops_launch / (avg_launch_ms * 1e-3) * 1e-12
    traffic = None
    tpath = traffic_path(L, variant, n)
    if os.path.exists(tpath):
        with open(tpath) as f:
            tr = json.load(f)
        if tr.get("kernel_source_hash") == kernel_source_hash():
            traffic = tr.get("hbm_bytes_per_launch")
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_F64_MFMA,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64_MFMA, 4), "traffic": traffic,
                "kernel": dominant_kernel(L, variant, n),
                "launches_per_step": launches,
                "exec_flops_per_launch": exec_flops_launch, "avg_launch_ms": round(avg_launch_ms, 3),
                "timing": "HIP event pair around each launch on the call's stream, timed steps"}
    if sums_launches:
        roofline["outer_sum_passes"] = {"launches_per_step": sums_launches // args.steps,
                                        "ms_per_step": round(sums_ms / args.steps, 3)}
    # the matrix cores' measured issue rate on this device, beside the datasheet peak
    f64_rate, _ = sx.probe_rates(stream)
    roofline["peak_measured"] = round(f64_rate, 2)
    roofline["frac_of_measured"] = round(achieved / f64_rate, 4)
    log(f"  measured FP64 MFMA issue rate {f64_rate:.2f} TFLOP/s")

    # ---- CPU baseline: the oracle on a bounded column sample -----------------------------------
    cpu = None
    if not args.no_cpu:
        from oracle import oracle_dgemm
        threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        if A_h is None:
            A_h = sx.to_host(A)
        Bh = sx.to_host(B)
        Ch = sx.to_host(C0)

        def run_cols(ncols):
            Bc = np.asfortranarray(Bh[:, :ncols])
            Cc = np.asfortranarray(Ch[:, :ncols])
            t = time.perf_counter()
            oracle_dgemm(A_h, Bc, Cc, 1.0, 1.0)
            return time.perf_counter() - t
        probe_cols = 32
        tp = run_cols(probe_cols)
        ncols = int(max(probe_cols, min(n, probe_cols * args.cpu_seconds / max(tp, 1e-6))))
        tc = run_cols(ncols)
        cpu_tflops = 2.0 * n * n * ncols / tc * 1e-12
        cpu = {"value": round(cpu_tflops, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"plain triple-loop oracle (FP64, sequential sum over k) on A {n}x{n} times "
                         f"the first {ncols} columns of B ({2.0 * n * n * ncols:.3e} flops, "
                         f"{tc:.1f} s); rate scaled to TFLOP/s"}
        log(f"cpu baseline: {cpu}")
        del A_h, Bh, Ch

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"strassen_dgemm L={L} {variant.upper()} m=n=k={n} FP64 "
                               f"C:=A*B+C, entries uniform[-1,1]",
                   "m": n, "n": n, "k": n, "levels": L, "variant": variant,
                   "outer_sums": (("staged" if sums_launches else "in the tile load") if L == 2 else
                                  ("staged, products on the classical kernel" if L == 1 and sums_launches
                                   else None)),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "variants": variants,
    }
    if variants:
        head = headline_key(L, variant, sums_launches)
        out["classical_tflops"] = variants["L0_abc"]["tflops"]
        out["headline_member"] = head
        out["speedup_vs_classical"] = variants[head]["speedup_vs_classical"]
        out["context_vendor_blas_fp64"] = dict(
            vendor, speedup_of_headline=round(vendor["ms"] / variants[head]["ms"], 4))
        out["ragged"] = ragged
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
