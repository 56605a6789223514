"""The learned selector: timings of the family's members, training of the network on the GPU
with the library's own kernels, and evaluation by regret against exhaustive timing.

Members (the network's seven outputs, also the C-ABI's member index):
    0 classical, 1 one-level ABC, 2 one-level AB, 3 one-level Naive,
    4 two-level ABC, 5 two-level AB, 6 two-level Naive.
dtype 0 is FP64 (strassen_dgemm); dtype 1 is BF16 products (strassen_gemm_ex with bf16
products, FP64 sums and update), where only the ABC members exist (the others time as +inf).

Data flow:  collect(shapes, dtypes) -> times (N x 7, ms)  ->  labels = argmin
            train(X, y) -> parameters (5383 floats)      ->  save / strassen_selector_load
            evaluate(params, X, times) -> regret of the network, of the analytical model and
            of every fixed member.
"""
import json
import math
import os
import time

import numpy as np

from . import check, dgemm, gemm_ex, lib, set_workspace, workspace_size, workspace_size_ex

MEMBERS = [(0, "abc"), (1, "abc"), (1, "ab"), (1, "naive"), (2, "abc"), (2, "ab"), (2, "naive")]
D_IN = 11
N_PARAMS = 64 * D_IN + 64 + 64 * 64 + 64 + 7 * 64 + 7   # 5383
DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_data")
WEIGHTS = os.path.join(DATA_DIR, "weights.json")
TIMINGS = os.path.join(DATA_DIR, "timings.npz")


def features(m, n, k, dtype):
    """Network inputs (N x 11 float32) for arrays of sizes and dtype flags, from the library's
    strassen_selector_features: the sizes on a log scale, the dtype flag, and the analytical
    model's time ratios min(ln(t_c / t_best), 1) of the seven members."""
    import ctypes
    m, n, k, d = (np.atleast_1d(np.asarray(a)) for a in np.broadcast_arrays(m, n, k, dtype))
    out = np.empty((len(m), D_IN), dtype=np.float32)
    x = (ctypes.c_float * D_IN)()
    for i in range(len(m)):
        check(lib().strassen_selector_features(int(m[i]), int(n[i]), int(k[i]), int(d[i]), x))
        out[i] = x[:]
    return out


def available(dtype):
    return [dtype == 0 or v == "abc" for _, v in MEMBERS]


# ---------------------------------------------------------------------------------------------
# timings
# ---------------------------------------------------------------------------------------------
def collect(shapes, dtypes, progress=None, log_every=20.0):
    """Time every member on every shape (one call each, HIP events, after a warm-up of every
    member); returns an N x 7 array of milliseconds (+inf where a member is not offered)."""
    import torch
    stream = torch.cuda.current_stream()
    mk = max(m * k for m, _, k in shapes)
    kn = max(k * n for _, n, k in shapes)
    mn = max(m * n for m, n, _ in shapes)
    A = torch.empty(mk, dtype=torch.float64, device="cuda").uniform_(-1, 1)
    B = torch.empty(kn, dtype=torch.float64, device="cuda").uniform_(-1, 1)
    C = torch.zeros(mn, dtype=torch.float64, device="cuda")
    # one workspace large enough for every call, so no call grows it inside its timing
    ws = 0
    for (m, n, k), d in zip(shapes, dtypes):
        if d == 0:
            for lv, v in MEMBERS:
                ws = max(ws, workspace_size(m, n, k, lv, v))
        else:
            for lv in (0, 1, 2):
                ws = max(ws, workspace_size_ex(m, n, k, lv, "bf16"))
    wbuf = torch.empty(max(ws, 256) // 8 + 32, dtype=torch.float64, device="cuda")
    set_workspace(wbuf)
    view = lambda buf, r, c: buf[:r * c].view(c, r).t()

    def call(shape, d, c):
        m, n, k = shape
        lv, v = MEMBERS[c]
        a, b, cc = view(A, m, k), view(B, k, n), view(C, m, n)
        if d == 0:
            dgemm(a, b, cc, 1.0, 0.0, lv, v, stream)
        else:
            gemm_ex(a, b, cc, 1.0, 0.0, lv, "bf16", "f64", "f64", "abc", stream)

    try:
        for d in (0, 1):   # warm-up: every member once at a moderate size
            for c in range(7):
                if available(d)[c]:
                    call((1024, 1024, 1024), d, c)
        torch.cuda.synchronize()
        times = np.full((len(shapes), 7), np.inf)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(7)]
        t_last = time.time()
        for i in range(len(shapes)):
            av = available(dtypes[i])
            for c in range(7):
                if av[c]:
                    ev[c][0].record(stream)
                    call(shapes[i], dtypes[i], c)
                    ev[c][1].record(stream)
            ev_last = [c for c in range(7) if av[c]][-1]
            ev[ev_last][1].synchronize()
            for c in range(7):
                if av[c]:
                    times[i, c] = ev[c][0].elapsed_time(ev[c][1])
            if progress and time.time() - t_last > log_every:
                progress(i + 1, len(shapes))
                t_last = time.time()
        return times
    finally:
        set_workspace(None)


# ---------------------------------------------------------------------------------------------
# training with the library's kernels
# ---------------------------------------------------------------------------------------------
def init_params(seed=0):
    """He-uniform weights, zero biases (float32, flat)."""
    g = np.random.default_rng(seed)
    parts = []
    for shape in [(64, D_IN), (64,), (64, 64), (64,), (7, 64), (7,)]:
        if len(shape) == 2:
            lim = math.sqrt(6.0 / shape[1])
            parts.append(g.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


class Trainer:
    """Device buffers for training on N samples (the network's forward, backward and Adam run
    in the library's kernels)."""

    def __init__(self, X, y, params):
        import torch
        self.torch = torch
        self.n = len(y)
        self.X = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32), device="cuda")
        self.y = torch.as_tensor(np.ascontiguousarray(y, dtype=np.int32), device="cuda")
        self.p = torch.as_tensor(np.ascontiguousarray(params, dtype=np.float32), device="cuda")
        self.g = torch.zeros(N_PARAMS, dtype=torch.float32, device="cuda")
        self.m = torch.zeros_like(self.g)
        self.v = torch.zeros_like(self.g)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        import ctypes
        b = ctypes.c_size_t()
        check(lib().strassen_mlp_work_size(self.n, ctypes.byref(b)))
        self.work = torch.empty(b.value // 4 + 1, dtype=torch.float32, device="cuda")
        self.t = 0

    def _stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def loss_grad(self, lo=0, hi=None):
        """Loss and gradient over samples [lo, hi) (device tensors)."""
        hi = self.n if hi is None else hi
        check(lib().strassen_mlp_loss_grad(self.p.data_ptr(), self.X[lo:hi].data_ptr(),
                                           self.y[lo:hi].data_ptr(), hi - lo,
                                           self.work.data_ptr(), self.g.data_ptr(),
                                           self.loss.data_ptr(), self._stream()))
        return self.loss, self.g

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        check(lib().strassen_mlp_adam(self.p.data_ptr(), self.g.data_ptr(), self.m.data_ptr(),
                                      self.v.data_ptr(), self.t, lr, b1, b2, eps, self._stream()))

    def params(self):
        return self.p.cpu().numpy()


def train(X, y, epochs=300, batch=2048, lr=3e-3, seed=0, log=None, weights=None):
    """Minibatch Adam on (X, y) with the library's kernels.  Each epoch the host draws the
    sample order (the device copy is reordered): a permutation, or with `weights` (e.g. each
    shape's best time, so that the loss counts shapes as the regret does) a draw with
    replacement proportional to them."""
    import torch
    g = np.random.default_rng(seed)
    tr = Trainer(X, y, init_params(seed))
    Xh, yh = np.asarray(X, dtype=np.float32), np.asarray(y, dtype=np.int32)
    pw = None
    if weights is not None:
        pw = np.asarray(weights, dtype=np.float64)
        pw = pw / pw.sum()
    for ep in range(epochs):
        perm = g.permutation(len(yh)) if pw is None else g.choice(len(yh), len(yh), p=pw)
        tr.X.copy_(torch.as_tensor(Xh[perm]))
        tr.y.copy_(torch.as_tensor(yh[perm]))
        rate = lr * (0.5 * (1 + math.cos(math.pi * ep / epochs)))
        for lo in range(0, len(yh), batch):
            tr.loss_grad(lo, min(len(yh), lo + batch))
            tr.adam(rate)
        if log and (ep % 25 == 0 or ep == epochs - 1):
            tr.X.copy_(torch.as_tensor(Xh))
            tr.y.copy_(torch.as_tensor(yh))
            L, _ = tr.loss_grad()
            log(f"epoch {ep}: loss {float(L.item()):.4f}")
    return tr.params()


def predict(params, X):
    """Scores of the network for X (N x 4) by the library's forward kernel (N x 7)."""
    import torch
    p = torch.as_tensor(np.asarray(params, dtype=np.float32), device="cuda")
    x = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32), device="cuda")
    out = torch.empty((len(X), 7), dtype=torch.float32, device="cuda")
    check(lib().strassen_mlp_forward(p.data_ptr(), x.data_ptr(), len(X), out.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream))
    return out.cpu().numpy()


def choose(scores, dtypes):
    """Arg-max over the members offered for each sample's dtype."""
    s = np.array(scores, dtype=np.float64, copy=True)
    for i, d in enumerate(dtypes):
        s[i, ~np.array(available(int(d)))] = -np.inf
    return s.argmax(axis=1)


def model_choice(shapes, dtypes):
    """Arg-min of the library's analytical cost model."""
    import ctypes
    out = np.empty(len(shapes), dtype=np.int64)
    sec = (ctypes.c_double * 7)()
    for i, ((m, n, k), d) in enumerate(zip(shapes, dtypes)):
        check(lib().strassen_cost_model(m, n, k, int(d), sec))
        out[i] = int(np.argmin(np.array(sec[:])))
    return out


def regret(times, choice):
    best = times.min(axis=1)
    chosen = times[np.arange(len(choice)), choice]
    return float(chosen.sum() / best.sum() - 1.0)


def evaluate(params, shapes, dtypes, times):
    """Regret of the network, of the analytical model and of each fixed member (where offered,
    falling back to classical) on the given timings."""
    X = features(*np.array(shapes).T, dtypes)
    out = {"network": regret(times, choose(predict(params, X), dtypes)),
           "cost_model": regret(times, model_choice(shapes, dtypes))}
    for c, (lv, v) in enumerate(MEMBERS):
        ch = np.array([c if available(int(d))[c] else 0 for d in dtypes])
        out[f"always_L{lv}_{v}"] = regret(times, ch)
    out["best_fixed"] = min(v for k_, v in out.items() if k_.startswith("always_"))
    return out


def save(params, path=WEIGHTS, meta=None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"params": [float(v) for v in np.asarray(params, dtype=np.float32)],
                   "meta": meta or {}}, f)


def load(path=WEIGHTS):
    with open(path) as f:
        return np.asarray(json.load(f)["params"], dtype=np.float32)


# None: the committed network is installed on the first select(); True/False: decided already
_network_state = None


def install(params):
    """Hand the network to the library: strassen_select uses it from now on."""
    global _network_state
    a = np.ascontiguousarray(params, dtype=np.float32)
    check(lib().strassen_selector_load(a.ctypes.data))
    _network_state = True


def uninstall():
    """Back to the analytical cost model (also for later select() calls)."""
    global _network_state
    check(lib().strassen_selector_load(None))
    _network_state = False


def install_committed():
    """Install the network trained on this library's own timings (selector_data/weights.json),
    if present; returns whether a network is installed."""
    global _network_state
    if _network_state is None:
        if os.path.exists(WEIGHTS):
            install(load())
        else:
            _network_state = False
    return bool(_network_state)


def select(m, n, k, dtype=0):
    """(levels, variant) chosen by the library for one shape: by the committed network unless
    uninstall() was called or none is committed, else by the analytical cost model."""
    import ctypes
    install_committed()
    lv, var = ctypes.c_int(), ctypes.c_int()
    check(lib().strassen_select(m, n, k, dtype, ctypes.byref(lv), ctypes.byref(var)))
    return lv.value, ["abc", "ab", "naive"][var.value]


# ---------------------------------------------------------------------------------------------
# command line: timing collection (in parts) and training
# ---------------------------------------------------------------------------------------------
def dataset(count=22000, seed=0):
    """The selector's shapes: m, n, k log-uniform in [256, 20000] (rounded), dtype flags drawn
    with the same seed; the first 20000 train, the last 2000 are held out."""
    import workloads as W
    shapes = W.selector_shapes(seed, count)
    dtypes = [int(d) for d in np.random.default_rng(seed + 1).integers(0, 2, count)]
    return shapes, dtypes


def main(argv=None):
    import argparse
    import sys
    ap = argparse.ArgumentParser(prog="python -m paper_1605_01078_amd.selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect", help="time every member on one part of the dataset")
    c.add_argument("--part", type=int, required=True)
    c.add_argument("--parts", type=int, required=True)
    c.add_argument("--count", type=int, default=22000)
    c.add_argument("--out", required=True)
    t = sub.add_parser("train", help="train on the collected parts, evaluate, write the weights")
    t.add_argument("inputs", nargs="+", help="timings .npz parts (or one merged file)")
    t.add_argument("--train", type=int, default=20000)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--lr", type=float, default=3e-3, help="peak Adam step (cosine schedule)")
    t.add_argument("--seed", type=int, default=0, help="initial weights and sample order")
    t.add_argument("--weights", default=WEIGHTS)
    t.add_argument("--merged", default=TIMINGS)
    a = ap.parse_args(argv)
    say = lambda *x: print(*x, file=sys.stderr, flush=True)
    if a.cmd == "collect":
        shapes, dtypes = dataset(a.count)
        idx = np.array_split(np.arange(len(shapes)), a.parts)[a.part]
        say(f"part {a.part}/{a.parts}: {len(idx)} shapes")
        t0 = time.time()
        times = collect([shapes[i] for i in idx], [dtypes[i] for i in idx],
                        progress=lambda i, n: say(f"  {i}/{n} shapes, {time.time() - t0:.0f} s"))
        np.savez(a.out, index=idx, times=times)
        say(f"done in {time.time() - t0:.0f} s -> {a.out}")
        return
    shapes, dtypes = dataset()
    times = np.full((len(shapes), 7), np.nan)
    for path in a.inputs:
        z = np.load(path)
        times[z["index"] if "index" in z else np.arange(len(shapes))] = z["times"]
    if np.isnan(times).any():
        raise SystemExit("missing timings for some shapes")
    np.savez_compressed(a.merged, times=times.astype(np.float32))
    X = features(*np.array(shapes).T, dtypes)
    y = times.argmin(axis=1)
    n = a.train
    # shapes weighted by their best time: the regret is a ratio of summed times
    params = train(X[:n], y[:n], epochs=a.epochs, lr=a.lr, seed=a.seed, log=say,
                   weights=times[:n].min(axis=1))
    res_test = evaluate(params, shapes[n:], dtypes[n:], times[n:])
    res_train = evaluate(params, shapes[:n], dtypes[:n], times[:n])
    say(json.dumps({"held_out": res_test, "train": res_train}))
    save(params, a.weights, meta={"held_out": res_test, "train": res_train,
                                  "epochs": a.epochs, "lr": a.lr, "seed": a.seed,
                                  "train_shapes": n,
                                  "held_out_shapes": len(shapes) - n})


if __name__ == "__main__":
    main()
