"""The selector's performance-model network, oracle side (FP64 numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network maps a GEMM shape to scores over the seven members of the family the selector picks
from (classical; one-level ABC, AB, Naive; two-level ABC, AB, Naive):

    x  = (f(m), f(n), f(k), d, r_0 .. r_6)
                                    f(s) = (ln s - ln 256) / (ln 20000 - ln 256),  d = 0 FP64, 1 BF16,
                                    r_c = min(ln(t_c / min_j t_j), 1) for the seven members' times
                                    t_c under a time model supplied by the caller (1 where t_c
                                    is infinite: a member not offered)
    h1 = relu(W1 x + b1)            W1: 64 x 11
    h2 = relu(W2 h1 + b2)           W2: 64 x 64
    z  = W3 h2 + b3                 W3: 7 x 64
    loss = mean over the batch of  -log softmax(z)[label]

Parameters are one flat vector in the order W1 (row-major), b1, W2, b2, W3, b3 (5383 values);
the library's kernels take the same layout.  Training uses Adam (Kingma and Ba, 2015):
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
import numpy as np

D_IN, H, D_OUT = 11, 64, 7
SHAPES = [(H, D_IN), (H,), (H, H), (H,), (D_OUT, H), (D_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)   # 5383
LOG_LO, LOG_HI = np.log(256.0), np.log(20000.0)


def features(m, n, k, dtype_flag, model_times):
    """Network input for shapes (arrays or scalars); dtype_flag 0 = FP64, 1 = BF16;
    model_times: the seven members' times under the caller's time model (N x 7, +inf for a
    member not offered)."""
    f = lambda s: (np.log(np.asarray(s, dtype=np.float64)) - LOG_LO) / (LOG_HI - LOG_LO)
    m, n, k, d = np.broadcast_arrays(f(m), f(n), f(k), np.asarray(dtype_flag, dtype=np.float64))
    size = np.stack([m, n, k, d], axis=-1).reshape(-1, 4)
    t = np.asarray(model_times, dtype=np.float64).reshape(-1, D_OUT)
    best = t.min(axis=1, keepdims=True)
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(np.isfinite(t), np.minimum(np.log(t / best), 1.0), 1.0)
    return np.concatenate([size, r], axis=1)


def unpack(p):
    """Views of the flat parameter vector as (W1, b1, W2, b2, W3, b3)."""
    p = np.asarray(p)
    out, o = [], 0
    for s in SHAPES:
        cnt = int(np.prod(s))
        out.append(p[o:o + cnt].reshape(s))
        o += cnt
    return out


def init(seed=0):
    """He-uniform weights, zero biases (FP64)."""
    g = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            parts.append(g.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def forward(p, X):
    """(logits, cache) for a batch X (N x 11)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return z, (X, a1, h1, a2, h2)


def log_softmax(z):
    zmax = z.max(axis=1, keepdims=True)
    return z - zmax - np.log(np.exp(z - zmax).sum(axis=1, keepdims=True))


def loss(p, X, y):
    z, _ = forward(p, X)
    return float(-log_softmax(z)[np.arange(len(y)), y].mean())


def loss_grad(p, X, y):
    """(loss, gradient as a flat vector) by backpropagation."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z, (X, a1, h1, a2, h2) = forward(p, X)
    N = X.shape[0]
    ls = log_softmax(z)
    L = float(-ls[np.arange(N), y].mean())
    dz = np.exp(ls)
    dz[np.arange(N), y] -= 1.0
    dz /= N
    gW3 = dz.T @ h2
    gb3 = dz.sum(axis=0)
    dh2 = dz @ W3
    da2 = dh2 * (a2 > 0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return L, np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict(p, X):
    z, _ = forward(p, X)
    return z.argmax(axis=1)


def regret(times, choice):
    """Total time of the chosen members over the total of the best ones, minus one.
    times: N x 7 (inf where a member is not available); choice: N indices."""
    times = np.asarray(times, dtype=np.float64)
    best = times.min(axis=1)
    chosen = times[np.arange(len(choice)), choice]
    return float(chosen.sum() / best.sum() - 1.0)
