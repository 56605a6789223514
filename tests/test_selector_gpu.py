"""Selector network on the GPU: the library's forward, backward and Adam kernels against the
FP64 oracle (oracle/mlp.py); training reduces the loss; the installed network drives
strassen_select; the committed network's regret on the held-out timings."""
import os

import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")
from paper_1605_01078_amd import selector as S

pytestmark = pytest.mark.gpu


def _data(seed, n):
    g = np.random.default_rng(seed)
    m, nn, k = (np.exp(g.uniform(np.log(256), np.log(20000), n)) for _ in range(3))
    d = g.integers(0, 2, n)
    return mlp.features(m, nn, k, d, np.exp(g.uniform(0, 1.5, (n, 7)))), g.integers(0, 7, n)


def test_forward_matches_oracle():
    p = (mlp.init(1) + 0.05).astype(np.float32)
    X, _ = _data(2, 1000)
    got = S.predict(p, X)
    want, _ = mlp.forward(p.astype(np.float64), X.astype(np.float32).astype(np.float64))
    assert np.abs(got - want).max() <= 1e-4 * (1 + np.abs(want).max())


def test_loss_and_gradient_match_oracle():
    p = (mlp.init(3) + 0.02).astype(np.float32)
    X, y = _data(4, 3000)
    tr = S.Trainer(X, y, p)
    L, g = tr.loss_grad()
    torch.cuda.synchronize()
    Lw, gw = mlp.loss_grad(p.astype(np.float64), X.astype(np.float32).astype(np.float64), y)
    assert abs(float(L.item()) - Lw) <= 1e-5 * (1 + abs(Lw))
    gg = g.cpu().numpy()
    assert np.abs(gg - gw).max() <= 1e-4 * np.abs(gw).max() + 1e-7


def test_adam_matches_oracle():
    p = (mlp.init(5)).astype(np.float32)
    X, y = _data(6, 500)
    tr = S.Trainer(X, y, p)
    pw, mw, vw = p.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for t in range(1, 4):
        _, g = tr.loss_grad()
        gh = g.cpu().numpy().astype(np.float64)
        tr.adam(2e-3)
        pw, mw, vw = mlp.adam_step(pw, gh, mw, vw, t, lr=2e-3)
        assert np.abs(tr.params() - pw).max() <= 1e-6 + 1e-5 * np.abs(pw).max()


def test_training_learns_a_rule():
    g = np.random.default_rng(7)
    n = 6000
    m, nn, k = (np.exp(g.uniform(np.log(256), np.log(20000), n)) for _ in range(3))
    d = g.integers(0, 2, n)
    X = S.features(m, nn, k, d)
    y = np.clip((X[:, :3].sum(axis=1) * 7 / 3).astype(int), 0, 6)   # a smooth rule of size
    p = S.train(X[:5000], y[:5000], epochs=60, batch=1000, lr=5e-3)
    pred = S.predict(p, X[5000:]).argmax(axis=1)
    assert (pred == y[5000:]).mean() > 0.8


def test_installed_network_drives_select():
    p = np.zeros(mlp.N_PARAMS, dtype=np.float32)
    p[-7:] = [0, 0, 9, 0, 5, 0, 0]          # scores: member 2 (one-level AB) first, then 4
    S.install(p)
    try:
        assert S.select(4096, 4096, 4096, 0) == (1, "ab")
        assert S.select(4096, 4096, 4096, 1) == (2, "abc")   # BF16: ABC members only
    finally:
        S.uninstall()


def test_installed_network_sees_model_features():
    """A hand-set network scoring member c as -x[4 + c] (minus the model's time ratio) picks
    the analytical model's member: the inputs reach the inference kernel in their layout."""
    W1, b1, W2, b2, W3, b3 = (np.zeros(s) for s in mlp.SHAPES)
    for c in range(7):
        W1[c, 4 + c] = 1.0
        W2[c, c] = 1.0
        W3[c, c] = -1.0
    p = np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float32)
    shapes = [(256, 256, 256, 0), (16384, 16384, 16384, 0), (16383, 16384, 16383, 0),
              (3000, 12000, 5000, 0), (8192, 8192, 8192, 1), (20000, 300, 20000, 1)]
    S.uninstall()
    want = [S.select(*s) for s in shapes]
    S.install(p)
    try:
        assert [S.select(*s) for s in shapes] == want
    finally:
        S.uninstall()


@pytest.mark.skipif(not os.path.exists(S.WEIGHTS) or not os.path.exists(S.TIMINGS),
                    reason="selector not trained yet")
def test_trained_network_regret_on_held_out_timings():
    shapes, dtypes = S.dataset()
    times = np.load(S.TIMINGS)["times"].astype(np.float64)
    p = S.load()
    res = S.evaluate(p, shapes[20000:], dtypes[20000:], times[20000:])
    print("held-out regret", res)
    assert res["network"] <= 0.05
    assert res["network"] < res["cost_model"]
    assert res["network"] < res["best_fixed"]
