"""Pins of the selector network's oracle (oracle/mlp.py): backpropagation against central
finite differences, closed forms of the loss, log-softmax against scipy, Adam against torch."""
import numpy as np
import pytest

from oracle import mlp


def _batch(seed, n=37):
    g = np.random.default_rng(seed)
    m, nn, k = (np.exp(g.uniform(np.log(256), np.log(20000), n)) for _ in range(3))
    X = mlp.features(m, nn, k, g.integers(0, 2, n), np.exp(g.uniform(0, 1.5, (n, 7))))
    y = g.integers(0, mlp.D_OUT, n)
    return X, y


def test_parameter_count_and_features():
    assert mlp.N_PARAMS == 64 * 11 + 64 + 64 * 64 + 64 + 7 * 64 + 7 == 5383
    # sizes at the ends and the geometric middle of the range; the model's best member gets 0,
    # a member e times slower 1, a slower one or one not offered is clipped at 1
    e = np.e
    t = [2.0, 2.0 * np.sqrt(e), 2.0 * e, 2.0 * e * e, np.inf, 2.0 * e ** 0.25, 2.0]
    x = mlp.features(256, 20000, np.sqrt(256 * 20000), 1, t)
    assert np.allclose(x, [[0.0, 1.0, 0.5, 1.0, 0.0, 0.5, 1.0, 1.0, 1.0, 0.25, 0.0]], rtol=0, atol=1e-12)


def test_gradient_matches_finite_differences():
    p = mlp.init(1) + 0.01
    X, y = _batch(2)
    L, g = mlp.loss_grad(p, X, y)
    assert abs(L - mlp.loss(p, X, y)) < 1e-14
    rng = np.random.default_rng(3)
    idx = rng.choice(mlp.N_PARAMS, size=120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, y) - mlp.loss(p - e, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_loss_closed_forms():
    X, y = _batch(4, 11)
    p = mlp.init(5)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    # zero output layer: logits are the bias for every sample
    W3[...] = 0.0
    b3[...] = np.arange(7) * 0.25
    z = b3
    want = float(np.mean(np.log(np.exp(z).sum()) - z[y]))
    assert abs(mlp.loss(p, X, y) - want) < 1e-13
    # all-equal logits: loss = log 7
    b3[...] = 2.0
    assert abs(mlp.loss(p, X, y) - np.log(7.0)) < 1e-13


def test_log_softmax_matches_scipy():
    from scipy.special import log_softmax
    z = np.random.default_rng(6).normal(size=(20, 7)) * 30
    assert np.allclose(mlp.log_softmax(z), log_softmax(z, axis=1), rtol=0, atol=1e-12)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(7)
    p = g.normal(size=50)
    t_p = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([t_p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 6):
        grad = g.normal(size=50)
        t_p.grad = torch.tensor(grad.copy())
        opt.step()
        p, m, v = mlp.adam_step(p, grad, m, v, t, lr=3e-3)
        assert np.allclose(p, t_p.detach().numpy(), rtol=0, atol=1e-12)


def test_regret_definition():
    times = np.array([[1.0, 2.0, np.inf], [3.0, 1.5, 2.0]])
    assert mlp.regret(times, np.array([0, 1])) == 0.0
    assert abs(mlp.regret(times, np.array([1, 0])) - ((2.0 + 3.0) / 2.5 - 1.0)) < 1e-15
