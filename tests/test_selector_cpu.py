"""Selector, host side: the analytical cost model and the model-based choice (no device)."""
import ctypes
import math

import numpy as np
import pytest

sx = pytest.importorskip("paper_1605_01078_amd")
from paper_1605_01078_amd import selector as S
from oracle import mlp


def _model(m, n, k, d):
    sec = (ctypes.c_double * 7)()
    sx.check(sx.lib().strassen_cost_model(m, n, k, d, sec))
    return list(sec)


def test_cost_model_members():
    t = _model(4096, 4096, 4096, 0)
    assert all(math.isfinite(v) and v > 0 for v in t)
    tb = _model(4096, 4096, 4096, 1)
    assert [math.isfinite(v) for v in tb] == [True, True, False, False, True, False, False]
    # classical time grows like m n k once the GPU is full
    a, b = _model(8192, 8192, 8192, 0)[0], _model(16384, 16384, 16384, 0)[0]
    assert 7.0 < b / a < 9.0


def test_model_choice_valid_and_strassen_at_large_sizes():
    S.uninstall()   # the analytical cost model decides
    for shape in [(256, 256, 256), (1000, 3000, 700), (20000, 300, 20000)]:
        for d in (0, 1):
            lv, var = S.select(*shape, d)
            assert lv in (0, 1, 2) and (d == 0 or var == "abc")
    # at 16384 the measured order (two-level ABC, one-level ABC, classical) is reproduced
    t = _model(16384, 16384, 16384, 0)
    assert t[4] < t[1] < t[0] and S.select(16384, 16384, 16384, 0) == (2, "abc")
    # where the all-products layout does not fit, ABC pays for its block-padded copies
    assert _model(16383, 16384, 16383, 0)[1] > _model(16384, 16384, 16384, 0)[1]
    assert S.select(20000, 20000, 20000, 1)[1] == "abc"


def test_select_argument_errors():
    L = sx.lib()
    a, b = ctypes.c_int(), ctypes.c_int()
    assert L.strassen_select(-1, 1, 1, 0, ctypes.byref(a), ctypes.byref(b)) == -1
    assert L.strassen_select(1, 1, 1, 2, ctypes.byref(a), ctypes.byref(b)) == -4
    assert L.strassen_select(1, 1, 1, 0, None, ctypes.byref(b)) == -5
    bad = np.full(mlp.N_PARAMS, np.nan, dtype=np.float32)
    assert L.strassen_selector_load(bad.ctypes.data) == -1
    assert L.strassen_selector_load(None) == 0
    sz = ctypes.c_size_t()
    assert L.strassen_mlp_work_size(10, ctypes.byref(sz)) == 0 and sz.value == 10 * 271 * 4


def test_features_match_oracle_definition():
    """The library's network input (strassen_selector_features) against the oracle's definition
    of it, fed the library's analytical model times."""
    g = np.random.default_rng(0)
    m, n, k = (g.integers(256, 20001, 50) for _ in range(3))
    d = g.integers(0, 2, 50)
    t = np.array([_model(int(a), int(b), int(c), int(e)) for a, b, c, e in zip(m, n, k, d)])
    got = S.features(m, n, k, d)
    assert got.shape == (50, mlp.D_IN)
    assert np.allclose(got, mlp.features(m, n, k, d, t), rtol=0, atol=1e-6)
    # the model's pick scores 0; BF16 rows mark AB and Naive as not offered
    assert (got[:, 4:].min(axis=1) == 0).all()
    assert (got[d == 1][:, [6, 7, 9, 10]] == 1).all()
    L = sx.lib()
    x = (ctypes.c_float * 11)()
    assert L.strassen_selector_features(-1, 1, 1, 0, x) == -1
    assert L.strassen_selector_features(1, 1, 1, 2, x) == -4
    assert L.strassen_selector_features(1, 1, 1, 0, None) == -5


def test_committed_network_file():
    """The committed network: every parameter finite, in the kernels' layout, with the held-out
    evaluation it was accepted on."""
    import json
    import os
    assert os.path.exists(S.WEIGHTS) and os.path.exists(S.TIMINGS)
    p = S.load()
    assert p.shape == (mlp.N_PARAMS,) and np.isfinite(p).all()
    meta = json.load(open(S.WEIGHTS))["meta"]
    assert meta["train_shapes"] == 20000 and meta["held_out_shapes"] == 2000
    assert meta["held_out"]["network"] <= 0.05
    times = np.load(S.TIMINGS)["times"]
    assert times.shape == (22000, 7)
    # the held-out regret recorded with the weights is the oracle network's on the stored timings
    shapes, dtypes = S.dataset()
    X = S.features(*np.array(shapes[20000:]).T, dtypes[20000:])
    z, _ = mlp.forward(p.astype(np.float64), X.astype(np.float32).astype(np.float64))
    ch = S.choose(z, dtypes[20000:])
    r = mlp.regret(times[20000:].astype(np.float64), ch)
    assert abs(r - meta["held_out"]["network"]) < 2e-3
