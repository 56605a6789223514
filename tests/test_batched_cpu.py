"""Batched mode, host side (no device needed): plans, the default choice rule, argument checks."""
import ctypes

import pytest

import workloads as W

sx = pytest.importorskip("paper_1605_01078_amd")


def test_plan_explicit_and_default_choices():
    shapes = [(256, 256, 256), (4096, 4096, 4096), (320, 4096, 64), (0, 5, 5)]
    b = sx.Batched(shapes, levels=[2, -1, 1, -1], cfg=[1, -1, 0, -1])
    ch = b.choices()
    assert ch[0] == (2, 1) and ch[2] == (1, 0)
    # default rule: classical, 128 x 128 tiles
    assert ch[1] == (0, 0) and ch[3] == (0, 0)
    b.close()
    b.close()   # idempotent


def test_plan_workload_c4_shapes():
    shapes = W.batched_shapes(0)
    assert len(shapes) == 512
    assert all(256 <= d <= 4096 and d % 64 == 0 for s in shapes for d in s)
    b = sx.Batched(shapes)
    assert len(b.choices()) == 512
    b.close()


def test_plan_argument_errors():
    L = sx.lib()
    i64 = ctypes.c_int64 * 2
    ci = ctypes.c_int * 2
    m, n, k = i64(4, 4), i64(4, 4), i64(4, 4)
    plan = ctypes.c_void_p()
    assert L.strassen_batched_plan(-1, m, n, k, None, None, ctypes.byref(plan)) == -1
    assert L.strassen_batched_plan(2, None, n, k, None, None, ctypes.byref(plan)) == -2
    assert L.strassen_batched_plan(2, i64(4, -1), n, k, None, None, ctypes.byref(plan)) == -2
    assert L.strassen_batched_plan(2, m, n, k, ci(0, 3), None, ctypes.byref(plan)) == -5
    assert L.strassen_batched_plan(2, m, n, k, None, ci(4, 0), ctypes.byref(plan)) == -6
    assert L.strassen_batched_plan(2, m, n, k, None, ci(0, -2), ctypes.byref(plan)) == -6
    assert L.strassen_batched_plan(2, m, n, k, None, None, None) == -7
    assert L.strassen_batched_plan(2, m, n, k, ci(1, 0), ci(2, 2), ctypes.byref(plan)) == 0
    lv, cf = ctypes.c_int(), ctypes.c_int()
    assert L.strassen_batched_choice(plan, 0, ctypes.byref(lv), ctypes.byref(cf)) == 0
    assert (lv.value, cf.value) == (1, 2)
    assert L.strassen_batched_destroy(plan) == 0
    assert L.strassen_batched_plan(2, m, n, k, None, None, ctypes.byref(plan)) == 0
    lv, cf = ctypes.c_int(), ctypes.c_int()
    assert L.strassen_batched_choice(plan, 2, ctypes.byref(lv), ctypes.byref(cf)) == -2
    assert L.strassen_batched_choice(None, 0, ctypes.byref(lv), ctypes.byref(cf)) == -1
    assert L.strassen_batched_replay(plan, None) == -1    # nothing recorded
    assert L.strassen_batched_autotune(plan, -1, 0, None) == -2
    assert L.strassen_batched_destroy(plan) == 0
    assert L.strassen_batched_destroy(None) == 0
