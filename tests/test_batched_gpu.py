"""Batched mode on the GPU: every problem of a batch (persistent-kernel tiles, its own
all-products launches, or its own launches on a side stream) equals (bitwise) the single call
with the same level and tile choice;
graph replays equal the eager run; the autotuner's choices are valid and run correctly;
scale-only problems."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, rel_fro

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-12, 2: 1e-11}


def _mixed_batch(seed, count):
    g = np.random.default_rng(seed)
    shapes, levels, cfg = [], [], []
    for i in range(count):
        m, n, k = (int(64 * g.integers(1, 11)) for _ in range(3))
        shapes.append((m, n, k))
        levels.append(int(g.integers(0, 3)))
        cfg.append(int(g.integers(0, 3)))
    # ragged problems (odd sizes: the general load path)
    shapes += [(130, 70, 200), (301, 259, 271)]
    levels += [2, 1]
    cfg += [0, 1]
    return shapes, levels, cfg


def _operands(shapes, seed):
    ops = []
    for i, (m, n, k) in enumerate(shapes):
        A, B, C = W.problem(seed + i, m, n, k, "uniform")
        ops.append((A, B, C))
    return ops


def _single(A, B, C, alpha, beta, level, cfg):
    # batched tile choice 2 (own all-products launches) = tile configuration 4 of a single call;
    # 3 (side streams) = the default dispatch
    sx.set_tile_config({2: 4, 3: -1}.get(cfg, cfg))
    try:
        dC = sx.to_device(C)
        sx.dgemm(sx.to_device(A), sx.to_device(B), dC, alpha, beta, level, "abc")
        torch.cuda.synchronize()
        return sx.to_host(dC)
    finally:
        sx.set_tile_config(-1)


def test_batched_equals_single_calls():
    shapes, levels, cfg = _mixed_batch(50, 22)
    print(f"case batched mixed {len(shapes)} problems", flush=True)
    ops = _operands(shapes, 500)
    b = sx.Batched(shapes, levels, cfg)
    assert b.choices() == list(zip(levels, cfg))
    dA = [sx.to_device(A) for A, _, _ in ops]
    dB = [sx.to_device(B) for _, B, _ in ops]
    dC = [sx.to_device(C) for _, _, C in ops]
    b.run(dA, dB, dC, -0.5, 2.5)
    torch.cuda.synchronize()
    for i, ((A, B, C), lv, cf) in enumerate(zip(ops, levels, cfg)):
        got = sx.to_host(dC[i])
        want = _single(A, B, C, -0.5, 2.5, lv, cf)
        assert np.array_equal(got, want), (i, shapes[i], lv, cf)
        ref = oracle_dgemm(A, B, C.copy(order="F"), -0.5, 2.5)
        assert rel_fro(got, ref) <= TOL[lv]
    b.close()


def test_batched_graph_replays():
    shapes, levels, cfg = _mixed_batch(51, 12)
    print(f"case batched graph {len(shapes)} problems", flush=True)
    ops = _operands(shapes, 600)
    b = sx.Batched(shapes, levels, cfg)
    dA = [sx.to_device(A) for A, _, _ in ops]
    dB = [sx.to_device(B) for _, B, _ in ops]
    C0 = [sx.to_device(C) for _, _, C in ops]
    dC = [c.clone() for c in C0]
    b.run(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    eager = [sx.to_host(c) for c in dC]
    for c, c0 in zip(dC, C0):
        c.copy_(c0)
    b.capture(dA, dB, dC, 1.0, 1.0)
    for rep in range(3):
        for c, c0 in zip(dC, C0):      # eager work between replays: reset C
            c.copy_(c0)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for i, c in enumerate(dC):
            assert np.array_equal(sx.to_host(c), eager[i]), (rep, i)
    # a run discards the recording
    b.run(dA, dB, dC, 1.0, 1.0)
    with pytest.raises(sx.StrassenError):
        b.replay()
    b.close()


def test_batched_autotune():
    shapes = [(64 * a, 64 * b_, 64 * c) for a, b_, c in
              [(4, 4, 4), (16, 8, 32), (40, 40, 40), (8, 48, 16), (32, 32, 64), (6, 6, 6)]]
    print(f"case batched autotune {len(shapes)} problems", flush=True)
    ops = _operands(shapes, 700)
    b = sx.Batched(shapes)
    b.autotune(sample=0, seed=3)
    ch = b.choices()
    assert all(lv in (0, 1, 2) and cf in (0, 1, 2, 3) for lv, cf in ch)
    assert all(cf != 2 or lv == 1 for lv, cf in ch)     # the rule gives own launches to L1 only
    assert all(cf != 3 or lv <= 1 for lv, cf in ch)     # side streams: no staging workspace
    dA = [sx.to_device(A) for A, _, _ in ops]
    dB = [sx.to_device(B) for _, B, _ in ops]
    dC = [sx.to_device(C) for _, _, C in ops]
    b.run(dA, dB, dC, 1.0, 0.5)
    torch.cuda.synchronize()
    for i, ((A, B, C), (lv, cf)) in enumerate(zip(ops, ch)):
        assert np.array_equal(sx.to_host(dC[i]), _single(A, B, C, 1.0, 0.5, lv, cf)), (i, lv, cf)
    b.close()


def test_batched_scale_only():
    """alpha == 0: every problem is C := beta*C (run eagerly; capture refuses it)."""
    shapes = [(256, 192, 320), (130, 70, 200)]
    print("case batched alpha=0", flush=True)
    ops = _operands(shapes, 800)
    b = sx.Batched(shapes, [1, 2], [0, 1])
    dA = [sx.to_device(A) for A, _, _ in ops]
    dB = [sx.to_device(B) for _, B, _ in ops]
    dC = [sx.to_device(C) for _, _, C in ops]
    b.run(dA, dB, dC, 0.0, 0.5)
    torch.cuda.synchronize()
    for i, (_, _, C) in enumerate(ops):
        assert np.array_equal(sx.to_host(dC[i]), 0.5 * C)
    with pytest.raises(sx.StrassenError):
        b.capture(dA, dB, dC, 0.0, 0.5)
    b.close()


def test_batched_all_products_launches():
    """Problems on their own all-products launches (whole-tile and masked one-level kernels, the
    seven in-load two-level launches, a level-0 problem whose choice falls back to the persistent
    kernel) beside persistent-kernel problems: eager run and graph replays equal single calls."""
    shapes = [(1024, 1024, 1024), (1024, 704, 512), (960, 1088, 768), (512, 512, 1024),
              (768, 640, 512), (260, 300, 200), (640, 640, 640), (301, 259, 271)]
    levels = [1, 1, 1, 2, 0, 1, 0, 1]
    cfg = [2, 2, 2, 2, 2, 2, 0, 2]     # the last: layout does not apply, persistent kernel
    print(f"case batched all-products {shapes}", flush=True)
    ops = _operands(shapes, 800)
    b = sx.Batched(shapes, levels, cfg)
    assert b.choices() == list(zip(levels, cfg))
    dA = [sx.to_device(A) for A, _, _ in ops]
    dB = [sx.to_device(B) for _, B, _ in ops]
    C0 = [sx.to_device(C) for _, _, C in ops]
    dC = [c.clone() for c in C0]
    b.run(dA, dB, dC, 0.75, -1.25)
    torch.cuda.synchronize()
    want = [_single(A, B, C, 0.75, -1.25, lv, cf) for (A, B, C), lv, cf in zip(ops, levels, cfg)]
    for i, c in enumerate(dC):
        assert np.array_equal(sx.to_host(c), want[i]), (i, shapes[i])
        A, B, C = ops[i]
        ref = oracle_dgemm(A, B, C.copy(order="F"), 0.75, -1.25)
        assert rel_fro(want[i], ref) <= TOL[levels[i]]
    b.capture(dA, dB, dC, 0.75, -1.25)
    for rep in range(3):
        for c, c0 in zip(dC, C0):      # eager work between replays: reset C
            c.copy_(c0)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for i, c in enumerate(dC):
            assert np.array_equal(sx.to_host(c), want[i]), (rep, i)
    b.close()


def test_batched_side_streams():
    """Problems on side streams (tile choice 3: their own single-call launches without
    workspace, spread over streams forked from and joined into the caller's) beside
    persistent-kernel and all-products problems: the classical kernel, the all-products kernel,
    the tile kernel for ragged shapes (where a single call would pad: bitwise the same), two
    levels with the outer sums in the load; eager run and graph replays equal single calls."""
    shapes = [(4096, 2048, 512), (1024, 1024, 1024), (1024, 704, 512), (301, 259, 271),
              (512, 512, 1024), (768, 640, 512), (130, 70, 200), (640, 640, 640), (2048, 1024, 768)]
    levels = [0, 1, 1, 1, 2, 0, 0, 1, 0]
    cfg = [3, 3, 3, 3, 3, 3, 0, 2, 3]
    print(f"case batched side streams {shapes}", flush=True)
    ops = _operands(shapes, 900)
    b = sx.Batched(shapes, levels, cfg)
    assert b.choices() == list(zip(levels, cfg))
    dA = [sx.to_device(A) for A, _, _ in ops]
    dB = [sx.to_device(B) for _, B, _ in ops]
    C0 = [sx.to_device(C) for _, _, C in ops]
    dC = [c.clone() for c in C0]
    b.run(dA, dB, dC, -0.75, 1.5)
    torch.cuda.synchronize()
    want = [_single(A, B, C, -0.75, 1.5, lv, cf) for (A, B, C), lv, cf in zip(ops, levels, cfg)]
    for i, c in enumerate(dC):
        assert np.array_equal(sx.to_host(c), want[i]), (i, shapes[i])
        A, B, C = ops[i]
        ref = oracle_dgemm(A, B, C.copy(order="F"), -0.75, 1.5)
        assert rel_fro(want[i], ref) <= TOL[levels[i]]
    b.capture(dA, dB, dC, -0.75, 1.5)
    for rep in range(3):
        for c, c0 in zip(dC, C0):      # eager work between replays: reset C
            c.copy_(c0)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for i, c in enumerate(dC):
            assert np.array_equal(sx.to_host(c), want[i]), (rep, i)
    b.close()
