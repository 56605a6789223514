"""Parity at the full benchmark sizes, in the configuration bench.py times (needs an MI355X).

m = n = k = 16384 (square), m = n = 16384, k = 1024 (rank-k) and m = n = k = 16383 (every
dimension odd: ABC on block-padded copies), A, B, C uniform[-1, 1] drawn on the device from
seeds, alpha = beta = 1:
  * 64 randomly chosen columns of C from classical, one-level ABC and two-level ABC (default
    path: staged outer sums) against the plain-definition oracle on those columns — relative
    Frobenius error 1e-12 / 1e-11 for Strassen, the any-order rounding bound for classical;
  * a Freivalds projection of the whole result, ||C x - (A (B x) + C0 x)|| / ||A (B x) + C0 x||
    with random x, computed on the host in FP64;
  * AB, Naive and the unstaged two-level ABC bitwise equal to ABC of the same level (the shared
    association and accumulation order).
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm, rel_fro

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
TOL = {0: None, 1: 1e-12, 2: 1e-11}


def _case(m, n, k, seed):
    A = W.device_uniform(seed, m, k)
    B = W.device_uniform(seed + 1, k, n)
    C0 = W.device_uniform(seed + 2, m, n)
    return A, B, C0


def _call(A, B, C0, levels, variant, cfg=-1):
    C = C0.clone()
    sx.set_tile_config(cfg)
    try:
        sx.dgemm(A, B, C, 1.0, 1.0, levels, variant)
        torch.cuda.synchronize()
    finally:
        sx.set_tile_config(-1)
    return C


@pytest.mark.parametrize("shape", [(16384, 16384, 16384), (16384, 16384, 1024), (16383, 16383, 16383)])
def test_full_size_sampled_columns_and_projection(shape):
    m, n, k = shape
    print(f"case full size {shape}", flush=True)
    A, B, C0 = _case(m, n, k, 61)
    g = np.random.default_rng(5)
    cols = np.sort(g.choice(n, size=64, replace=False))
    A_h = sx.to_host(A)
    Bc = np.asfortranarray(sx.to_host(B[:, torch.as_tensor(cols, device="cuda")]))
    Cc = np.asfortranarray(sx.to_host(C0[:, torch.as_tensor(cols, device="cuda")]))
    ref = oracle_dgemm(A_h, Bc, Cc.copy(order="F"), 1.0, 1.0)
    # Freivalds: the whole result projected on a random vector, on the host in FP64
    x = g.uniform(-1, 1, n)
    B_h = sx.to_host(B)
    C0_h = sx.to_host(C0)
    want_x = A_h @ (B_h @ x) + C0_h @ x
    del B_h
    bound = 2 * (k + 2) * U / (1 - (k + 2) * U) * (np.abs(A_h) @ np.abs(Bc) + np.abs(Cc))
    idx = torch.as_tensor(cols, device="cuda")
    results = {}
    for levels in (0, 1, 2):
        C = _call(A, B, C0, levels, "abc")
        got = sx.to_host(C[:, idx])
        if levels == 0:
            assert (np.abs(got - ref) <= bound).all()
        else:
            err = rel_fro(got, ref)
            print(f"  L={levels} ABC sampled rel err {err:.3e}", flush=True)
            assert err <= TOL[levels]
        proj = sx.to_host(C) @ x
        perr = np.linalg.norm(proj - want_x) / np.linalg.norm(want_x)
        print(f"  L={levels} ABC projection rel err {perr:.3e}", flush=True)
        assert perr <= (1e-13 if levels == 0 else TOL[levels])
        results[levels] = C
    for levels in (1, 2):
        for v in ("ab", "naive"):
            assert torch.equal(_call(A, B, C0, levels, v), results[levels]), (levels, v)
    # two-level ABC with the outer sums formed in the load (tile configuration 4)
    assert torch.equal(_call(A, B, C0, 2, "abc", cfg=4), results[2])
