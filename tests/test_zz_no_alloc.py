"""strassen_dgemm_noalloc: the entry point for callers that cannot allocate (its workspace is
the library's static scratch).  Checked against strassen_dgemm on the same inputs, bit for bit
(both run the same kernels in the same order), on two calls in a row, the second smaller; the
device's free memory must not shrink across the calls; sizes beyond the scratch are refused."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle_dgemm

torch = pytest.importorskip("torch")
sx = pytest.importorskip("paper_1605_01078_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _first_call_setup():
    """The first call on a device resolves the scratch's device address (set-up); the checks
    of the device's free memory below start after it."""
    A, B, C = W.problem(70, 64, 64, 64, "uniform")
    sx.dgemm_noalloc(sx.to_device(A), sx.to_device(B), sx.to_device(C), 1.0, 1.0, 1, "ab")
    torch.cuda.synchronize()


def _pair(shape, seed, levels, variant, kind="uniform", alpha=0.75, beta=-1.25):
    m, n, k = shape
    A, B, C = W.problem(seed, m, n, k, kind)
    dA, dB = sx.to_device(A), sx.to_device(B)
    ref_c, got_c = sx.to_device(C), sx.to_device(C)
    sx.dgemm(dA, dB, ref_c, alpha, beta, levels, variant)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sx.dgemm_noalloc(dA, dB, got_c, alpha, beta, levels, variant)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return A, B, C, sx.to_host(ref_c), sx.to_host(got_c), free0 - free1


@pytest.mark.parametrize("levels,variant", [(0, "abc"), (1, "abc"), (2, "abc"), (1, "ab"),
                                            (2, "ab"), (1, "naive"), (2, "naive")])
def test_noalloc_matches_dgemm_two_calls(levels, variant):
    for shape, seed in (((1536, 1280, 1152), 71), ((301, 259, 270), 72)):
        print(f"case noalloc {shape} L={levels} {variant}", flush=True)
        A, B, C, ref, got, drop = _pair(shape, seed, levels, variant)
        assert np.array_equal(got, ref), shape
        assert drop < (16 << 20), drop
    # integer inputs: exact, so also equal to the oracle
    A, B, C = W.problem(73, 300, 260, 270, "integer")
    want = oracle_dgemm(A, B, C.copy(order="F"), 1.0, 1.0)
    dC = sx.to_device(C)
    sx.dgemm_noalloc(sx.to_device(A), sx.to_device(B), dC, 1.0, 1.0, levels, variant)
    torch.cuda.synchronize()
    assert np.array_equal(sx.to_host(dC), want)


def test_noalloc_allocates_nothing_where_dgemm_would():
    """AB at 3000^3 keeps 126 MB of temporaries: with the library-owned workspace released,
    strassen_dgemm_noalloc leaves the device's free memory as it was."""
    sx.release_workspace()
    shape = (3000, 3000, 3000)
    print(f"case noalloc free memory {shape}", flush=True)
    m, n, k = shape
    A, B, C = W.problem(74, m, n, k, "uniform")
    dA, dB, dC = sx.to_device(A), sx.to_device(B), sx.to_device(C)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sx.dgemm_noalloc(dA, dB, dC, 1.0, 1.0, 1, "ab")
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (16 << 20), free0 - free1
    got = sx.to_host(dC)
    ref_c = sx.to_device(C)
    sx.dgemm(dA, dB, ref_c, 1.0, 1.0, 1, "ab")
    torch.cuda.synchronize()
    assert np.array_equal(got, sx.to_host(ref_c))


def test_noalloc_abc_beyond_scratch_runs_workspace_free():
    """Ragged ABC whose block-padded copies exceed the scratch runs the workspace-free path
    (the general tile kernel): same bits as strassen_dgemm with its copies."""
    shape = (6001, 2999, 3001)   # copies of A, B, C: about 330 MB
    print(f"case noalloc abc beyond scratch {shape}", flush=True)
    m, n, k = shape
    assert sx.workspace_size(m, n, k, 1, "abc") > sx.NOALLOC_SCRATCH_BYTES
    A, B, C, ref, got, drop = _pair(shape, 75, 1, "abc")
    assert np.array_equal(got, ref)


def test_noalloc_refuses_ab_beyond_scratch():
    m, n, k = 5000, 5000, 64
    print(f"case noalloc refuse {(m, n, k)}", flush=True)
    assert sx.workspace_size(m, n, k, 1, "ab") > sx.NOALLOC_SCRATCH_BYTES
    A, B, C = W.problem(76, m, n, k, "uniform")
    dA, dB, dC = sx.to_device(A), sx.to_device(B), sx.to_device(C)
    with pytest.raises(sx.StrassenError) as ei:
        sx.dgemm_noalloc(dA, dB, dC, 1.0, 1.0, 1, "ab")
    assert ei.value.code == 2 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert np.array_equal(sx.to_host(dC), C)
