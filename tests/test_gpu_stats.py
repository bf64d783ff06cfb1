"""The step statistics reported by the kernels are exact.

delta of a step is max |W_{k+1} - W_k| over the whole state; every kernel
family forms it per element in FP64 (exact for FP32 and FP64 states) and
reduces it over lanes, waves and workgroups by max, which is exact in any
order.  So the delta that the library reports must equal, bit for bit, the
maximum of the difference of the two exported iterates.  A reduction that left
out lanes, rows or workgroups would report less.  Covered: the general tiles
(FP64, FP32, BF16), the large-tile FP32, BF16 and FP64 steps, the small-problem
batch kernel (through dpt_solve's delta history) and the CSR product.
"""
import numpy as np
import pytest

import workloads
from helpers import small_problem

pytestmark = pytest.mark.gpu

dpt = pytest.importorskip("paper_2002_12872_amd.dpt")


def delta_matches(theta, delta, precision, k=2):
    spec = dpt.ProblemSpec(theta, delta, 1.0, stream=0)
    h = dpt.dpt_init(spec, dpt.options(tol=1e-30, max_iter=1000, precision=precision))
    try:
        dpt.dpt_step(h, k)
        z0 = dpt.dpt_eigenvectors(h)
        reported = dpt.dpt_step(h, 1)
        z1 = dpt.dpt_eigenvectors(h)
    finally:
        dpt.dpt_destroy(h)
    expect = float(np.max(np.abs(z1 - z0)))
    assert expect > 0.0
    assert reported == expect, (reported, expect)


@pytest.mark.parametrize("n", [37, 300])
@pytest.mark.parametrize("precision", [dpt.DPT_FP64, dpt.DPT_FP32, dpt.DPT_BF16_FP32])
def test_general_tile_delta_is_exact(n, precision):
    theta, delta = small_problem(n, 3)
    delta_matches(theta, delta, precision)


@pytest.mark.parametrize("n, precision", [(4096, dpt.DPT_FP32), (2048, dpt.DPT_BF16_FP32),
                                          (2048, dpt.DPT_FP64)])
def test_large_tile_delta_is_exact(n, precision):
    theta, delta = workloads.dense_unsym(1, n=n)
    delta_matches(theta, delta.astype(np.float64) if precision == dpt.DPT_FP64 else delta, precision)


@pytest.mark.parametrize("precision", [dpt.DPT_FP64, dpt.DPT_FP32])
def test_small_batch_delta_history_is_exact(precision):
    """Order 64 runs dpt_solve in batches of steps in one workgroup: the delta of
    iteration k + 1 against the iterates after k and k + 1 iterations."""
    theta, delta = small_problem(64, 5, symmetric=True)
    k = 4
    z = {}
    for cap in (k, k + 1):
        h = dpt.dpt_init(dpt.ProblemSpec(theta, delta, 1.0, stream=0),
                         dpt.options(tol=1e-30, max_iter=cap, precision=precision))
        try:
            res = dpt.dpt_solve(h, history_cap=16)
            z[cap] = dpt.dpt_eigenvectors(h)
        finally:
            dpt.dpt_destroy(h)
        assert res["iters"] == cap
    assert res["history"][k] == float(np.max(np.abs(z[k + 1] - z[k])))


@pytest.mark.parametrize("precision", [dpt.DPT_FP64, dpt.DPT_FP32])
def test_sparse_delta_is_exact(precision):
    theta, ip, ix, v = workloads.sparse_sym(2, n=300, dtype=np.float64 if precision == dpt.DPT_FP64 else np.float32)
    delta_matches(theta, (ip, ix, v), precision)
