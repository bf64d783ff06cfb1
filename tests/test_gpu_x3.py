"""The split-BF16 sweep form (DPT_BF16_X3, an experiment).

BF16 steps as in DPT_BF16_FP32, then FP32-grade sweeps whose product is formed
on BF16 matrix cores from split operands: x = h + l with h = bf16(x) and
l = bf16(x - h) (round to nearest even), and C = D^T + Wh Dh^T + Wl Dh^T + Wh Dl^T
with FP32 accumulation over the three products (only the l x l term is left
out).  The sweep is pinned against that definition written out here in float64
from a state exported just before it, and against the exact product, which it
may miss by the dropped terms: |Wl||Dl| + |W - Wh - Wl||D| + |W||D - Dh - Dl|,
at most 3 * 2^-18 of the magnitude sum.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from helpers import gap_matrix, rel_eig_error, small_problem

pytestmark = pytest.mark.gpu

dpt = pytest.importorskip("paper_2002_12872_amd.dpt")


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split(x32):
    h = bf16_round(x32)
    l = bf16_round((x32 - h).astype(np.float32))
    return h.astype(np.float64), l.astype(np.float64)


def state(theta, delta32, lam, max_iter):
    h = dpt.dpt_init(dpt.ProblemSpec(theta, delta32, lam, stream=0),
                     dpt.options(tol=1e-6, max_iter=max_iter, precision=dpt.DPT_BF16_X3))
    res = dpt.dpt_solve(h)
    z = dpt.dpt_eigenvectors(h)
    dpt.dpt_destroy(h)
    return res, z


@pytest.mark.parametrize("n", [1100, 2048])
def test_split_sweep_equals_split_product_definition(n):
    theta, delta = small_problem(n, 21, symmetric=(n == 2048))
    delta32 = delta.astype(np.float32)
    lam = 0.9
    full, _ = state(theta, delta32, lam, 200)
    nb = full["iters_bf16"]
    assert full["status"] == dpt.DPT_OK and nb >= 2 and full["iters_fp32"] >= 1
    r0, z0 = state(theta, delta32, lam, nb)        # the BF16 phase only
    r1, z1 = state(theta, delta32, lam, nb + 1)    # and one split sweep
    assert r0["iters_fp32"] == 0 and r1["iters_fp32"] == 1
    w = (z0 - np.eye(n)).astype(np.float32)
    wh, wl = split(w)
    dh, dl = split(delta32)
    d64 = delta32.astype(np.float64)
    prod = wh @ dh.T + wl @ dh.T + wh @ dl.T
    c = d64.T + prod
    w64 = w.astype(np.float64)
    dvec = np.diag(d64) + np.sum(w64 * d64, axis=1)
    g = gap_matrix(theta)
    expect = lam * g * (c - dvec[:, None] * w64)
    got = z1 - np.eye(n)
    # FP32 accumulation over K = 3 ld terms and the FP32 epilogue
    ld = 1280 if n == 1100 else 2048
    k = 8 + math.sqrt(3 * ld)
    prod_mag = np.abs(wh) @ np.abs(dh).T + np.abs(wl) @ np.abs(dh).T + np.abs(wh) @ np.abs(dl).T
    mag = np.abs(c) + np.abs(dvec)[:, None] * np.abs(w64)
    tol = (np.abs(lam * g) * 1.5 * (k * 2.0 ** -24 * (prod_mag + mag)) + 4 * 2.0 ** -24 * np.abs(expect) + 1e-300)
    assert np.all(np.abs(got - expect) <= tol), float(np.max(np.abs(got - expect) / tol))
    # against the exact-operand product: the dropped terms on top
    exact = lam * g * (d64.T + w64 @ d64.T - dvec[:, None] * w64)
    exact_mag = np.abs(w64) @ np.abs(d64).T
    tol2 = tol + np.abs(lam * g) * 3 * 2.0 ** -18 * exact_mag
    assert np.all(np.abs(got - exact) <= tol2), float(np.max(np.abs(got - exact) / tol2))


def test_split_solve_reaches_fp32_target():
    n = 2048
    theta, delta = small_problem(n, 5, symmetric=True)
    delta32 = delta.astype(np.float32)
    h = dpt.dpt_init(dpt.ProblemSpec(theta, delta32, 1.0, stream=0),
                     dpt.options(tol=1e-6, max_iter=100, precision=dpt.DPT_BF16_X3))
    res = dpt.dpt_solve(h)
    e = dpt.dpt_eigenvalues(h)
    z = dpt.dpt_eigenvectors(h)
    dpt.dpt_destroy(h)
    assert res["status"] == dpt.DPT_OK and res["iters_bf16"] >= 1 and res["iters_fp32"] >= 1
    rows = workloads.sample_rows(n, 64)
    ref = oracle.iterate(theta, delta32.astype(np.float64), 1.0, rows=rows, max_iter=200, tol=1e-14)
    assert rel_eig_error(e[rows], ref["e"], theta) <= 1e-5
    assert np.max(np.abs(z[rows] - ref["z"])) / np.max(np.abs(ref["z"] - np.eye(n)[rows])) <= 1e-5


def test_split_form_only_for_large_dense_problems():
    theta, delta = small_problem(300, 1, symmetric=True)
    with pytest.raises(dpt.DptError) as ei:
        dpt.dpt_init(dpt.ProblemSpec(theta, delta.astype(np.float32), 1.0, stream=0),
                     dpt.options(precision=dpt.DPT_BF16_X3))
    assert ei.value.code == dpt.DPT_EINVAL
    th, ip, ix, v = workloads.sparse_sym(0, n=2048)
    with pytest.raises(dpt.DptError) as ei:
        dpt.dpt_init(dpt.ProblemSpec(th, (ip, ix, v), 1.0, stream=0), dpt.options(precision=dpt.DPT_BF16_X3))
    assert ei.value.code == dpt.DPT_EINVAL
