"""The block-scaled FP8 product form (DPT_FP8_FP32, an experiment: no parity
target with the FP64 oracle beyond the FP32 refinement reaching its own).

The FP8 step is pinned against its definition written out here in float64:
both operands quantised to OCP E4M3 (1 sign, 4 exponent bits with bias 7,
3 mantissa bits, largest value 448, round to nearest even) with one E8M0
power-of-two scale 2^X per 32 consecutive values of a row, X the smallest
integer with max|v| <= 448 * 2^X; then the update of eq. (dyn) in FP32 terms.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from helpers import gap_matrix, rel_eig_error, small_problem

pytestmark = pytest.mark.gpu

dpt = pytest.importorskip("paper_2002_12872_amd.dpt")


def e4m3_round(y):
    """Round float64 values with |y| <= 448 to E4M3 (nearest even), as float64."""
    a = np.abs(y)
    mant, ex = np.frexp(a)                       # a = mant * 2^ex, mant in [0.5, 1)
    e = np.where(a > 0, ex - 1, 0)               # floor(log2 a)
    e = np.maximum(e, -6)                        # subnormals share the step 2^-9
    step = np.ldexp(1.0, (e - 3).astype(np.int64))
    return np.sign(y) * np.round(a / step) * step


def quantise_blocks(x32):
    """Dequantised value of each entry of a float32 (rows, cols) matrix after
    block-scaled E4M3 quantisation with 32-value blocks along the rows."""
    x = x32.astype(np.float64)
    rows, cols = x.shape
    xb = x.reshape(rows, cols // 32, 32)
    amax = np.max(np.abs(xb), axis=2)
    mant, ex = np.frexp(amax)
    xs = np.where(mant <= 0.875, ex - 9, ex - 8)
    xs = np.where(amax > 0, xs, -127).clip(-127, 127)
    scale = np.ldexp(1.0, xs.astype(np.int64))[:, :, None]
    q = e4m3_round(np.clip(xb / scale, -448.0, 448.0)) * scale
    return q.reshape(rows, cols)


def test_e4m3_rounding_helper():
    # the grid of E4M3 values around 1 (step 1/8), 16 (step 2), the top (448) and subnormals
    assert e4m3_round(np.array([1.0625]))[0] == 1.0       # tie -> even mantissa
    assert e4m3_round(np.array([1.1875]))[0] == 1.25
    assert e4m3_round(np.array([17.0]))[0] == 16.0
    assert e4m3_round(np.array([447.0]))[0] == 448.0
    assert e4m3_round(np.array([3 * 2.0 ** -10]))[0] == 2.0 ** -8
    # scales: 1024 = 0.5 * 2^11 -> 2^2, exact; 448 * 8 -> 2^3, exact; 1000 = 250 * 2^2 -> 256 * 2^2
    assert np.all(quantise_blocks(np.full((1, 32), 1024.0, np.float32)) == 1024.0)
    assert np.all(quantise_blocks(np.full((1, 32), 3584.0, np.float32)) == 3584.0)
    assert np.all(quantise_blocks(np.full((1, 32), 1000.0, np.float32)) == 1024.0)


def gpu_state(theta, delta32, lam, steps):
    spec = dpt.ProblemSpec(theta, delta32, lam, stream=0)
    h = dpt.dpt_init(spec, dpt.options(precision=dpt.DPT_FP8_FP32, max_iter=200))
    dpt.dpt_step(h, steps)
    z = dpt.dpt_eigenvectors(h)
    dpt.dpt_destroy(h)
    return z


@pytest.mark.parametrize("n", [1100, 2048])
def test_fp8_step_equals_block_scaled_operand_product(n):
    theta, delta = small_problem(n, 8, symmetric=False)
    delta32 = delta.astype(np.float32)
    lam = 0.9
    zk = gpu_state(theta, delta32, lam, 2)
    zk1 = gpu_state(theta, delta32, lam, 3)
    ld = 1280 if n == 1100 else 2048
    w = zk.copy()
    np.fill_diagonal(w, 0.0)
    wpad = np.zeros((ld, ld), np.float32)
    wpad[:n, :n] = w
    dpad = np.zeros((ld, ld), np.float32)
    dpad[:n, :n] = delta32
    wq = quantise_blocks(wpad)[:n, :n]
    dq = quantise_blocks(dpad)[:n, :n]
    d64 = delta32.astype(np.float64)
    c = d64.T + wq @ dq.T
    dvec = np.diag(d64) + np.sum(w * d64, axis=1)
    g = gap_matrix(theta)
    expect = lam * g * (c - dvec[:, None] * w)
    # The block-scaled FP8 MFMA does not accumulate to FP32 accuracy: against
    # the exact product of the dequantised operands its results deviate by up to
    # ~1.5e-4 of the magnitude sum (median ~1e-6) at K = 1280.  The bound allows
    # 2^-11 of the magnitude sum for the product and FP32 rounding for the rest;
    # a quantisation, scale or layout mistake moves terms by ~2^-4 relative and
    # still fails it.
    prod_mag = np.abs(wq) @ np.abs(dq).T
    mag = np.abs(c) + np.abs(dvec)[:, None] * np.abs(w)
    tol = (np.abs(lam * g) * (2.0 ** -11 * prod_mag + (8 + math.sqrt(n)) * 2.0 ** -24 * mag)
           + 4 * 2.0 ** -24 * np.abs(expect) + 1e-300)
    got = zk1 - np.eye(n)
    assert np.all(np.abs(got - expect) <= tol), float(np.max(np.abs(got - expect) / tol))


def test_fp8_solve_reaches_fp32_target():
    n = 1100
    theta, delta = small_problem(n, 5, symmetric=True)
    delta32 = delta.astype(np.float32)
    spec = dpt.ProblemSpec(theta, delta32, 1.0, stream=0)
    h = dpt.dpt_init(spec, dpt.options(tol=1e-6, max_iter=100, precision=dpt.DPT_FP8_FP32))
    res = dpt.dpt_solve(h)
    e = dpt.dpt_eigenvalues(h)
    z = dpt.dpt_eigenvectors(h)
    assert res["status"] == dpt.DPT_OK
    assert res["iters_bf16"] >= 1 and res["iters_fp32"] >= 1
    rows = workloads.sample_rows(n, 64)
    ref = oracle.iterate(theta, delta32.astype(np.float64), 1.0, rows=rows, max_iter=200, tol=1e-14)
    assert rel_eig_error(e[rows], ref["e"], theta) <= 1e-5
    assert np.max(np.abs(z[rows] - ref["z"])) / np.max(np.abs(ref["z"] - np.eye(n)[rows])) <= 1e-5


def test_fp8_only_for_large_dense_problems():
    theta, delta = small_problem(300, 1, symmetric=True)
    with pytest.raises(dpt.DptError) as ei:
        dpt.dpt_init(dpt.ProblemSpec(theta, delta.astype(np.float32), 1.0, stream=0),
                     dpt.options(precision=dpt.DPT_FP8_FP32))
    assert ei.value.code == dpt.DPT_EINVAL
    th, ip, ix, v = workloads.sparse_sym(0, n=2048)
    with pytest.raises(dpt.DptError) as ei:
        dpt.dpt_init(dpt.ProblemSpec(th, (ip, ix, v), 1.0, stream=0), dpt.options(precision=dpt.DPT_FP8_FP32))
    assert ei.value.code == dpt.DPT_EINVAL
