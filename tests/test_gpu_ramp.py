"""GPU parity of the coupling ramp (Supplement E): the k-th application of the
map uses lambda_k = lambda (1 - alpha^k) while alpha^k >= 2^-53, lambda after.

Compared with the oracle's ramp (itself pinned in test_oracle_extensions.py to
the 2x2 recurrence and to library eigenpairs where the autonomous map
diverges): fixed steps element by element (FP64 1e-12, FP32 by the FP32
one-step scale), full solves to the FP64 and FP32 targets, CSR and dominant
mode, and the rejections.
"""
import numpy as np
import pytest

import oracle
import workloads
from helpers import rel_eig_error, small_problem

pytestmark = pytest.mark.gpu

dpt = pytest.importorskip("paper_2002_12872_amd.dpt")

THETA4 = np.arange(4.0)
DELTA4 = np.array([[0.0, 0.4, -0.25, 1.15], [0.4, 0.0, 0.9, -1.05],
                   [-0.25, 0.9, 0.0, 0.4], [1.15, -1.05, 0.4, 0.0]])


def test_ramp_converges_where_the_autonomous_map_diverges():
    spec = dpt.ProblemSpec(THETA4, DELTA4, 0.75, stream=0)
    plain = dpt.dpt_solve(dpt.dpt_init(spec, dpt.options(tol=1e-13, max_iter=3000, precision=dpt.DPT_FP64)))
    assert plain["status"] == dpt.DPT_DIVERGED
    h = dpt.dpt_init(spec, dpt.options(tol=1e-13, max_iter=3000, precision=dpt.DPT_FP64, ramp_alpha=0.9))
    res = dpt.dpt_solve(h)
    ref = oracle.ramp(THETA4, DELTA4, 0.75, 0.9, max_iter=3000, tol=1e-13)
    assert res["status"] == dpt.DPT_OK and ref["status"] == oracle.OR_OK
    assert res["iters"] == ref["iters"]
    assert np.max(np.abs(dpt.dpt_eigenvectors(h) - ref["z"])) <= 1e-12
    assert np.max(np.abs(dpt.dpt_eigenvalues(h) - ref["e"])) <= 1e-12
    w = np.linalg.eigvalsh(np.diag(THETA4) + 0.75 * DELTA4)
    assert np.max(np.abs(dpt.dpt_eigenvalues(h) - w)) <= 1e-12


@pytest.mark.parametrize("n,sym", [(64, True), (300, False), (1100, True)])
def test_ramp_steps_match_oracle_fp64(n, sym):
    theta, delta = small_problem(n, 5, symmetric=sym)
    rows = workloads.sample_rows(n, 40)
    spec = dpt.ProblemSpec(theta, delta, 1.0, stream=0)
    h = dpt.dpt_init(spec, dpt.options(precision=dpt.DPT_FP64, ramp_alpha=0.7))
    for k in range(1, 5):
        dpt.dpt_step(h, 1)
        ref = oracle.ramp(theta, delta, 1.0, 0.7, rows=rows, max_iter=k, fixed_steps=True)
        z = dpt.dpt_eigenvectors(h)[rows]
        assert np.max(np.abs(z - ref["z"])) <= 1e-12 * max(1.0, np.abs(ref["z"]).max()), k
        assert rel_eig_error(dpt.dpt_eigenvalues(h)[rows], ref["e"], theta) <= 1e-12


@pytest.mark.parametrize("precision", [dpt.DPT_FP32, dpt.DPT_BF16_FP32])
def test_ramp_solve_reaches_the_fp32_target(precision):
    n = 1100
    theta, delta = small_problem(n, 6, symmetric=True)
    delta = delta.astype(np.float32)
    spec = dpt.ProblemSpec(theta, delta, 1.0, stream=0)
    h = dpt.dpt_init(spec, dpt.options(tol=1e-6, max_iter=200, precision=precision, ramp_alpha=0.5))
    res = dpt.dpt_solve(h)
    assert res["status"] == dpt.DPT_OK and res["iters"] > 53      # 0.5^k >= 2^-53 for k <= 53
    rows = workloads.sample_rows(n, 32)
    ref = oracle.iterate(theta, delta.astype(np.float64), 1.0, rows=rows, max_iter=200, tol=1e-14)
    assert rel_eig_error(dpt.dpt_eigenvalues(h)[rows], ref["e"], theta) <= 1e-5
    z = dpt.dpt_eigenvectors(h)[rows]
    assert np.max(np.abs(z - ref["z"])) / np.max(np.abs(ref["z"] - np.eye(n)[rows])) <= 1e-5


def test_ramp_csr_steps_and_dominant_mode_match_oracle():
    n = 2000
    theta, ip, ix, v = workloads.sparse_sym(3, n=n, dtype=np.float64)
    spec = dpt.ProblemSpec(theta, (ip, ix, v), 1.0, stream=0)
    rows = workloads.sample_rows(n, 32)
    h = dpt.dpt_init(spec, dpt.options(precision=dpt.DPT_FP64, ramp_alpha=0.6))
    dpt.dpt_step(h, 3)
    ref = oracle.ramp(theta, (ip, ix, v), 1.0, 0.6, rows=rows, max_iter=3, fixed_steps=True)
    assert np.max(np.abs(dpt.dpt_eigenvectors(h)[rows] - ref["z"])) <= 1e-12
    ev, vec, res = dpt.dpt_dominant(spec, dpt.options(tol=1e-13, max_iter=200, precision=dpt.DPT_FP64,
                                                      ramp_alpha=0.6))
    rd = oracle.ramp(theta, (ip, ix, v), 1.0, 0.6, rows=[n - 1], max_iter=200, tol=1e-13)
    assert res["status"] == dpt.DPT_OK and res["iters"] == rd["iters"] and res["iters"] > 70
    assert abs(ev - rd["e"][0]) <= 1e-12 * abs(rd["e"][0])
    assert np.max(np.abs(vec - rd["z"][0])) <= 1e-12


def test_ramp_rejections():
    theta, delta = small_problem(50, 1)
    spec = dpt.ProblemSpec(theta, delta.astype(np.float32), 1.0, stream=0)
    for alpha in (-0.1, 1.0, 1.5):
        with pytest.raises(dpt.DptError):
            dpt.dpt_init(spec, dpt.options(ramp_alpha=alpha))
    srv = dpt.dpt_serve_open(64 << 20, max_slots=4)
    with pytest.raises(dpt.DptError):
        dpt.dpt_serve_submit(srv, spec, dpt.options(precision=dpt.DPT_BF16_FP32, ramp_alpha=0.5))
    dpt.dpt_serve_close(srv)
