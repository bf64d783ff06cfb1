"""Warm start and resume (Sec. II.H, last paragraph: refining approximate
eigenvectors; the iterate is the whole state of the method, eq. dyn).

* Resume: k1 steps, export the iterate, start a new handle from it and take k2
  more steps: the result equals k1 + k2 uninterrupted steps bit for bit (dense
  and CSR, FP32 and FP64), and an FP64 solve resumed after a few steps stops on
  the same step with the same result.
* Refinement: eigenvectors accurate to ~1 % (the converged oracle rows times
  1 + 0.01 noise) converge to the oracle's fixed point, dense and CSR.
"""
import numpy as np
import pytest

import oracle
import workloads
from helpers import rel_eig_error, small_problem

pytestmark = pytest.mark.gpu

dpt = pytest.importorskip("paper_2002_12872_amd.dpt")


def make(kind, precision, n):
    dtype = np.float64 if precision == dpt.DPT_FP64 else np.float32
    if kind == "dense":
        theta, delta = small_problem(n, 21, symmetric=False)
        return theta, delta.astype(dtype)
    theta, ip, ix, v = workloads.sparse_sym(21, n=n, dtype=dtype)
    return theta, (ip, ix, v)


def z_dtype(precision):
    return np.float64 if precision == dpt.DPT_FP64 else np.float32


@pytest.mark.parametrize("kind,n", [("dense", 300), ("dense", 1100), ("csr", 1000)])
@pytest.mark.parametrize("precision", [dpt.DPT_FP64, dpt.DPT_FP32])
def test_resume_equals_uninterrupted_steps(kind, n, precision):
    theta, delta = make(kind, precision, n)
    spec = dpt.ProblemSpec(theta, delta, 1.0, stream=0)
    opts = dpt.options(precision=precision)
    full = dpt.dpt_init(spec, opts)
    dpt.dpt_step(full, 5)
    z_full = dpt.dpt_eigenvectors(full, dtype=z_dtype(precision))
    e_full = dpt.dpt_eigenvalues(full)
    first = dpt.dpt_init(spec, opts)
    dpt.dpt_step(first, 2)
    z_mid = dpt.dpt_eigenvectors(first, dtype=z_dtype(precision))
    second = dpt.dpt_init(spec, opts, z_mid)
    dpt.dpt_step(second, 3)
    assert np.array_equal(dpt.dpt_eigenvectors(second, dtype=z_dtype(precision)), z_full)
    assert np.array_equal(dpt.dpt_eigenvalues(second), e_full)


@pytest.mark.parametrize("kind,n", [("dense", 257), ("csr", 2000)])
def test_resumed_fp64_solve_stops_on_the_same_step(kind, n):
    theta, delta = make(kind, dpt.DPT_FP64, n)
    spec = dpt.ProblemSpec(theta, delta, 1.0, stream=0)
    opts = dpt.options(tol=1e-13, max_iter=100, precision=dpt.DPT_FP64)
    full = dpt.dpt_init(spec, opts)
    r_full = dpt.dpt_solve(full)
    first = dpt.dpt_init(spec, opts)
    dpt.dpt_step(first, 3)
    second = dpt.dpt_init(spec, opts, dpt.dpt_eigenvectors(first))
    r_second = dpt.dpt_solve(second)
    assert r_full["status"] == r_second["status"] == dpt.DPT_OK
    assert r_second["iters"] + 3 == r_full["iters"]
    assert np.array_equal(dpt.dpt_eigenvectors(second), dpt.dpt_eigenvectors(full))
    assert np.array_equal(dpt.dpt_eigenvalues(second), dpt.dpt_eigenvalues(full))


@pytest.mark.parametrize("mem", ["host", "device"])
def test_csr_warm_start_refines_approximate_eigenvectors(mem):
    n = 2000
    theta, (ip, ix, v) = make("csr", dpt.DPT_FP64, n)
    ref = oracle.iterate(theta, (ip, ix, v), 1.0, max_iter=100, tol=1e-15)
    rng = np.random.default_rng(3)
    z0 = ref["z"] * (1 + 0.01 * rng.standard_normal(ref["z"].shape))   # ~1 % accurate
    arrs = (theta, (ip, ix, v), z0)
    if mem == "device":
        import torch
        arrs = (torch.from_numpy(theta).cuda(),
                tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (ip, ix, v)),
                torch.from_numpy(z0).cuda())
    spec = dpt.ProblemSpec(arrs[0], arrs[1], 1.0, stream=None if mem == "device" else 0)
    h = dpt.dpt_init(spec, dpt.options(tol=1e-13, max_iter=100, precision=dpt.DPT_FP64), arrs[2])
    res = dpt.dpt_solve(h)
    assert res["status"] == dpt.DPT_OK
    z = dpt.dpt_eigenvectors(h)
    assert np.max(np.abs(z - ref["z"])) <= 1e-11
    assert rel_eig_error(dpt.dpt_eigenvalues(h), ref["e"], theta) <= 1e-11
    # the start is a genuine warm start: fewer steps than from the identity
    cold = dpt.dpt_solve(dpt.dpt_init(dpt.ProblemSpec(theta, (ip, ix, v), 1.0, stream=0),
                                      dpt.options(tol=1e-13, max_iter=100, precision=dpt.DPT_FP64)))
    assert res["iters"] <= cold["iters"]
