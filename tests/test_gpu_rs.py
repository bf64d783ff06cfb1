"""The Rayleigh-Schroedinger comparator on the GPU (eq. ARS-alpha, Supplement B)
and the D-PT vs RS comparison of Sec. II.F on the delta-potential.

Coefficients are compared with the oracle's recursion (``oracle.rs``, pinned in
test_oracle_pins.py by the O(lambda^(k+1)) containment, the explicit second
iterate and the second-order eigenvalues): order by order to 1e-12 of each
order's magnitude, FP64 on both sides, ragged and multi-tile orders, zero and
non-zero diagonals.  The comparison reproduces the paper's qualitative claims:
at lambda = 1.5 D-PT needs fewer iterations than RS needs orders for the same
eigenvalue accuracy, at lambda = 2.5 the RS partial sums diverge while D-PT
converges.
"""
import numpy as np
import pytest

import oracle
import workloads
from helpers import small_problem

pytestmark = pytest.mark.gpu

dpt = pytest.importorskip("paper_2002_12872_amd.dpt")


@pytest.mark.parametrize("n,sym,diag", [(37, True, False), (130, False, True), (300, True, True)])
def test_rs_coefficients_match_oracle(n, sym, diag):
    theta, delta = small_problem(n, 4, symmetric=sym, diag=diag)
    order = 8
    lam = 0.7
    eps, cmax, z = dpt.dpt_rs_series(dpt.ProblemSpec(theta, delta, lam, stream=0), order)
    ref_eps = oracle.rs_eigenvalue_coefficients(theta, delta, order)
    ref_a = oracle.rs_coefficients(theta, delta, order)
    for ell in range(1, order + 1):
        scale = max(np.abs(ref_eps[ell - 1]).max(), 1e-300)
        assert np.max(np.abs(eps[ell - 1] - ref_eps[ell - 1])) <= 1e-12 * scale, ell
        assert abs(cmax[ell - 1] - np.abs(ref_a[ell]).max()) <= 1e-12 * np.abs(ref_a[ell]).max(), ell
    ref_z = oracle.rs_partial_sum(theta, delta, lam, order)
    assert np.max(np.abs(z - ref_z)) <= 1e-12 * np.abs(ref_z).max()


def test_rs_device_problem_matches_host():
    import torch
    theta, delta = small_problem(200, 5, symmetric=True)
    h_eps, h_max, h_z = dpt.dpt_rs_series(dpt.ProblemSpec(theta, delta, 0.5, stream=0), 5)
    spec = dpt.ProblemSpec(torch.from_numpy(theta).cuda(), torch.from_numpy(delta).cuda(), 0.5)
    d_eps, d_max, d_z = dpt.dpt_rs_series(spec, 5)
    assert np.array_equal(h_eps, d_eps) and np.array_equal(h_max, d_max)
    assert np.array_equal(h_z, d_z.cpu().numpy())


def rs_eigenvalue_errors(eps, theta, lam, exact):
    """max relative eigenvalue error of E_RS^(k) for k = 1..order."""
    powers = lam ** np.arange(1, eps.shape[0] + 1)
    partial = theta[None, :] + np.cumsum(powers[:, None] * eps, axis=0)
    return np.max(np.abs(partial - exact[None, :]) / np.abs(exact)[None, :], axis=1)


def dpt_eigenvalue_errors(theta, delta, lam, steps, exact):
    h = dpt.dpt_init(dpt.ProblemSpec(theta, delta, lam, stream=0), dpt.options(precision=dpt.DPT_FP64))
    errs = []
    for _ in range(steps):
        dpt.dpt_step(h, 1)
        e = dpt.dpt_eigenvalues(h)
        errs.append(np.max(np.abs(e - exact) / np.abs(exact)))
    return np.array(errs)


def test_section_2f_dpt_beats_rs_at_lambda_1_5():
    theta, delta = workloads.delta_potential(100)
    lam = 1.5
    exact = np.linalg.eigvalsh(np.diag(theta) + lam * delta)   # rank-one positive: order kept
    eps, _, _ = dpt.dpt_rs_series(dpt.ProblemSpec(theta, delta, lam, stream=0), 120, want_z=False)
    rs = rs_eigenvalue_errors(eps, theta, lam, exact)
    dp = dpt_eigenvalue_errors(theta, delta, lam, 120, exact)
    target = 1e-8
    k_rs = int(np.argmax(rs < target)) + 1
    k_dpt = int(np.argmax(dp < target)) + 1
    assert rs.min() < target and dp.min() < target
    assert k_dpt < k_rs, (k_dpt, k_rs)


def test_section_2f_rs_diverges_at_lambda_2_5_while_dpt_converges():
    theta, delta = workloads.delta_potential(100)
    lam = 2.5
    exact = np.linalg.eigvalsh(np.diag(theta) + lam * delta)
    eps, cmax, _ = dpt.dpt_rs_series(dpt.ProblemSpec(theta, delta, lam, stream=0), 120, want_z=False)
    rs = rs_eigenvalue_errors(eps, theta, lam, exact)
    assert rs[-1] > 1.0 and rs[-1] > rs[60]          # growing: beyond the RS radius (about 2.2)
    h = dpt.dpt_init(dpt.ProblemSpec(theta, delta, lam, stream=0),
                     dpt.options(tol=1e-12, max_iter=1000, precision=dpt.DPT_FP64))
    res = dpt.dpt_solve(h)
    assert res["status"] == dpt.DPT_OK
    assert np.max(np.abs(dpt.dpt_eigenvalues(h) - exact) / np.abs(exact)) <= 1e-10


def test_rs_rejections():
    theta, delta = small_problem(20, 1)
    spec = dpt.ProblemSpec(theta, delta, 0.5, stream=0)
    for order in (0, 5000):
        with pytest.raises(dpt.DptError):
            dpt.dpt_rs_series(spec, order)
    th, ip, ix, v = workloads.sparse_sym(0, n=100)
    with pytest.raises(dpt.DptError):
        dpt.dpt_rs_series(dpt.ProblemSpec(th, (ip, ix, v), 0.5, stream=0), 3)
