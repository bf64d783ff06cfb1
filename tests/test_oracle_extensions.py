"""Pins of the oracle's domain extensions (Sec. III homotopy, Supplement E ramp).

Each extension is checked against what the mathematics fixes independently of
the oracle: the closed-form eigenpairs of the 2x2 example (eq. 2by2) at
couplings where the plain iteration cycles or diverges, library eigensolvers on
the delta-potential beyond the plain iteration's radius (Sec. II.F) and on an
unsymmetric matrix, and the 2x2 recurrence x_k = lambda_k (x_{k-1}^2 - 1) with a
per-step coupling.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import OR_DIVERGED, OR_NOT_CONVERGED, OR_OK


def two_by_two_eigenpairs(lam):
    """M = [[0, lam], [lam, 1]]: E_0 < E_1, z_0 = (1, E_0/lam), z_1 = (lam/E_1, 1)."""
    r = math.sqrt(1 + 4 * lam * lam)
    e0, e1 = (1 - r) / 2, (1 + r) / 2
    return np.array([e0, e1]), np.array([[1.0, e0 / lam], [lam / e1, 1.0]])


# ------------------------------------------------------------------ homotopy
@pytest.mark.parametrize("lam,stages", [(0.9, 2), (0.9, 8), (3.0, 6), (10.0, 16), (-3.0, 6)])
def test_homotopy_reaches_the_2x2_closed_form_outside_the_domain(lam, stages):
    theta, delta = workloads.two_by_two()
    plain = oracle.iterate(theta, delta, lam, max_iter=500, tol=1e-14)
    assert plain["status"] in (OR_NOT_CONVERGED, OR_DIVERGED)     # |lam| > sqrt(3)/2
    r = oracle.homotopy(theta, delta, lam, stages)
    e, z = two_by_two_eigenpairs(lam)
    assert r["status"] == OR_OK and len(r["iters"]) == stages
    assert np.max(np.abs(r["e"] - e)) <= 1e-13 * max(1.0, abs(lam))
    assert np.max(np.abs(r["z"] - z)) <= 1e-13


def test_homotopy_with_one_stage_is_the_plain_iteration():
    theta, delta = workloads.dense_sym_small(1)
    a = oracle.iterate(theta, delta, 1.0, max_iter=200, tol=1e-13)
    b = oracle.homotopy(theta, delta, 1.0, 1, tol=1e-13, max_iter=200)
    assert np.array_equal(a["e"], b["e"]) and np.array_equal(a["z"], b["z"])


@pytest.mark.parametrize("lam,stages", [(4.0, 2), (8.0, 4)])
def test_homotopy_beyond_the_delta_potential_radius(lam, stages):
    """Sec. II.F: the plain iteration's radius is about 2.9 for this problem."""
    theta, delta = workloads.delta_potential(100)
    assert oracle.iterate(theta, delta, lam, max_iter=500, tol=1e-13)["status"] != OR_OK
    r = oracle.homotopy(theta, delta, lam, stages)
    assert r["status"] == OR_OK
    m = np.diag(theta) + lam * delta
    w, v = np.linalg.eigh(m)
    # a rank-one positive perturbation keeps the order of the levels
    assert np.max(np.abs(r["e"] - w)) <= 1e-12 * w.max()
    vz = (v / np.diag(v)[None, :]).T
    assert np.max(np.abs(r["z"] - vz)) <= 1e-10
    res, _, _ = oracle.residual(theta, delta, lam, r["z"], r["e"])
    assert res.max() <= 1e-11 * w.max()


def test_homotopy_unsymmetric():
    """A real spectrum (checked) that the plain iteration does not reach."""
    rng = np.random.default_rng(13)
    n = 40
    theta = np.arange(n, dtype=np.float64)
    delta = rng.normal(0.0, 1.0, (n, n))
    np.fill_diagonal(delta, 0.0)
    lam = 0.3
    assert oracle.iterate(theta, delta, lam, max_iter=500, tol=1e-13)["status"] != OR_OK
    r = oracle.homotopy(theta, delta, lam, 4)
    assert r["status"] == OR_OK
    w, v = np.linalg.eig(np.diag(theta) + lam * delta)
    assert np.max(np.abs(w.imag)) == 0.0
    w, v = w.real, v.real
    # one-to-one pairing with the library's eigenpairs (eigenvalues >= 0.1 apart)
    j = np.array([int(np.argmin(np.abs(w - x))) for x in r["e"]])
    assert sorted(j) == list(range(n)) and np.min(np.diff(np.sort(w))) > 0.1
    assert np.max(np.abs(r["e"] - w[j])) <= 1e-11 * np.abs(w).max()
    zlib = (v[:, j] / v[np.arange(n), j][None, :]).T      # eigenvector of E_n, chart z_n[n] = 1
    assert np.max(np.abs(r["z"] - zlib)) <= 1e-9


# ------------------------------------------------------------------ ramp
def test_ramp_follows_the_2x2_recurrence_with_per_step_coupling():
    """Row 0 of the 2x2 iterate is (1, x_k) with x_k = lambda_k (x_{k-1}^2 - 1)."""
    theta, delta = workloads.two_by_two()
    lam, alpha = 0.6, 0.7
    x, ak = 0.0, 1.0
    for k in range(1, 30):
        ak *= alpha
        lk = lam * (1 - ak) if ak >= 2.0 ** -53 else lam
        x = lk * (x * x - 1)
        r = oracle.ramp(theta, delta, lam, alpha, rows=[0], max_iter=k, fixed_steps=True)
        assert abs(r["z"][0, 1] - x) <= 1e-15, k


def test_ramp_converges_where_the_autonomous_map_diverges():
    """theta = (0, 1, 2, 3), lambda = 0.75: every eigenvalue is real and simple,
    but the autonomous iteration from the identity leaves the basin and diverges;
    the ramped iteration follows the fixed point from small couplings and ends on
    the eigenpairs continued from e_n."""
    theta = np.arange(4.0)
    delta = np.array([[0.0, 0.4, -0.25, 1.15], [0.4, 0.0, 0.9, -1.05],
                      [-0.25, 0.9, 0.0, 0.4], [1.15, -1.05, 0.4, 0.0]])
    lam = 0.75
    assert oracle.iterate(theta, delta, lam, max_iter=3000, tol=1e-13)["status"] == OR_DIVERGED
    r = oracle.ramp(theta, delta, lam, 0.9, max_iter=3000, tol=1e-13)
    assert r["status"] == OR_OK
    assert r["iters"] > 342              # the ramp itself: 0.9^k >= 2^-53 for k <= 342
    w, v = np.linalg.eigh(np.diag(theta) + lam * delta)
    assert np.max(np.abs(r["e"] - w)) <= 1e-12
    assert np.max(np.abs(r["z"] - (v / np.diag(v)[None, :]).T)) <= 1e-10


def test_ramp_ends_on_the_autonomous_fixed_point():
    theta, delta = workloads.dense_sym_small(2)
    a = oracle.iterate(theta, delta, 1.0, max_iter=500, tol=1e-13)
    b = oracle.ramp(theta, delta, 1.0, 0.5, max_iter=500, tol=1e-13)
    assert a["status"] == b["status"] == OR_OK and b["iters"] > 53
    assert np.max(np.abs(a["z"] - b["z"])) <= 1e-12
    assert np.max(np.abs(a["e"] - b["e"])) <= 1e-12 * 64


def test_ramp_rejects_alpha_outside_the_unit_interval():
    theta, delta = workloads.two_by_two()
    for alpha in (-0.1, 1.0, 2.0):
        with pytest.raises(ValueError):
            oracle.ramp(theta, delta, 0.5, alpha)


# ------------------------------------------------------------------ per-row stop
def test_per_row_stop_on_two_independent_2x2_blocks():
    """theta = (0, g1, 10, 10 + g2), Delta block-diagonal with off-diagonal b1, b2:
    row 0 of each block evolves as (1, x_k) with x_k = c (x_{k-1}^2 - 1), c = lambda b / g
    (row 1 as (-x_k, 1)), so each pair of rows freezes on the first step with
    |x_k - x_{k-1}| < tol, which differs between the blocks."""
    g1, b1, g2, b2, lam, tol = 1.0, 0.2, 2.0, 1.2, 1.0, 1e-12
    theta = np.array([0.0, g1, 10.0, 10.0 + g2])
    delta = np.zeros((4, 4))
    delta[0, 1] = delta[1, 0] = b1
    delta[2, 3] = delta[3, 2] = b2
    r = oracle.iterate(theta, delta, lam, max_iter=200, tol=tol, per_row=True)
    assert r["status"] == OR_OK
    expect_steps, expect_x = [], []
    for c in (lam * b1 / g1, lam * b2 / g2):
        x, k = 0.0, 0
        while True:
            xn = c * (x * x - 1)
            k += 1
            done = abs(xn - x) < tol
            x = xn
            if done:
                break
        expect_steps += [k, k]
        expect_x.append(x)
    assert list(r["row_iters"]) == expect_steps and expect_steps[0] != expect_steps[2]
    assert r["iters"] == max(expect_steps)
    assert abs(r["z"][0, 1] - expect_x[0]) <= 1e-15 and abs(r["z"][1, 0] + expect_x[0]) <= 1e-15
    assert abs(r["z"][2, 3] - expect_x[1]) <= 1e-15 and abs(r["z"][3, 2] + expect_x[1]) <= 1e-15
    # without the per-row stop every row runs to the slowest block's step
    s = oracle.iterate(theta, delta, lam, max_iter=200, tol=tol)
    assert s["iters"] == max(expect_steps)
