"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: printed
closed forms (eq. 2by2), printed polynomials (Supplement E), textbook/library
eigensolvers, the trace invariant, the Rayleigh-Schroedinger recursion
(eq. ARS-alpha, Supplement C), and properties stated in Secs. II.C and II.F.
The mutation tests at the end compile the oracle with a planted mistake and
show that the pins reject it.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle import OR_DIVERGED, OR_NOT_CONVERGED, OR_OK

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers
def quad_map_iterates(lam, k):
    """f(x) = lam (x^2 - 1) iterated k times from 0 (eq. 2by2 closed form)."""
    x = 0.0
    out = []
    for _ in range(k):
        x = lam * (x * x - 1.0)
        out.append(x)
    return out


def load_multiplier_polynomials():
    terms = {}
    with open(os.path.join(GOLDEN, "si_3x3_multiplier_polynomials.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            n, a, b, c = line.split()
            terms.setdefault(int(n), []).append((int(a), int(b), float(c)))
    return terms


def poly_residual(terms, lam, mu):
    """|P(lam, mu)| / sum |terms|  (scale-free)."""
    vals = [c * lam ** a * mu ** b for a, b, c in terms]
    return abs(sum(vals)) / sum(abs(v) for v in vals)


def chart_multipliers(it, theta, delta, lam, n, z, h=1e-6):
    """Eigenvalues of the Jacobian of F_n in the chart coordinates m != n,
    by central differences of one oracle step."""
    free = [m for m in range(len(theta)) if m != n]
    jac = np.zeros((len(free), len(free)))
    for col, k in enumerate(free):
        zp, zm = z.copy(), z.copy()
        zp[k] += h
        zm[k] -= h
        fp = it(theta, delta, lam, rows=[n], z0=zp, max_iter=1, fixed_steps=True)["z"][0]
        fm = it(theta, delta, lam, rows=[n], z0=zm, max_iter=1, fixed_steps=True)["z"][0]
        jac[:, col] = (fp[free] - fm[free]) / (2 * h)
    return np.linalg.eigvals(jac)


def eig_rows_normalised(mat):
    """Right eigenvectors of ``mat`` as rows scaled so that component n = 1,
    matched to index n by the largest component (continuation from e_n)."""
    w, v = np.linalg.eig(mat)
    n = mat.shape[0]
    rows = np.zeros((n, n), dtype=v.dtype)
    vals = np.zeros(n, dtype=w.dtype)
    for j in range(n):
        k = int(np.argmax(np.abs(v[:, j])))
        rows[k] = v[:, j] / v[k, j]
        vals[k] = w[j]
    return vals, rows


# ---------------------------------------------------------------- 2x2, eq. (2by2)
@pytest.mark.parametrize("lam", [0.1, 0.3, -0.45, 0.8])
def test_two_by_two_every_iterate_matches_closed_form(lam):
    theta, delta = workloads.two_by_two()
    xs = quad_map_iterates(lam, 12)
    for k in range(1, 13):
        r = oracle.iterate(theta, delta, lam, max_iter=k, fixed_steps=True)
        z = r["z"]
        assert z[0, 0] == 1.0 and z[1, 1] == 1.0
        assert abs(z[0, 1] - xs[k - 1]) <= 1e-15
        assert abs(z[1, 0] + xs[k - 1]) <= 1e-15


@pytest.mark.parametrize("lam", [0.1, 0.3, -0.6, 0.7])
def test_two_by_two_eigenvalues_closed_form(lam):
    theta, delta = workloads.two_by_two()
    r = oracle.iterate(theta, delta, lam, max_iter=5000, tol=1e-15)
    assert r["status"] == OR_OK
    root = math.sqrt(1 + 4 * lam * lam)
    assert abs(r["e"][0] - (1 - root) / 2) <= 1e-14
    assert abs(r["e"][1] - (1 + root) / 2) <= 1e-14


def test_two_by_two_convergence_rate():
    # |f^k(0) - x*| ~ |1 - sqrt(1 + 4 lam^2)|^k  (Sec. II.E)
    lam = 0.3
    theta, delta = workloads.two_by_two()
    xstar = (1 - math.sqrt(1 + 4 * lam * lam)) / 2 / lam
    errs = []
    for k in (8, 9):
        z = oracle.iterate(theta, delta, lam, max_iter=k, fixed_steps=True)["z"]
        errs.append(abs(z[0, 1] - xstar))
    ratio = errs[1] / errs[0]
    assert abs(ratio - abs(1 - math.sqrt(1 + 4 * lam * lam))) < 1e-3


def test_two_by_two_dynamics_outside_domain():
    theta, delta = workloads.two_by_two()
    # flip bifurcation at sqrt(3)/2: lam = 0.9 settles on a 2-cycle
    r = oracle.iterate(theta, delta, 0.9, max_iter=400, tol=1e-14)
    assert r["status"] == OR_NOT_CONVERGED
    xs = quad_map_iterates(0.9, 400)
    assert abs(xs[-1] - xs[-3]) < 1e-12 and abs(xs[-1] - xs[-2]) > 0.1
    # far outside: divergence to infinity
    r = oracle.iterate(theta, delta, 3.0, max_iter=100, tol=1e-14)
    assert r["status"] == OR_DIVERGED
    # just inside the domain: slow but convergent
    r = oracle.iterate(theta, delta, 0.85, max_iter=20000, tol=1e-13)
    assert r["status"] == OR_OK


# ---------------------------------------------------------------- 3x3, Supplement E
@pytest.mark.parametrize("lam", [0.1, 0.25, -0.3])
@pytest.mark.parametrize("n", [0, 1, 2])
def test_three_by_three_multipliers_are_roots_of_printed_polynomials(lam, n):
    theta, delta = workloads.three_by_three()
    terms = load_multiplier_polynomials()[n + 1]
    r = oracle.iterate(theta, delta, lam, rows=[n], max_iter=5000, tol=1e-15)
    assert r["status"] == OR_OK
    mus = chart_multipliers(oracle.iterate, theta, delta, lam, n, r["z"][0])
    assert len(mus) == 2
    for mu in mus:
        assert abs(mu) < 1.0                      # attracting fixed point
        assert poly_residual(terms, lam, mu) < 1e-8


def test_three_by_three_transcription_special_points():
    # the mu^6 coefficient vanishes where a multiplier escapes to infinity:
    # lambda ~ 0.45 (n=1), 0.56 (n=2), 1.2 (n=3)
    terms = load_multiplier_polynomials()
    expect = {1: 0.45, 2: 0.56, 3: 1.2}
    for n, lam_text in expect.items():
        c = {a: coef for a, b, coef in terms[n] if b == 6}
        root = -c[0] / c[1]
        assert abs(root - lam_text) < 0.01


# ---------------------------------------------------------------- eigensolver pins
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_symmetric_against_hand_written_jacobi(seed):
    theta, delta = workloads.dense_sym_small(seed)
    r = oracle.iterate(theta, delta, 1.0, max_iter=200, tol=1e-12)
    assert r["status"] == OR_OK and r["iters"] < 40
    m = np.diag(theta) + delta
    w, v = oracle.jacobi_eigh(m)
    scale = np.abs(theta).max()
    for n in range(len(theta)):
        j = int(np.argmax(np.abs(v[n, :])))       # eigenvector continued from e_n
        assert abs(r["e"][n] - w[j]) <= 1e-12 * scale
        vec = v[:, j] / v[n, j]
        assert np.max(np.abs(r["z"][n] - vec)) <= 1e-10
    res, mz, _ = oracle.residual(theta, delta, 1.0, r["z"], r["e"])
    assert res.max() <= 1e-12 * scale


def test_jacobi_against_library_eigh():
    theta, delta = workloads.dense_sym_small(5, n=40)
    m = np.diag(theta) + delta
    w, v = oracle.jacobi_eigh(m)
    assert np.allclose(np.sort(w), np.linalg.eigvalsh(m), atol=1e-12, rtol=0)
    assert np.allclose(v.T @ v, np.eye(40), atol=1e-12)
    assert np.allclose(m @ v, v * w, atol=1e-12)


@pytest.mark.parametrize("lam", [1.0, 0.7, -1.3])
def test_unsymmetric_against_library_eig(lam):
    theta, delta = workloads.dense_unsym(0, n=96)
    delta = delta.astype(np.float64)
    r = oracle.iterate(theta, delta, lam, max_iter=300, tol=1e-14)
    assert r["status"] == OR_OK
    vals, rows = eig_rows_normalised(np.diag(theta) + lam * delta)
    assert np.max(np.abs(r["e"] - vals.real)) <= 1e-11
    assert np.max(np.abs(vals.imag)) == 0.0
    assert np.max(np.abs(r["z"] - rows.real)) <= 1e-11
    res, _, _ = oracle.residual(theta, delta, lam, r["z"], r["e"])
    assert res.max() <= 1e-11


def test_nonzero_diagonal_against_library_eig():
    rng = np.random.default_rng(11)
    n = 50
    theta = np.arange(n) * 1.0 + rng.uniform(0, 0.3, n)
    delta = rng.normal(0, 0.05, (n, n))            # keeps its diagonal
    r = oracle.iterate(theta, delta, 1.0, max_iter=300, tol=1e-14)
    assert r["status"] == OR_OK
    vals, rows = eig_rows_normalised(np.diag(theta) + delta)
    assert np.max(np.abs(r["e"] - vals.real)) <= 1e-11
    assert np.max(np.abs(r["z"] - rows.real)) <= 1e-11


# ---------------------------------------------------------------- invariants
def test_trace_exact_after_first_iterate_and_at_fixed_point():
    theta, delta = workloads.dense_unsym(3, n=200)
    delta = delta.astype(np.float64)
    lam = 0.8
    r1 = oracle.iterate(theta, delta, lam, max_iter=1, fixed_steps=True)
    # zero diagonal: sum_n (A_1 Delta')_nn = lam sum G_nk Delta_kn Delta_nk = 0 (G antisymmetric)
    assert abs(r1["e"].sum() - theta.sum()) <= 1e-9
    r2 = oracle.iterate(theta, delta, lam, max_iter=2, fixed_steps=True)
    assert abs(r2["e"].sum() - theta.sum()) > 1e-9          # not exact at k = 2
    r = oracle.iterate(theta, delta, lam, max_iter=300, tol=1e-14)
    assert r["status"] == OR_OK
    assert abs(r["e"].sum() - theta.sum()) <= 1e-9
    # with a diagonal: sum E = sum theta + lam tr(Delta)
    delta2 = delta + np.diag(np.linspace(-0.1, 0.1, 200))
    r = oracle.iterate(theta, delta2, lam, max_iter=300, tol=1e-14)
    assert abs(r["e"].sum() - (theta.sum() + lam * np.trace(delta2))) <= 1e-9


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_contains_rayleigh_schroedinger_to_order_k(k):
    # A_D^(k) = A_RS^(k) + O(lam^(k+1))  (Sec. II.D, Supplement C)
    theta, delta = workloads.dense_unsym(1, n=14)
    delta = delta.astype(np.float64) * 10.0
    errs = []
    for lam in (0.02, 0.01, 0.005):
        ad = oracle.iterate(theta, delta, lam, max_iter=k, fixed_steps=True)["z"]
        errs.append(np.max(np.abs(ad - oracle.rs_partial_sum(theta, delta, lam, k))))
    if k == 1:
        assert max(errs) <= 1e-16
        return
    for a, b in zip(errs, errs[1:]):
        assert abs(a / b - 2 ** (k + 1)) < 0.05 * 2 ** (k + 1)


def test_second_iterate_explicit_form():
    # A_D^(2) = A_RS^(2) - lam^3 theta*[((theta*Delta')Delta') |> (theta*Delta')]
    theta, delta = workloads.dense_unsym(2, n=20)
    delta = delta.astype(np.float64) * 10
    lam = 0.37
    g = np.zeros((20, 20))
    off = ~np.eye(20, dtype=bool)
    g[off] = 1.0 / (theta[:, None] - theta[None, :])[off]
    t1 = g * delta.T
    corr = g * (np.diag(t1 @ delta.T)[:, None] * t1)
    ad = oracle.iterate(theta, delta, lam, max_iter=2, fixed_steps=True)["z"]
    ars = oracle.rs_partial_sum(theta, delta, lam, 2)
    assert np.max(np.abs(ad - (ars - lam ** 3 * corr))) <= 1e-15


def test_eigenvalue_second_order():
    theta, delta = workloads.dense_sym_small(4, n=30)
    base = theta + np.einsum("nm,mn->n", delta * 0, delta)
    diffs = []
    for lam in (0.2, 0.1):
        r = oracle.iterate(theta, delta, lam, max_iter=200, tol=1e-15)
        g = np.zeros((30, 30))
        off = ~np.eye(30, dtype=bool)
        g[off] = 1.0 / (theta[:, None] - theta[None, :])[off]
        e2 = base + lam * np.diag(delta) + lam ** 2 * np.sum(delta * delta.T * g, axis=1)
        diffs.append(np.max(np.abs(r["e"] - e2)))
    assert abs(diffs[0] / diffs[1] - 8.0) < 0.8      # O(lam^3)


def test_rs_eigenvalue_coefficients_match_textbook_second_order():
    theta, delta = workloads.dense_unsym(4, n=10)
    delta = delta.astype(np.float64)
    eps = oracle.rs_eigenvalue_coefficients(theta, delta, 2)
    g = np.zeros((10, 10))
    off = ~np.eye(10, dtype=bool)
    g[off] = 1.0 / (theta[:, None] - theta[None, :])[off]
    assert np.allclose(eps[0], np.diag(delta), atol=0)
    assert np.allclose(eps[1], np.sum(delta * delta.T * g, axis=1), atol=1e-16)


# ---------------------------------------------------------------- Sec. II.F, delta potential
def test_delta_potential_beyond_rs_radius():
    theta, delta = workloads.delta_potential(100)
    # lambda = 1.5: D-PT converges in fewer iterations than RS needs orders
    r = oracle.iterate(theta, delta, 1.5, max_iter=500, tol=1e-14)
    assert r["status"] == OR_OK and 30 <= r["iters"] <= 60
    w = np.linalg.eigvalsh(np.diag(theta) + 1.5 * delta)
    assert np.max(np.abs(np.sort(r["e"]) - w)) <= 1e-12
    assert np.max(np.abs(r["e"] - w)) <= 1e-12          # index order preserved
    a_star = r["z"]
    k_dpt = int(np.argmax(r["hist"] < 1e-8)) + 1
    err_rs = np.max(np.abs(oracle.rs_partial_sum(theta, delta, 1.5, k_dpt) - a_star))
    assert err_rs > 1e-7                                # RS at the same order lags
    # lambda = 2.5: RS diverges, D-PT still converges
    r = oracle.iterate(theta, delta, 2.5, max_iter=2000, tol=1e-13)
    assert r["status"] == OR_OK
    w = np.linalg.eigvalsh(np.diag(theta) + 2.5 * delta)
    assert np.max(np.abs(r["e"] - w)) <= 1e-11
    e60 = np.max(np.abs(oracle.rs_partial_sum(theta, delta, 2.5, 60) - r["z"]))
    e120 = np.max(np.abs(oracle.rs_partial_sum(theta, delta, 2.5, 120) - r["z"]))
    assert e120 > e60 > 1.0


def test_hermite_values():
    # phi_0(0) = pi^(-1/4), phi_2(0) = -pi^(-1/4)/sqrt(2), phi_4(0) = pi^(-1/4) sqrt(3/8)
    phi = workloads.hermite_even_at_zero(3)
    c = math.pi ** -0.25
    assert np.allclose(phi, [c, -c / math.sqrt(2), c * math.sqrt(3 / 8)], rtol=1e-15)


# ---------------------------------------------------------------- Sec. II.C, Banach ball
@pytest.mark.parametrize("seed", range(4))
def test_converges_inside_banach_ball(seed):
    rng = np.random.default_rng(100 + seed)
    n = 40
    theta = np.sort(rng.uniform(0, 40, n))
    delta = rng.normal(0, 1, (n, n))
    np.fill_diagonal(delta, 0)
    g = np.zeros((n, n))
    off = ~np.eye(n, dtype=bool)
    g[off] = 1.0 / (theta[:, None] - theta[None, :])[off]
    bound = (3 - 2 * math.sqrt(2)) / (np.linalg.norm(g, 2) * np.linalg.norm(delta, 2))
    lam = 0.99 * bound
    r = oracle.iterate(theta, delta, lam, max_iter=500, tol=1e-14)
    assert r["status"] == OR_OK
    res, _, _ = oracle.residual(theta, delta, lam, r["z"], r["e"])
    assert res.max() <= 1e-12 * np.abs(theta).max()


# ---------------------------------------------------------------- sparse / rows / dominant
def test_csr_equals_dense_bitwise():
    theta, indptr, indices, values = workloads.sparse_sym(0, n=300)
    dense = workloads.csr_to_dense(300, indptr, indices, values)
    a = oracle.iterate(theta, (indptr, indices, values), 1.0, max_iter=6, fixed_steps=True)
    b = oracle.iterate(theta, dense, 1.0, max_iter=6, fixed_steps=True)
    assert np.array_equal(a["z"], b["z"]) and np.array_equal(a["e"], b["e"])


def test_rows_evolve_independently():
    theta, delta = workloads.dense_unsym(5, n=80)
    full = oracle.iterate(theta, delta, 1.0, max_iter=7, fixed_steps=True)
    rows = np.array([0, 13, 79])
    part = oracle.iterate(theta, delta, 1.0, rows=rows, max_iter=7, fixed_steps=True)
    assert np.array_equal(part["z"], full["z"][rows])
    assert np.array_equal(part["e"], full["e"][rows])


def test_dominant_eigenpair_sparse():
    theta, indptr, indices, values = workloads.sparse_sym(1, n=3000)
    n = 3000
    r = oracle.iterate(theta, (indptr, indices, values), 1.0, rows=[n - 1], max_iter=50,
                       tol=1e-15)
    assert r["status"] == OR_OK and r["iters"] <= 6
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    m = sp.diags(theta) + sp.csr_matrix((values.astype(np.float64), indices, indptr),
                                        shape=(n, n))
    top = spl.eigsh(m, k=1, which="LA", tol=1e-14)[0][0]
    assert abs(r["e"][0] - top) <= 1e-12 * n


def test_rejects_degenerate_and_bad_inputs():
    theta = np.array([0.0, 1.0, 1.0])
    with pytest.raises(ValueError):
        oracle.iterate(theta, np.zeros((3, 3)), 0.1)
    with pytest.raises(ValueError):
        oracle.iterate(np.array([0.0, 1.0]), np.zeros((2, 2)), float("nan"))
    with pytest.raises(ValueError):   # column index out of range
        oracle.iterate(np.array([0.0, 1.0]),
                       (np.array([0, 1, 1]), np.array([5], np.int32), np.array([1.0])), 0.1)
    r = oracle.iterate(np.array([2.0]), np.array([[0.5]]), 0.3, max_iter=10, tol=1e-12)
    assert r["e"][0] == 2.0 + 0.3 * 0.5 and r["z"][0, 0] == 1.0


def test_degenerate_theta_away_from_requested_rows():
    """Row n's single-line map divides only by theta_n - theta_m (Sec. II.H): a
    repeated value elsewhere is accepted and the converged row is still an
    eigenvector of M (checked by the plain eigen-equation); asking for one of
    the repeated rows is rejected."""
    n = 40
    rng = np.random.default_rng(5)
    theta = np.arange(n, dtype=np.float64)
    theta[3] = theta[4]
    delta = rng.normal(0.0, 0.05, (n, n))
    delta = 0.5 * (delta + delta.T)
    r = oracle.iterate(theta, delta, 1.0, rows=[n - 1, 20], max_iter=500, tol=1e-14)
    assert r["status"] == 0
    res, mz, zn = oracle.residual(theta, delta, 1.0, r["z"], r["e"])
    assert np.max(res / mz) <= 1e-12
    with pytest.raises(ValueError):
        oracle.iterate(theta, delta, 1.0, rows=[3], max_iter=5, tol=1e-12)
    with pytest.raises(ValueError):
        oracle.iterate(theta, delta, 1.0, max_iter=5, tol=1e-12)


# ---------------------------------------------------------------- planted mistakes
MUTANTS = {
    "bracket_sign": ("(c[m] - cn * z[m])", "(cn * z[m] - c[m])"),
    "dropped_rescale": ("(c[m] - cn * z[m])", "(c[m])"),
    "transposed_delta": ("s += row[l] * z[l];", "s += p->dense[l * p->n + m] * z[l];"),
    "gap_index": ("(p->theta[nidx] - p->theta[m])", "(p->theta[m] - p->theta[nidx])"),
    "readout_without_lambda": ("p->theta[rows[r]] + p->lambda * delta_row_dot",
                               "p->theta[rows[r]] + delta_row_dot"),
    "rescale_wrong_index": ("const double cn = c[nidx];", "const double cn = c[0];"),
}


def _pin_battery(it):
    """Return the list of pins that fail for the oracle build ``it``."""
    failed = []
    # 2x2 closed form at every iterate, lam = 0.3
    theta, delta = workloads.two_by_two()
    xs = quad_map_iterates(0.3, 6)
    z = it(theta, delta, 0.3, max_iter=6, fixed_steps=True)["z"]
    if abs(z[0, 1] - xs[-1]) > 1e-15 or abs(z[1, 0] + xs[-1]) > 1e-15:
        failed.append("2x2 iterates")
    r = it(theta, delta, 0.3, max_iter=2000, tol=1e-15)
    if abs(r["e"][0] - (1 - math.sqrt(1.36)) / 2) > 1e-13:
        failed.append("2x2 eigenvalue")
    # 3x3 printed multiplier polynomial
    theta, delta = workloads.three_by_three()
    terms = load_multiplier_polynomials()[3]
    r = it(theta, delta, 0.25, rows=[2], max_iter=2000, tol=1e-15)
    if r["status"] != OR_OK:
        failed.append("3x3 convergence")
    else:
        mus = chart_multipliers(it, theta, delta, 0.25, 2, r["z"][0])
        if max(poly_residual(terms, 0.25, mu) for mu in mus) > 1e-8:
            failed.append("3x3 polynomial")
    # unsymmetric problem against the library eigensolver, lam != 1
    theta, delta = workloads.dense_unsym(0, n=40)
    delta = delta.astype(np.float64)
    r = it(theta, delta, 0.7, max_iter=300, tol=1e-14)
    vals, rows = eig_rows_normalised(np.diag(theta) + 0.7 * delta)
    if (r["status"] != OR_OK or np.max(np.abs(r["e"] - vals.real)) > 1e-11
            or np.max(np.abs(r["z"] - rows.real)) > 1e-11):
        failed.append("unsymmetric eig")
    return failed


def test_pin_battery_passes_on_the_oracle():
    assert _pin_battery(oracle.iterate) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "dpt_oracle.c")).read()
    assert src.count(old) == 1, "mutation anchor not found"
    path = tmp_path / ("mutant_%s.c" % name)
    path.write_text(src.replace(old, new))
    lib = oracle.OracleLib(oracle.build(src=str(path), out=str(tmp_path / "libmut.so")))
    assert _pin_battery(lib.iterate) != []
