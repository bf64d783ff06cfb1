"""GPU parity of the dense path (C ABI through the ctypes binding) against the FP64 oracle.

Tolerances: FP64 paths 1e-12 relative per step (accumulation order only);
FP32/BF16 single steps by the elementwise bound of ``helpers.one_step_bound``
(operand rounding 2^-24 / 2^-8 plus accumulation); solves at the stated targets,
1e-5 (FP32 results) and 1e-10 (FP64 results).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from helpers import gap_matrix, one_step_bound, rel_eig_error, small_problem

pytestmark = pytest.mark.gpu

dpt = pytest.importorskip("paper_2002_12872_amd.dpt")


def bf16_round(x):
    """Round float32 values to bfloat16 (round to nearest even), returned as float32."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def gpu_run(theta, delta, lam, precision, steps=None, tol=1e-6, max_iter=200, fp64_final_tol=0.0,
            z0=None, out_dtype=np.float64):
    spec = dpt.ProblemSpec(theta, delta, lam, stream=0)
    h = dpt.dpt_init(spec, dpt.options(tol=tol, max_iter=max_iter, precision=precision,
                                       fp64_final_tol=fp64_final_tol), z0)
    res = None
    if steps is not None:
        res = {"last_delta": dpt.dpt_step(h, steps)}
    else:
        res = dpt.dpt_solve(h)
    e = dpt.dpt_eigenvalues(h)
    z = dpt.dpt_eigenvectors(h, dtype=out_dtype)
    return h, res, e, z


SIZES = [1, 2, 3, 31, 33, 64, 127, 257, 300, 1000, 1100]


# ------------------------------------------------------------------ FP64
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp64_solve_small_symmetric_matches_oracle_and_jacobi(seed):
    theta, delta = workloads.dense_sym_small(seed)
    h, res, e, z = gpu_run(theta, delta, 1.0, dpt.DPT_FP64, tol=1e-12, max_iter=200)
    ref = oracle.iterate(theta, delta, 1.0, max_iter=200, tol=1e-12)
    assert res["status"] == dpt.DPT_OK and ref["status"] == oracle.OR_OK
    assert abs(res["iters"] - ref["iters"]) <= 1
    assert rel_eig_error(e, ref["e"], theta) <= 1e-10
    assert np.max(np.abs(z - ref["z"])) <= 1e-10
    w, v = oracle.jacobi_eigh(np.diag(theta) + delta)
    for n in range(64):
        j = int(np.argmax(np.abs(v[n])))
        assert abs(e[n] - w[j]) <= 1e-10 * max(abs(w[j]), 1e-12 * 63)
    r = dpt.dpt_residuals(h, np.arange(64))
    norm_ub = np.abs(theta).max() + np.linalg.norm(delta)
    assert np.max(r / (norm_ub * np.linalg.norm(z, axis=1))) <= 1e-10


@pytest.mark.parametrize("n", SIZES + [2048, 4100, 6000])
@pytest.mark.parametrize("sym", [False, True])
def test_fp64_steps_match_oracle(n, sym):
    """N = 2048, 4100 and 6000 (padded to 2048, 4352 and 6144) run the
    large-tile FP64 step (128 x 128 tiles, two workgroups per CU, direct-to-LDS
    loads); the smaller orders the general one."""
    theta, delta = small_problem(n, 1, symmetric=sym)
    lam = -0.8 if sym else 1.0
    rows = workloads.sample_rows(n, 48)
    for k in (1, 2, 3):
        _, _, e, z = gpu_run(theta, delta, lam, dpt.DPT_FP64, steps=k)
        ref = oracle.iterate(theta, delta, lam, rows=rows, max_iter=k, fixed_steps=True)
        scale = max(1.0, np.abs(ref["z"]).max())
        assert np.max(np.abs(z[rows] - ref["z"])) <= 1e-12 * scale, k
        assert rel_eig_error(e[rows], ref["e"], theta) <= 1e-12


def test_fp64_nonzero_diagonal_first_iterates():
    theta, delta = small_problem(70, 3, diag=True)
    for k in (1, 2, 4):
        _, _, e, z = gpu_run(theta, delta, 0.9, dpt.DPT_FP64, steps=k)
        ref = oracle.iterate(theta, delta, 0.9, max_iter=k, fixed_steps=True)
        assert np.max(np.abs(z - ref["z"])) <= 1e-12
        assert np.max(np.abs(e - ref["e"])) <= 1e-12 * np.abs(theta).max()


# --------------------------------------------------------- FP32 / BF16 steps
def _state_after(theta, delta32, lam, precision, k):
    """GPU state after k steps (exported exactly as float64) and after k+1 steps."""
    _, _, _, zk = gpu_run(theta, delta32, lam, precision, steps=k)
    _, _, ek1, zk1 = gpu_run(theta, delta32, lam, precision, steps=k + 1)
    return zk, zk1, ek1


@pytest.mark.parametrize("n", [31, 64, 257, 1000, 1100, 4096, 4100])
@pytest.mark.parametrize("sym", [False, True])
def test_fp32_step_within_rounding_bound(n, sym):
    """4096 runs the 256 x 256-tile FP32 step, 4100 (padded to 4352, a third of
    a wave of those tiles) the general 128 x 128 one."""
    theta, delta = small_problem(n, 2, symmetric=sym)
    delta32 = delta.astype(np.float32)
    d64 = delta32.astype(np.float64)
    rows = workloads.sample_rows(n, 40)
    for k in (0, 2):
        zk, zk1, _ = _state_after(theta, delta32, 1.0, dpt.DPT_FP32, k)
        ref = oracle.iterate(theta, d64, 1.0, rows=rows, z0=zk[rows], max_iter=1, fixed_steps=True)
        bound = one_step_bound(theta, d64, 1.0, zk[rows], 2.0 ** -24, 8 + math.sqrt(n), rows=rows)
        err = np.abs(zk1[rows] - ref["z"])
        assert np.all(err <= bound), (k, float(np.max(err / bound)))


@pytest.mark.parametrize("n", [31, 64, 257, 1000, 1100, 2048, 4100])
@pytest.mark.parametrize("sym", [False, True])
def test_bf16_step_within_rounding_bound(n, sym):
    """2048 and 4100 (padded to 4352) run the 256 x 256-tile BF16 step."""
    theta, delta = small_problem(n, 3, symmetric=sym)
    delta32 = delta.astype(np.float32)
    d64 = delta32.astype(np.float64)
    rows = workloads.sample_rows(n, 40)
    for k in (1, 2):
        zk, zk1, _ = _state_after(theta, delta32, 1.0, dpt.DPT_BF16_FP32, k)
        ref = oracle.iterate(theta, d64, 1.0, rows=rows, z0=zk[rows], max_iter=1, fixed_steps=True)
        bound = one_step_bound(theta, d64, 1.0, zk[rows], 2.0 ** -8, 8 + math.sqrt(n), rows=rows)
        err = np.abs(zk1[rows] - ref["z"])
        assert np.all(err <= bound), (k, float(np.max(err / bound)))


@pytest.mark.parametrize("n", [64, 300, 1100])
def test_bf16_step_equals_rounded_operand_product(n):
    """The BF16 step is the FP32 update applied to bf16(W) bf16(Delta)^T + Delta^T."""
    theta, delta = small_problem(n, 4, symmetric=False)
    delta32 = delta.astype(np.float32)
    zk, zk1, _ = _state_after(theta, delta32, 0.9, dpt.DPT_BF16_FP32, 2)
    w = zk.copy()
    np.fill_diagonal(w, 0.0)
    wb = bf16_round(w.astype(np.float32)).astype(np.float64)
    db = bf16_round(delta32).astype(np.float64)
    d64 = delta32.astype(np.float64)
    c = d64.T + wb @ db.T
    dvec = np.diag(d64) + np.sum(w * d64, axis=1)     # pre-pass uses the FP32 state, FP64 sums
    g = gap_matrix(theta)
    expect = 0.9 * g * (c - dvec[:, None] * w)
    mag = np.abs(wb) @ np.abs(db).T + np.abs(c) + np.abs(dvec)[:, None] * np.abs(w)
    tol = np.abs(0.9 * g) * (8 + math.sqrt(n)) * 2.0 ** -24 * mag + 4 * 2.0 ** -24 * np.abs(expect) + 1e-300
    got = zk1 - np.eye(n)
    assert np.all(np.abs(got - expect) <= tol), float(np.max(np.abs(got - expect) / tol))


# ------------------------------------------------------------------ solves
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("sym", [False, True])
def test_solve_reaches_fp32_target(precision, sym):
    n = 1100
    theta, delta = small_problem(n, 5, symmetric=sym)
    delta32 = delta.astype(np.float32)
    prec = dpt.DPT_FP32 if precision == "fp32" else dpt.DPT_BF16_FP32
    h, res, e, z = gpu_run(theta, delta32, 1.0, prec, tol=1e-6, max_iter=100)
    assert res["status"] == dpt.DPT_OK
    if precision == "bf16":
        assert res["iters_bf16"] >= 1 and res["iters_fp32"] >= 1
    rows = workloads.sample_rows(n, 64)
    ref = oracle.iterate(theta, delta32.astype(np.float64), 1.0, rows=rows, max_iter=200, tol=1e-14)
    assert rel_eig_error(e[rows], ref["e"], theta) <= 1e-5
    ez = np.max(np.abs(z[rows] - ref["z"])) / np.max(np.abs(ref["z"] - np.eye(n)[rows]))
    assert ez <= 1e-5
    r = dpt.dpt_residuals(h, rows)
    norm_ub = np.abs(theta).max() + np.linalg.norm(delta32.astype(np.float64))
    assert np.max(r / (norm_ub * np.linalg.norm(z[rows], axis=1))) <= 1e-5


def test_bf16_then_fp64_final_sweeps_reach_1e10():
    n = 300
    theta, delta = small_problem(n, 6, symmetric=True)
    delta32 = delta.astype(np.float32)
    h, res, e, z = gpu_run(theta, delta32, 1.0, dpt.DPT_BF16_FP32, tol=1e-6, max_iter=100,
                           fp64_final_tol=1e-13)
    assert res["status"] == dpt.DPT_OK and res["iters_fp64"] >= 1
    ref = oracle.iterate(theta, delta32.astype(np.float64), 1.0, max_iter=200, tol=1e-15)
    assert rel_eig_error(e, ref["e"], theta) <= 1e-10
    assert np.max(np.abs(z - ref["z"])) <= 1e-10


# ------------------------------------------------------------- edge cases
def test_order_one():
    h, res, e, z = gpu_run(np.array([2.5]), np.array([[0.75]]), 0.4, dpt.DPT_FP64, tol=1e-12)
    assert res["status"] == dpt.DPT_OK
    assert e[0] == 2.5 + 0.4 * 0.75 and z[0, 0] == 1.0


def test_zero_iterations_returns_identity():
    theta, delta = small_problem(40, 7, diag=True)
    h, res, e, z = gpu_run(theta, delta, 0.5, dpt.DPT_FP64, max_iter=0)
    assert res["status"] == dpt.DPT_NOT_CONVERGED and res["iters"] == 0
    assert np.array_equal(z, np.eye(40))
    assert np.allclose(e, theta + 0.5 * np.diag(delta), rtol=0, atol=1e-14)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_two_by_two_dynamics(precision):
    theta, delta = workloads.two_by_two()
    d = delta.astype(np.float32) if precision else delta
    # inside the domain: closed-form eigenvalues
    _, res, e, _ = gpu_run(theta, d, 0.3, precision, tol=1e-6 if precision else 1e-14, max_iter=500)
    assert res["status"] == dpt.DPT_OK
    root = math.sqrt(1 + 4 * 0.09)
    assert abs(e[0] - (1 - root) / 2) <= (1e-6 if precision else 1e-14)
    # flip bifurcation: 2-cycle runs to the cap
    _, res, _, _ = gpu_run(theta, d, 0.9, precision, tol=1e-9, max_iter=300)
    assert res["status"] == dpt.DPT_NOT_CONVERGED and res["iters"] == 300
    # divergence to infinity
    _, res, _, _ = gpu_run(theta, d, 3.0, precision, tol=1e-9, max_iter=300)
    assert res["status"] == dpt.DPT_DIVERGED


def test_nan_in_delta_diverges():
    theta, delta = small_problem(100, 8)
    delta[3, 7] = np.nan
    _, res, _, _ = gpu_run(theta, delta.astype(np.float32), 1.0, dpt.DPT_BF16_FP32, max_iter=20)
    assert res["status"] == dpt.DPT_DIVERGED


def test_fp32_floor_reports_stall():
    theta, delta = small_problem(200, 9)
    _, res, _, _ = gpu_run(theta, delta.astype(np.float32), 1.0, dpt.DPT_FP32, tol=1e-30, max_iter=200)
    assert res["status"] == dpt.DPT_STALLED and res["iters"] < 200


def test_warm_start_refines_approximate_eigenvectors():
    theta, delta = small_problem(257, 10, symmetric=True)
    ref = oracle.iterate(theta, delta, 1.0, max_iter=200, tol=1e-15)
    rng = np.random.default_rng(0)
    z0 = ref["z"] * (1 + 0.01 * rng.standard_normal(ref["z"].shape))   # ~1 % accurate
    _, res, e, z = gpu_run(theta, delta, 1.0, dpt.DPT_FP64, tol=1e-13, z0=z0)
    assert res["status"] == dpt.DPT_OK
    assert np.max(np.abs(z - ref["z"])) <= 1e-11
    assert rel_eig_error(e, ref["e"], theta) <= 1e-11


def test_warm_start_must_match_the_problem_memory_kind():
    """A device z0 given with a host problem (and a host z0 with a device
    problem) is rejected by the library itself, not dereferenced."""
    import ctypes
    import torch
    n = 64
    theta, delta = small_problem(n, 12)
    z_host = np.eye(n)
    z_dev = torch.eye(n, dtype=torch.float64, device="cuda")
    lib = dpt.load_library()
    o = dpt.options(precision=dpt.DPT_FP64)
    for spec, z0 in ((dpt.ProblemSpec(theta, delta, 1.0, stream=0), z_dev.data_ptr()),
                     (dpt.ProblemSpec(torch.from_numpy(theta).cuda(), torch.from_numpy(delta).cuda(), 1.0),
                      z_host.ctypes.data)):
        h = ctypes.c_void_p()
        rc = lib.dpt_init(ctypes.byref(h), ctypes.byref(spec.struct), ctypes.byref(o), z0)
        assert rc == dpt.DPT_EINVAL and not h.value
    with pytest.raises(ValueError):
        dpt.dpt_init(dpt.ProblemSpec(theta, delta, 1.0, stream=0), o, z_dev)


def test_device_inputs_are_borrowed_and_match_host_inputs():
    import torch
    n = 1024
    theta, delta = small_problem(n, 11, symmetric=True)
    delta32 = delta.astype(np.float32)
    _, r_host, e_host, z_host = gpu_run(theta, delta32, 1.0, dpt.DPT_BF16_FP32, tol=1e-6)
    th_d = torch.from_numpy(theta).cuda()
    de_d = torch.from_numpy(delta32).cuda()
    spec = dpt.ProblemSpec(th_d, de_d, 1.0)
    h = dpt.dpt_init(spec, dpt.options(tol=1e-6, precision=dpt.DPT_BF16_FP32))
    res = dpt.dpt_solve(h)
    e_dev = torch.empty(n, dtype=torch.float64, device="cuda")
    dpt.dpt_eigenvalues(h, e_dev)
    z_dev = torch.empty((n, n), dtype=torch.float32, device="cuda")
    dpt.dpt_eigenvectors(h, z_dev)
    torch.cuda.synchronize()
    assert res["iters"] == r_host["iters"]
    assert np.array_equal(e_dev.cpu().numpy(), e_host)
    assert np.array_equal(z_dev.cpu().numpy(), z_host.astype(np.float32))
    assert torch.equal(de_d.cpu(), torch.from_numpy(delta32))     # input untouched


def test_unaligned_device_delta_is_copied_and_matches():
    """A device Delta whose address is not 16-byte aligned (a view one element
    into a buffer) cannot be borrowed by the 16-byte vector loads; it is copied
    instead and gives the same result bit for bit."""
    import torch
    n = 1024
    theta, delta = small_problem(n, 13, symmetric=True)
    delta32 = delta.astype(np.float32)
    _, r_host, e_host, z_host = gpu_run(theta, delta32, 1.0, dpt.DPT_BF16_FP32, tol=1e-6)
    flat = torch.zeros(n * n + 1, dtype=torch.float32, device="cuda")
    flat[1:] = torch.from_numpy(delta32.reshape(-1)).cuda()
    de_d = flat[1:].view(n, n)
    assert de_d.data_ptr() % 16 == 4
    h = dpt.dpt_init(dpt.ProblemSpec(torch.from_numpy(theta).cuda(), de_d, 1.0),
                     dpt.options(tol=1e-6, precision=dpt.DPT_BF16_FP32))
    res = dpt.dpt_solve(h)
    e = dpt.dpt_eigenvalues(h)
    z = dpt.dpt_eigenvectors(h, dtype=np.float64)
    dpt.dpt_destroy(h)
    assert res["iters"] == r_host["iters"]
    assert np.array_equal(e, e_host) and np.array_equal(z, z_host)


@pytest.mark.parametrize("precision,n,sym,lam,tol,max_iter", [
    (dpt.DPT_FP64, 64, True, 1.0, 1e-12, 200),   # stops inside the first batch of 16
    (dpt.DPT_FP64, 33, False, 2.0, 1e-300, 37),  # slow contraction: the cap, over three batches
    (dpt.DPT_FP32, 50, False, 1.0, 1e-6, 200),
    (dpt.DPT_FP32, 64, True, 4.0, 1e-300, 20),   # the cap, over two batches
    (dpt.DPT_FP64, 40, True, 6.0, 1e-12, 200),   # diverges inside the first batch (the batch ends there)
    (dpt.DPT_FP32, 40, True, 6.0, 1e-6, 200),
])
def test_small_problem_batches_equal_single_steps(precision, n, sym, lam, tol, max_iter):
    """Problems with padded order 64 run several steps per launch in dpt_solve;
    the iterate returned and the delta history are those of one launch per step
    (dpt_step), bit for bit, whichever step the stopping rule ends on."""
    theta, delta = small_problem(n, 14, symmetric=sym)
    d = delta if precision == dpt.DPT_FP64 else delta.astype(np.float32)
    _, res, e1, z1 = gpu_run(theta, d, lam, precision, tol=tol, max_iter=max_iter)
    if lam == 6.0:
        assert res["status"] == dpt.DPT_DIVERGED
    steps = res["iters"]
    assert (steps < 16) if tol > 1e-100 else (steps == max_iter)
    spec = dpt.ProblemSpec(theta, d, lam, stream=0)
    h = dpt.dpt_init(spec, dpt.options(tol=tol, max_iter=max_iter, precision=precision))
    deltas = [dpt.dpt_step(h, 1) for _ in range(steps)]
    e2 = dpt.dpt_eigenvalues(h)
    z2 = dpt.dpt_eigenvectors(h, dtype=np.float64)
    dpt.dpt_destroy(h)
    assert np.array_equal(e1, e2) and np.array_equal(z1, z2)
    assert np.array_equal(res["history"][:steps], np.array(deltas))


def test_runs_are_deterministic():
    theta, delta = small_problem(1000, 12)
    d32 = delta.astype(np.float32)
    _, r1, e1, z1 = gpu_run(theta, d32, 1.0, dpt.DPT_BF16_FP32)
    _, r2, e2, z2 = gpu_run(theta, d32, 1.0, dpt.DPT_BF16_FP32)
    assert r1["iters"] == r2["iters"] and np.array_equal(e1, e2) and np.array_equal(z1, z2)


def test_recycled_buffers_leave_no_trace():
    """Small device buffers are recycled across handles (they come back holding
    the previous handle's data): solves of different orders and precisions,
    interleaved, with handles destroyed and created again, must repeat their
    first results exactly, including at the identity (max_iter = 0)."""
    cases = [(64, dpt.DPT_FP64, 200), (300, dpt.DPT_FP32, 200), (64, dpt.DPT_FP32, 0), (257, dpt.DPT_BF16_FP32, 200),
             (33, dpt.DPT_FP64, 0)]
    probs = {n: small_problem(n, 20 + n) for n, _, _ in cases}
    first = {}
    for rep in range(3):
        for n, prec, mi in cases:
            theta, delta = probs[n]
            d = delta if prec == dpt.DPT_FP64 else delta.astype(np.float32)
            h, r, e, z = gpu_run(theta, d, 0.7, prec, max_iter=mi)
            dpt.dpt_destroy(h)
            if rep == 0:
                first[(n, prec, mi)] = (r["iters"], e, z)
                if mi == 0:
                    assert np.array_equal(z, np.eye(n))
            else:
                it0, e0, z0 = first[(n, prec, mi)]
                assert r["iters"] == it0 and np.array_equal(e, e0) and np.array_equal(z, z0), (rep, n, prec)


def test_device_rejects_duplicate_theta():
    import torch
    theta = torch.tensor([0.0, 1.0, 1.0], dtype=torch.float64, device="cuda")
    delta = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(dpt.DptError) as ei:
        dpt.dpt_init(dpt.ProblemSpec(theta, delta, 0.1))
    assert ei.value.code == dpt.DPT_EINVAL


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("sym", [False, True])
def test_estimate_stop_rule_certifies_accuracy_with_fewer_products(precision, sym):
    n = 1100
    theta, delta = small_problem(n, 13, symmetric=sym)
    delta32 = delta.astype(np.float32)
    prec = dpt.DPT_FP32 if precision == "fp32" else dpt.DPT_BF16_FP32
    runs = {}
    for rule in (dpt.DPT_STOP_DELTA, dpt.DPT_STOP_ESTIMATE):
        spec = dpt.ProblemSpec(theta, delta32, 1.0, stream=0)
        h = dpt.dpt_init(spec, dpt.options(tol=1e-6, max_iter=100, precision=prec, stop_rule=rule))
        runs[rule] = (dpt.dpt_solve(h), dpt.dpt_eigenvalues(h), dpt.dpt_eigenvectors(h))
    (rd, ed, zd), (re_, ee, ze) = runs[dpt.DPT_STOP_DELTA], runs[dpt.DPT_STOP_ESTIMATE]
    assert rd["status"] == dpt.DPT_OK and re_["status"] == dpt.DPT_OK
    assert re_["iters"] <= rd["iters"]
    if precision == "bf16":
        assert re_["iters_fp32"] >= 1
    rows = workloads.sample_rows(n, 64)
    ref = oracle.iterate(theta, delta32.astype(np.float64), 1.0, rows=rows, max_iter=200, tol=1e-14)
    # the certified distance to the fixed point (tol) plus FP32 rounding of the state
    assert np.max(np.abs(ze[rows] - ref["z"])) <= 1e-6 + 1e-6 * np.max(np.abs(ref["z"] - np.eye(n)[rows]))
    assert rel_eig_error(ee[rows], ref["e"], theta) <= 1e-5
