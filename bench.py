#!/usr/bin/env python3
"""Benchmark of the D-PT hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): dense symmetric
N = 16384, theta_i = i/4, Delta = (R + R^T)/2 with R off-diagonal iid
N(0, (0.25/sqrt(N))^2), zero diagonal, lambda = 1, FP32 input values.  One
"step" is one whole solve through the C ABI: dpt_init on device-resident
inputs (staging, BF16 copy, symmetry test), dpt_solve in the BF16 -> FP32 form
to tol 1e-6, and the eigenvalue readout.  The stopping rule (default: the
a-posteriori contraction bound, DPT_STOP_ESTIMATE) is the same for the plain
FP32 solve timed beside it; the other rule is reported for context.

Printed: one JSON line with value = D-PT iterations per second of the BF16 ->
FP32 solve, the roofline of the kernel that dominates the solve time (HIP
events on its stream) and of both fused product kernels, the error of the
result against the converged FP64 oracle on 64 sampled rows, and the FP64 CPU
oracle timed on that sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DPT iter/s + TFLOP/s at N=16384 (bf16→fp32 vs fp32); solves/s, p50/p99 lat"
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix cores
PEAK_FP8_TFLOPS = 5000.0
CSRC = os.path.join(ROOT, "paper_2002_12872_amd", "csrc")
# per fused product kernel: profile class, traffic summary, source file, peak
KERNELS = {
    "gemm_bf16": {"name": "k_step_bf16_large (256x256 tile, 4 waves of 128x128, K-tiles of 64 via direct-to-LDS loads)",
                  "traffic": os.path.join(ROOT, "profiles", "traffic_gemm_bf16_n16384.txt"),
                  "source": os.path.join(CSRC, "kernels_gemm_large.hip"), "peak": PEAK_BF16_TFLOPS},
    "gemm_fp32": {"name": "k_step_f32_large (256x256 tile, 4 waves of 128x128, K-tiles of 32 via direct-to-LDS loads)",
                  "traffic": os.path.join(ROOT, "profiles", "traffic_gemm_fp32_n16384.txt"),
                  "source": os.path.join(CSRC, "kernels_gemm_large.hip"), "peak": PEAK_FP32_TFLOPS},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--stop-rule", choices=["estimate", "delta"], default="estimate",
                    help="stopping rule of the timed solves (both precision forms)")
    ap.add_argument("--kernel-precision", choices=["bf16", "fp32", "fp64"], default="bf16",
                    help="precision of the --kernel-only steps")
    ap.add_argument("--spmm-only", action="store_true",
                    help="profiling mode: CSR product steps of the N = 32768 sparse workload only")
    ap.add_argument("--serve-only", action="store_true",
                    help="profiling mode: the serving engine on the first --serve-requests trace requests, burst")
    ap.add_argument("--fp32-solves", type=int, default=2)
    ap.add_argument("--skip-cpu", action="store_true", help="do not time the CPU oracle")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU oracle work")
    ap.add_argument("--kernel-only", action="store_true",
                    help="profiling mode: init once, run --steps BF16 steps (after --warmup), no solve")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="profiling mode: plain device-to-device copy of MIB MiB, --steps times")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="serving trace length (0 skips the serving measurement)")
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--skip-secondary", action="store_true",
                    help="skip the small/unsymmetric/sparse configuration lines")
    ap.add_argument("--no-paper-scale", dest="paper_scale", action="store_false",
                    help="skip the N = 2^22 (1.34e8 nnz) dominant-pair line")
    ap.add_argument("--secondary-only", action="store_true",
                    help="run only the small/unsymmetric/sparse configuration lines")
    return ap.parse_args()


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def serving_bench(args):
    """Continuous batching vs one-at-a-time FP32 solves on the serving trace.

    Trace: N log-uniform in [32, 2048], half symmetric, theta_i = i + U(0, 0.5),
    Delta ~ N(0, (0.4/sqrt N)^2), tol 1e-5, BF16->FP32 in the engine (tile
    shapes of the grouped step chosen by the autotuner when it opens).  The
    one-at-a-time FP32 service rate mu_1 is measured first on the trace's
    problems; arrivals are Poisson at rate mu_1.  Engine latencies come from its
    own submit/finish timestamps; the one-at-a-time latencies from its measured
    service times through a FIFO single-server queue on the same arrivals, and
    observed in real time on the same arrivals (one_at_a_time_fp32_observed).
    """
    import numpy as np

    import workloads
    from paper_2002_12872_amd import dpt
    count = args.serve_requests
    trace = workloads.serving_trace(0, count=count, rate=None)
    probs = [workloads.request_matrices(r) for r in trace]
    specs = [dpt.ProblemSpec(th, de, 1.0, stream=0) for th, de in probs]
    sizes = [th.shape[0] for th, _ in probs]
    o_fp32 = dpt.options(tol=1e-5, max_iter=100, precision=dpt.DPT_FP32)
    o_mixed = dpt.options(tol=1e-5, max_iter=100, precision=dpt.DPT_BF16_FP32)
    # one-at-a-time FP32 solves: service time of every request
    svc = np.empty(count)
    ok = 0
    base_flop = 0.0
    for i, sp in enumerate(specs):
        t = time.perf_counter()
        h = dpt.dpt_init(sp, o_fp32)
        r = dpt.dpt_solve(h, history_cap=0)
        dpt.dpt_eigenvalues(h)
        dpt.dpt_destroy(h)
        svc[i] = time.perf_counter() - t
        ok += r["status"] == dpt.DPT_OK
        base_flop += 2.0 * float(sizes[i]) ** 3 * max(r["iters"] - 1, 0)
    mu1 = count / svc.sum()
    rng = np.random.default_rng(5_100)
    arrivals = np.cumsum(rng.exponential(1.0 / mu1, size=count))
    finish = np.empty(count)
    prev = 0.0
    for i in range(count):
        prev = max(arrivals[i], prev) + svc[i]
        finish[i] = prev
    lat_base = finish - arrivals
    base = {"solves_per_s": round(count / (finish[-1] - arrivals[0]), 2),
            "p50_ms": round(1e3 * percentile(lat_base, 50), 3),
            "p99_ms": round(1e3 * percentile(lat_base, 99), 3),
            "mean_service_ms": round(1e3 * svc.mean(), 3), "converged": int(ok),
            "gemm_tflops_while_busy": round(base_flop / svc.sum() / 1e12, 2)}
    def engine_run(arr, specs=specs):
        """Engine in real time on the arrival times arr (None: all at t = 0)."""
        srv = dpt.dpt_serve_open(int(args.serve_budget_gib * (1 << 30)), max_slots=1024, use_graph=True,
                                 autotune=True)
        tickets = []
        t0 = time.perf_counter()
        for i, sp in enumerate(specs):
            if arr is not None:
                delay = arr[i] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            tickets.append(dpt.dpt_serve_submit(srv, sp, o_mixed))
        res = [dpt.dpt_serve_poll(srv, t, wait_ms=-1) for t in tickets]
        st = dpt.dpt_serve_stats_read(srv)
        dpt.dpt_serve_close(srv)
        lat = np.array([r["times"]["finish"] - r["times"]["submit"] for r in res])
        span = max(r["times"]["finish"] for r in res) - min(r["times"]["submit"] for r in res)
        # products run: every iteration after the closed-form first one costs 2 N^3
        flop = sum(2.0 * float(nr) ** 3 * max(r["iters"] - 1, 0) for nr, r in zip(sizes, res))
        return {"solves_per_s": round(count / span, 2), "gemm_tflops": round(flop / span / 1e12, 2),
                "p50_ms": round(1e3 * percentile(lat, 50), 3),
                "p99_ms": round(1e3 * percentile(lat, 99), 3),
                "converged": int(sum(r["status"] == dpt.DPT_OK for r in res)),
                "steps": st["steps"], "peak_active": st["peak_active"],
                "peak_arena_gib": round(st["peak_bytes"] / 2 ** 30, 3),
                "tile_shape_bf16_fp32": st["tile_shape"]}

    def base_at(rate_mult):
        arr = arrivals / rate_mult
        fin = np.empty(count)
        prev = 0.0
        for i in range(count):
            prev = max(arr[i], prev) + svc[i]
            fin[i] = prev
        lat_b = fin - arr
        return {"solves_per_s": round(count / (fin[-1] - arr[0]), 2),
                "p50_ms": round(1e3 * percentile(lat_b, 50), 3), "p99_ms": round(1e3 * percentile(lat_b, 99), 3)}

    def base_observed(arr):
        """One-at-a-time FP32 solves in real time on the arrival times arr: each
        request starts when it has arrived and the previous one is done."""
        t0 = time.perf_counter()
        lat = np.empty(count)
        for i, sp in enumerate(specs):
            delay = arr[i] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            h = dpt.dpt_init(sp, o_fp32)
            dpt.dpt_solve(h, history_cap=0)
            dpt.dpt_eigenvalues(h)
            dpt.dpt_destroy(h)
            lat[i] = (time.perf_counter() - t0) - arr[i]
        span = (time.perf_counter() - t0) - arr[0]
        return {"solves_per_s": round(count / span, 2), "p50_ms": round(1e3 * percentile(lat, 50), 3),
                "p99_ms": round(1e3 * percentile(lat, 99), 3), "observed": True}

    eng = engine_run(arrivals)
    eng2 = engine_run(arrivals / 2.0)
    burst = engine_run(None)
    # the same problems already resident in HBM (FP32 Delta, FP64 theta), submitted at once
    import torch
    dev = [(torch.from_numpy(th).cuda(), torch.from_numpy(de).float().cuda()) for th, de in probs]
    torch.cuda.synchronize()
    burst_dev = engine_run(None, [dpt.ProblemSpec(th, de, 1.0) for th, de in dev])
    del dev
    torch.cuda.empty_cache()
    base2 = base_at(2.0)
    base_obs = base_observed(arrivals)
    return {"requests": count, "arrival_rate_per_s": round(mu1, 2), "tol": 1e-5,
            "engine_bf16_fp32": eng, "one_at_a_time_fp32": base,
            "one_at_a_time_fp32_observed": base_obs,
            "p99_speedup": round(base["p99_ms"] / eng["p99_ms"], 2),
            "p99_speedup_observed": round(base_obs["p99_ms"] / eng["p99_ms"], 2),
            "at_2x_rate": {"engine_bf16_fp32": eng2, "one_at_a_time_fp32": base2},
            "burst_all_at_t0": {"engine_solves_per_s": burst["solves_per_s"],
                                "one_at_a_time_solves_per_s": round(mu1, 2),
                                "engine_p99_ms": burst["p99_ms"], "peak_active": burst["peak_active"],
                                "engine_solves_per_s_device_inputs": burst_dev["solves_per_s"],
                                "engine_p99_ms_device_inputs": burst_dev["p99_ms"],
                                "converged_device_inputs": burst_dev["converged"]}}


def secondary_bench(args):
    """The other measured configurations, one line each (not the headline)."""
    import numpy as np
    import torch

    import workloads
    from paper_2002_12872_amd import dpt
    out = {}
    # small dense symmetric FP64, N = 64, to max|dZ| < 1e-12
    th, de = workloads.dense_sym_small(0)
    spec = dpt.ProblemSpec(torch.from_numpy(th).cuda(), torch.from_numpy(de).cuda(), 1.0)
    o = dpt.options(tol=1e-12, max_iter=200, precision=dpt.DPT_FP64)
    for _ in range(3):
        dpt.dpt_destroy(dpt.dpt_init(spec, o))
    t = time.perf_counter()
    reps = 50
    for _ in range(reps):
        h = dpt.dpt_init(spec, o)
        r = dpt.dpt_solve(h, history_cap=0)
        dpt.dpt_eigenvalues(h)
        dpt.dpt_destroy(h)
    out["dense_sym_n64_fp64"] = {"us_per_solve": round(1e6 * (time.perf_counter() - t) / reps, 1),
                                 "iters": r["iters"], "status": r["status"]}
    # dense unsymmetric FP32, N = 4096, 30 steps
    n = 4096
    th, de = workloads.dense_unsym(0, n=n)
    spec = dpt.ProblemSpec(torch.from_numpy(th).cuda(), torch.from_numpy(de).cuda(), 1.0)
    h = dpt.dpt_init(spec, dpt.options(precision=dpt.DPT_FP32))
    dpt.dpt_step(h, 2)
    dpt.dpt_profile_enable(h, True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    dpt.dpt_step(h, 30)
    el = time.perf_counter() - t
    pr = dpt.dpt_profile_read(h)
    gms = pr["gemm_fp32"][0] / pr["gemm_fp32"][1]
    out["dense_unsym_n4096_fp32"] = {"iter_s": round(30 / el, 2), "ms_per_step": round(1e3 * el / 30, 3),
                                     "gemm_fp32_ms": round(gms, 4),
                                     "gemm_tflops": round(2.0 * n ** 3 / (gms * 1e-3) / 1e12, 2),
                                     "frac_fp32_peak": round(2.0 * n ** 3 / (gms * 1e-3) / 1e12 / 157.3, 3)}
    dpt.dpt_destroy(h)
    # sparse symmetric N = 32768: SpMM full update and dominant eigenvector
    n = 32768
    th, ip, ix, v = workloads.sparse_sym(0, n=n)
    csr = (torch.from_numpy(ip).cuda(), torch.from_numpy(ix).cuda(), torch.from_numpy(v).cuda())
    spec = dpt.ProblemSpec(torch.from_numpy(th).cuda(), csr, 1.0)
    h = dpt.dpt_init(spec, dpt.options(precision=dpt.DPT_FP32))
    dpt.dpt_step(h, 4)                                   # the state is dense after a few steps
    dpt.dpt_profile_enable(h, True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    dpt.dpt_step(h, 20)
    el = time.perf_counter() - t
    pr = dpt.dpt_profile_read(h)
    sms = pr["spmm"][0] / pr["spmm"][1]
    nnz = int(v.shape[0])
    step_bytes = 2 * 4 * n * n + 8 * nnz + 4 * (n + 1)   # Z in + Z' out + CSR
    gather = 4 * nnz * n
    out["sparse_sym_n32768_spmm_fp32"] = {
        "nnz": nnz, "ms_per_step": round(1e3 * el / 20, 3), "spmm_ms": round(sms, 4),
        "hbm_gbs": round(step_bytes / (sms * 1e-3) / 1e9, 1),
        "frac_hbm_peak": round(step_bytes / (sms * 1e-3) / 1e9 / PEAK_HBM_GBS, 3),
        "l2_gather_gbs": round(gather / (sms * 1e-3) / 1e9, 1),
        "algorithmic_bytes_per_step": step_bytes}
    # gather roof: random 512-byte runs from one panel of the same size (16 MiB),
    # as many as the product gathers per step
    p_ms, p_gbs = dpt.dpt_probe_gather(n, nnz * (n // 128), 5)
    out["sparse_sym_n32768_spmm_fp32"].update({
        "gather_roof_gbs": round(p_gbs, 1), "gather_roof_ms": round(p_ms, 3),
        "frac_gather_roof": round((gather / (sms * 1e-3) / 1e9) / p_gbs, 3)})
    dpt.dpt_destroy(h)
    o = dpt.options(tol=1e-6, max_iter=50, precision=dpt.DPT_FP32)
    for _ in range(3):
        dpt.dpt_dominant(spec, o)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = 20
    for _ in range(reps):
        ev, vec, r = dpt.dpt_dominant(spec, o)
    torch.cuda.synchronize()
    out["sparse_sym_n32768_dominant_fp32"] = {"us_per_solve": round(1e6 * (time.perf_counter() - t) / reps, 1),
                                              "iters": r["iters"], "eigenvalue": ev}
    del csr, spec
    if args.paper_scale:
        out["sparse_sym_n4194304_dominant_fp32"] = paper_scale_dominant()
    return out


def paper_scale_dominant():
    """Dominant pair of a sparse symmetric matrix of the size of the paper's Fig. 5
    example (1e8 non-zeros): N = 2^22, 16 random columns per row symmetrised
    (1.34e8 nnz, 1.07 GB CSR), device-resident, FP32, tol 1e-6.  The SpMV
    iteration rate is the difference of calls capped at 4 and at 1 iterations."""
    import numpy as np
    import torch

    import workloads
    from paper_2002_12872_amd import dpt
    n = 1 << 22
    t = time.perf_counter()
    th, ip, ix, v = workloads.sparse_sym(0, n=n)
    gen_s = time.perf_counter() - t
    nnz = int(v.shape[0])
    spec = dpt.ProblemSpec(torch.from_numpy(th).cuda(), (torch.from_numpy(ip).cuda(), torch.from_numpy(ix).cuda(),
                                                          torch.from_numpy(v).cuda()), 1.0)
    del th, ip, ix, v
    o = dpt.options(tol=1e-6, max_iter=50, precision=dpt.DPT_FP32)
    ev, vec, r = dpt.dpt_dominant(spec, o)
    torch.cuda.synchronize()
    reps = 5
    t = time.perf_counter()
    for _ in range(reps):
        ev, vec, r = dpt.dpt_dominant(spec, o)
    torch.cuda.synchronize()
    per_solve = (time.perf_counter() - t) / reps

    def capped(k):
        oc = dpt.options(tol=1e-30, max_iter=k, precision=dpt.DPT_FP32)
        dpt.dpt_dominant(spec, oc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            dpt.dpt_dominant(spec, oc)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps
    per_iter = (capped(4) - capped(1)) / 3.0
    it_bytes = nnz * 8 + 8 * (n + 1) + 2 * 4 * n          # CSR stream + z read + z' write (gathers: cache)
    # machine precision, as in the paper: FP64 iteration to max|dz| < 1e-14
    o64 = dpt.options(tol=1e-14, max_iter=50, precision=dpt.DPT_FP64)
    dpt.dpt_dominant(spec, o64)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ev64, _, r64 = dpt.dpt_dominant(spec, o64)
    torch.cuda.synchronize()
    fp64 = {"ms_per_solve": round(1e3 * (time.perf_counter() - t), 3), "iters": r64["iters"],
            "status": r64["status"], "eigenvalue": ev64}
    return {"n": n, "nnz": nnz, "csr_gb": round((nnz * 8 + 8 * (n + 1)) / 1e9, 3), "iters": r["iters"],
            "fp64_to_1e-14": fp64, "status": r["status"], "ms_per_solve": round(1e3 * per_solve, 3),
            "ms_per_iteration": round(1e3 * per_iter, 3),
            "hbm_gbs_per_iteration": round(it_bytes / per_iter / 1e9, 1),
            "frac_hbm_peak": round(it_bytes / per_iter / 1e9 / PEAK_HBM_GBS, 3),
            "eigenvalue": ev, "generation_s": round(gen_s, 1),
            "paper": "4 iterations, 3 s (Mathematica on a desktop CPU, 1e8 nnz; Sec. II.H)"}


def vendor_gemm_reference(n):
    """The vendor library's plain GEMM (torch.matmul -> hipBLASLt) at the same
    size, for context: the fused steps add the update, the BF16 shadow and the
    statistics to a product of this shape."""
    import torch
    out = {}
    for name, dt, reps in (("bf16", torch.bfloat16, 5), ("fp32", torch.float32, 3)):
        a = torch.randn(n, n, device="cuda").to(dt)
        b = torch.randn(n, n, device="cuda").to(dt)
        torch.matmul(a, b)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            torch.matmul(a, b)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        peak = PEAK_BF16_TFLOPS if name == "bf16" else PEAK_FP32_TFLOPS
        tf = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
        out[name] = {"ms": round(ms, 3), "tflops": round(tf, 1), "frac_peak": round(tf / peak, 3)}
        del a, b
    torch.cuda.empty_cache()
    return out


def next_rows_bench():
    """Per-row retirement, homotopy continuation, Rayleigh-Schroedinger comparator
    and the coupling ramp, one line each (device-resident inputs)."""
    import numpy as np
    import torch

    import workloads
    from paper_2002_12872_amd import dpt
    out = {}

    def dev(x):
        return torch.from_numpy(np.ascontiguousarray(x)).cuda()

    # per-row retirement on the delta-potential (Sec. II.F): the lowest level
    # converges last, most rows freeze after 6-7 steps
    n = 8192
    th, de = workloads.delta_potential(n)
    spec = dpt.ProblemSpec(dev(th), dev(de), 1.0)
    line = {"workload": "delta-potential N=%d (theta_n = 2n + 1/2, Delta = phi phi^T), lambda = 1, FP64, "
                        "tol 1e-12" % n}
    for name, rule in (("delta_rule", dpt.DPT_STOP_DELTA), ("per_row", dpt.DPT_STOP_ROW)):
        o = dpt.options(tol=1e-12, max_iter=200, precision=dpt.DPT_FP64, stop_rule=rule)
        dpt.dpt_destroy(dpt.dpt_init(spec, o))
        torch.cuda.synchronize()
        t = time.perf_counter()
        h = dpt.dpt_init(spec, o)
        r = dpt.dpt_solve(h, history_cap=0)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        at, rows_mult = dpt.dpt_row_status(h)
        line[name] = {"ms_per_solve": round(1e3 * el, 2), "iters": r["iters"], "status": r["status"]}
        if rule == dpt.DPT_STOP_ROW:
            full = n * (r["iters"] - 1)
            line[name]["rows_multiplied"] = int(rows_mult)
            line[name]["products_saved"] = round(1.0 - rows_mult / full, 3)
            line[name]["rows_frozen_by_step"] = {int(k): int(v) for k, v in
                                                 zip(*np.unique(at, return_counts=True))}
        dpt.dpt_destroy(h)
    line["speedup"] = round(line["delta_rule"]["ms_per_solve"] / line["per_row"]["ms_per_solve"], 3)
    out["per_row_retirement"] = line
    del spec
    # homotopy: the delta-potential beyond the plain iteration's radius (about 2.9)
    n = 2048
    th, de = workloads.delta_potential(n)
    spec = dpt.ProblemSpec(dev(th), dev(de), 4.0)
    o = dpt.options(tol=1e-12, max_iter=500, precision=dpt.DPT_FP64)
    plain = dpt.dpt_solve(dpt.dpt_init(spec, o), history_cap=0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    e, z, r = dpt.dpt_homotopy(spec, o, 2)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    w = np.linalg.eigvalsh(np.diag(th) + 4.0 * de)
    out["homotopy"] = {"workload": "delta-potential N=%d, lambda = 4, 2 stages, FP64 tol 1e-12" % n,
                       "plain_status": plain["status"], "status": r["status"], "iters": r["iters"],
                       "ms": round(1e3 * el, 2),
                       "max_rel_eigenvalue_error_vs_eigvalsh": float(np.max(np.abs(e.cpu().numpy() - w) /
                                                                            np.abs(w)))}
    del spec, z
    # Rayleigh-Schroedinger comparator (Sec. II.F): orders vs D-PT iterations
    th, de = workloads.delta_potential(100)
    rs = {}
    for lam in (1.5, 2.5):
        exact = np.linalg.eigvalsh(np.diag(th) + lam * de)
        eps, _, _ = dpt.dpt_rs_series(dpt.ProblemSpec(th, de, lam, stream=0), 120, want_z=False)
        partial = th[None, :] + np.cumsum((lam ** np.arange(1, 121))[:, None] * eps, axis=0)
        err_rs = np.max(np.abs(partial - exact) / np.abs(exact), axis=1)
        h = dpt.dpt_init(dpt.ProblemSpec(th, de, lam, stream=0), dpt.options(precision=dpt.DPT_FP64))
        err_d = []
        for _ in range(400):
            dpt.dpt_step(h, 1)
            err_d.append(float(np.max(np.abs(dpt.dpt_eigenvalues(h) - exact) / np.abs(exact))))
            if err_d[-1] < 1e-12:
                break
        hit = lambda errs: int(np.argmax(np.asarray(errs) < 1e-8)) + 1 if min(errs) < 1e-8 else None
        rs["lambda_%g" % lam] = {"rs_orders_to_1e-8": hit(err_rs), "dpt_iterations_to_1e-8": hit(err_d),
                                 "rs_error_at_order_120": float(err_rs[-1]), "dpt_error_final": err_d[-1]}
    n = 4096
    th, de = small_problem_sym(n)
    spec = dpt.ProblemSpec(dev(th), dev(de), 0.5)
    dpt.dpt_rs_series(spec, 2, want_z=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    dpt.dpt_rs_series(spec, 10, want_z=False)
    torch.cuda.synchronize()
    rs["n4096_fp64_ms_per_order"] = round(1e3 * (time.perf_counter() - t) / 10, 3)
    rs["workload"] = "delta-potential N=100 (Sec. II.F); timing: dense symmetric N=4096, 10 orders"
    out["rs_comparator"] = rs
    # coupling ramp (Supplement E) on the 4x4 example whose plain iteration diverges
    th4 = np.arange(4.0)
    de4 = np.array([[0.0, 0.4, -0.25, 1.15], [0.4, 0.0, 0.9, -1.05], [-0.25, 0.9, 0.0, 0.4],
                    [1.15, -1.05, 0.4, 0.0]])
    sp4 = dpt.ProblemSpec(th4, de4, 0.75, stream=0)
    r_plain = dpt.dpt_solve(dpt.dpt_init(sp4, dpt.options(tol=1e-13, max_iter=3000, precision=dpt.DPT_FP64)))
    t = time.perf_counter()
    h = dpt.dpt_init(sp4, dpt.options(tol=1e-13, max_iter=3000, precision=dpt.DPT_FP64, ramp_alpha=0.9))
    r_ramp = dpt.dpt_solve(h, history_cap=0)
    el = time.perf_counter() - t
    w = np.linalg.eigvalsh(np.diag(th4) + 0.75 * de4)
    out["ramp"] = {"workload": "4x4, theta = (0,1,2,3), lambda = 0.75, alpha = 0.9, FP64 tol 1e-13",
                   "plain_status": r_plain["status"], "status": r_ramp["status"], "iters": r_ramp["iters"],
                   "ms": round(1e3 * el, 2),
                   "max_abs_eigenvalue_error": float(np.max(np.abs(dpt.dpt_eigenvalues(h) - w)))}
    return out


def small_problem_sym(n, seed=0):
    """Dense symmetric test matrix: theta_i = i + U(0, 0.5) sorted, Delta = (R + R^T)/2,
    R off-diagonal iid N(0, (0.5/sqrt n)^2)."""
    import numpy as np
    rng = np.random.default_rng(77_000 + seed)
    theta = np.sort(np.arange(n, dtype=np.float64) + rng.uniform(0, 0.5, n))
    r = rng.normal(0, 0.5 / np.sqrt(n), (n, n))
    np.fill_diagonal(r, 0.0)
    return theta, 0.5 * (r + r.T)


def host_info():
    """CPU of the machine the baseline runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def cpu_baselines(threads):
    """The FP64 oracle on the other configurations (host cores, and one core):
    full solves where they fit a few seconds (N = 64), per-row samples scaled by
    N / rows otherwise (rows evolve independently, so a sample's time per row is
    the full solve's), and the serving mix on its first requests."""
    import numpy as np

    import oracle
    import workloads
    out = {"host": host_info(), "threads": threads}
    th, de = workloads.dense_sym_small(0)
    t = time.perf_counter()
    reps = 5
    for _ in range(reps):
        r = oracle.iterate(th, de, 1.0, max_iter=200, tol=1e-12)
    out["dense_sym_n64_fp64_full_solve"] = {"us_per_solve": round(1e6 * (time.perf_counter() - t) / reps, 1),
                                            "iters": r["iters"]}
    n = 4096
    th, de = workloads.dense_unsym(0, n=n)
    rows = workloads.sample_rows(n, 32)
    t = time.perf_counter()
    oracle.iterate(th, de.astype(np.float64), 1.0, rows=rows, max_iter=30, fixed_steps=True)
    el = time.perf_counter() - t
    out["dense_unsym_n4096_30_steps"] = {"iter_s": round(30 * len(rows) / n / el, 4),
                                         "sample": "%d of %d rows, 30 FP64 steps in %.2f s, scaled by rows/N"
                                                   % (len(rows), n, el)}
    trace = workloads.serving_trace(0, count=4096, rate=None)
    count = 32
    t = time.perf_counter()
    for req in trace[:count]:
        th, de = workloads.request_matrices(req)
        oracle.iterate(th, de.astype(np.float64), 1.0, max_iter=100, tol=1e-5)
    el = time.perf_counter() - t
    out["serving_mix_full_solves"] = {"solves_per_s": round(count / el, 3),
                                      "sample": "first %d of 4096 trace requests, full FP64 solves to tol 1e-5 "
                                                "in %.2f s" % (count, el)}
    n = 16384
    th, de = workloads.dense_sym_large(0, n=n)
    rows = workloads.sample_rows(n, 64)[:4]
    t = time.perf_counter()
    r = oracle.iterate(th, de.astype(np.float64), 1.0, rows=rows, max_iter=40, tol=1e-14, nthreads=1)
    el = time.perf_counter() - t
    out["one_core_dense_sym_n16384"] = {"iter_s": round(r["iters"] * len(rows) / n / el, 7), "cores": 1,
                                        "sample": "%d rows, %d FP64 iterations in %.2f s on one thread, scaled "
                                                  "by rows/N" % (len(rows), r["iters"], el)}
    return out


def kernel_only(args):
    """Fused product steps of one precision at size n only (for counter
    collection with rocprofv3): BF16 steps of the BF16 -> FP32 form, or FP32 steps."""
    import torch

    import workloads
    from paper_2002_12872_amd import dpt
    theta, delta = workloads.dense_sym_large(0, n=args.n)
    spec = dpt.ProblemSpec(torch.from_numpy(theta).cuda(), torch.from_numpy(delta).cuda(), 1.0)
    prec = {"bf16": dpt.DPT_BF16_FP32, "fp32": dpt.DPT_FP32, "fp64": dpt.DPT_FP64}[args.kernel_precision]
    h = dpt.dpt_init(spec, dpt.options(precision=prec))
    dpt.dpt_step(h, 1 + args.warmup)            # first iterate (no product) + warm-up steps
    dpt.dpt_profile_enable(h, True)
    last = dpt.dpt_step(h, args.steps)
    prof = dpt.dpt_profile_read(h)
    print(json.dumps({"mode": "kernel-only", "precision": args.kernel_precision, "n": args.n,
                      "steps": args.steps, "last_delta": last,
                      "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in prof.items()}}), flush=True)


def spmm_only(args):
    """CSR product steps of the sparse workload (N = 32768, ~1.05e6 non-zeros,
    FP32) after 4 warm-up steps (the state is dense by then)."""
    import torch

    import workloads
    from paper_2002_12872_amd import dpt
    n = 32768
    th, ip, ix, v = workloads.sparse_sym(0, n=n)
    spec = dpt.ProblemSpec(torch.from_numpy(th).cuda(), (torch.from_numpy(ip).cuda(), torch.from_numpy(ix).cuda(),
                                                          torch.from_numpy(v).cuda()), 1.0)
    h = dpt.dpt_init(spec, dpt.options(precision=dpt.DPT_FP32))
    dpt.dpt_step(h, 4)
    dpt.dpt_profile_enable(h, True)
    last = dpt.dpt_step(h, args.steps)
    prof = dpt.dpt_profile_read(h)
    print(json.dumps({"mode": "spmm-only", "n": n, "nnz": int(v.shape[0]), "steps": args.steps,
                      "last_delta": last, "kernel_ms": {k: x[0] / max(x[1], 1) for k, x in prof.items()}}),
          flush=True)


def serve_only(args):
    """The serving engine on the first --serve-requests requests of the trace,
    all submitted at once (BF16 -> FP32, tol 1e-5)."""
    import workloads
    from paper_2002_12872_amd import dpt
    trace = workloads.serving_trace(0, count=4096, rate=None)[:args.serve_requests]
    specs = [dpt.ProblemSpec(th, de, 1.0, stream=0) for th, de in (workloads.request_matrices(r) for r in trace)]
    o = dpt.options(tol=1e-5, max_iter=100, precision=dpt.DPT_BF16_FP32)
    srv = dpt.dpt_serve_open(int(args.serve_budget_gib * (1 << 30)), max_slots=1024, use_graph=True, autotune=True)
    t = time.perf_counter()
    tickets = [dpt.dpt_serve_submit(srv, sp, o) for sp in specs]
    res = [dpt.dpt_serve_poll(srv, x, wait_ms=-1) for x in tickets]
    el = time.perf_counter() - t
    st = dpt.dpt_serve_stats_read(srv)
    dpt.dpt_serve_close(srv)
    print(json.dumps({"mode": "serve-only", "requests": len(specs), "solves_per_s": round(len(specs) / el, 2),
                      "converged": sum(r["status"] == dpt.DPT_OK for r in res), "steps": st["steps"]}),
          flush=True)


def copy_probe(args):
    """Plain copy of a known number of bytes (calibrates HBM byte counters)."""
    import torch
    count = args.copy_probe * (1 << 20) // 4
    src = torch.ones(count, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy-probe", "bytes_read": count * 4, "bytes_written": count * 4,
                      "launches": args.steps}), flush=True)


def source_hash(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def read_traffic(kind, n):
    """HBM bytes per launch of a fused product kernel from its committed
    rocprofv3 --pmc summary, if that was taken on the current kernel source at
    this n; None otherwise."""
    info = KERNELS[kind]
    if not os.path.exists(info["traffic"]):
        return None
    vals = {}
    for line in open(info["traffic"]):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != source_hash(info["source"]) or int(vals.get("n", -1)) != n:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def solve_once(dpt, spec, opts, n, profile):
    import torch
    h = dpt.dpt_init(spec, opts)
    if profile:
        dpt.dpt_profile_enable(h, True)
    res = dpt.dpt_solve(h, history_cap=64)
    e = torch.empty(n, dtype=torch.float64, device="cuda")
    dpt.dpt_eigenvalues(h, e)
    return h, res, e


def timed_solves(dpt, spec, opts, n, count, warmup):
    """count solves after warmup ones; returns (elapsed s, results, handles, profile sums, last E)."""
    import torch
    for _ in range(warmup):
        h, _, _ = solve_once(dpt, spec, opts, n, False)
        dpt.dpt_destroy(h)
    torch.cuda.synchronize()
    handles, results = [], []
    t0 = time.perf_counter()
    for _ in range(count):
        h, res, e = solve_once(dpt, spec, opts, n, True)
        handles.append(h)
        results.append(res)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {}
    for h in handles:
        for k, (ms, cnt) in dpt.dpt_profile_read(h).items():
            acc = prof.setdefault(k, [0.0, 0])
            acc[0] += ms
            acc[1] += cnt
    return elapsed, results, handles, prof, e


def roofline_of(kind, prof, n):
    ms, cnt = prof.get(kind, (0.0, 0))
    if cnt == 0:
        return None
    info = KERNELS[kind]
    avg = ms / cnt
    flop = 2.0 * n ** 3
    achieved = flop / (avg * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": info["peak"], "unit": "TFLOP/s",
            "frac": round(achieved / info["peak"], 4), "traffic": read_traffic(kind, n), "kernel": info["name"],
            "avg_launch_ms": round(avg, 4), "launches": cnt, "algorithmic_flop_per_launch": flop}


def accuracy(dpt, h, e_dev, theta, ref, rows, z_scale, z64=False):
    """Errors of a handle's result against the converged FP64 oracle rows
    (eigenvectors exported in FP32, or FP64 with z64)."""
    import numpy as np
    import torch
    n = theta.shape[0]
    z = torch.empty((n, n), dtype=torch.float64 if z64 else torch.float32, device="cuda")
    dpt.dpt_eigenvectors(h, z)
    zr = z[torch.as_tensor(rows, device="cuda")].double().cpu().numpy()
    del z
    e = e_dev.cpu().numpy()[rows]
    e_e = float(np.max(np.abs(e - ref["e"]) / np.maximum(np.abs(ref["e"]), 1e-12 * np.abs(theta).max())))
    e_z = float(np.max(np.abs(zr - ref["z"])) / z_scale)
    return {"max_rel_eigenvalue": e_e, "max_abs_eigenvalue": float(np.max(np.abs(e - ref["e"]))),
            "e_Z": e_z}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the D-PT path runs on a single MI355X "
              "(no multi-GPU path); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.kernel_only:
        return kernel_only(args)
    if args.copy_probe:
        return copy_probe(args)
    if args.spmm_only:
        return spmm_only(args)
    if args.serve_only:
        return serve_only(args)
    if args.secondary_only:
        print(json.dumps({"mode": "secondary-only", "secondary": secondary_bench(args)}), flush=True)
        return
    import numpy as np
    import torch

    import workloads
    from paper_2002_12872_amd import dpt

    n = args.n
    dev = torch.device("cuda:0")
    theta, delta = workloads.dense_sym_large(0, n=n)
    th_d = torch.from_numpy(theta).to(dev)
    de_d = torch.from_numpy(delta).to(dev)
    torch.cuda.synchronize()
    spec = dpt.ProblemSpec(th_d, de_d, 1.0)
    rules = {"estimate": dpt.DPT_STOP_ESTIMATE, "delta": dpt.DPT_STOP_DELTA}
    rule = rules[args.stop_rule]
    other = "delta" if args.stop_rule == "estimate" else "estimate"

    def opts(precision, stop_rule):
        return dpt.options(tol=args.tol, max_iter=100, precision=precision, stop_rule=stop_rule)

    # ---- BF16 -> FP32 solves (the timed steps)
    elapsed, results, handles, prof, e_mixed = timed_solves(dpt, spec, opts(dpt.DPT_BF16_FP32, rule), n,
                                                            args.steps, args.warmup)
    print("# mixed solves: %d in %.3f s, iterations %s" % (args.steps, elapsed,
          [(r["iters_bf16"], r["iters_fp32"]) for r in results]), file=sys.stderr, flush=True)
    iters_total = sum(r["iters"] for r in results)
    gemm_steps = sum(r["iters"] - 1 for r in results)   # the first iterate needs no product
    flop = 2.0 * n ** 3
    value = iters_total / elapsed
    ms_per_solve = 1e3 * elapsed / args.steps

    # roofline: the product kernel with the largest share of the solve time, plus both
    by_kernel = {k: roofline_of(k, prof, n) for k in KERNELS}
    dominant = max((k for k in KERNELS if by_kernel[k]), key=lambda k: prof[k][0])
    roofline = dict(by_kernel[dominant])
    roofline["share_of_solve_gpu_time"] = round(prof[dominant][0] / sum(v[0] for v in prof.values()), 3)
    # the BF16 step, which runs most of the iterations, beside it: fraction of the
    # BF16 matrix-core peak against the 0.6 target
    if by_kernel.get("gemm_bf16"):
        roofline["bf16_step_frac"] = by_kernel["gemm_bf16"]["frac"]
        roofline["bf16_step_target_frac"] = 0.6
        roofline["bf16_step_ms"] = by_kernel["gemm_bf16"]["avg_launch_ms"]

    # ---- plain FP32 solves, same tolerance and stopping rule
    fp32 = None
    f_handles = []
    if args.fp32_solves > 0:
        f_el, f_res, f_handles, f_prof, e_fp32 = timed_solves(dpt, spec, opts(dpt.DPT_FP32, rule), n,
                                                              args.fp32_solves, 1)
        f_avg = f_prof["gemm_fp32"][0] / max(f_prof["gemm_fp32"][1], 1)
        fp32 = {"iter_s": round(sum(r["iters"] for r in f_res) / f_el, 3),
                "ms_per_solve": round(1e3 * f_el / args.fp32_solves, 2),
                "iters": f_res[0]["iters"],
                "gemm_fp32_avg_ms": round(f_avg, 3),
                "gemm_fp32_tflops": round(flop / (f_avg * 1e-3) / 1e12, 2)}

    # ---- the other stopping rule, one solve of each form (context)
    other_rule = {}
    for name, prec in (("bf16_fp32", dpt.DPT_BF16_FP32), ("fp32", dpt.DPT_FP32)):
        el, rs, hs, _, _ = timed_solves(dpt, spec, opts(prec, rules[other]), n, 1, 0)
        other_rule[name] = {"ms_per_solve": round(1e3 * el, 2), "iters": [rs[0]["iters_bf16"], rs[0]["iters_fp32"]]}
        for h in hs:
            dpt.dpt_destroy(h)
    other_rule["speedup_bf16_fp32_vs_fp32"] = round(other_rule["fp32"]["ms_per_solve"] /
                                                    other_rule["bf16_fp32"]["ms_per_solve"], 3)

    # ---- FP8 experiment: block-scaled E4M3 products until stall, then FP32 (same rule)
    el8, rs8, hs8, prof8, e_fp8 = timed_solves(dpt, spec, opts(dpt.DPT_FP8_FP32, rule), n, 1, 1)
    g8 = prof8.get("gemm_fp8", (float("nan"), 1))
    fp8 = {"ms_per_solve": round(1e3 * el8, 2), "iters": [rs8[0]["iters_bf16"], rs8[0]["iters_fp32"]],
           "gemm_fp8_ms": round(g8[0] / max(g8[1], 1), 4),
           "gemm_fp8_tflops": round(flop / (g8[0] / max(g8[1], 1) * 1e-3) / 1e12, 2),
           "frac_fp8_peak": round(flop / (g8[0] / max(g8[1], 1) * 1e-3) / 1e12 / PEAK_FP8_TFLOPS, 4)}

    # ---- split-BF16 sweeps (experiment): BF16 steps, then FP32-grade sweeps whose
    # product is three BF16 products of split operands (same rule)
    elx, rsx, hsx, profx, e_x3 = timed_solves(dpt, spec, opts(dpt.DPT_BF16_X3, rule), n, 1, 1)
    gx = profx.get("gemm_x3", (float("nan"), 1))
    gx_ms = gx[0] / max(gx[1], 1)
    x3 = {"ms_per_solve": round(1e3 * elx, 2), "iters": [rsx[0]["iters_bf16"], rsx[0]["iters_fp32"]],
          "gemm_x3_ms": round(gx_ms, 4),
          "fp32_equivalent_tflops": round(flop / (gx_ms * 1e-3) / 1e12, 2),
          "bf16_tflops_executed": round(3 * flop / (gx_ms * 1e-3) / 1e12, 2),
          "frac_bf16_peak": round(3 * flop / (gx_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS, 4),
          "speedup_vs_bf16_fp32": round(ms_per_solve / (1e3 * elx), 3)}

    # ---- optional FP64 final sweeps to 1e-10 after the FP32 phase (same rule)
    o64 = dpt.options(tol=args.tol, max_iter=100, precision=dpt.DPT_BF16_FP32, fp64_final_tol=1e-10,
                      stop_rule=rule)
    el64, rs64, hs64, prof64, e_f64 = timed_solves(dpt, spec, o64, n, 1, 0)
    g64 = prof64.get("gemm_fp64", (float("nan"), 1))
    g64_ms = g64[0] / max(g64[1], 1)
    fp64_final = {"ms_per_solve": round(1e3 * el64, 2), "status": rs64[0]["status"],
                  "iters": [rs64[0]["iters_bf16"], rs64[0]["iters_fp32"], rs64[0]["iters_fp64"]],
                  "gemm_fp64_ms": round(g64_ms, 3),
                  "gemm_fp64_tflops": round(flop / (g64_ms * 1e-3) / 1e12, 2),
                  "frac_fp64_peak": round(flop / (g64_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_solve, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16->fp32", "data": "synthetic",
        "config": {"workload": "dense symmetric N=%d, theta_i=i/4, Delta=(R+R^T)/2, "
                               "R~N(0,(0.25/sqrt N)^2) zero diagonal, lambda=1; "
                               "BF16->FP32 solve to tol %g (%s stopping rule)" % (n, args.tol, args.stop_rule),
                   "n": n, "tol": args.tol, "stop_rule": args.stop_rule,
                   "step": "one full solve (init+solve+readout)"},
        "iters_per_solve": [r["iters"] for r in results],
        # the first application of the map is the closed form F(I): one product fewer
        "products_per_solve": [r["iters"] - 1 for r in results],
        "product_steps_per_s": round(gemm_steps / elapsed, 3),
        "iters_bf16_fp32": [results[0]["iters_bf16"], results[0]["iters_fp32"]],
        "delta_history": [float("%.3g" % x) for x in results[0]["history"]],
        "solve_tflops": round(gemm_steps * flop / elapsed / 1e12, 2),
        "kernel_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()},
        "roofline": roofline,
        "roofline_by_kernel": by_kernel,
        "fp32": fp32,
        "speedup_vs_fp32": (round(fp32["ms_per_solve"] / ms_per_solve, 3) if fp32 else None),
        "other_stop_rule": {"rule": other, **other_rule},
        "vendor_plain_gemm_same_size": vendor_gemm_reference(n),
        "fp8_fp32_experiment": fp8,
        "bf16_x3_experiment": x3,
        "bf16_fp32_fp64_to_1e-10": fp64_final,
    }

    # ---- FP64 oracle on 64 sampled rows: converged reference and CPU baseline
    if not args.skip_cpu:
        import oracle
        threads = oracle.max_threads()
        rows = workloads.sample_rows(n, 64)
        d64 = delta.astype(np.float64)
        t = time.perf_counter()
        ref = oracle.iterate(theta, d64, 1.0, rows=rows, max_iter=40, tol=1e-14)
        cpu_t = time.perf_counter() - t
        k = ref["iters"]
        out["cpu_baseline"] = {"value": round(k * (len(rows) / n) / cpu_t, 6), "unit": "iter/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "%d of %d eigenvector rows (rows evolve independently), %d FP64 "
                                         "iterations to max|dz| < 1e-14 in %.1f s, scaled by rows/N"
                                         % (len(rows), n, k, cpu_t)}
        print("# CPU oracle on the other configurations", file=sys.stderr, flush=True)
        out["cpu_baseline"]["other_configs"] = cpu_baselines(threads)
        z_scale = float(np.max(np.abs(ref["z"] - np.eye(n)[rows])))
        err = {"reference": "FP64 oracle, %d rows, %d iterations" % (len(rows), k),
               "bf16_fp32": accuracy(dpt, handles[-1], e_mixed, theta, ref, rows, z_scale)}
        res = dpt.dpt_residuals(handles[-1], rows)
        norm_ub = np.abs(theta).max() + np.sqrt(np.sum(d64 ** 2))
        zr = dpt.dpt_eigenvectors(handles[-1])[rows] if n <= 4096 else None
        if zr is None:
            zt = torch.empty((n, n), dtype=torch.float32, device="cuda")
            dpt.dpt_eigenvectors(handles[-1], zt)
            zr = zt[torch.as_tensor(rows, device="cuda")].double().cpu().numpy()
            del zt
        # ||M z - E z||_2 / (||M||_ub ||z||_2), ||M||_ub = max|theta| + |lambda| ||Delta||_F
        err["bf16_fp32"]["residual_rel"] = float(np.max(res / (norm_ub * np.linalg.norm(zr, axis=1))))
        err["bf16_fp32"]["residual_norm"] = "||Mz - Ez||_2 / ((max|theta| + |lambda| ||Delta||_F) ||z||_2)"
        if f_handles:
            err["fp32"] = accuracy(dpt, f_handles[-1], e_fp32, theta, ref, rows, z_scale)
        err["fp8_fp32"] = accuracy(dpt, hs8[-1], e_fp8, theta, ref, rows, z_scale)
        err["bf16_x3"] = accuracy(dpt, hsx[-1], e_x3, theta, ref, rows, z_scale)
        err["bf16_fp32_fp64"] = accuracy(dpt, hs64[-1], e_f64, theta, ref, rows, z_scale, z64=True)
        out["error_vs_fp64_oracle"] = err
    for h in handles + f_handles + hs8 + hsx + hs64:
        dpt.dpt_destroy(h)
    if args.serve_requests > 0:
        print("# serving trace of %d requests" % args.serve_requests, file=sys.stderr, flush=True)
        out["serving"] = serving_bench(args)
    if not args.skip_secondary:
        print("# secondary configurations", file=sys.stderr, flush=True)
        out["secondary"] = secondary_bench(args)
        print("# per-row retirement, homotopy, RS comparator, ramp", file=sys.stderr, flush=True)
        out["next_rows"] = next_rows_bench()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
