"""dpt_dominant_noalloc: the dominant mode with its work buffers in the library's
fixed per-device array, checked against dpt_dominant (which allocates them).

Both entry points run the same kernels in the same order on the same inputs,
so eigenvalue, eigenvector and the delta history must agree bitwise.  Two
calls in a row (the second on a smaller problem) show that the contents the
first call leaves in the shared array do not leak into the next.
"""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

dpt = pytest.importorskip("paper_2002_12872_amd.dpt")


def device(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def csr_spec(n, seed, dtype):
    theta, ip, ix, v = workloads.sparse_sym(seed, n=n, dtype=dtype)
    return dpt.ProblemSpec(device(theta), (device(ip), device(ix), device(v)), 1.0)


def dense_spec(n, seed, dtype):
    rng = np.random.default_rng(500 + seed)
    theta = np.sort(np.arange(n, dtype=np.float64) + rng.uniform(0, 0.5, n))
    delta = rng.normal(0, 0.5 / np.sqrt(n), (n, n))
    np.fill_diagonal(delta, 0.0)
    return dpt.ProblemSpec(device(theta), device(delta.astype(dtype)), 0.8)


def both(spec, opts, dtype, index=-1):
    import torch
    n = spec.struct.n
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    ev_a, vec_a, res_a = dpt.dpt_dominant(spec, opts, index=index)
    out = torch.full((n,), float("nan"), dtype=tdt, device="cuda")
    ev_b, vec_b, res_b = dpt.dpt_dominant_noalloc(spec, opts, out, index=index)
    torch.cuda.synchronize()
    assert res_a["status"] == res_b["status"] and res_a["iters"] == res_b["iters"]
    assert ev_a == ev_b
    assert torch.equal(vec_a, vec_b)
    assert np.array_equal(res_a["history"], res_b["history"])
    return ev_b, res_b


@pytest.mark.parametrize("precision,dtype", [(dpt.DPT_FP32, np.float32), (dpt.DPT_FP64, np.float64)])
def test_noalloc_equals_dominant_csr_twice_then_smaller(precision, dtype):
    opts = dpt.options(tol=1e-12 if precision == dpt.DPT_FP64 else 1e-6, max_iter=60, precision=precision)
    ev1, r1 = both(csr_spec(40000, 1, dtype), opts, dtype)
    assert r1["status"] == dpt.DPT_OK and r1["iters"] >= 2
    ev2, r2 = both(csr_spec(40000, 1, dtype), opts, dtype)          # same problem again
    assert ev2 == ev1
    ev3, r3 = both(csr_spec(3000, 2, dtype), opts, dtype, index=1234)  # smaller, explicit index
    assert r3["status"] == dpt.DPT_OK


@pytest.mark.parametrize("precision,dtype", [(dpt.DPT_FP32, np.float32), (dpt.DPT_FP64, np.float64)])
def test_noalloc_equals_dominant_dense(precision, dtype):
    opts = dpt.options(tol=1e-12 if precision == dpt.DPT_FP64 else 1e-6, max_iter=80, precision=precision)
    both(dense_spec(700, 3, dtype), opts, dtype)
    both(dense_spec(130, 4, dtype), opts, dtype, index=17)


def test_noalloc_rejections():
    import torch
    lib = dpt.load_library()
    spec = csr_spec(2000, 5, np.float32)
    out = torch.empty(2000, dtype=torch.float32, device="cuda")
    ev = ctypes.c_double()
    r = dpt.Result()
    # iteration cap above the fixed statistics area
    rc = lib.dpt_dominant_noalloc(ctypes.byref(spec.struct), ctypes.byref(dpt.options(max_iter=4097)), -1,
                                  ctypes.byref(ev), out.data_ptr(), ctypes.byref(r))
    assert rc == dpt.DPT_EINVAL
    # FP64 precision on FP32 values (would need a conversion copy)
    rc = lib.dpt_dominant_noalloc(ctypes.byref(spec.struct), ctypes.byref(dpt.options(precision=dpt.DPT_FP64)), -1,
                                  ctypes.byref(ev), out.data_ptr(), ctypes.byref(r))
    assert rc == dpt.DPT_EINVAL
    # host-resident problem
    theta, ip, ix, v = workloads.sparse_sym(5, n=2000)
    host = dpt.ProblemSpec(theta, (ip, ix, v), 1.0, stream=0)
    rc = lib.dpt_dominant_noalloc(ctypes.byref(host.struct), ctypes.byref(dpt.options()), -1,
                                  ctypes.byref(ev), out.data_ptr(), ctypes.byref(r))
    assert rc == dpt.DPT_EINVAL
    # an order beyond the fixed iterate area is refused before any device work
    big = dpt.Problem()
    ctypes.memmove(ctypes.byref(big), ctypes.byref(spec.struct), ctypes.sizeof(dpt.Problem))
    big.n = 8388609
    rc = lib.dpt_dominant_noalloc(ctypes.byref(big), ctypes.byref(dpt.options()), -1,
                                  ctypes.byref(ev), out.data_ptr(), ctypes.byref(r))
    assert rc == dpt.DPT_EINVAL
    # a malformed device CSR is caught by the device check
    ip_bad = ip.copy()
    ip_bad[1000] = ip_bad[1001] + 1
    bad = dpt.ProblemSpec(device(theta), (device(ip_bad), device(ix), device(v)), 1.0)
    with pytest.raises(dpt.DptError):
        dpt.dpt_dominant_noalloc(bad, dpt.options(), out)
    # and a valid call right after still matches the allocating entry point
    both(spec, dpt.options(tol=1e-6, max_iter=50), np.float32)
