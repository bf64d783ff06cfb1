"""Thin ctypes binding of the C ABI declared in ``include/dpt.h``.

Argument marshalling only: every step of the method runs in the HIP library
``_lib/libdpt.so``.  Importing this module fails loudly when the library has not
been built; there is no CPU fallback.

Inputs may be numpy arrays / CPU tensors (host memory, copied by the library) or
torch device tensors (borrowed by the library; keep them alive and unchanged
while the handle lives).  Function names mirror the C entry points.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libdpt.so")

DPT_OK, DPT_NOT_CONVERGED, DPT_STALLED, DPT_DIVERGED, DPT_EAGAIN = 0, 1, 2, 3, 4
DPT_EINVAL, DPT_ENOMEM, DPT_EDEVICE, DPT_ESTATE = -1, -2, -3, -4
DPT_FP64, DPT_FP32, DPT_BF16_FP32, DPT_FP8_FP32, DPT_BF16_X3 = 0, 1, 2, 3, 4
DPT_DENSE, DPT_CSR = 0, 1
DPT_MEM_HOST, DPT_MEM_DEVICE = 0, 1
DPT_DTYPE_F64, DPT_DTYPE_F32 = 0, 1
DPT_STOP_DELTA, DPT_STOP_ESTIMATE, DPT_STOP_ROW = 0, 1, 2


class DptError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s%s" % (what + ": " if what else "", status_str(code)))


class Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("theta", ctypes.c_void_p),
        ("delta", ctypes.c_void_p),
        ("indptr", ctypes.c_void_p),
        ("indices", ctypes.c_void_p),
        ("nnz", ctypes.c_int64),
        ("lam", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("format", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("mem", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("fp64_final_tol", ctypes.c_double),
        ("stall_ratio", ctypes.c_double),
        ("blowup", ctypes.c_double),
        ("ramp_alpha", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("stall_patience", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("stop_rule", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("last_delta", ctypes.c_double),
        ("delta_history", ctypes.c_void_p),
        ("history_cap", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("iters_bf16", ctypes.c_int32),
        ("iters_fp32", ctypes.c_int32),
        ("iters_fp64", ctypes.c_int32),
    ]


DPT_PROF_KINDS = 8
PROF_NAMES = ["first_iterate", "prepass", "gemm_bf16", "gemm_fp32", "gemm_fp64", "spmm", "gemm_fp8", "gemm_x3"]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * DPT_PROF_KINDS), ("launches", ctypes.c_int64 * DPT_PROF_KINDS)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class ServeTimes(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("first_step_s", ctypes.c_double), ("finish_s", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("peak_active", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("active", ctypes.c_int64), ("pending", ctypes.c_int64), ("busy_s", ctypes.c_double),
                ("tile_shape", (ctypes.c_int32 * 4) * 2), ("graph_steps", ctypes.c_int64)]


_FUNCS = {
    "dpt_options_default": (None, [ctypes.POINTER(Options)]),
    "dpt_validate": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options)]),
    "dpt_init": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Problem),
                                ctypes.POINTER(Options), ctypes.c_void_p]),
    "dpt_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "dpt_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Result)]),
    "dpt_eigenvalues": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "dpt_eigenvectors": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "dpt_residuals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "dpt_dominant": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                    ctypes.POINTER(Result)]),
    "dpt_dominant_noalloc": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                            ctypes.POINTER(Result)]),
    "dpt_homotopy": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Result)]),
    "dpt_rs_series": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int]),
    "dpt_row_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "dpt_probe_gather": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "dpt_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "dpt_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Profile)]),
    "dpt_serve_open": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ServeConfig)]),
    "dpt_serve_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "dpt_serve_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(Result),
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.POINTER(ServeTimes)]),
    "dpt_serve_stats_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServeStats)]),
    "dpt_serve_close": (None, [ctypes.c_void_p]),
    "dpt_destroy": (None, [ctypes.c_void_p]),
    "dpt_status_str": (ctypes.c_char_p, [ctypes.c_int]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdpt.so (raises if it has not been built: no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("libdpt.so not found at %s; run paper_2002_12872_amd.build.build()" % path)
        # torch ships its own HIP runtime with the same soname (libamdhip64.so.7).
        # Loading torch first makes libdpt.so bind to that copy, so a process that
        # uses both has exactly one HIP runtime (two copies cannot share the GPU).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        for name, (res, args) in _FUNCS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def library_path() -> str:
    return LIB_PATH


def status_str(code: int) -> str:
    return load_library().dpt_status_str(int(code)).decode()


dpt_status_str = status_str


# ------------------------------------------------------------ marshalling
def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _info(x):
    """(pointer, dtype code or None, is_device, keep-alive object) of an array-like."""
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        dev = x.is_cuda
        dt = str(x.dtype)
        return x.data_ptr(), dt, dev, x
    a = np.ascontiguousarray(x)
    return a.ctypes.data, str(a.dtype), False, a


def _dtype_code(dt):
    if dt in ("float64", "torch.float64"):
        return DPT_DTYPE_F64
    if dt in ("float32", "torch.float32"):
        return DPT_DTYPE_F32
    raise ValueError("delta values must be float32 or float64, got %s" % dt)


class ProblemSpec:
    """A ``dpt_problem`` plus references keeping its arrays alive."""

    def __init__(self, theta, delta, lam, stream=None):
        keep = []
        tp, tdt, tdev, tk = _info(theta if _is_torch(theta) else np.asarray(theta, np.float64))
        if tdt not in ("float64", "torch.float64"):
            raise ValueError("theta must be float64")
        keep.append(tk)
        st = Problem()
        st.theta = tp
        st.lam = float(lam)
        st.reserved = 0
        if isinstance(delta, tuple):
            indptr, indices, values = delta
            ip, ipdt, ipdev, ipk = _info(indptr if _is_torch(indptr) else np.asarray(indptr, np.int64))
            ix, ixdt, ixdev, ixk = _info(indices if _is_torch(indices) else np.asarray(indices, np.int32))
            vp, vdt, vdev, vk = _info(values)
            if ipdt not in ("int64", "torch.int64") or ixdt not in ("int32", "torch.int32"):
                raise ValueError("CSR needs int64 indptr and int32 indices")
            devs = {tdev, ipdev, ixdev, vdev}
            keep += [ipk, ixk, vk]
            st.format = DPT_CSR
            st.indptr, st.indices, st.delta = ip, ix, vp
            st.nnz = int(values.shape[0])
            st.n = int(indptr.shape[0]) - 1
            st.dtype = _dtype_code(vdt)
        else:
            dp, ddt, ddev, dk = _info(delta)
            devs = {tdev, ddev}
            keep.append(dk)
            st.format = DPT_DENSE
            st.delta = dp
            st.indptr = st.indices = None
            st.nnz = 0
            st.n = int(delta.shape[0])
            if tuple(delta.shape) != (st.n, st.n):
                raise ValueError("dense delta must be square")
            st.dtype = _dtype_code(ddt)
        if len(devs) != 1:
            raise ValueError("all inputs must live in the same memory kind")
        device = devs.pop()
        st.mem = DPT_MEM_DEVICE if device else DPT_MEM_HOST
        if int(theta.shape[0]) != st.n:
            raise ValueError("theta length does not match delta")
        if stream is None and device:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        st.stream = stream
        self.struct = st
        self.keep = keep
        self.device = device


def options(tol=1e-6, max_iter=200, precision=DPT_FP32, fp64_final_tol=0.0, stall_ratio=0.5,
            stall_patience=2, check_every=1, blowup=1e6, stop_rule=DPT_STOP_DELTA, ramp_alpha=0.0):
    o = Options()
    load_library().dpt_options_default(ctypes.byref(o))
    o.tol, o.max_iter, o.precision = tol, max_iter, precision
    o.fp64_final_tol, o.stall_ratio, o.stall_patience = fp64_final_tol, stall_ratio, stall_patience
    o.check_every, o.blowup, o.stop_rule, o.ramp_alpha = check_every, blowup, stop_rule, ramp_alpha
    return o


def dpt_options_default():
    o = Options()
    load_library().dpt_options_default(ctypes.byref(o))
    return o


def dpt_validate(problem: ProblemSpec, opts: Options = None) -> int:
    return load_library().dpt_validate(ctypes.byref(problem.struct),
                                       ctypes.byref(opts) if opts is not None else None)


class Handle:
    def __init__(self, ptr, problem):
        self.ptr = ptr
        self.problem = problem      # keeps borrowed device inputs alive
        self.n = problem.struct.n

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.dpt_destroy(self.ptr)
            self.ptr = None


def dpt_init(problem: ProblemSpec, opts: Options = None, z0=None) -> Handle:
    h = ctypes.c_void_p()
    zp = None
    keep = None
    if z0 is not None:
        zp, _, zdev, keep = _info(z0)
        if zdev != problem.device:
            raise ValueError("z0 must live in the same memory kind as the problem's arrays")
    rc = load_library().dpt_init(ctypes.byref(h), ctypes.byref(problem.struct),
                                 ctypes.byref(opts) if opts is not None else None, zp)
    del keep
    if rc != DPT_OK:
        raise DptError(rc, "dpt_init")
    return Handle(h.value, problem)


def dpt_step(h: Handle, nsteps: int) -> float:
    d = ctypes.c_double()
    rc = load_library().dpt_step(h.ptr, int(nsteps), ctypes.byref(d))
    if rc < 0:
        raise DptError(rc, "dpt_step")
    return d.value


def dpt_solve(h: Handle, history_cap: int = 256) -> dict:
    hist = np.full(max(history_cap, 1), np.nan)
    r = Result()
    r.delta_history = hist.ctypes.data if history_cap > 0 else None
    r.history_cap = history_cap
    rc = load_library().dpt_solve(h.ptr, ctypes.byref(r))
    if rc < 0:
        raise DptError(rc, "dpt_solve")
    return {"status": r.status, "iters": r.iters, "iters_bf16": r.iters_bf16,
            "iters_fp32": r.iters_fp32, "iters_fp64": r.iters_fp64,
            "last_delta": r.last_delta, "history": hist[:min(r.iters, history_cap)].copy()}


def dpt_eigenvalues(h: Handle, out=None):
    """Host numpy array by default; pass a float64 device tensor of length n to fill it."""
    if out is None:
        out = np.empty(h.n, np.float64)
    p, dt, dev, keep = _info(out)
    if dt not in ("float64", "torch.float64"):
        raise ValueError("eigenvalues are float64")
    rc = load_library().dpt_eigenvalues(h.ptr, p, DPT_MEM_DEVICE if dev else DPT_MEM_HOST)
    if rc != DPT_OK:
        raise DptError(rc, "dpt_eigenvalues")
    return out


def dpt_eigenvectors(h: Handle, out=None, dtype=np.float64):
    """Z[k, m] = component m of eigenvector k (row k, Z[k, k] = 1)."""
    if out is None:
        out = np.empty((h.n, h.n), dtype=dtype)
    p, dt, dev, keep = _info(out)
    rc = load_library().dpt_eigenvectors(h.ptr, p, _dtype_code(dt),
                                         DPT_MEM_DEVICE if dev else DPT_MEM_HOST)
    if rc != DPT_OK:
        raise DptError(rc, "dpt_eigenvectors")
    return out


def dpt_residuals(h: Handle, rows):
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    res = np.empty(rows.shape[0], np.float64)
    rc = load_library().dpt_residuals(h.ptr, rows.shape[0], rows.ctypes.data, res.ctypes.data)
    if rc != DPT_OK:
        raise DptError(rc, "dpt_residuals")
    return res


def dpt_dominant(problem: ProblemSpec, opts: Options = None, index: int = -1, out=None,
                 history_cap: int = 64):
    """Returns (eigval, eigvec, result dict).  eigvec has the problem's dtype and memory kind."""
    st = problem.struct
    if out is None:
        if problem.device:
            import torch
            out = torch.empty(st.n, dtype=torch.float64 if st.dtype == DPT_DTYPE_F64 else torch.float32,
                              device="cuda")
        else:
            out = np.empty(st.n, np.float64 if st.dtype == DPT_DTYPE_F64 else np.float32)
    p, _, _, keep = _info(out)
    ev = ctypes.c_double()
    hist = np.full(max(history_cap, 1), np.nan)
    r = Result()
    r.delta_history = hist.ctypes.data
    r.history_cap = history_cap
    rc = load_library().dpt_dominant(ctypes.byref(st), ctypes.byref(opts) if opts is not None else None,
                                     int(index), ctypes.byref(ev), p, ctypes.byref(r))
    if rc < 0:
        raise DptError(rc, "dpt_dominant")
    return ev.value, out, {"status": r.status, "iters": r.iters, "last_delta": r.last_delta,
                           "history": hist[:min(r.iters, history_cap)].copy()}


def dpt_dominant_noalloc(problem: ProblemSpec, opts: Options, out, index: int = -1, history_cap: int = 64):
    """Dominant mode without device allocation: device-resident problem, ``out`` a
    device tensor of n values of the problem's dtype.  Returns (eigval, out, result dict)."""
    st = problem.struct
    p, _, dev, keep = _info(out)
    if not dev or not problem.device:
        raise ValueError("dpt_dominant_noalloc takes device-resident inputs and output")
    ev = ctypes.c_double()
    hist = np.full(max(history_cap, 1), np.nan)
    r = Result()
    r.delta_history = hist.ctypes.data
    r.history_cap = history_cap
    rc = load_library().dpt_dominant_noalloc(ctypes.byref(st), ctypes.byref(opts) if opts is not None else None,
                                             int(index), ctypes.byref(ev), p, ctypes.byref(r))
    if rc < 0:
        raise DptError(rc, "dpt_dominant_noalloc")
    return ev.value, out, {"status": r.status, "iters": r.iters, "last_delta": r.last_delta,
                           "history": hist[:min(r.iters, history_cap)].copy()}


def dpt_homotopy(problem: ProblemSpec, opts: Options, stages: int, E=None, Z=None, z_dtype=np.float64):
    """Homotopy continuation in ``stages`` FP64 stages.  Outputs default to host
    arrays (device tensors for a device problem).  Returns (E, Z, result dict)."""
    st = problem.struct
    n = st.n
    if E is None or Z is None:
        if problem.device:
            import torch
            E = torch.empty(n, dtype=torch.float64, device="cuda") if E is None else E
            Z = torch.empty((n, n), dtype=torch.float64 if z_dtype == np.float64 else torch.float32,
                            device="cuda") if Z is None else Z
        else:
            E = np.empty(n, np.float64) if E is None else E
            Z = np.empty((n, n), z_dtype) if Z is None else Z
    ep, _, _, ek = _info(E)
    zp, zdt, _, zk = _info(Z)
    r = Result()
    rc = load_library().dpt_homotopy(ctypes.byref(st), ctypes.byref(opts), int(stages), ep, zp, _dtype_code(zdt),
                                     ctypes.byref(r))
    if rc < 0:
        raise DptError(rc, "dpt_homotopy")
    return E, Z, {"status": r.status, "iters": r.iters}


def dpt_rs_series(problem: ProblemSpec, order: int, want_z: bool = True):
    """Rayleigh-Schroedinger coefficients on the GPU.  Returns (eps (order, n),
    coef_max (order,), Z partial sum (n, n) host array or None); a device problem
    gets Z as a device tensor."""
    st = problem.struct
    n = st.n
    eps = np.empty((order, n), np.float64)
    cmax = np.empty(order, np.float64)
    z = None
    zp = None
    if want_z:
        if problem.device:
            import torch
            z = torch.empty((n, n), dtype=torch.float64, device="cuda")
        else:
            z = np.empty((n, n), np.float64)
        zp, _, _, _ = _info(z)
    rc = load_library().dpt_rs_series(ctypes.byref(st), int(order), eps.ctypes.data, cmax.ctypes.data, zp,
                                      DPT_DTYPE_F64)
    if rc != DPT_OK:
        raise DptError(rc, "dpt_rs_series")
    return eps, cmax, z


def dpt_row_status(h: Handle):
    """(retired_at (n,) int32, rows_multiplied) of a DPT_STOP_ROW solve."""
    out = np.zeros(h.n, np.int32)
    rm = ctypes.c_int64()
    rc = load_library().dpt_row_status(h.ptr, out.ctypes.data, ctypes.byref(rm))
    if rc != DPT_OK:
        raise DptError(rc, "dpt_row_status")
    return out, rm.value


def dpt_probe_gather(panel_rows: int, gathers: int, reps: int = 5):
    """(ms per pass, GB/s) of random 512-byte row gathers from a panel (measurement probe)."""
    ms, gbs = ctypes.c_double(), ctypes.c_double()
    rc = load_library().dpt_probe_gather(int(panel_rows), int(gathers), int(reps), ctypes.byref(ms),
                                         ctypes.byref(gbs))
    if rc != DPT_OK:
        raise DptError(rc, "dpt_probe_gather")
    return ms.value, gbs.value


def dpt_profile_enable(h: Handle, on: bool = True) -> None:
    rc = load_library().dpt_profile_enable(h.ptr, int(bool(on)))
    if rc != DPT_OK:
        raise DptError(rc, "dpt_profile_enable")


def dpt_profile_read(h: Handle) -> dict:
    """{kernel class: (total device ms, launches)} from HIP events on the handle's stream."""
    p = Profile()
    rc = load_library().dpt_profile_read(h.ptr, ctypes.byref(p))
    if rc != DPT_OK:
        raise DptError(rc, "dpt_profile_read")
    return {PROF_NAMES[i]: (p.ms[i], int(p.launches[i])) for i in range(DPT_PROF_KINDS)
            if p.launches[i] > 0}


def dpt_destroy(h: Handle) -> None:
    if h.ptr:
        load_library().dpt_destroy(h.ptr)
        h.ptr = None


# ------------------------------------------------------------------ serving
class Server:
    """Handle of a serving engine (continuous batching); remembers each ticket's order."""

    def __init__(self, ptr):
        self.ptr = ptr
        self.tickets = {}

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.dpt_serve_close(self.ptr)
            self.ptr = None


def dpt_serve_open(budget_bytes, max_slots=256, use_graph=True, grid_blocks=0, autotune=False,
                   stream=None, tile_shape=None) -> Server:
    """stream: a hipStream_t (e.g. torch.cuda.Stream().cuda_stream) for the server's work, or None.
    tile_shape: 0, 1 or 2 (64x64, 128x64, 128x128) for every order class instead of the defaults
    or the autotuner."""
    mode = int(bool(autotune)) if tile_shape is None else -int(tile_shape) - 1
    cfg = ServeConfig(int(budget_bytes), int(max_slots), int(bool(use_graph)), int(grid_blocks), mode, stream)
    h = ctypes.c_void_p()
    rc = load_library().dpt_serve_open(ctypes.byref(h), ctypes.byref(cfg))
    if rc != DPT_OK:
        raise DptError(rc, "dpt_serve_open")
    return Server(h.value)


def dpt_serve_submit(srv: Server, problem: ProblemSpec, opts: Options = None,
                     want_eigenvectors: bool = False) -> int:
    """Host (numpy) or device (torch cuda, finished) theta/Delta.  Device arrays
    are read when the request is admitted: the ticket keeps the spec (and so its
    tensors) alive until the result is polled."""
    t = ctypes.c_int64()
    rc = load_library().dpt_serve_submit(srv.ptr, ctypes.byref(problem.struct),
                                         ctypes.byref(opts) if opts is not None else None,
                                         int(bool(want_eigenvectors)), ctypes.byref(t))
    if rc != DPT_OK:
        raise DptError(rc, "dpt_serve_submit")
    srv.tickets[t.value] = (int(problem.struct.n), bool(want_eigenvectors), problem)
    return t.value


def dpt_serve_poll(srv: Server, ticket: int, wait_ms: int = 0):
    """None while pending; else dict(status, iters..., E, Z (or None), times)."""
    n, want_z, _ = srv.tickets[ticket]
    e = np.empty(n, np.float64)
    z = np.empty((n, n), np.float64) if want_z else None
    r = Result()
    times = ServeTimes()
    rc = load_library().dpt_serve_poll(srv.ptr, int(ticket), int(wait_ms), ctypes.byref(r), e.ctypes.data,
                                       z.ctypes.data if z is not None else None, DPT_DTYPE_F64,
                                       ctypes.byref(times))
    if rc == DPT_EAGAIN:
        return None
    del srv.tickets[ticket]
    if rc < 0:
        raise DptError(rc, "dpt_serve_poll")
    return {"status": rc, "iters": r.iters, "iters_bf16": r.iters_bf16, "iters_fp32": r.iters_fp32,
            "last_delta": r.last_delta, "E": e, "Z": z,
            "times": {"submit": times.submit_s, "admit": times.admit_s,
                      "first_step": times.first_step_s, "finish": times.finish_s}}


def dpt_serve_stats_read(srv: Server) -> dict:
    st = ServeStats()
    rc = load_library().dpt_serve_stats_read(srv.ptr, ctypes.byref(st))
    if rc != DPT_OK:
        raise DptError(rc, "dpt_serve_stats_read")
    out = {k: getattr(st, k) for k, _ in ServeStats._fields_}
    out["tile_shape"] = [list(row) for row in st.tile_shape]
    return out


def dpt_serve_close(srv: Server) -> None:
    if srv.ptr:
        load_library().dpt_serve_close(srv.ptr)
        srv.ptr = None
