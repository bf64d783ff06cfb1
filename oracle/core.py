"""ctypes front-end of the C oracle plus the plain residual definition.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

OR_OK = 0
OR_NOT_CONVERGED = 1
OR_DIVERGED = 3
OR_EINVAL = -1
OR_ENOMEM = -2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpt_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle.so")
_lib = None


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("theta", ctypes.c_void_p),
        ("dense", ctypes.c_void_p),
        ("indptr", ctypes.c_void_p),
        ("indices", ctypes.c_void_p),
        ("values", ctypes.c_void_p),
        ("lam", ctypes.c_double),
    ]


def build(force: bool = True, src: str = _SRC, out: str = _LIB_PATH, defines=()) -> str:
    """Compile the C oracle (gcc, FP64, OpenMP) into a shared library; returns its path."""
    if not force and os.path.exists(out):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = (["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall"]
           + ["-D%s" % d for d in defines] + ["-o", tmp, src, "-lm"])
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class OracleLib:
    """One loaded build of the C oracle."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        lib.or_iterate.restype = ctypes.c_int
        lib.or_iterate.argtypes = [
            ctypes.POINTER(_Problem), ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
            ctypes.c_void_p,
        ]
        lib.or_max_threads.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def max_threads(self) -> int:
        return int(self.lib.or_max_threads())

    def iterate(self, theta, delta, lam, rows=None, z0=None, max_iter=200, tol=1e-12,
                fixed_steps=False, blowup=1e6, nthreads=0, ramp_alpha=0.0, per_row=False):
        """Run the D-PT iteration on the eigenvector rows ``rows`` (default: all).

        ``ramp_alpha`` in (0, 1) selects the non-autonomous coupling of
        Supplement E, lambda_k = lambda (1 - ramp_alpha^k) (see dpt_oracle.c).
        ``per_row`` stops each row on its own delta (frozen rows keep their
        iterate); the result then has ``row_iters``, the step each row froze on.

        ``delta`` is a dense (n, n) array, Delta[m, l], or a CSR triple
        ``(indptr, indices, values)``.  Returns a dict with
        ``z`` (len(rows), n), ``e`` (len(rows),), ``hist`` (iters,), ``iters``, ``status``.
        """
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        n = theta.shape[0]
        prob = _Problem()
        prob.n = n
        prob.theta = _ptr(theta)
        keep = [theta]
        if isinstance(delta, tuple):
            indptr = np.ascontiguousarray(delta[0], dtype=np.int64)
            indices = np.ascontiguousarray(delta[1], dtype=np.int32)
            values = np.ascontiguousarray(delta[2], dtype=np.float64)
            if indptr.shape[0] != n + 1 or indices.shape[0] != values.shape[0]:
                raise ValueError("bad CSR shapes")
            prob.dense = None
            prob.indptr, prob.indices, prob.values = _ptr(indptr), _ptr(indices), _ptr(values)
            keep += [indptr, indices, values]
        else:
            dense = np.ascontiguousarray(delta, dtype=np.float64)
            if dense.shape != (n, n):
                raise ValueError("delta must be (n, n)")
            prob.dense = _ptr(dense)
            prob.indptr = prob.indices = prob.values = None
            keep.append(dense)
        prob.lam = float(lam)
        if rows is None:
            rows = np.arange(n, dtype=np.int64)
        rows = np.ascontiguousarray(np.atleast_1d(rows), dtype=np.int64)
        nrows = rows.shape[0]
        if z0 is not None:
            z0 = np.ascontiguousarray(z0, dtype=np.float64).reshape(nrows, n)
        z = np.zeros((nrows, n), dtype=np.float64)
        e = np.zeros(nrows, dtype=np.float64)
        hist = np.full(max(max_iter, 1), np.nan, dtype=np.float64)
        iters = ctypes.c_int(0)
        row_iters = np.zeros(nrows, dtype=np.int32)
        rc = self.lib.or_iterate(ctypes.byref(prob), nrows, _ptr(rows), _ptr(z0), int(max_iter),
                                 float(tol), int(bool(fixed_steps)), float(blowup), int(nthreads),
                                 float(ramp_alpha), int(bool(per_row)), _ptr(z), _ptr(e), _ptr(hist),
                                 ctypes.byref(iters), _ptr(row_iters))
        del keep
        if rc < 0:
            raise ValueError("oracle rejected the problem (code %d)" % rc)
        k = iters.value
        return {"z": z, "e": e, "hist": hist[:k].copy(), "iters": k, "status": rc,
                "rows": rows, "row_iters": row_iters}


def _default():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        _lib = OracleLib(_LIB_PATH)
    return _lib


def max_threads() -> int:
    return _default().max_threads()


def _ptr(a):
    return None if a is None else a.ctypes.data


def iterate(*args, **kwargs):
    """D-PT iteration with the default oracle build (see ``OracleLib.iterate``)."""
    return _default().iterate(*args, **kwargs)


def _delta_matvec(delta, x):
    """Delta @ x for dense or CSR Delta (x: (n,) or (n, r))."""
    if isinstance(delta, tuple):
        import scipy.sparse as sp
        indptr, indices, values = delta
        n = len(indptr) - 1
        mat = sp.csr_matrix((np.asarray(values, np.float64), np.asarray(indices),
                             np.asarray(indptr)), shape=(n, n))
        return mat @ x
    return np.asarray(delta, np.float64) @ x


def residual(theta, delta, lam, z_rows, e):
    """||M z_n - E_n z_n||_2 for each row z_n of ``z_rows`` (M = diag(theta) + lam Delta).

    Plain definition of an eigenpair (Sec. II.A): returns (res, mz_norm, z_norm),
    all of shape (len(e),).
    """
    theta = np.asarray(theta, np.float64)
    z = np.atleast_2d(np.asarray(z_rows, np.float64))
    e = np.atleast_1d(np.asarray(e, np.float64))
    mz = theta[:, None] * z.T + lam * _delta_matvec(delta, z.T)   # (n, r)
    r = mz - z.T * e[None, :]
    return (np.linalg.norm(r, axis=0), np.linalg.norm(mz, axis=0),
            np.linalg.norm(z, axis=1))
