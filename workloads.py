"""Seeded synthetic inputs for the D-PT hot path.

This module only *builds inputs* (unperturbed eigenvalues theta, perturbation
Delta, request traces).  It contains none of the method's arithmetic and is the
only code shared by the oracle side and the GPU side.  Every generator is a pure
function of its seed (numpy PCG64 via ``default_rng``).

Workload families (sizes and distributions of the five measured configurations,
plus the paper's analytic examples):

* ``dense_sym_small``  N=64, theta_i = i, Delta = (R + R^T)/2, R off-diagonal
  iid N(0, 0.05^2), zero diagonal, FP64.
* ``dense_unsym``      N=4096, theta_i = i + U(0, 0.5) (sorted), Delta = R with R
  off-diagonal iid N(0, (0.5/sqrt(N))^2), zero diagonal, FP32 values.
* ``sparse_sym``       N=32768, theta_i = i, R has 16 distinct random off-diagonal
  columns per row with values N(0, 0.02^2); Delta = (R + R^T)/2 (pattern union),
  CSR with int32 column indices sorted within rows, FP32 values.
* ``dense_sym_large``  N=16384, theta_i = i/4, Delta = (R + R^T)/2 with R
  off-diagonal iid N(0, (0.25/sqrt(N))^2), zero diagonal, FP32 values.
* ``serving_trace``    4096 requests, N log-uniform in [32, 2048], 50 % symmetric,
  theta_i = i + U(0, 0.5), R off-diagonal iid N(0, (0.4/sqrt(N))^2), Poisson arrivals.
* ``two_by_two``       eq. (2by2) of the paper.
* ``three_by_three``   the Supplement E example.
* ``delta_potential``  the harmonic oscillator with a delta potential, Sec. II.F:
  D_nn = 2n + 1/2, Delta_nm = phi_2n(0) phi_2m(0).

FP32 workloads return FP32 arrays: the problem *is* those FP32 values, so the
FP64 oracle (which upcasts them exactly) and the GPU solve the same matrix.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = {"dense_sym_small": 1000, "dense_unsym": 2000, "sparse_sym": 3000,
             "dense_sym_large": 4000, "serving": 5000}


def _rng(family, seed):
    return np.random.default_rng(SEED_BASE[family] + int(seed))


def _zero_diag(a):
    np.fill_diagonal(a, 0)
    return a


def dense_sym_small(seed=0, n=64, sigma=0.05):
    """theta (float64), Delta (float64, symmetric, zero diagonal)."""
    rng = _rng("dense_sym_small", seed)
    theta = np.arange(n, dtype=np.float64)
    r = _zero_diag(rng.normal(0.0, sigma, size=(n, n)))
    delta = 0.5 * (r + r.T)
    return theta, delta


def dense_unsym(seed=0, n=4096, scale=0.5):
    """theta (float64, sorted), Delta (float32, unsymmetric, zero diagonal)."""
    rng = _rng("dense_unsym", seed)
    theta = np.sort(np.arange(n, dtype=np.float64) + rng.uniform(0.0, 0.5, size=n))
    delta = rng.standard_normal(size=(n, n), dtype=np.float32)
    delta *= np.float32(scale / math.sqrt(n))
    _zero_diag(delta)
    return theta, delta


def dense_sym_large(seed=0, n=16384, scale=0.25):
    """theta (float64), Delta (float32, symmetric, zero diagonal)."""
    rng = _rng("dense_sym_large", seed)
    theta = np.arange(n, dtype=np.float64) / 4.0
    r = rng.standard_normal(size=(n, n), dtype=np.float32)
    r *= np.float32(scale / math.sqrt(n))
    _zero_diag(r)
    delta = r + r.T
    del r
    delta *= np.float32(0.5)
    return theta, delta


def _distinct_offdiag_columns(rng, n, per_row):
    """(n, per_row) int64 columns, distinct within a row and never equal to the row."""
    k = min(per_row, n - 1)
    cols = rng.integers(0, n - 1, size=(n, k))
    todo = np.arange(n)
    while True:
        c = cols[todo]
        c = np.where(c >= todo[:, None], c + 1, c)         # skip the diagonal
        cs = np.sort(c, axis=1)
        dup = np.any(cs[:, 1:] == cs[:, :-1], axis=1) if k > 1 else np.zeros(len(todo), bool)
        cols[todo] = c
        if not dup.any():
            break
        todo = todo[dup]
        cols[todo] = rng.integers(0, n - 1, size=(len(todo), k))
    return cols


def sparse_sym(seed=0, n=32768, per_row=16, sigma=0.02, dtype=np.float32):
    """theta (float64), CSR (indptr int64, indices int32, values dtype) of (R + R^T)/2."""
    import scipy.sparse as sp
    rng = _rng("sparse_sym", seed)
    theta = np.arange(n, dtype=np.float64)
    cols = _distinct_offdiag_columns(rng, n, per_row)
    vals = rng.normal(0.0, sigma, size=cols.shape).astype(dtype)
    rows = np.repeat(np.arange(n), cols.shape[1])
    r = sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(n, n), dtype=dtype)
    s = (r + r.T).tocsr()
    s.sum_duplicates()
    s.sort_indices()
    values = (s.data * dtype(0.5)).astype(dtype)
    return (theta, np.asarray(s.indptr, np.int64), np.asarray(s.indices, np.int32), values)


def csr_to_dense(n, indptr, indices, values, dtype=np.float64):
    out = np.zeros((n, n), dtype=dtype)
    for m in range(n):
        sl = slice(indptr[m], indptr[m + 1])
        out[m, indices[sl]] = values[sl]
    return out


def serving_request(rng, n, symmetric):
    theta = np.arange(n, dtype=np.float64) + rng.uniform(0.0, 0.5, size=n)
    theta.sort()
    r = rng.normal(0.0, 0.4 / math.sqrt(n), size=(n, n)).astype(np.float32)
    _zero_diag(r)
    if symmetric:
        r = ((r + r.T) * np.float32(0.5)).astype(np.float32)
    return theta, r


def serving_trace(seed=0, count=4096, rate=None, nmin=32, nmax=2048):
    """Request descriptors: list of dicts (n, symmetric, seed, arrival_s).

    Sizes are log-uniform in [nmin, nmax] (rounded), half the requests symmetric;
    inter-arrival times exponential with the given rate (requests/s), or all zero
    when ``rate`` is None.  Matrices are built lazily with ``serving_request``
    from the per-request seed.
    """
    rng = _rng("serving", seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=count))).astype(int)
    sym = rng.random(count) < 0.5
    seeds = rng.integers(0, 2**62, size=count)
    if rate is None:
        arrivals = np.zeros(count)
    else:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    return [{"n": int(sizes[i]), "symmetric": bool(sym[i]), "seed": int(seeds[i]),
             "arrival_s": float(arrivals[i])} for i in range(count)]


def request_matrices(req):
    rng = np.random.default_rng(req["seed"])
    return serving_request(rng, req["n"], req["symmetric"])


def two_by_two():
    """eq. (2by2): D = diag(0, 1), Delta = [[0, 1], [1, 0]]."""
    return np.array([0.0, 1.0]), np.array([[0.0, 1.0], [1.0, 0.0]])


def three_by_three():
    """Supplement E example: D = diag(0, 1, 3), Delta = [[0,1,2],[1,0,3],[2,3,0]]."""
    return (np.array([0.0, 1.0, 3.0]),
            np.array([[0.0, 1.0, 2.0], [1.0, 0.0, 3.0], [2.0, 3.0, 0.0]]))


def hermite_even_at_zero(n):
    """phi_{2k}(0) for k = 0..n-1, phi_j the normalised Hermite functions.

    phi_0(0) = pi^(-1/4) and phi_{2k}(0) = -sqrt((2k-1)/(2k)) phi_{2k-2}(0), which
    follows from H_{2k}(0) = (-1)^k (2k)!/k! and the normalisation (2^j j! sqrt(pi))^(-1/2).
    """
    out = np.empty(n, dtype=np.float64)
    out[0] = math.pi ** -0.25
    for k in range(1, n):
        out[k] = -math.sqrt((2 * k - 1) / (2 * k)) * out[k - 1]
    return out


def delta_potential(n=100):
    """Sec. II.F: theta_n = 2n + 1/2, Delta = phi phi^T (rank one, non-zero diagonal)."""
    phi = hermite_even_at_zero(n)
    return 2.0 * np.arange(n, dtype=np.float64) + 0.5, np.outer(phi, phi)


def sample_rows(n, count=64, seed=0):
    """{0, n-1} plus (count-2) distinct seeded uniform rows, sorted."""
    if n <= count:
        return np.arange(n, dtype=np.int64)
    rng = np.random.default_rng(7_000_000 + seed)
    inner = rng.choice(np.arange(1, n - 1), size=count - 2, replace=False)
    return np.sort(np.concatenate([[0, n - 1], inner])).astype(np.int64)
