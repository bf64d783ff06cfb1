"""Shared helpers for the GPU parity tests (no method arithmetic beyond error metrics)."""
import math

import numpy as np


def small_problem(n, seed, symmetric=False, diag=False, scale=0.5):
    """theta_i = i + U(0, 0.5) sorted; Delta iid N(0, (scale/sqrt(n))^2), float64."""
    rng = np.random.default_rng(90_000 + 7 * n + seed)
    theta = np.sort(np.arange(n, dtype=np.float64) + rng.uniform(0, 0.5, n))
    delta = rng.normal(0, scale / math.sqrt(max(n, 1)), (n, n))
    if symmetric:
        delta = 0.5 * (delta + delta.T)
    if not diag:
        np.fill_diagonal(delta, 0.0)
    return theta, delta


def gap_matrix(theta):
    g = np.zeros((len(theta), len(theta)))
    off = ~np.eye(len(theta), dtype=bool)
    g[off] = 1.0 / (theta[:, None] - theta[None, :])[off]
    return g


def one_step_bound(theta, delta, lam, z, u_prod, k_eff, rows=None):
    """Elementwise bound on |F(Z)_gpu - F(Z)_exact| for one step from Z.

    The product W Delta' (W = Z - I) is formed with per-term relative error
    u_prod (operand rounding) and an accumulation error of k_eff * 2^-24 per
    magnitude sum; the identity part Delta' is exact; the update multiplies by
    |lambda gap|.  Rows of z correspond to ``rows`` (default all).  The FP32
    matrix-core accumulation over K terms behaves like a drift of order
    sqrt(K) ulps of the magnitude sum, hence callers pass k_eff = 8 + sqrt(K).
    """
    n = len(theta)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    w = z.copy()
    w[np.arange(len(rows)), rows] = 0.0
    mag = np.abs(w) @ np.abs(delta).T                       # sum_k |W_nk Delta_mk|
    c = w @ delta.T + delta.T[rows]                         # C = Delta' + W Delta'
    d = c[np.arange(len(rows)), rows]
    g = gap_matrix(theta)[rows]
    acc = 2.0 ** -24 * k_eff
    term = (u_prod + acc) * mag + acc * (np.abs(c) + np.abs(d)[:, None] * np.abs(w))
    out = np.abs(lam * g) * term * 1.5
    new = lam * g * (c - d[:, None] * w)
    return out + 4 * 2.0 ** -24 * np.abs(new) + 1e-300


def rel_eig_error(e, e_ref, theta):
    """max |E - E*| / max(|E*|, 1e-12 max|theta|)."""
    floor = 1e-12 * max(np.abs(theta).max(), 1.0)
    return float(np.max(np.abs(e - e_ref) / np.maximum(np.abs(e_ref), floor)))
