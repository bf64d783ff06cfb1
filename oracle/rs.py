"""Rayleigh-Schroedinger (RS) perturbation coefficients, eq. (ARS-alpha).

Test infrastructure only.  Matrix form of the recursion derived in Supplement B:

    a^(0) = I,
    a^(l) = theta * ( a^(l-1) Delta'  -  sum_{s=0}^{l-1} (a^(s) Delta') |> a^(l-1-s) ),

where ``*`` is the Hadamard product, ``'`` the transpose, ``A |> B = diag(A) B``
(row n of B scaled by A[n, n]) and theta[n, m] = 1 / (theta_n - theta_m) off the
diagonal, 0 on it.  The eigenvalue coefficients are eps^(l) = (a^(l-1) Delta')_nn
(Supplement B), so E_RS^(k) = theta + sum_{l=1}^{k} lam^l eps^(l)  (eps^(1) carries
diag(Delta)).  The order-k partial sum is A_RS^(k) = sum_{l<=k} lam^l a^(l).
"""
from __future__ import annotations

import numpy as np


def _gap_matrix(theta):
    theta = np.asarray(theta, np.float64)
    diff = theta[:, None] - theta[None, :]
    with np.errstate(divide="ignore"):
        g = 1.0 / diff
    np.fill_diagonal(g, 0.0)
    return g


def rs_coefficients(theta, delta, order):
    """Return [a^(0), ..., a^(order)] (dense numpy arrays)."""
    g = _gap_matrix(theta)
    d = np.asarray(delta, np.float64)
    dt = d.T
    n = g.shape[0]
    coeffs = [np.eye(n)]
    prods = [coeffs[0] @ dt]            # a^(s) Delta'
    for ell in range(1, order + 1):
        acc = prods[ell - 1].copy()
        for s in range(ell):
            acc -= np.diag(prods[s])[:, None] * coeffs[ell - 1 - s]
        a = g * acc
        coeffs.append(a)
        prods.append(a @ dt)
    return coeffs


def rs_partial_sum(theta, delta, lam, order):
    """A_RS^(order) = sum_{l=0}^{order} lam^l a^(l)."""
    coeffs = rs_coefficients(theta, delta, order)
    out = np.zeros_like(coeffs[0])
    for ell, a in enumerate(coeffs):
        out += (lam ** ell) * a
    return out


def rs_eigenvalue_coefficients(theta, delta, order):
    """[eps^(1), ..., eps^(order)] with eps^(l) = diag(a^(l-1) Delta')."""
    coeffs = rs_coefficients(theta, delta, max(order - 1, 0))
    dt = np.asarray(delta, np.float64).T
    return [np.diag(coeffs[ell - 1] @ dt).copy() for ell in range(1, order + 1)]
