"""Hand-written cyclic Jacobi eigensolver for small real symmetric matrices (FP64).

Test infrastructure only.  Textbook method (Golub & Van Loan, "Matrix
Computations", Sec. 8.5, cyclic-by-row Jacobi): sweep over all (p, q) pairs,
zero the off-diagonal entry with a plane rotation, repeat until the
off-diagonal Frobenius norm is negligible.  Used as an independent pin for the
D-PT oracle on symmetric problems with N <= 64.
"""
from __future__ import annotations

import math

import numpy as np


def jacobi_eigh(a, tol=1e-15, max_sweeps=100):
    """Eigenpairs of the symmetric matrix ``a``.

    Returns ``(w, v)`` with ``a @ v[:, i] = w[i] * v[:, i]``, columns of ``v``
    orthonormal, in the order the diagonal settles (no sorting).
    """
    a = np.array(a, dtype=np.float64, copy=True)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("square matrix required")
    if not np.array_equal(a, a.T):
        raise ValueError("symmetric matrix required")
    v = np.eye(n)
    scale = max(np.abs(a).max(), 1e-300)
    for _ in range(max_sweeps):
        off = math.sqrt(float(np.sum(np.tril(a, -1) ** 2)))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = a[p, q]
                if apq == 0.0:
                    continue
                # rotation angle that annihilates a[p, q]
                tau = (a[q, q] - a[p, p]) / (2.0 * apq)
                t = math.copysign(1.0, tau) / (abs(tau) + math.sqrt(1.0 + tau * tau))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                # A <- J^T A J with J the (p, q) rotation
                ap = a[:, p].copy()
                aq = a[:, q].copy()
                a[:, p] = c * ap - s * aq
                a[:, q] = s * ap + c * aq
                ap = a[p, :].copy()
                aq = a[q, :].copy()
                a[p, :] = c * ap - s * aq
                a[q, :] = s * ap + c * aq
                a[p, q] = a[q, p] = 0.0
                vp = v[:, p].copy()
                vq = v[:, q].copy()
                v[:, p] = c * vp - s * vq
                v[:, q] = s * vp + c * vq
    else:
        raise RuntimeError("Jacobi did not converge")
    return np.diag(a).copy(), v
