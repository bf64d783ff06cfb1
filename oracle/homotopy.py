"""Domain extensions of the D-PT iteration (Sec. III and Supplement E).

TEST INFRASTRUCTURE ONLY (see the package docstring): plain FP64, built on the
oracle's own iteration ``core.iterate``; nothing here is shared with the HIP
library.

``homotopy``  Sec. III (Discussion): when the iteration does not converge at
              lambda, split lambda into Q equal parts.  Stage q diagonalises
              M_q = D + (q lambda / Q) Delta by D-PT, written in the eigenbasis
              B of M_{q-1}: there M_q = diag(E_{q-1}) + (lambda/Q) B^-1 Delta B,
              a problem whose unperturbed part is the diagonal matrix obtained at
              the previous stage.  The eigenvectors found (rows y_n, chart
              y_n[n] = 1) update the basis, B <- B Y^T, and their eigenvalues
              become the next stage's diagonal.  After Q stages the columns of B
              are the eigenvectors of M continued from e_n; they are returned in
              the chart z_n[n] = 1.  B^-1 is taken with a library inverse (a plain
              step of the definition).
``ramp``      Supplement E: the non-autonomous iteration z <- F(z, lambda_k) with
              lambda_k = lambda (1 - alpha^k), which continues the steady state
              from small lambda.  Delegates to the C oracle (``ramp_alpha``).
"""
from __future__ import annotations

import numpy as np

from . import core


def homotopy(theta, delta, lam, stages, tol=1e-14, max_iter=500):
    """Eigenpairs of diag(theta) + lam * delta by ``stages`` D-PT stages of lam/stages.

    Returns dict(z (n, n) rows z_n with z_n[n] = 1, e (n,), iters (list per
    stage), status (worst stage status)).
    """
    theta = np.asarray(theta, np.float64)
    delta = np.asarray(delta, np.float64)
    n = theta.shape[0]
    basis = np.eye(n)            # columns: eigenvectors of M_q in the original coordinates
    diag = theta.copy()
    iters, status = [], core.OR_OK
    for _ in range(stages):
        stage_delta = np.linalg.inv(basis) @ delta @ basis
        r = core.iterate(diag, stage_delta, lam / stages, max_iter=max_iter, tol=tol)
        iters.append(r["iters"])
        status = max(status, r["status"])
        basis = basis @ r["z"].T
        diag = r["e"]
    z = basis.T / np.diag(basis)[:, None]
    return {"z": z, "e": diag, "iters": iters, "status": status}


def ramp(theta, delta, lam, alpha, **kwargs):
    """D-PT with the per-step coupling lambda_k = lam (1 - alpha^k) (see ``core.iterate``)."""
    return core.iterate(theta, delta, lam, ramp_alpha=alpha, **kwargs)
