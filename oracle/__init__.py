"""FP64 CPU oracle for dynamical perturbation theory (arXiv:2002.12872).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  It shares no code with the HIP
library in ``paper_2002_12872_amd`` and neither package imports the other.

Contents
--------
``iterate``        the D-PT iteration itself (C, ``dpt_oracle.c``), eq. (single_line_dyn)
                   applied row by row = eq. (dyn) from A^(0) = I, Sec. II.B.
``residual``       eigen-equation residual  ||M z - E z||_2  per row (Sec. II.A definition).
``jacobi_eigh``    hand-written cyclic Jacobi eigensolver (textbook method), a pin for
                   symmetric N <= 64.
``rs_coefficients`` Rayleigh-Schroedinger recursion eq. (ARS-alpha) / Supplement B.
``homotopy``       Sec. III: Q stages of lambda/Q, each diagonalised by D-PT in the
                   eigenbasis of the previous stage.
``ramp``           Supplement E: the non-autonomous coupling lambda (1 - alpha^k).
"""
from .core import (  # noqa: F401
    OR_OK,
    OR_NOT_CONVERGED,
    OR_DIVERGED,
    OR_EINVAL,
    OR_ENOMEM,
    OracleLib,
    build,
    iterate,
    max_threads,
    residual,
)
from .homotopy import homotopy, ramp  # noqa: F401
from .jacobi import jacobi_eigh  # noqa: F401
from .rs import rs_coefficients, rs_partial_sum, rs_eigenvalue_coefficients  # noqa: F401
