"""Oracle: eigenvalues of the preconditioned operator J M^{-1} (Sec. 4.3).

Test infrastructure only (like the rest of this package).

Following the paper's eigenvalue study, the inner solves of M are exact
(sparse LU in place of each AMG V-cycle: A_pp for CPR, A_ss and the
approximate Schur complement for BF), while the first CPR stage stays
ILU(0).  J M^{-1} is formed densely, one column M^{-1} e_j at a time, and
its spectrum computed with LAPACK (numpy.linalg.eigvals).  The summary
statistics describe what the paper reads off its plots: how far the
spectrum stays from the origin and how tightly it clusters.
"""
from __future__ import annotations

import numpy as np

from . import precond, tpfa


def preconditioned_matrix(kind, row_ptr, col_idx, vals, grid, p1="ilu"):
    """Dense J M^{-1} with exact inner solves."""
    J = tpfa.bcsr_to_dense(row_ptr, col_idx, vals)
    M = precond.Preconditioner(kind, row_ptr, col_idx, vals, grid, inner="exact", p1=p1)
    n = J.shape[0]
    Minv = np.column_stack([M.apply(e) for e in np.eye(n)])
    return J @ Minv


def summary(ev):
    """Spectrum statistics: extreme moduli, the share of eigenvalues near the
    origin (|lambda| < 0.1) and within 0.5 of 1, and the real-part range."""
    a = np.abs(ev)
    return {"n": int(len(ev)), "min_abs": float(a.min()), "max_abs": float(a.max()),
            "frac_abs_below_0.1": float(np.mean(a < 0.1)),
            "frac_within_0.5_of_1": float(np.mean(np.abs(ev - 1.0) < 0.5)),
            "re_min": float(ev.real.min()), "re_max": float(ev.real.max()),
            "max_abs_imag": float(np.abs(ev.imag).max())}


def spectrum(case, kind, p1="ilu"):
    """Eigenvalues of J M^{-1} at the case's state, and their summary."""
    rp, ci, v = tpfa.jacobian(case, case.u, case.u_old)
    ev = np.linalg.eigvals(preconditioned_matrix(kind, rp, ci, v, (case.nx, case.ny, case.nz),
                                                 p1=p1))
    return ev, summary(ev)
