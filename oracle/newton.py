"""Oracle: Newton linearisation of Sec. 3, J(u_k) delta = -F(u_k),
u_{k+1} = u_k + delta.  The paper's 'variant of Newton's method' is not
specified; the reading used here: each saturation increment is limited to
[-ds_max, ds_max] (a per-cell saturation chop, when ds_max > 0), then S_n is
clamped to [0,1]; no line search."""
from __future__ import annotations

import numpy as np

from . import tpfa
from .fgmres import fgmres
from .precond import Preconditioner


def linear_system(case):
    """(row_ptr, col_idx, vals, b) with b = -F(u) point ordered."""
    rp, ci, v = tpfa.jacobian(case, case.u, case.u_old)
    R = tpfa.residual(case, case.u, case.u_old)
    return rp, ci, v, -R.reshape(-1)


def solve(case, kind="bf", rtol=1e-8, restart=30, maxit=1000, inner="vcycle", amg_opts=None):
    rp, ci, v, b = linear_system(case)
    M = Preconditioner(kind, rp, ci, v, (case.nx, case.ny, case.nz), inner=inner,
                       amg_opts=amg_opts)
    J = tpfa.bcsr_matrix(rp, ci, v).tocsr()
    x, info = fgmres(lambda z: J @ z, M.apply, b, rtol=rtol, restart=restart, maxit=maxit)
    return x, info, (rp, ci, v, b, M)


def update(u, delta, ds_max=0.0):
    d = delta.reshape(-1, 2).copy()
    if ds_max > 0:
        d[:, 1] = np.clip(d[:, 1], -ds_max, ds_max)
    un = u + d
    un[:, 1] = np.clip(un[:, 1], 0.0, 1.0)
    return un


def sequence(case, n_jacobians, kind="bf", ds_max=0.2, rtol=1e-8, amg_opts=None):
    """Consecutive Newton Jacobians of one time step: returns the list of
    (||F||, linear-solve info) and the final state."""
    u = case.u.copy()
    out = []
    for _ in range(n_jacobians):
        ck = case.replace(u=u)
        x, info, _ = solve(ck, kind, rtol=rtol, amg_opts=amg_opts)
        Fn = float(np.linalg.norm(tpfa.residual(ck, ck.u, ck.u_old)))
        out.append((Fn, info))
        u = update(u, x, ds_max)
    return out, u
