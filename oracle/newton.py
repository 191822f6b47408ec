"""Oracle: Newton linearisation of Sec. 3, J(u_k) delta = -F(u_k),
u_{k+1} = u_k + delta, with S_n clamped to [0,1] (the paper's 'variant of
Newton's method' is not specified further; no line search)."""
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


def update(u, delta):
    un = u + delta.reshape(-1, 2)
    un[:, 1] = np.clip(un[:, 1], 0.0, 1.0)
    return un
