"""Oracle: the fully implicit time loop around the linear solve.

Test infrastructure only (like the rest of this package): plain NumPy/SciPy.

Backward Euler in time (Sec. 2, Eq. fully_discrete_system: every flux,
source and mobility at the new time level), and in every time step Newton's
method (Sec. 3, J(u_k) delta = -F(u_k), u_{k+1} = u_k + delta) until
||F(u_k)|| <= newton_tol (Sec. 4.1 solver settings: 1e-6).  The reading of
the paper's unspecified Newton variant is the one of newton.update: each
saturation increment limited to [-ds_max, ds_max], then S_n clamped to
[0, 1]; no line search and no time-step cuts.  A time step whose Newton
iteration has not met the tolerance after max_newton linear solves, or whose
linear solve does not converge, ends the simulation as diverged (the
paper's '-').  Counts: NI = Newton iterations (linear solves), LI = their
total Krylov iterations (the paper's tables of NI, LI and LI/NI).
"""
from __future__ import annotations

import numpy as np

from . import newton, tpfa
from .fgmres import CONVERGED


def simulate(case, kind, t_final, dt=None, newton_tol=1e-6, max_newton=25, rtol=1e-8,
             ds_max=0.2, amg_opts=None):
    """Returns (record, final state).  record: per time step the residual
    norms before each Newton iteration, the Krylov iterations of each solve,
    the step's status and its final state; totals NI, LI and the overall
    status."""
    dt = case.dt if dt is None else dt
    n_steps = int(round(t_final / dt))
    u = case.u.copy()
    steps = []
    status = "converged"
    for _ in range(n_steps):
        c = case.replace(u=u.copy(), u_old=u.copy(), dt=dt)
        fnorms, its = [], []
        st = "diverged"
        while True:
            fn = float(np.linalg.norm(tpfa.residual(c, c.u, c.u_old)))
            fnorms.append(fn)
            if not np.isfinite(fn):
                break
            if fn <= newton_tol:
                st = "converged"
                break
            if len(its) >= max_newton:
                break
            x, info, _ = newton.solve(c, kind, rtol=rtol, amg_opts=amg_opts)
            its.append(int(info["iterations"]))
            if info["status"] != CONVERGED:
                break
            c = c.replace(u=newton.update(c.u, x, ds_max))
        steps.append(dict(fnorms=fnorms, iterations=its, status=st, u=c.u.copy()))
        u = c.u
        if st != "converged":
            status = "diverged"
            break
    ni = sum(len(s["iterations"]) for s in steps)
    li = sum(sum(s["iterations"]) for s in steps)
    return dict(steps=steps, NI=ni, LI=li, LI_per_NI=li / ni if ni else 0.0,
                status=status), u
