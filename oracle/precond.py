"""Oracle: the paper's preconditioners M^{-1} r (Sec. 3.2-3.4).

* AMG   black-box AMG on the point-ordered scalar Jacobian (Sec. 3.2).
* CPR1  Algorithm 1 / Eq. m_comb: u = P_1^{-1} r; r' = r - J u;
        u += R_p^T A_pp^{-1} R_p r'.
* CPR2  Algorithm 2 / Eq. m_add: as CPR1 plus R_s^T A_ss^{-1} R_s r' from
        the same updated residual.
* BF    Algorithm 3 / Eq. m_bf: s = A_ss^{-1} R_s r; t = R_p r - A_ps s;
        p = S~^{-1} t; u = (p, s).

Inner solves A^{-1} are one AMG V-cycle each (Sec. 4.1: one V-cycle), or
exact sparse LU (``inner='exact'``) for the matrix-form checks.  P_1 is
block ILU(0), or the exact inverse of J with ``p1='exact'``.

AMG interpolation per operator (unless ``amg_opts['interp']`` is given):
extended+i for the pressure-like operators (S~, A_pp) and direct
interpolation for A_ss and the point-ordered J of black-box AMG.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import blocks
from .amg import Hierarchy
from .ilu import Bilu0
from .tpfa import bcsr_matrix


class Exact:
    def __init__(self, A):
        self.lu = spla.splu(A.tocsc())

    def vcycle(self, b):
        return self.lu.solve(b)


def inner_solver(A, inner, amg_opts, interp):
    if inner == "exact":
        return Exact(A)
    opts = dict(amg_opts or {})
    opts.setdefault("interp", interp)
    return Hierarchy(A, **opts)


class Preconditioner:
    def __init__(self, kind, row_ptr, col_idx, vals, grid, inner="vcycle", p1="ilu",
                 amg_opts=None):
        self.kind = kind
        self.J = bcsr_matrix(row_ptr, col_idx, vals).tocsr()
        if kind == "amg":
            self.Js = blocks.scalarize(row_ptr, col_idx, vals)
            self.H = inner_solver(self.Js, inner, amg_opts, "direct")
            return
        self.App = blocks.block(row_ptr, col_idx, vals, 0, 0)
        self.Aps = blocks.block(row_ptr, col_idx, vals, 0, 1)
        self.Asp = blocks.block(row_ptr, col_idx, vals, 1, 0)
        self.Ass = blocks.block(row_ptr, col_idx, vals, 1, 1)
        if kind in ("cpr1", "cpr2"):
            if p1 == "exact":
                self.P1 = Exact(self.J)
                self.p1_apply = self.P1.vcycle
            else:
                self.P1 = Bilu0(row_ptr, col_idx, vals, *grid)
                self.p1_apply = self.P1.apply
            self.Hp = inner_solver(self.App, inner, amg_opts, "ext+i")
            if kind == "cpr2":
                self.Hs = inner_solver(self.Ass, inner, amg_opts, "direct")
        elif kind == "bf":
            self.S = blocks.schur_simple(self.App, self.Aps, self.Asp, self.Ass)
            self.Hs = inner_solver(self.Ass, inner, amg_opts, "direct")
            self.Hschur = inner_solver(self.S, inner, amg_opts, "ext+i")
        else:
            raise ValueError(kind)

    def apply(self, r):
        k = self.kind
        if k == "amg":
            return self.H.vcycle(r)
        if k in ("cpr1", "cpr2"):
            u = self.p1_apply(r)
            r2 = r - self.J @ u
            u = u + blocks.R_pT(self.Hp.vcycle(blocks.R_p(r2)))
            if k == "cpr2":
                u = u + blocks.R_sT(self.Hs.vcycle(blocks.R_s(r2)))
            return u
        # bf
        s = self.Hs.vcycle(blocks.R_s(r))
        t = blocks.R_p(r) - self.Aps @ s
        p = self.Hschur.vcycle(t)
        z = np.empty(len(r))
        z[0::2] = p
        z[1::2] = s
        return z
