"""Oracle: right-preconditioned flexible GMRES(m) (paper Eq. precon-system:
J M^{-1} c^ = q, c = M^{-1} c^; GMRES as in Sec. 3).

Reading (the paper gives no variant, restart or start vector): x_0 = 0,
restart m = 30, classical Gram-Schmidt applied twice (CGS2), Givens
rotations on the Hessenberg matrix, stop a cycle when the estimated
residual |g_{j+1}| <= rtol ||b|| or h_{j+1,j} = 0, then x += Z y; converged
iff the true residual ||b - J x|| <= rtol ||b||, else restart until maxit
Arnoldi steps in total.  The iteration count is the number of Arnoldi steps.
"""
from __future__ import annotations

import math

import numpy as np

CONVERGED, MAX_ITERS, BREAKDOWN, NONFINITE = 0, 1, 2, 3


def fgmres(matvec, precond, b, rtol=1e-8, restart=30, maxit=1000, history=None):
    n = len(b)
    x = np.zeros(n)
    beta0 = float(np.linalg.norm(b))
    if beta0 == 0.0:
        return x, dict(status=CONVERGED, iterations=0, relres=0.0, relres_est=0.0)
    if not math.isfinite(beta0):
        return x, dict(status=NONFINITE, iterations=0, relres=float("nan"), relres_est=float("nan"))
    m = restart
    total = 0
    r = b.copy()
    status = MAX_ITERS
    est = 1.0
    while True:
        beta = float(np.linalg.norm(r))
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        breakdown = False
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            col = np.zeros(m + 1)
            col[:j + 1] = h
            col[j + 1] = hn
            for i in range(j):
                a, c = col[i], col[i + 1]
                col[i] = cs[i] * a + sn[i] * c
                col[i + 1] = -sn[i] * a + cs[i] * c
            d = math.hypot(col[j], col[j + 1])
            total += 1
            k = j + 1
            if d == 0.0 or not math.isfinite(d):
                breakdown = True
                k = j
                break
            cs[j] = col[j] / d
            sn[j] = col[j + 1] / d
            col[j] = d
            col[j + 1] = 0.0
            H[:, j] = col
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1]) / beta0
            if history is not None:
                history.append(est)
            if hn != 0.0:
                V[j + 1] = w / hn
            if abs(g[j + 1]) <= rtol * beta0 or hn == 0.0 or total >= maxit:
                break
        if k > 0:
            y = np.zeros(k)
            for i in range(k - 1, -1, -1):
                y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
            x = x + Z[:k].T @ y
        r = b - matvec(x)
        rn = float(np.linalg.norm(r))
        if not math.isfinite(rn):
            status = NONFINITE
            break
        if rn <= rtol * beta0:
            status = CONVERGED
            break
        if breakdown:
            status = BREAKDOWN
            break
        if total >= maxit:
            status = MAX_ITERS
            break
    return x, dict(status=status, iterations=total, relres=rn / beta0, relres_est=est)
