"""Oracle: ILU(0), the first stage P_1 of the two-stage preconditioners
(paper Sec. 3.3: 'incomplete factorization with no fill ILU(0)').

Reading: block ILU(0) with 2x2 blocks on the point-ordered, lexicographic
Jacobian (the paper's black-box ordering of Sec. 3.2).  ``bilu0_generic``
is the textbook IKJ elimination restricted to the block pattern.  On the
5/7-point block stencil no update ever lands off the diagonal inside the
pattern, so the factorisation reduces to new pivot blocks only,
D_i = A_ii - sum_{k<i, k nbr i} A_ik D_k^{-1} A_ki,
and M = (D + L_A) D^{-1} (D + U_A) with the strictly lower/upper blocks of J;
``Bilu0`` computes that recurrence one anti-diagonal wavefront
(ix+iy+iz = const) at a time, and the tests assert both forms agree.
"""
from __future__ import annotations

import numpy as np


def bilu0_generic(row_ptr, col_idx, vals):
    """Block IKJ ILU(0): returns LU values on the same block pattern
    (unit lower factor implied, L blocks stored left of the diagonal)."""
    N = len(row_ptr) - 1
    lu = vals.copy()
    pos = [dict() for _ in range(N)]
    for i in range(N):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            pos[i][int(col_idx[e])] = e
    for i in range(N):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            k = int(col_idx[e])
            if k >= i:
                break
            ukk = lu[pos[k][k]]
            lu[e] = lu[e] @ np.linalg.inv(ukk)
            for f in range(row_ptr[k], row_ptr[k + 1]):
                j = int(col_idx[f])
                if j <= k:
                    continue
                if j in pos[i]:
                    lu[pos[i][j]] = lu[pos[i][j]] - lu[e] @ lu[f]
    return lu


def wavefronts(nx, ny, nz):
    N = nx * ny * nz
    i = np.arange(N)
    lev = (i % nx) + (i // nx) % ny + i // (nx * ny)
    order = np.argsort(lev, kind="stable")
    counts = np.bincount(lev, minlength=nx + ny + nz - 2)
    return lev, order, counts


def inv2(b):
    det = b[..., 0, 0] * b[..., 1, 1] - b[..., 0, 1] * b[..., 1, 0]
    out = np.empty_like(b)
    out[..., 0, 0] = b[..., 1, 1] / det
    out[..., 0, 1] = -b[..., 0, 1] / det
    out[..., 1, 0] = -b[..., 1, 0] / det
    out[..., 1, 1] = b[..., 0, 0] / det
    return out, det


class Bilu0:
    """Pivot form of block ILU(0) and its apply z = M^{-1} r."""

    def __init__(self, row_ptr, col_idx, vals, nx, ny, nz):
        N = len(row_ptr) - 1
        self.N = N
        self.row_ptr, self.col_idx, self.vals = row_ptr, col_idx, vals
        lev, order, counts = wavefronts(nx, ny, nz)
        self.fronts = np.split(order, np.cumsum(counts)[:-1])
        slot = np.empty(N, np.int64)          # position of a cell inside its front
        for fr in self.fronts:
            slot[fr] = np.arange(len(fr))
        self.slot = slot
        rows = np.repeat(np.arange(N), np.diff(row_ptr))
        cols = col_idx.astype(np.int64)
        self.rows, self.cols = rows, cols
        key = rows.astype(np.int64) * N + cols

        def by_front(entries):
            lv = lev[rows[entries]]
            o = np.argsort(lv, kind="stable")
            e = entries[o]
            c = np.bincount(lv, minlength=len(self.fronts))
            return np.split(e, np.cumsum(c)[:-1])

        lo = np.nonzero(cols < rows)[0]
        up = np.nonzero(cols > rows)[0]
        self.lo_f = by_front(lo)
        self.up_f = by_front(up)
        diagpos = np.nonzero(cols == rows)[0]
        D = vals[diagpos].copy()
        Dinv = np.zeros_like(D)
        self.min_det = np.inf
        for fr, ee in zip(self.fronts, self.lo_f):
            acc = np.zeros((len(fr), 2, 2))
            if len(ee):
                k = cols[ee]
                eT = np.searchsorted(key, k * N + rows[ee])   # A_ki, the mirror block
                contrib = vals[ee] @ Dinv[k] @ vals[eT]
                np.add.at(acc, slot[rows[ee]], contrib)
            D[fr] = D[fr] - acc
            Dinv[fr], det = inv2(D[fr])
            self.min_det = min(self.min_det, float(np.min(np.abs(det))))
        self.D = D
        self.Dinv = Dinv

    def apply(self, r):
        """Forward (D+L) w = r, then (I + D^{-1} U) z = w, wavefront order."""
        N = self.N
        rb = r.reshape(N, 2)
        w = np.zeros((N, 2))
        for fr, ee in zip(self.fronts, self.lo_f):
            acc = np.zeros((len(fr), 2))
            if len(ee):
                np.add.at(acc, self.slot[self.rows[ee]],
                          np.einsum("eab,eb->ea", self.vals[ee], w[self.cols[ee]]))
            w[fr] = np.einsum("eab,eb->ea", self.Dinv[fr], rb[fr] - acc)
        z = np.zeros((N, 2))
        for fr, ee in zip(reversed(self.fronts), reversed(self.up_f)):
            acc = np.zeros((len(fr), 2))
            if len(ee):
                np.add.at(acc, self.slot[self.rows[ee]],
                          np.einsum("eab,eb->ea", self.vals[ee], z[self.cols[ee]]))
            z[fr] = w[fr] - np.einsum("eab,eb->ea", self.Dinv[fr], acc)
        return z.reshape(-1)


def generic_apply(row_ptr, col_idx, lu, r):
    """z = (LU)^{-1} r with the generic factors (unit lower L)."""
    N = len(row_ptr) - 1
    rb = r.reshape(N, 2)
    y = np.zeros((N, 2))
    for i in range(N):
        acc = rb[i].copy()
        for e in range(row_ptr[i], row_ptr[i + 1]):
            k = col_idx[e]
            if k < i:
                acc -= lu[e] @ y[k]
        y[i] = acc
    z = np.zeros((N, 2))
    for i in range(N - 1, -1, -1):
        acc = y[i].copy()
        d = None
        for e in range(row_ptr[i], row_ptr[i + 1]):
            k = col_idx[e]
            if k > i:
                acc -= lu[e] @ z[k]
            elif k == i:
                d = lu[e]
        z[i] = np.linalg.solve(d, acc)
    return z.reshape(-1)


def ilu0_scalar(A):
    """Scalar IKJ ILU(0) of a CSR matrix (dense 2x2 block pattern when A is
    the point-ordered Jacobian); returns dense L (unit lower) and U."""
    A = A.tocsr()
    n = A.shape[0]
    W = A.toarray()
    pat = _structural(A)
    for i in range(1, n):
        for k in range(i):
            if not pat[i, k]:
                continue
            W[i, k] = W[i, k] / W[k, k]
            for j in range(k + 1, n):
                if pat[i, j] and pat[k, j]:
                    W[i, j] -= W[i, k] * W[k, j]
    L = np.tril(W, -1) + np.eye(n)
    U = np.triu(W)
    return L, U


def _structural(A):
    n = A.shape[0]
    P = np.zeros((n, n), bool)
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    P[rows, A.indices] = True
    return P
