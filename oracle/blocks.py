"""Oracle: block views of the Jacobian (paper Sec. 3.1, Eq. jacobian),
the point-ordered scalar matrix used by black-box AMG (Sec. 3.2), the
restrictions R_p, R_s (Sec. 3.3) and the SIMPLE-type approximate Schur
complement of Sec. 3.4 (Eq. SIMPLE-Schur, read with A_sp as the trailing
factor, as in the exact Schur complement S = A_pp - A_ps A_ss^{-1} A_sp).

Patterns are symbolic: every stored block of J is kept even if its value is
zero, and product patterns are computed from unit values so that numerical
cancellation never removes an entry.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def block(row_ptr, col_idx, vals, a, b):
    """Scalar CSR (N x N) holding component (a, b) of every 2x2 block."""
    N = len(row_ptr) - 1
    return sp.csr_matrix((vals[:, a, b].copy(), col_idx.copy(), row_ptr.copy()), shape=(N, N))


def scalarize(row_ptr, col_idx, vals):
    """Point-ordered 2N x 2N CSR: unknown 2i is P_w of cell i, 2i+1 is S_n;
    row 2i+a holds, for each block (i,j) in column order, entries
    (2j, vals[a][0]) and (2j+1, vals[a][1])."""
    N = len(row_ptr) - 1
    nb = np.diff(row_ptr)
    rp = np.zeros(2 * N + 1, np.int64)
    per_row = np.repeat(2 * nb, 2)
    np.cumsum(per_row, out=rp[1:])
    cols = np.empty(4 * len(col_idx), np.int64)
    data = np.empty(4 * len(col_idx))
    for i in range(N):
        s, e = row_ptr[i], row_ptr[i + 1]
        cj = col_idx[s:e].astype(np.int64)
        for a in range(2):
            o = rp[2 * i + a]
            cols[o:o + 2 * (e - s):2] = 2 * cj
            cols[o + 1:o + 2 * (e - s):2] = 2 * cj + 1
            data[o:o + 2 * (e - s):2] = vals[s:e, a, 0]
            data[o + 1:o + 2 * (e - s):2] = vals[s:e, a, 1]
    return sp.csr_matrix((data, cols, rp), shape=(2 * N, 2 * N))


def R_p(x):
    """Restriction to the pressure unknowns."""
    return x[0::2].copy()


def R_s(x):
    """Restriction to the saturation unknowns."""
    return x[1::2].copy()


def R_pT(p):
    """Prolongation of a pressure vector, saturation entries zero."""
    y = np.zeros(2 * len(p))
    y[0::2] = p
    return y


def R_sT(s):
    y = np.zeros(2 * len(s))
    y[1::2] = s
    return y


def ones_like_pattern(A):
    B = A.copy()
    B.data = np.ones_like(B.data)
    return B


def place_on_pattern(pattern, values):
    """CSR with the (sorted) pattern of ``pattern`` and the entries of
    ``values`` (whose pattern must be a subset); missing entries are 0."""
    P = pattern.tocsr()
    P.sort_indices()
    Vv = values.tocsr()
    Vv.sort_indices()
    n, m = P.shape
    rp = np.repeat(np.arange(n, dtype=np.int64), np.diff(P.indptr))
    kp = rp * m + P.indices
    rv = np.repeat(np.arange(n, dtype=np.int64), np.diff(Vv.indptr))
    kv = rv * m + Vv.indices
    pos = np.searchsorted(kp, kv)
    assert np.all(kp[pos] == kv), "value pattern not contained in symbolic pattern"
    data = np.zeros(len(kp))
    data[pos] = Vv.data
    return sp.csr_matrix((data, P.indices.copy(), P.indptr.copy()), shape=(n, m))


def symbolic_product(*mats):
    """Pattern of the product of the given matrices, from unit values."""
    out = ones_like_pattern(mats[0])
    for M in mats[1:]:
        out = out @ ones_like_pattern(M)
    out = out.tocsr()
    out.sort_indices()
    return out


def schur_simple(App, Aps, Asp, Ass):
    """S~ = A_pp - (A_ps diag(A_ss)^{-1}) A_sp on the symbolic pattern
    pat(A_pp) U pat(A_ps) pat(A_sp)."""
    dinv = 1.0 / Ass.diagonal()
    Y = Aps.tocsr().copy()
    Y.data = Y.data * dinv[Y.indices]
    prod = Y @ Asp
    pat = (ones_like_pattern(App) + symbolic_product(Aps, Asp)).tocsr()
    pat.sort_indices()
    S = place_on_pattern(pat, App) - place_on_pattern(pat, prod)
    # subtraction in scipy can drop exact zeros: rebuild on the pattern
    return place_on_pattern(pat, S) if S.nnz != pat.nnz else S
