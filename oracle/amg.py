"""Oracle: classical algebraic multigrid as chosen for this build.

The paper applies one AMG V-cycle per inner solve (Sec. 3.2-3.4, Sec. 4.1
solver settings) with hypre BoomerAMG (CLJP coarsening, classical
interpolation, hybrid Gauss-Seidel).  The build replaces those components by
deterministic, data-parallel ones; this module states exactly those:

1. strength: s_i = sign(a_ii) (+1 for a_ii >= 0), m_i = max_{k!=i} -s_i a_ik;
   j is strong for i iff m_i > 0 and -s_i a_ij >= theta m_i;
2. PMIS coarsening (De Sterck, Yang, Heys), or CLJP (see cljp()): weights w_i = |S^T_i| + u_i with
   u_i = (splitmix64(seed ^ i) >> 40) * 2^-24; points with |S^T_i| = 0 start
   as F; each round an undecided i becomes C iff (w_i, i) beats (w_j, j)
   lexicographically for every undecided j in S_i u S^T_i; then every
   undecided j with a new C point in S_j becomes F;
3. direct interpolation (Stueben): for an F point i with P_i = C n S_i,
   w_ij = -alpha_i a_ij / a~_ii, alpha_i = sum_{k!=i} a_ik^- / sum_{k in P_i} a_ik^-,
   where ^- marks entries of sign opposite to a_ii and a~_ii = a_ii plus the
   same-signed off-diagonal entries (strong points always have the opposite
   sign, so the same-signed part is always lumped); C rows are injection,
   coarse points are numbered in ascending fine order;
   or extended+i interpolation (De Sterck, Falgout, Nolting, Yang, 2008) for
   an F point i: C^_i = (C n S_i) u (C n S_k over strong F neighbours k);
   with a-bar_kl = a_kl when its sign is opposite to a_kk (else 0) and
   d_ik = sum over l in C^_i u {i} of a-bar_kl,
   w_ij = -(a_ij + sum_k a_ik a-bar_kj / d_ik) / a~_ii,
   a~_ii = a_ii + (off-diagonal entries of row i that are neither in C^_i
   nor strong F) + sum_k a_ik a-bar_ki / d_ik, and a strong F neighbour with
   d_ik = 0 is lumped into a~_ii;
   or classical interpolation (Ruge, Stueben 1987; Stueben 2001, in the
   modified form that filters signs, as BoomerAMG's classical interpolation
   does) for an F point i: C_i = C n S_i, d_ik = sum over m in C_i of
   a-bar_km for each strong F neighbour k (a-bar as above),
   w_ij = -(a_ij + sum_k a_ik a-bar_kj / d_ik) / a~_ii,
   a~_ii = a_ii + (weak off-diagonal entries of row i) + (a_ik of every
   strong F neighbour with d_ik = 0);
3a. interpolation truncation (a setting of this build; the paper leaves the
   sparsity of P to its AMG package): with pmax > 0 or factor > 0, each row
   of P ranks its entries by |w_ij| rounded to FP32 (larger first; the lower
   column first among equal magnitudes) and keeps those ranked below pmax
   (all when pmax = 0) whose rounded magnitude is at least factor times the
   row's largest; the kept positive entries are then scaled by
   (sum of the row's positive entries) / (sum of the kept positive ones),
   and the negative ones likewise, so each sign's row sum is unchanged
   (a sign with no kept entry loses its sum); sums run in ascending column
   order.  Default pmax = 3, factor = 0 on every level;
4. R = P^T, A_c = R (A P) with the symbolic pattern (no dropping);
5. stop when n <= coarse_max, n_c == 0, n_c > 0.9 n, or max_levels; the
   coarsest level is solved by dense LU with partial pivoting when it has at
   most dense_max rows, otherwise by two l1-Jacobi sweeps;
6. V(nu1, nu2) cycle, zero initial guess on every level, with nu1 pre- and
   nu2 post-smoothing steps (default 1 and 1) of either smoother:
   * l1-Jacobi (Baker, Falgout, Kolev, Yang 2011): x <- x + D^{-1}(b - A x),
     d_i = a_ii + s_i sum_{j!=i} |a_ij| (rows with d_i = 0 are not smoothed);
   * Chebyshev of degree k on D^{-1} A (D the same l1 diagonal): the
     three-term Chebyshev iteration (Saad, Iterative Methods, Alg. 12.1)
     for the interval [lo, hi], hi = 1.1 lambda^ and lo = 0.3 hi, where
     lambda^ estimates the largest eigenvalue of D^{-1} A by power
     iteration from the PMIS hash vector; its error propagator is the
     scaled Chebyshev polynomial T_k((c - t)/h) / T_k(c/h), c = (hi+lo)/2,
     h = (hi-lo)/2, in t = D^{-1} A;
   * multicolour Gauss-Seidel, standing in for the paper's hybrid
     Gauss-Seidel (Sec. 4.1 solver settings), which is sequential within a
     process: the points are coloured so that no two neighbours in the
     pattern of A + A^T share a colour (round r colours the points whose
     hash key beats every uncoloured neighbour's), and a sweep updates
     x_i <- x_i + (b_i - (A x)_i) / a_ii colour by colour, in ascending
     colour order before the coarse-grid correction and descending after
     it.  The l1-Jacobi and Chebyshev smoothers are polynomials in A
     applied row-parallel.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .blocks import place_on_pattern, symbolic_product

UNDECIDED, C_PT, F_PT = 0, 1, 2
MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output function (Steele, Lea, Flood 2014) of state x."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_vec(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def pmis_random(n: int, seed: int) -> np.ndarray:
    i = np.arange(n, dtype=np.uint64)
    z = splitmix64_vec(np.uint64(seed) ^ i)
    return (z >> np.uint64(40)).astype(np.float64) * 2.0 ** -24


def row_index(A):
    return np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))


def diag_sign(A):
    return np.where(A.diagonal() < 0, -1.0, 1.0)


def strength(A, theta=0.25):
    """Boolean mask over the stored entries of A (CSR, sorted)."""
    n = A.shape[0]
    rows = row_index(A)
    cols = A.indices
    s = diag_sign(A)
    offd = cols != rows
    neg = -s[rows] * A.data
    m = np.full(n, -np.inf)
    np.maximum.at(m, rows[offd], neg[offd])
    mr = m[rows]
    return offd & (mr > 0) & (neg >= theta * mr)


def strength_matrix(A, mask):
    rows = row_index(A)
    return sp.csr_matrix((np.ones(int(mask.sum()), np.int8), (rows[mask], A.indices[mask])),
                         shape=A.shape)


def pmis(A, mask, seed):
    """C/F splitting (array of C_PT / F_PT) and the number of rounds."""
    n = A.shape[0]
    S = strength_matrix(A, mask)
    ST = S.T.tocsr()
    nst = np.diff(ST.indptr)
    w = nst + pmis_random(n, seed)
    state = np.full(n, UNDECIDED, np.int8)
    state[nst == 0] = F_PT
    G = ((S + ST) > 0).tocsr()
    gr = row_index(G)
    gc = G.indices
    Sr = row_index(S)
    Sc = S.indices
    rounds = 0
    while np.any(state == UNDECIDED):
        rounds += 1
        und = state == UNDECIDED
        live = und[gr] & und[gc]
        beats = live & ((w[gc] > w[gr]) | ((w[gc] == w[gr]) & (gc > gr)))
        lose = np.zeros(n, bool)
        lose[gr[beats]] = True
        newc = und & ~lose
        state[newc] = C_PT
        hasc = np.zeros(n, bool)
        hasc[Sr[newc[Sc]]] = True
        state[und & ~newc & hasc] = F_PT
    return state, rounds


def cljp(A, mask, seed):
    """CLJP C/F splitting (Cleary, Falgout, Henson, Jones 1998), the
    coarsening of the paper's BoomerAMG settings (Sec. 4.1).  S is the
    strength graph (edge i -> j when i depends on j, j in S_i).

    w_i = |S^T_i| + u_i (u_i the PMIS hash weight); points with w_i < 1 are
    F from the start.  Each round, on the edges not yet removed:
      1. D = undecided points whose (w_i, i) beats that of every undecided
         point joined to them by an edge (either direction); D becomes C;
      2. for c in D: every j that c depends on loses 1 (edge c -> j
         removed); for every j and k that both depend on c with k depending
         on j, j loses 1 and the edge k -> j is removed (j is less needed
         as a C point: k can take its value from c); then the edges into c
         are removed;
      3. undecided points with w < 1 become F.
    Each removed edge lowers its target's weight once, so a round does not
    depend on the order in which D is processed.  Returns (splitting,
    number of rounds)."""
    n = A.shape[0]
    S = strength_matrix(A, mask).tocsr()
    S.sort_indices()
    ST = S.T.tocsr()
    ST.sort_indices()
    alive = {(int(i), int(j)) for i, j in zip(row_index(S), S.indices)}
    out_nb = [set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist()) for i in range(n)]
    in_nb = [set(ST.indices[ST.indptr[i]:ST.indptr[i + 1]].tolist()) for i in range(n)]
    w = np.diff(ST.indptr) + pmis_random(n, seed)
    state = np.full(n, UNDECIDED, np.int8)
    state[w < 1.0] = F_PT
    rounds = 0
    while np.any(state == UNDECIDED):
        rounds += 1
        und = state == UNDECIDED
        D = []
        for i in np.flatnonzero(und):
            nb = [j for j in out_nb[i] if (i, j) in alive] + [j for j in in_nb[i] if (j, i) in alive]
            if all(not und[j] or (w[i], i) > (w[j], j) for j in nb if j != i):
                D.append(int(i))
        removed = set()
        for c in D:
            for j in out_nb[c]:
                if (c, j) in alive:
                    removed.add((c, j))
            deps = [j for j in in_nb[c] if (j, c) in alive]
            for j in deps:
                for k in deps:
                    if k != j and (k, j) in alive:
                        removed.add((k, j))
        for (_, j) in removed:
            w[j] -= 1.0
        alive -= removed
        for c in D:
            alive -= {(j, c) for j in in_nb[c]}
        state[D] = C_PT
        state[(state == UNDECIDED) & (w < 1.0)] = F_PT
    return state, rounds


def coarsen(A, mask, seed, kind="pmis"):
    return cljp(A, mask, seed) if kind == "cljp" else pmis(A, mask, seed)


def direct_interpolation(A, mask, cf):
    """P (n x n_c CSR, columns ascending) and the coarse index map."""
    n = A.shape[0]
    rows = row_index(A)
    cols = A.indices
    vals = A.data
    diag = A.diagonal()
    s = diag_sign(A)
    offd = cols != rows
    opp = offd & (s[rows] * vals < 0)
    same = offd & (s[rows] * vals > 0)
    isc = cf == C_PT
    cidx = np.cumsum(isc) - 1
    nc = int(isc.sum())
    pmask = mask & isc[cols]
    sum_n_opp = np.bincount(rows[opp], vals[opp], minlength=n)
    sum_n_same = np.bincount(rows[same], vals[same], minlength=n)
    sum_p_opp = np.bincount(rows[pmask], vals[pmask], minlength=n)
    atil = diag + sum_n_same
    frow = ~isc[rows]
    emask = pmask & frow
    er = rows[emask]
    alpha = sum_n_opp[er] / sum_p_opp[er]
    wv = -alpha * vals[emask] / atil[er]
    crow = np.nonzero(isc)[0]
    r_all = np.concatenate([er, crow])
    c_all = np.concatenate([cidx[cols[emask]], cidx[crow]])
    v_all = np.concatenate([wv, np.ones(len(crow))])
    order = np.lexsort((c_all, r_all))
    P = sp.csr_matrix((v_all[order], (r_all[order], c_all[order])), shape=(n, nc))
    # csr_matrix from COO sums duplicates (there are none) and keeps zeros
    P.sort_indices()
    return P, cidx


def extended_i_interpolation(A, mask, cf):
    """Extended+i interpolation, one F row at a time (see module docstring)."""
    A = A.tocsr()
    n = A.shape[0]
    rp, ci, av = A.indptr, A.indices, A.data
    diag = A.diagonal()
    s = diag_sign(A)
    isc = cf == C_PT
    cidx = np.cumsum(isc) - 1
    nc = int(isc.sum())
    r_out, c_out, v_out = [], [], []
    for i in range(n):
        if isc[i]:
            r_out.append(i)
            c_out.append(cidx[i])
            v_out.append(1.0)
            continue
        row = range(rp[i], rp[i + 1])
        strong_f = [e for e in row if mask[e] and ci[e] != i and not isc[ci[e]]]
        chat = {int(ci[e]) for e in row if mask[e] and isc[ci[e]]}
        for e in strong_f:
            k = ci[e]
            chat |= {int(ci[f]) for f in range(rp[k], rp[k + 1]) if mask[f] and isc[ci[f]]}
        w = dict.fromkeys(chat, 0.0)
        atil = diag[i]
        sf = set(strong_f)
        for e in row:
            j = int(ci[e])
            if j == i:
                continue
            if j in chat:
                w[j] += av[e]
            elif e not in sf:
                atil += av[e]
        for e in strong_f:
            k = ci[e]
            aik = av[e]
            kr = range(rp[k], rp[k + 1])
            d = sum(av[f] for f in kr
                    if s[k] * av[f] < 0 and (int(ci[f]) in chat or ci[f] == i))
            if d == 0.0:
                atil += aik
                continue
            for f in kr:
                l = int(ci[f])
                if s[k] * av[f] < 0:
                    if l in chat:
                        w[l] += aik * av[f] / d
                    elif l == i:
                        atil += aik * av[f] / d
        for j in sorted(chat):
            r_out.append(i)
            c_out.append(cidx[j])
            v_out.append(-w[j] / atil)
    P = sp.csr_matrix((np.array(v_out, float), (np.array(r_out, np.int64), np.array(c_out, np.int64))),
                      shape=(n, nc))
    P.sort_indices()
    return P, cidx


def classical_interpolation(A, mask, cf):
    """Classical (Ruge-Stueben) interpolation in its modified form, one F
    row at a time (see module docstring): interpolatory set C_i = C n S_i;
    each strong F neighbour k is distributed over C_i through the entries of
    row k whose sign is opposite to a_kk, or lumped into the diagonal when
    none of them falls in C_i; weak entries are lumped into the diagonal."""
    A = A.tocsr()
    n = A.shape[0]
    rp, ci, av = A.indptr, A.indices, A.data
    diag = A.diagonal()
    s = diag_sign(A)
    isc = cf == C_PT
    cidx = np.cumsum(isc) - 1
    nc = int(isc.sum())
    r_out, c_out, v_out = [], [], []
    for i in range(n):
        if isc[i]:
            r_out.append(i)
            c_out.append(cidx[i])
            v_out.append(1.0)
            continue
        row = range(rp[i], rp[i + 1])
        ci_set = sorted(int(ci[e]) for e in row if mask[e] and isc[ci[e]])
        strong_f = [e for e in row if mask[e] and ci[e] != i and not isc[ci[e]]]
        w = dict.fromkeys(ci_set, 0.0)
        atil = diag[i]
        for e in row:
            j = int(ci[e])
            if j == i:
                continue
            if j in w and mask[e]:
                w[j] += av[e]
            elif not mask[e]:
                atil += av[e]
        for e in strong_f:
            k = ci[e]
            aik = av[e]
            kr = range(rp[k], rp[k + 1])
            d = sum(av[f] for f in kr if s[k] * av[f] < 0 and int(ci[f]) in w)
            if d == 0.0:
                atil += aik
                continue
            for f in kr:
                m = int(ci[f])
                if s[k] * av[f] < 0 and m in w:
                    w[m] += aik * av[f] / d
        for j in ci_set:
            r_out.append(i)
            c_out.append(cidx[j])
            v_out.append(-w[j] / atil)
    P = sp.csr_matrix((np.array(v_out, float), (np.array(r_out, np.int64), np.array(c_out, np.int64))),
                      shape=(n, nc))
    P.sort_indices()
    return P, cidx


TRUNC_PMAX = 3       # default: at most three interpolatory points per row
TRUNC_FACTOR = 0.0


def truncate_interpolation(P, pmax, factor=0.0):
    """Interpolation truncation (module docstring, item 3a)."""
    P = P.tocsr()
    P.sort_indices()
    if pmax <= 0 and factor <= 0.0:
        return P
    rp, ci, pv = P.indptr, P.indices, P.data
    keep = np.ones(P.nnz, bool)
    val = pv.astype(float).copy()
    lengths = np.diff(rp)
    # rows that can change (factor < 1: a single entry is always kept, and
    # with factor = 0 a row of at most pmax entries keeps all of them)
    may_change = lengths > 1 if factor > 0.0 else lengths > pmax
    for i in np.flatnonzero(may_change):
        ents = list(range(rp[i], rp[i + 1]))        # ascending column
        key = {e: float(np.float32(abs(pv[e]))) for e in ents}
        largest = max(key.values())
        ranked = sorted(ents, key=lambda e: (-key[e], ci[e]))
        kept = {e for r, e in enumerate(ranked)
                if (pmax <= 0 or r < pmax) and key[e] >= factor * largest}
        pos_all = neg_all = pos_kept = neg_kept = 0.0
        for e in ents:
            if pv[e] > 0:
                pos_all += pv[e]
                if e in kept:
                    pos_kept += pv[e]
            elif pv[e] < 0:
                neg_all += pv[e]
                if e in kept:
                    neg_kept += pv[e]
        for e in ents:
            if e not in kept:
                keep[e] = False
            elif pv[e] > 0:
                val[e] = pv[e] * (pos_all / pos_kept)
            elif pv[e] < 0:
                val[e] = pv[e] * (neg_all / neg_kept)
    rows = np.repeat(np.arange(P.shape[0]), lengths)[keep]
    Q = sp.csr_matrix((val[keep], (rows, ci[keep])), shape=P.shape)
    Q.sort_indices()
    return Q


def interpolation(A, mask, cf, kind, pmax=0, factor=0.0):
    """P of the given kind, then truncated (item 3a) when pmax or factor is set."""
    if kind == "ext+i":
        P, cidx = extended_i_interpolation(A, mask, cf)
    elif kind == "classical":
        P, cidx = classical_interpolation(A, mask, cf)
    else:
        P, cidx = direct_interpolation(A, mask, cf)
    return truncate_interpolation(P, pmax, factor), cidx


def galerkin(A, P):
    """A_c = R (A P), R = P^T, on the symbolic pattern (no dropping)."""
    R = P.T.tocsr()
    R.sort_indices()
    AP = A @ P
    val = R @ AP
    pat = symbolic_product(R, A, P)
    return place_on_pattern(pat, val), R


def l1_diag(A):
    rows = row_index(A)
    offd = A.indices != rows
    s = diag_sign(A)
    off = np.bincount(rows[offd], np.abs(A.data[offd]), minlength=A.shape[0])
    return A.diagonal() + s * off


def power_max_eig(A, dinv, iters, seed):
    """Estimate of the largest eigenvalue magnitude of D^{-1} A: `iters`
    power steps v <- w / ||w||, w = D^{-1} A v, from v = the PMIS hash
    vector (u_i - 1/2) normalised; returns ||w|| of the last step."""
    v = pmis_random(A.shape[0], seed) - 0.5
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = dinv * (A @ v)
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            return 0.0
        v = w / lam
    return lam


def chebyshev_bounds(lam, hi_factor=1.1, lo_fraction=0.3):
    hi = hi_factor * lam
    return lo_fraction * hi, hi


def l1_jacobi_smooth(A, dinv, b, x):
    """One l1-Jacobi step x + D^{-1}(b - A x)."""
    return x + dinv * (b - A @ x)


def chebyshev_smooth(A, dinv, b, x, lo, hi, degree):
    """Chebyshev iteration of the given degree on D^{-1} A x = D^{-1} b over
    the interval [lo, hi] (Saad, Alg. 12.1): with c = (hi+lo)/2, h =
    (hi-lo)/2, sigma = c/h and rho_0 = 1/sigma,
      d_0 = D^{-1}(b - A x_0) / c,  x_1 = x_0 + d_0,
      rho_k = 1/(2 sigma - rho_{k-1}),
      d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / h) D^{-1}(b - A x_k),
      x_{k+1} = x_k + d_k."""
    c = 0.5 * (hi + lo)
    h = 0.5 * (hi - lo)
    sigma = c / h
    rho = 1.0 / sigma
    d = dinv * (b - A @ x) / c
    x = x + d
    for _ in range(degree - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / h) * (dinv * (b - A @ x))
        x = x + d
        rho = rho_new
    return x


def gs_colors(A, seed):
    """Colouring for the multicolour Gauss-Seidel smoother.  The graph is
    the stored off-diagonal pattern of A + A^T.  Round r gives colour r to
    every uncoloured point whose key (u_i, i) exceeds the key of each
    uncoloured neighbour, u_i being the PMIS hash weight; points of one
    colour are therefore never neighbours.  Returns (colour per point,
    number of colours)."""
    A = A.tocsr()
    n = A.shape[0]
    pat = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    G = (pat + pat.T).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    rows = np.repeat(np.arange(n), np.diff(G.indptr))
    k = (splitmix64_vec(np.uint64(seed) ^ np.arange(n, dtype=np.uint64)) >> np.uint64(40)).astype(np.int64)
    key = (k << 32) | np.arange(n, dtype=np.int64)
    color = np.full(n, -1, np.int64)
    r = 0
    while (color < 0).any():
        und = color < 0
        nb = np.where(und[G.indices], key[G.indices], -1)
        best = np.full(n, -1, np.int64)
        np.maximum.at(best, rows, nb)
        pick = und & (key > best)
        color[pick] = r
        r += 1
    return color, r


def gs_sweep(A, diag, color_rows, b, x, reverse):
    """One multicolour Gauss-Seidel sweep, colours in ascending order
    (backward: descending): for the points i of each colour,
    x_i <- x_i + (b_i - (A x)_i) / a_ii with the x of the colours already
    swept; points with a_ii = 0 are left as they are."""
    x = x.copy()
    order = range(len(color_rows) - 1, -1, -1) if reverse else range(len(color_rows))
    for c in order:
        idx, Ac = color_rows[c]
        d = diag[idx]
        r = b[idx] - Ac @ x
        x[idx] += np.divide(r, d, out=np.zeros_like(r), where=d != 0)
    return x


class Level:
    def __init__(self, A):
        self.A = A.tocsr()
        self.A.sort_indices()
        self.n = A.shape[0]
        d = l1_diag(self.A)
        # a zero l1 row (a decoupled, empty row) is left unsmoothed
        self.dinv = np.divide(1.0, d, out=np.zeros_like(d), where=d != 0)
        self.P = None
        self.R = None
        self.mask = None
        self.cf = None
        self.cheb = None  # (lo, hi) of the Chebyshev smoother
        self.gs = None    # (colour per point, [(points, their rows of A)] per colour)

    def smooth(self, b, x, H, post=False):
        # multicolour Gauss-Seidel: forward sweeps before the coarse-grid
        # correction, backward after it (a symmetric cycle)
        if H.smoother == "gs":
            return gs_sweep(self.A, self.A.diagonal(), self.gs[1], b, x, reverse=post)
        # a zero eigenvalue estimate (D^{-1} A = 0) leaves l1-Jacobi sweeps
        if H.smoother == "chebyshev" and self.cheb[1] > 0.0:
            lo, hi = self.cheb
            return chebyshev_smooth(self.A, self.dinv, b, x, lo, hi, H.cheb_degree)
        return l1_jacobi_smooth(self.A, self.dinv, b, x)


class Hierarchy:
    """AMG hierarchy; ``levels[-1]`` is the coarsest."""

    def __init__(self, A, theta=0.25, coarse_max=128, max_levels=25, seed=0x5eed,
                 dense_max=1024, interp="direct", smoother="l1jacobi", nu1=1, nu2=1,
                 cheb_degree=2, cheb_eig_iters=10, coarsening="pmis", trunc_pmax=TRUNC_PMAX,
                 trunc_factor=TRUNC_FACTOR):
        self.levels = []
        self.interp = interp
        self.dense_max = dense_max
        self.smoother, self.nu1, self.nu2 = smoother, nu1, nu2
        self.cheb_degree, self.cheb_eig_iters, self.seed = cheb_degree, cheb_eig_iters, seed
        A = A.tocsr()
        A.sort_indices()
        while True:
            lvl = Level(A)
            self.levels.append(lvl)
            if lvl.n <= coarse_max or len(self.levels) >= max_levels:
                break
            mask = strength(lvl.A, theta)
            cf, _ = coarsen(lvl.A, mask, seed, coarsening)
            nc = int((cf == C_PT).sum())
            if nc == 0 or nc > 0.9 * lvl.n:
                break
            P, _ = interpolation(lvl.A, mask, cf, interp, trunc_pmax, trunc_factor)
            Ac, R = galerkin(lvl.A, P)
            lvl.mask, lvl.cf, lvl.P, lvl.R = mask, cf, P, R
            A = Ac
        last = self.levels[-1]
        self.coarse_dense = last.n <= dense_max
        if self.coarse_dense:
            self.lu = sla.lu_factor(last.A.toarray())
        self.smoother_setup()

    def smoother_setup(self):
        if self.smoother == "chebyshev":
            for L in self.levels[:-1]:
                lam = power_max_eig(L.A, L.dinv, self.cheb_eig_iters, self.seed)
                L.cheb = chebyshev_bounds(lam)
        if self.smoother == "gs":
            for L in self.levels[:-1]:
                color, nc = gs_colors(L.A, self.seed)
                rows = [np.flatnonzero(color == c) for c in range(nc)]
                L.gs = (color, [(idx, L.A[idx]) for idx in rows])

    def coarse_solve(self, b):
        last = self.levels[-1]
        if self.coarse_dense:
            return sla.lu_solve(self.lu, b)
        x = last.dinv * b
        return x + last.dinv * (b - last.A @ x)

    def vcycle(self, b, level=0):
        """One V(nu1, nu2) cycle with zero initial guess."""
        if level == len(self.levels) - 1:
            return self.coarse_solve(b)
        L = self.levels[level]
        x = np.zeros_like(b)
        for _ in range(self.nu1):
            x = L.smooth(b, x, self)
        r = b - L.A @ x
        xc = self.vcycle(L.R @ r, level + 1)
        x = x + L.P @ xc
        for _ in range(self.nu2):
            x = L.smooth(b, x, self, post=True)
        return x

    def stats(self):
        rows = [L.n for L in self.levels]
        nnz = [L.A.nnz for L in self.levels]
        return dict(levels=len(rows), rows=rows, nnz=nnz,
                    operator_complexity=sum(nnz) / nnz[0], grid_complexity=sum(rows) / rows[0])


def hierarchy_from_levels(As, Ps, dense_max=1024, smoother="l1jacobi", nu1=1, nu2=1,
                          cheb_degree=2, cheb_eig_iters=10, seed=0x5eed):
    """An oracle Hierarchy holding given level operators and interpolations
    (used to apply the oracle's V-cycle to matrices produced elsewhere)."""
    H = Hierarchy.__new__(Hierarchy)
    H.levels = []
    H.dense_max = dense_max
    H.smoother, H.nu1, H.nu2 = smoother, nu1, nu2
    H.cheb_degree, H.cheb_eig_iters, H.seed = cheb_degree, cheb_eig_iters, seed
    for l, A in enumerate(As):
        L = Level(A)
        if l < len(Ps):
            L.P = Ps[l].tocsr()
            L.R = L.P.T.tocsr()
            L.R.sort_indices()
        H.levels.append(L)
    last = H.levels[-1]
    H.coarse_dense = last.n <= dense_max
    if H.coarse_dense:
        H.lu = sla.lu_factor(last.A.toarray())
    H.smoother_setup()
    return H
