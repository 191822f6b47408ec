"""Pins for the oracle's block views, Schur complement, AMG, ILU(0),
preconditioners and FGMRES (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg, blocks, fgmres, ilu, newton, precond, tpfa
from paper_1611_00127_amd import inputs


def _small(nx=6, ny=5, nz=2, seed=1, **kw):
    """Small case with both phases mobile in every cell (S_n in (0.12, 0.88))."""
    c = inputs.small_case(nx, ny, nz, seed=seed, **kw)
    c = inputs.random_state(c, seed + 100, s_lo=0.12, s_hi=0.88)
    rp, ci, v = tpfa.jacobian(c, c.u, c.u_old)
    return c, rp, ci, v


def _perm_point_to_field(N):
    """Permutation matrix taking point order (p0,s0,p1,s1,..) to field order."""
    idx = np.concatenate([np.arange(0, 2 * N, 2), np.arange(1, 2 * N, 2)])
    return np.eye(2 * N)[idx]


# ----------------------------------------------------------------- blocks


def test_scalarize_and_spmv_match_dense():
    c, rp, ci, v = _small()
    D = tpfa.bcsr_to_dense(rp, ci, v)
    np.testing.assert_array_equal(blocks.scalarize(rp, ci, v).toarray(), D)
    x = inputs.random_vector(2 * c.N, 7)
    np.testing.assert_allclose(tpfa.bcsr_spmv(rp, ci, v, x), D @ x, rtol=0,
                               atol=1e-14 * np.abs(D).sum(axis=1).max() * np.abs(x).max())
    # field-ordered blocks are the quadrants of the permuted dense matrix
    Pm = _perm_point_to_field(c.N)
    F = Pm @ D @ Pm.T
    N = c.N
    for (a, b) in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        np.testing.assert_array_equal(blocks.block(rp, ci, v, a, b).toarray(),
                                      F[a * N:(a + 1) * N, b * N:(b + 1) * N])


def test_schur_matches_dense():
    c, rp, ci, v = _small(7, 6, 5, seed=5)
    App, Aps, Asp, Ass = (blocks.block(rp, ci, v, a, b) for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)])
    S = blocks.schur_simple(App, Aps, Asp, Ass).toarray()
    Sd = App.toarray() - Aps.toarray() @ np.diag(1.0 / Ass.diagonal()) @ Asp.toarray()
    np.testing.assert_allclose(S, Sd, rtol=0, atol=1e-13 * np.abs(Sd).max())
    # symbolic pattern: 7-point o 7-point = 25 offsets in the interior of a 3D grid
    Sc = blocks.schur_simple(App, Aps, Asp, Ass)
    assert np.diff(Sc.indptr).max() == 25


def test_schur_closed_form_total_mobility():
    """Uniform state, P_d = 0, no wells: A_ps = -phi V/dt I, A_ss = phi V/dt I,
    so S~ = A_pp + A_sp = the total-mobility TPFA operator."""
    c = inputs.config_c1().replace(pd=0.0, q=np.zeros((1024, 2)),
                                   prod_cells=np.zeros(0, np.int32), prod_wi=np.zeros(0),
                                   prod_pbh=np.zeros(0))
    rp, ci, v = tpfa.jacobian(c, c.u, c.u_old)
    App, Aps, Asp, Ass = (blocks.block(rp, ci, v, a, b) for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)])
    np.testing.assert_array_equal(Ass.toarray(), np.diag(c.poro / c.dt))
    S = blocks.schur_simple(App, Aps, Asp, Ass).toarray()
    # total mobility operator built independently: sum over faces T (lw+ln) (e_l-e_h)(e_l-e_h)^T
    sf = tpfa.sat_functions(c, c.u[:, 1])
    lt = sf["lw"][0] + sf["ln"][0]
    fl, fh, fd = tpfa.faces(c)
    T = tpfa.transmissibility(c, fl, fh, fd)
    B = sp.csr_matrix((np.concatenate([np.ones(len(fl)), -np.ones(len(fl))]),
                       (np.concatenate([np.arange(len(fl))] * 2), np.concatenate([fl, fh]))),
                      shape=(len(fl), c.N))
    L = (B.T @ sp.diags(T * lt) @ B).toarray()
    np.testing.assert_allclose(S, L, rtol=0, atol=1e-13 * np.abs(L).max())


# ----------------------------------------------------------------- AMG


def _laplace2d(n, eps=1.0):
    def d2(m):
        return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    return (sp.kron(sp.identity(n), d2(n)) + eps * sp.kron(d2(n), sp.identity(n))).tocsr()


def test_strength_closed_forms():
    """Isotropic Laplacian: every neighbour is strong.  Anisotropic with
    y-coupling eps < theta: only the x-neighbours are strong."""
    A = _laplace2d(6)
    m = amg.strength(A, 0.25)
    rows = amg.row_index(A)
    assert np.array_equal(m, A.indices != rows)
    B = _laplace2d(6, eps=0.1)
    mb = amg.strength(B, 0.25)
    xnb = np.abs(B.indices - rows) == 1
    assert np.array_equal(mb, xnb)


def test_pmis_invariants_and_determinism():
    """Every point is C or F; an F point that strongly influences someone has a
    C point among its strong dependencies; a C point i with a strong C
    dependency j was chosen in an earlier round, so (w_i, i) > (w_j, j); for a
    symmetric strength graph the C points are independent.  Re-running gives
    identical bits."""
    c, rp, ci, v = _small(12, 10, 3, seed=2)
    S = blocks.schur_simple(*(blocks.block(rp, ci, v, a, b) for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)]))
    mask = amg.strength(S, 0.25)
    cf, rounds = amg.pmis(S, mask, 17)
    cf2, _ = amg.pmis(S, mask, 17)
    assert np.array_equal(cf, cf2)
    assert set(np.unique(cf)) <= {amg.C_PT, amg.F_PT}
    Sm = amg.strength_matrix(S, mask)
    nst = np.diff(Sm.T.tocsr().indptr)
    w = nst + amg.pmis_random(S.shape[0], 17)
    srows = amg.row_index(Sm)
    isc = cf == amg.C_PT
    cc = isc[srows] & isc[Sm.indices]
    i, j = srows[cc], Sm.indices[cc]
    assert np.all((w[i] > w[j]) | ((w[i] == w[j]) & (i > j)))
    has_c = np.zeros(S.shape[0], bool)
    has_c[srows[isc[Sm.indices]]] = True
    assert np.all(has_c[(cf == amg.F_PT) & (nst > 0)])
    # symmetric strength graph (constant-coefficient Laplacian): independent set
    App = _laplace2d(11)
    App.sort_indices()
    m2 = amg.strength(App, 0.25)
    cf3, _ = amg.pmis(App, m2, 5)
    S2 = amg.strength_matrix(App, m2)
    r2 = amg.row_index(S2)
    isc3 = cf3 == amg.C_PT
    assert not np.any(isc3[r2] & isc3[S2.indices])


def _cljp_sequential(A, mask, seed):
    """CLJP as its definition reads, one C point at a time: D from the
    round's start, then each c of D (here in descending order) with its
    edges removed and weights lowered at once."""
    n = A.shape[0]
    S = amg.strength_matrix(A, mask).tocsr()
    S.sort_indices()
    ST = S.T.tocsr()
    edges = {(int(i), int(j)) for i, j in zip(amg.row_index(S), S.indices)}
    w = np.diff(ST.indptr) + amg.pmis_random(n, seed)
    state = np.full(n, amg.UNDECIDED, np.int8)
    state[w < 1] = amg.F_PT
    while (state == amg.UNDECIDED).any():
        und = state == amg.UNDECIDED
        D = []
        for i in np.flatnonzero(und):
            nb = [j for (a, j) in edges if a == i] + [a for (a, j) in edges if j == i]
            if all(not und[j] or (w[i], i) > (w[j], j) for j in nb if j != i):
                D.append(int(i))
        for c in sorted(D, reverse=True):
            for (a, j) in list(edges):
                if a == c:
                    w[j] -= 1
                    edges.discard((a, j))
            deps = [a for (a, j) in edges if j == c]
            for j in deps:
                for k in deps:
                    if k != j and (k, j) in edges:
                        w[j] -= 1
                        edges.discard((k, j))
            for j in deps:
                edges.discard((j, c))
        state[D] = amg.C_PT
        state[(state == amg.UNDECIDED) & (w < 1)] = amg.F_PT
    return state


@pytest.mark.parametrize("which", ["App", "Ass", "S"])
def test_cljp_equals_sequential_and_keeps_ff_pairs_covered(which):
    """CLJP on the blocks and S~ of a 3D case: the round-parallel form equals
    the algorithm run one C point at a time in another order (each removed
    edge lowers its target's weight once), every point is decided, and every
    strong F-F connection i -> j shares a C point (S_j n C_i nonempty): the
    property CLJP's second heuristic provides and classical interpolation
    relies on; PMIS gives no such guarantee and gives fewer C points."""
    c = inputs.random_state(inputs.config_c3(9, 8, 5), 5, s_lo=0.15, s_hi=0.85)
    rp, ci, v = tpfa.jacobian(c, c.u, c.u_old)
    blk = [blocks.block(rp, ci, v, a, b) for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)]]
    A = {"App": blk[0], "Ass": blk[3], "S": blocks.schur_simple(*blk)}[which].tocsr()
    A.sort_indices()
    m = amg.strength(A, 0.25)
    cf, rounds = amg.cljp(A, m, 0x5eed)
    assert rounds >= 2 and set(np.unique(cf)) == {amg.C_PT, amg.F_PT}
    np.testing.assert_array_equal(cf, _cljp_sequential(A, m, 0x5eed))
    S = amg.strength_matrix(A, m).tocsr()
    for i in np.flatnonzero(cf == amg.F_PT):
        Si = S.indices[S.indptr[i]:S.indptr[i + 1]]
        Ci = {j for j in Si if cf[j] == amg.C_PT}
        for j in Si:
            if cf[j] == amg.F_PT:
                assert set(S.indices[S.indptr[j]:S.indptr[j + 1]]) & Ci, (i, j)
    assert (cf == amg.C_PT).sum() > (amg.pmis(A, m, 0x5eed)[0] == amg.C_PT).sum()


def test_splitmix64_published_value():
    """SplitMix64 from state 0: first output 0xE220A8397B1DCDAF (the
    published reference sequence of the generator)."""
    assert amg.splitmix64(0) == 0xE220A8397B1DCDAF
    assert int(amg.splitmix64_vec(np.array([0], np.uint64))[0]) == 0xE220A8397B1DCDAF


def test_direct_interpolation_closed_forms():
    """1D Laplacian, alternating C/F: linear interpolation (1/2, 1/2).
    Zero-row-sum rows: P reproduces constants."""
    n = 9
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    mask = amg.strength(A, 0.25)
    cf = np.where(np.arange(n) % 2 == 0, amg.C_PT, amg.F_PT).astype(np.int8)
    P, _ = amg.direct_interpolation(A, mask, cf)
    Pd = P.toarray()
    for i in range(1, n, 2):
        np.testing.assert_allclose(Pd[i, [i // 2, i // 2 + 1]], [0.5, 0.5], rtol=1e-15)
    # 2D Neumann Laplacian (zero row sums everywhere)
    L = _laplace2d(8).tolil()
    L = sp.csr_matrix(L)
    L = L - sp.diags(np.asarray(L.sum(axis=1)).ravel())
    L = L.tocsr(); L.sort_indices()
    m = amg.strength(L, 0.25)
    cf, _ = amg.pmis(L, m, 3)
    P, _ = amg.direct_interpolation(L, m, cf)
    rs = np.asarray(P.sum(axis=1)).ravel()
    nonempty = np.diff(P.indptr) > 0
    np.testing.assert_allclose(rs[nonempty], 1.0, rtol=1e-14)


def test_extended_i_closed_forms():
    """1D Laplacian: C F C gives (1/2, 1/2) (no distance-two points, same as
    direct); C F F C gives linear interpolation (2/3, 1/3) for the F point
    next to the left C point.  Zero-row-sum rows reproduce constants."""
    n = 10
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    mask = amg.strength(A, 0.25)
    # pattern C F C F F C F F C C
    cf = np.array([1, 2, 1, 2, 2, 1, 2, 2, 1, 1], np.int8)
    P, cidx = amg.extended_i_interpolation(A, mask, cf)
    Pd = P.toarray()
    np.testing.assert_allclose(Pd[1, [0, 1]], [0.5, 0.5], rtol=1e-15)
    np.testing.assert_allclose(Pd[3, [1, 2]], [2 / 3, 1 / 3], rtol=1e-14)
    np.testing.assert_allclose(Pd[4, [1, 2]], [1 / 3, 2 / 3], rtol=1e-14)
    np.testing.assert_allclose(Pd[6, [2, 3]], [2 / 3, 1 / 3], rtol=1e-14)
    assert np.count_nonzero(Pd[3]) == 2
    Pdir, _ = amg.direct_interpolation(A, mask, np.array([1, 2, 1, 2, 1, 2, 1, 2, 1, 2], np.int8))
    Pext, _ = amg.extended_i_interpolation(A, mask, np.array([1, 2, 1, 2, 1, 2, 1, 2, 1, 2], np.int8))
    np.testing.assert_allclose(Pext.toarray(), Pdir.toarray(), rtol=1e-15)
    L = _laplace2d(9).tolil()
    L = sp.csr_matrix(L)
    L = (L - sp.diags(np.asarray(L.sum(axis=1)).ravel())).tocsr()
    L.sort_indices()
    m = amg.strength(L, 0.25)
    cf2, _ = amg.pmis(L, m, 3)
    P2, _ = amg.extended_i_interpolation(L, m, cf2)
    rs = np.asarray(P2.sum(axis=1)).ravel()
    nonempty = np.diff(P2.indptr) > 0
    np.testing.assert_allclose(rs[nonempty], 1.0, rtol=1e-13)


def _non_m_matrix():
    """Six points, not an M-matrix (positive off-diagonals, a negative
    diagonal).  Row 0 (diagonal 10, F): strong C point 1 (-4), strong F point
    2 (-4), weak C point 3 (-0.5 < 0.25 * 4), weak F point 4 (+1, positive),
    strong F point 5 (-2).  Row 2 (diagonal -5, F): entries +2 (point 0,
    strong F), -1 (point 1, same sign as its diagonal, so weak), +1.5
    (point 3, strong C).  Row 5 (diagonal 3): +1 to point 0 (same sign as
    its diagonal), -1 to point 4.  Points 1, 3, 4 have only a diagonal."""
    D = np.zeros((6, 6))
    D[0, [0, 1, 2, 3, 4, 5]] = [10.0, -4.0, -4.0, -0.5, 1.0, -2.0]
    D[1, 1] = 1.0
    D[2, [0, 1, 2, 3]] = [2.0, -1.0, -5.0, 1.5]
    D[3, 3] = 1.0
    D[4, 4] = 1.0
    D[5, [0, 4, 5]] = [1.0, -1.0, 3.0]
    A = sp.csr_matrix(D)
    A.sort_indices()
    cf = np.array([2, 1, 2, 1, 2, 2], np.int8)
    return A, cf


def test_extended_i_non_m_matrix_hand_weights():
    """Extended+i (De Sterck, Falgout, Nolting, Yang 2008) on a matrix that is
    not an M-matrix, weights worked out by hand.

    Row 0: C^_0 = {1} (strong C) u {3} (strong C of its strong F neighbour 2;
    point 5's only strong neighbour is the F point 4).  The filtered entries
    a-bar_2l keep the signs opposite to a_22 = -5, i.e. the positive ones:
    a-bar_20 = 2, a-bar_21 = 0, a-bar_23 = 1.5, so d_02 = 3.5.  Point 5 has
    no opposite-signed entry in C^_0 u {0} (a_50 = +1 shares a_55's sign),
    d_05 = 0, so a_05 = -2 is lumped into the diagonal, as is the weak F
    entry a_04 = +1, while the weak entry a_03 = -0.5 (3 in C^_0) stays in
    the numerator:
      a~_00 = 10 + 1 + (-4)(2)/3.5 + (-2) = 47/7
      w_01  = -(-4) / (47/7) = 28/47
      w_03  = -(-0.5 + (-4)(1.5)/3.5) / (47/7) = 31/94.
    Row 2 (negative diagonal): C^_2 = {3} u {1} (strong C of point 0); row 0's
    filtered entries keep the negative ones (a_00 > 0): d_20 = -4 - 0.5 - 4
    = -8.5 over {1, 3, 2}:
      a~_22 = -5 + 2(-4)/(-8.5) = -69/17
      w_21  = -(-1 + 2(-4)/(-8.5)) / (-69/17) = -1/69
      w_23  = -(1.5 + 2(-0.5)/(-8.5)) / (-69/17) = 55/138.
    Each of these moves if a-bar takes a_ii's sign instead of a_kk's, if a
    weak entry in C^_i is lumped, or if a d_ik = 0 neighbour is dropped."""
    A, cf = _non_m_matrix()
    mask = amg.strength(A, 0.25)
    rows = amg.row_index(A)
    strong = {(int(r), int(c)) for r, c, k in zip(rows, A.indices, mask) if k}
    assert strong == {(0, 1), (0, 2), (0, 5), (2, 0), (2, 3), (5, 4)}
    P, cidx = amg.extended_i_interpolation(A, mask, cf)
    Pd = P.toarray()
    assert list(cidx[[1, 3]]) == [0, 1]
    np.testing.assert_allclose(Pd[0], [28 / 47, 31 / 94], rtol=1e-15)
    np.testing.assert_allclose(Pd[2], [-1 / 69, 55 / 138], rtol=1e-14)
    np.testing.assert_array_equal(Pd[[1, 3]], np.eye(2))
    # rows 4 and 5 have no interpolatory set: empty rows
    assert np.diff(P.indptr)[4] == 0 and np.diff(P.indptr)[5] == 0


def test_classical_interpolation_non_m_matrix_hand_weights():
    """Classical (modified Ruge-Stueben) interpolation on the same matrix,
    weights worked out by hand.

    Row 0: C_0 = {1} (point 3 is a weak C neighbour).  Strong F neighbour 2:
    row 2 keeps its positive entries (a_22 = -5), and its only entry in C_0,
    a_21 = -1, is negative, so d_02 = 0 and a_02 = -4 is lumped; strong F
    neighbour 5 has no entry in C_0, so a_05 = -2 is lumped too.  The weak
    entries a_03 = -0.5 and a_04 = +1 are lumped:
      a~_00 = 10 - 0.5 + 1 - 4 - 2 = 4.5,  w_01 = -(-4) / 4.5 = 8/9.
    Row 2: C_2 = {3}.  Strong F neighbour 0 keeps its negative entries
    (a_00 > 0); in C_2 that is a_03 = -0.5 = d_20, so a_20 = 2 moves to point 3
    in full; the weak entry a_21 = -1 is lumped:
      a~_22 = -5 - 1 = -6,  w_23 = -(1.5 + 2 (-0.5) / (-0.5)) / (-6) = 7/12.
    Using a_ii's sign for the filter, or leaving the weak or d = 0 entries
    out of a~_ii, moves both weights."""
    A, cf = _non_m_matrix()
    mask = amg.strength(A, 0.25)
    P, cidx = amg.classical_interpolation(A, mask, cf)
    Pd = P.toarray()
    np.testing.assert_allclose(Pd[0], [8 / 9, 0.0], rtol=1e-15)
    np.testing.assert_allclose(Pd[2], [0.0, 7 / 12], rtol=1e-15)
    np.testing.assert_array_equal(Pd[[1, 3]], np.eye(2))
    assert np.diff(P.indptr)[4] == 0 and np.diff(P.indptr)[5] == 0


def test_classical_interpolation_closed_forms():
    """1D Laplacian: C F C gives (1/2, 1/2); in C F F C the F points have no
    common C point (d = 0), so each takes its one C neighbour with weight 1.
    On a zero-row-sum M-matrix every F row with a nonempty interpolatory set
    sums to exactly 1 whether or not a strong F neighbour is lumped:
    -(sum_C a_ij + sum_k a_ik) = a_ii + weak + lumped = a~_ii."""
    n = 10
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    mask = amg.strength(A, 0.25)
    cf = np.array([1, 2, 1, 2, 2, 1, 2, 2, 1, 1], np.int8)
    Pd = amg.classical_interpolation(A, mask, cf)[0].toarray()
    np.testing.assert_allclose(Pd[1, [0, 1]], [0.5, 0.5], rtol=1e-15)
    np.testing.assert_allclose(Pd[3], [0, 1, 0, 0, 0], rtol=0, atol=0)
    np.testing.assert_allclose(Pd[4], [0, 0, 1, 0, 0], rtol=0, atol=0)
    L = _laplace2d(9).tolil()
    L = sp.csr_matrix(L)
    L = (L - sp.diags(np.asarray(L.sum(axis=1)).ravel())).tocsr()
    L.sort_indices()
    m = amg.strength(L, 0.25)
    cf2, _ = amg.pmis(L, m, 3)
    P2, _ = amg.classical_interpolation(L, m, cf2)
    rs = np.asarray(P2.sum(axis=1)).ravel()
    nonempty = np.diff(P2.indptr) > 0
    assert nonempty.sum() == L.shape[0]
    np.testing.assert_allclose(rs, 1.0, rtol=1e-13)
    # the same rows and columns as direct interpolation (C n S_i)
    Pdir, _ = amg.direct_interpolation(L, m, cf2)
    np.testing.assert_array_equal(P2.indptr, Pdir.indptr)
    np.testing.assert_array_equal(P2.indices, Pdir.indices)


def _row(P, i):
    P = P.tocsr()
    sl = slice(P.indptr[i], P.indptr[i + 1])
    return list(P.indices[sl]), list(P.data[sl])


def test_truncation_hand_weights():
    """Interpolation truncation by hand.  Row 0 holds w = (0.5, -0.1, 0.3,
    0.3, 0.05, -0.2) in columns 0..5: its positive sum is 1.15, its negative
    sum -0.3.
    * pmax 3 keeps columns 0, 2, 3; the positives scale by 1.15/1.1 and the
      negative sum is lost (no negative kept);
    * pmax 2 keeps 0 and 2 (the tie of 0.3 goes to the lower column), scale
      1.15/0.8;
    * pmax 4 also keeps column 5, whose sign's sum -0.3 it then carries;
    * factor 0.5 alone drops everything below 0.25 (the same as pmax 3);
    * a large negative entry ranks by magnitude (row 1: (-0.9, 0.2, 0.1),
      pmax 1 keeps -0.9 unchanged);
    * magnitudes equal in FP32 tie (row 2: 0.3 and 0.3(1 + 2^-40), pmax 1
      keeps column 0 although column 1 is larger in FP64);
    * pmax 0 and factor 0 leave P as it is."""
    w0 = [0.5, -0.1, 0.3, 0.3, 0.05, -0.2]
    w2 = [0.3, 0.3 * (1 + 2.0 ** -40)]
    rows = [0] * 6 + [1] * 3 + [2] * 2
    cols = list(range(6)) + [0, 1, 2] + [0, 1]
    vals = w0 + [-0.9, 0.2, 0.1] + w2
    P = sp.csr_matrix((vals, (rows, cols)), shape=(3, 6))
    k = 1.15 / 1.1
    c, v = _row(amg.truncate_interpolation(P, 3), 0)
    assert c == [0, 2, 3]
    np.testing.assert_allclose(v, [0.5 * k, 0.3 * k, 0.3 * k], rtol=1e-15)
    c, v = _row(amg.truncate_interpolation(P, 2), 0)
    assert c == [0, 2]
    np.testing.assert_allclose(v, [0.5 * 1.15 / 0.8, 0.3 * 1.15 / 0.8], rtol=1e-15)
    c, v = _row(amg.truncate_interpolation(P, 4), 0)
    assert c == [0, 2, 3, 5]
    np.testing.assert_allclose(v, [0.5 * k, 0.3 * k, 0.3 * k, -0.3], rtol=1e-15)
    assert abs(sum(v) - sum(w0)) <= 1e-15
    c, v = _row(amg.truncate_interpolation(P, 0, 0.5), 0)
    assert c == [0, 2, 3]
    np.testing.assert_allclose(v, [0.5 * k, 0.3 * k, 0.3 * k], rtol=1e-15)
    assert _row(amg.truncate_interpolation(P, 1), 1) == ([0], [-0.9])
    c, v = _row(amg.truncate_interpolation(P, 1), 2)
    assert c == [0]
    np.testing.assert_allclose(v, [sum(w2)], rtol=1e-15)
    Q = amg.truncate_interpolation(P, 0, 0.0)
    assert (Q != P).nnz == 0


def test_truncation_keeps_row_sums_and_default_hierarchy():
    """On the S~ of the 3D workload family: with the default (pmax 3) every
    P row holds at most three entries, every row whose signs each keep an
    entry keeps its sum, rows of at most three entries are untouched, and
    the hierarchy's operator complexity falls below the untruncated one's."""
    c = inputs.config_c3(16, 16, 8)
    rp, ci, v, _ = newton.linear_system(c)
    M = precond.Preconditioner("bf", rp, ci, v, (16, 16, 8))
    S = M.S.tocsr()
    mask = amg.strength(S, 0.25)
    cf, _ = amg.pmis(S, mask, 0x5eed)
    P, _ = amg.extended_i_interpolation(S, mask, cf)
    Q, _ = amg.interpolation(S, mask, cf, "ext+i", amg.TRUNC_PMAX, amg.TRUNC_FACTOR)
    assert amg.TRUNC_PMAX == 3 and amg.TRUNC_FACTOR == 0.0
    lp, lq = np.diff(P.indptr), np.diff(Q.indptr)
    assert lq.max() <= 3 and (lp > 3).any()
    short = np.flatnonzero(lp <= 3)
    for i in short[:2000]:
        assert _row(P, i) == _row(Q, i)
    checked = 0
    for i in np.flatnonzero(lp > 3):
        _, pv = _row(P, i)
        _, qv = _row(Q, i)
        pv, qv = np.array(pv), np.array(qv)
        if ((qv > 0).any() or not (pv > 0).any()) and ((qv < 0).any() or not (pv < 0).any()):
            assert abs(qv.sum() - pv.sum()) <= 1e-14 * np.abs(pv).sum()
            checked += 1
    assert checked > 0
    Hd = amg.Hierarchy(S, interp="ext+i")
    Hn = amg.Hierarchy(S, interp="ext+i", trunc_pmax=0)
    assert all(np.diff(L.P.indptr).max() <= 3 for L in Hd.levels[:-1])
    assert Hd.stats()["operator_complexity"] < Hn.stats()["operator_complexity"]


def test_gs_coloring_and_sweeps_are_triangular_solves():
    """Multicolour Gauss-Seidel on a nonsymmetric TPFA block: no two
    neighbours of A + A^T share a colour, and a forward sweep equals the
    Gauss-Seidel step of A with its rows and columns ordered by colour,
    x' = (D + L)^{-1}(b - U x) (L, U strictly lower/upper in that order), a
    backward sweep (D + U)^{-1}(b - L x); the order inside a colour does not
    matter."""
    c, rp, ci, v = _small(7, 6, 2, seed=8)
    A = blocks.block(rp, ci, v, 0, 1) + blocks.block(rp, ci, v, 0, 0)
    A = A.tocsr()
    A.sort_indices()
    n = A.shape[0]
    color, nc = amg.gs_colors(A, 0x5eed)
    assert nc >= 2 and (color >= 0).all() and color.max() == nc - 1
    Ad = A.toarray()
    nbr = (Ad != 0) | (Ad.T != 0)
    np.fill_diagonal(nbr, False)
    ii, jj = np.nonzero(nbr)
    assert (color[ii] != color[jj]).all()
    perm = np.lexsort((np.arange(n), color))
    Ap = Ad[np.ix_(perm, perm)]
    Lo, Up, D = np.tril(Ap, -1), np.triu(Ap, 1), np.diag(np.diag(Ap))
    rng = np.random.default_rng(2)
    b, x = rng.standard_normal(n), rng.standard_normal(n)
    rows = [(np.flatnonzero(color == k), A[np.flatnonzero(color == k)]) for k in range(nc)]
    fwd = amg.gs_sweep(A, A.diagonal(), rows, b, x, reverse=False)
    bwd = amg.gs_sweep(A, A.diagonal(), rows, b, x, reverse=True)
    ref_f = np.linalg.solve(D + Lo, b[perm] - Up @ x[perm])
    ref_b = np.linalg.solve(D + Up, b[perm] - Lo @ x[perm])
    np.testing.assert_allclose(fwd[perm], ref_f, rtol=1e-12, atol=1e-12 * np.abs(ref_f).max())
    np.testing.assert_allclose(bwd[perm], ref_b, rtol=1e-12, atol=1e-12 * np.abs(ref_b).max())
    # within a colour the order is irrelevant: reversing it changes nothing
    rows_rev = [(idx[::-1].copy(), A[idx[::-1]]) for idx, _ in rows]
    np.testing.assert_allclose(amg.gs_sweep(A, A.diagonal(), rows_rev, b, x, False), fwd,
                               rtol=1e-14, atol=1e-14 * np.abs(fwd).max())


def test_extended_i_restores_scalable_schur_cycle():
    """On the heterogeneous S~ of the 3D workload family the direct
    interpolation cycle degrades with the grid while extended+i stays flat
    (the reason it is used for the pressure-like operators)."""
    its = {}
    for (nx, ny, nz) in [(16, 16, 8), (32, 32, 16)]:
        c = inputs.config_c3(nx, ny, nz)
        rp, ci, v, _ = newton.linear_system(c)
        M = precond.Preconditioner("bf", rp, ci, v, (nx, ny, nz))
        b = inputs.random_vector(M.S.shape[0], 1)
        for interp in ["direct", "ext+i"]:
            H = amg.Hierarchy(M.S, interp=interp)
            _, info = fgmres.fgmres(lambda z: M.S @ z, H.vcycle, b, rtol=1e-8, maxit=300)
            its[(nx, interp)] = info["iterations"]
    assert its[(32, "ext+i")] <= 16 and its[(32, "ext+i")] < its[(32, "direct")]


def test_galerkin_matches_dense_and_symmetry():
    c, rp, ci, v = _small(10, 9, 2, seed=3)
    App = blocks.block(rp, ci, v, 0, 0)
    H = amg.Hierarchy(App, coarse_max=20)
    L0 = H.levels[0]
    Ac = H.levels[1].A.toarray()
    dense = L0.P.T.toarray() @ L0.A.toarray() @ L0.P.toarray()
    np.testing.assert_allclose(Ac, dense, rtol=0, atol=1e-13 * np.abs(dense).max())
    assert np.allclose(Ac, Ac.T, rtol=0, atol=1e-13 * np.abs(Ac).max())


def test_two_level_cycle_matches_dense_formula():
    """Two levels with exact coarse solve: x = x_pre + D^{-1}(b - A x_pre')...
    compared with the dense two-grid formula, and iterating it converges to
    the dense direct solution."""
    c, rp, ci, v = _small(9, 8, 1, seed=4)
    App = blocks.block(rp, ci, v, 0, 0)
    H = amg.Hierarchy(App, coarse_max=40, max_levels=2)
    assert len(H.levels) == 2 and H.coarse_dense
    A = App.toarray()
    L0 = H.levels[0]
    P = L0.P.toarray()
    R = P.T
    Dinv = np.diag(L0.dinv)
    Ac = R @ A @ P
    b = inputs.random_vector(A.shape[0], 3)
    xpre = Dinv @ b
    x = xpre + P @ np.linalg.solve(Ac, R @ (b - A @ xpre))
    x = x + Dinv @ (b - A @ x)
    np.testing.assert_allclose(H.vcycle(b), x, rtol=0, atol=1e-13 * np.abs(x).max())
    # coarse-grid correction is a projector
    Q = P @ np.linalg.solve(Ac, R @ A)
    np.testing.assert_allclose(Q @ Q, Q, atol=1e-12)
    # stationary iteration with the two-grid cycle converges to the direct solve
    xe = np.linalg.solve(A, b)
    xk = np.zeros_like(b)
    for _ in range(200):
        xk = xk + H.vcycle(b - A @ xk)
    np.testing.assert_allclose(xk, xe, rtol=0, atol=1e-12 * np.abs(xe).max())


def test_vcycle_symmetric_for_symmetric_matrix():
    c, rp, ci, v = _small(10, 8, 2, seed=6)
    App = blocks.block(rp, ci, v, 0, 0)
    H = amg.Hierarchy(App, coarse_max=15)
    assert len(H.levels) >= 3
    n = App.shape[0]
    M = np.column_stack([H.vcycle(e) for e in np.eye(n)])
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())


def test_chebyshev_polynomial_on_diagonal_operator():
    """Chebyshev smoothing of degree k on D^{-1} A over [lo, hi] (Saad,
    Alg. 12.1) from x = 0: with A = diag(t) and D = I the error of each
    component is multiplied by the scaled Chebyshev polynomial
    T_k((c - t)/h) / T_k(c/h), c = (hi+lo)/2, h = (hi-lo)/2, with
    T_2(u) = 2u^2 - 1 and T_3(u) = 4u^3 - 3u."""
    t = np.linspace(0.0, 1.2, 25)
    A = sp.diags(t).tocsr()
    xt = inputs.random_vector(len(t), 50)
    b = A @ xt
    lo, hi = 0.3, 1.1
    c, h = 0.5 * (hi + lo), 0.5 * (hi - lo)
    T = {2: lambda u: 2 * u * u - 1, 3: lambda u: 4 * u ** 3 - 3 * u}
    for k in (2, 3):
        x = amg.chebyshev_smooth(A, np.ones(len(t)), b, np.zeros(len(t)), lo, hi, k)
        p = T[k]((c - t) / h) / T[k](c / h)
        np.testing.assert_allclose(xt - x, p * xt, rtol=0, atol=1e-14 * np.abs(xt).max())
    # degree one is a damped Jacobi step with weight 1/c
    x1 = amg.chebyshev_smooth(A, np.ones(len(t)), b, np.zeros(len(t)), lo, hi, 1)
    np.testing.assert_allclose(x1, b / c, rtol=1e-15)
    # power estimate on diag(t): K steps from v0 give ||t^K v0|| / ||t^(K-1) v0||
    v0 = amg.pmis_random(len(t), 9) - 0.5
    lam = amg.power_max_eig(A, np.ones(len(t)), 6, 9)
    np.testing.assert_allclose(lam, np.linalg.norm(t ** 6 * v0) / np.linalg.norm(t ** 5 * v0),
                               rtol=1e-14)
    assert lam <= t.max()


@pytest.mark.parametrize("smoother,nu", [("l1jacobi", 2), ("chebyshev", 1), ("chebyshev", 2),
                                         ("gs", 1), ("gs", 2)])
def test_vcycle_variants_symmetric_and_convergent(smoother, nu):
    """V(nu, nu) with l1-Jacobi, Chebyshev or multicolour Gauss-Seidel
    (forward sweeps before, backward after): for a symmetric matrix the cycle
    operator B is symmetric (the post-smoother is the pre-smoother's adjoint),
    and the stationary iteration x <- x + B(b - A x) converges: the spectral
    radius of I - B A is below 1 and no larger than with V(1,1) l1-Jacobi."""
    c, rp, ci, v = _small(10, 8, 2, seed=6)
    App = blocks.block(rp, ci, v, 0, 0)
    A = App.toarray()
    n = App.shape[0]

    def cycle_matrix(**kw):
        H = amg.Hierarchy(App, coarse_max=15, **kw)
        assert len(H.levels) >= 3
        return np.column_stack([H.vcycle(e) for e in np.eye(n)])

    M = cycle_matrix(smoother=smoother, nu1=nu, nu2=nu)
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())
    rho = np.abs(np.linalg.eigvals(np.eye(n) - M @ A)).max()
    rho1 = np.abs(np.linalg.eigvals(np.eye(n) - cycle_matrix() @ A)).max()
    assert rho < 1.0 and rho <= rho1 + 1e-12, (rho, rho1)


def test_single_level_is_exact():
    """n <= coarse_max: one level, dense LU -> AMG-GMRES converges in 1 step."""
    c, rp, ci, v = _small(5, 4, 2, seed=7)
    Js = blocks.scalarize(rp, ci, v)
    H = amg.Hierarchy(Js, coarse_max=256)
    assert len(H.levels) == 1
    b = inputs.random_vector(Js.shape[0], 1)
    x, info = fgmres.fgmres(lambda z: Js @ z, H.vcycle, b, rtol=1e-10)
    assert info["status"] == fgmres.CONVERGED and info["iterations"] == 1


# ----------------------------------------------------------------- ILU(0)


def test_bilu0_generic_reproduces_pattern_and_matches_pivot_form():
    c, rp, ci, v = _small(5, 4, 3, seed=8)
    lu = ilu.bilu0_generic(rp, ci, v)
    N = c.N
    L = np.eye(2 * N)
    U = np.zeros((2 * N, 2 * N))
    for i in range(N):
        for e in range(rp[i], rp[i + 1]):
            j = ci[e]
            blk = lu[e]
            if j < i:
                L[2 * i:2 * i + 2, 2 * j:2 * j + 2] = blk
            else:
                U[2 * i:2 * i + 2, 2 * j:2 * j + 2] = blk
    LU = L @ U
    D = tpfa.bcsr_to_dense(rp, ci, v)
    pat = np.kron((np.abs(D).reshape(N, 2, N, 2).sum(axis=(1, 3)) > 0) | np.eye(N, dtype=bool),
                  np.ones((2, 2), bool))
    blockpat = np.zeros((N, N), bool)
    for i in range(N):
        blockpat[i, ci[rp[i]:rp[i + 1]]] = True
    pat = np.kron(blockpat, np.ones((2, 2), bool))
    np.testing.assert_allclose(LU[pat], D[pat], rtol=0, atol=1e-12 * np.abs(D).max())
    # pivot (DILU) form gives the same preconditioner
    B = ilu.Bilu0(rp, ci, v, c.nx, c.ny, c.nz)
    r = inputs.random_vector(2 * N, 2)
    z1 = ilu.generic_apply(rp, ci, lu, r)
    z2 = B.apply(r)
    np.testing.assert_allclose(z2, z1, rtol=0, atol=1e-12 * np.abs(z1).max())
    # scalar ILU(0) on the point-ordered matrix is the same factorisation
    Ls, Us = ilu.ilu0_scalar(blocks.scalarize(rp, ci, v))
    zs = np.linalg.solve(Us, np.linalg.solve(Ls, r))
    np.testing.assert_allclose(zs, z1, rtol=0, atol=1e-11 * np.abs(z1).max())


def test_bilu0_exact_on_1d_grid():
    c, rp, ci, v = _small(12, 1, 1, seed=9)
    B = ilu.Bilu0(rp, ci, v, c.nx, c.ny, c.nz)
    r = inputs.random_vector(2 * c.N, 4)
    D = tpfa.bcsr_to_dense(rp, ci, v)
    np.testing.assert_allclose(B.apply(r), np.linalg.solve(D, r), rtol=0, atol=1e-11)


# ----------------------------------------------------------- preconditioners


def _dense_blocks(rp, ci, v, N):
    Pm = _perm_point_to_field(N)
    F = Pm @ tpfa.bcsr_to_dense(rp, ci, v) @ Pm.T
    return Pm, F[:N, :N], F[:N, N:], F[N:, :N], F[N:, N:]


@pytest.mark.parametrize("kind", ["cpr1", "cpr2", "bf"])
def test_precond_matches_matrix_form(kind):
    """With exact inner solves, Algorithms 1-3 equal Eqs. m_comb, m_add, m_bf."""
    c, rp, ci, v = _small(5, 4, 2, seed=10)
    N = c.N
    M = precond.Preconditioner(kind, rp, ci, v, (c.nx, c.ny, c.nz), inner="exact")
    r = inputs.random_vector(2 * N, 5)
    z = M.apply(r)
    Pm, App, Aps, Asp, Ass = _dense_blocks(rp, ci, v, N)
    J = tpfa.bcsr_to_dense(rp, ci, v)
    I2 = np.eye(2 * N)
    Rp = np.zeros((N, 2 * N)); Rp[np.arange(N), 2 * np.arange(N)] = 1
    Rs = np.zeros((N, 2 * N)); Rs[np.arange(N), 2 * np.arange(N) + 1] = 1
    if kind in ("cpr1", "cpr2"):
        B = ilu.Bilu0(rp, ci, v, c.nx, c.ny, c.nz)
        P1inv = np.column_stack([B.apply(e) for e in I2])
        P1 = np.linalg.inv(P1inv)
        corr = Rp.T @ np.linalg.inv(App) @ Rp
        if kind == "cpr2":
            corr = corr + Rs.T @ np.linalg.inv(Ass) @ Rs
        Minv = (I2 - corr @ (J - P1)) @ P1inv
    else:
        St = App - Aps @ np.diag(1 / np.diag(Ass)) @ Asp
        Sti = np.linalg.inv(St)
        Assi = np.linalg.inv(Ass)
        Mf = np.block([[Sti, -Sti @ Aps @ Assi], [np.zeros((N, N)), Assi]])
        Minv = Pm.T @ Mf @ Pm
    ze = Minv @ r
    # the dense side goes through explicit inverses (cond ~ 1e4 here)
    np.testing.assert_allclose(z, ze, rtol=0, atol=1e-10 * np.abs(ze).max())


def test_exact_block_factorisations_gmres_steps():
    """Full LDU with exact S -> 1 step; the upper-triangular M with exact S
    and A_ss -> at most 2 steps; A_sp = 0 -> M = J -> 1 step."""
    c, rp, ci, v = _small(5, 4, 1, seed=12)
    N = c.N
    Pm, App, Aps, Asp, Ass = _dense_blocks(rp, ci, v, N)
    J = tpfa.bcsr_to_dense(rp, ci, v)
    b = inputs.random_vector(2 * N, 8)
    S = App - Aps @ np.linalg.solve(Ass, Asp)
    I = np.eye(N)
    Z = np.zeros((N, N))
    Uf = np.block([[I, Aps @ np.linalg.inv(Ass)], [Z, I]])
    Df = np.block([[S, Z], [Z, Ass]])
    Lf = np.block([[I, Z], [np.linalg.solve(Ass, Asp), I]])
    for Mf, steps in [(Uf @ Df @ Lf, 1), (Uf @ Df, 2)]:
        Mp = Pm.T @ Mf @ Pm
        _, info = fgmres.fgmres(lambda z: J @ z, lambda r: np.linalg.solve(Mp, r), b, rtol=1e-10)
        assert info["status"] == fgmres.CONVERGED and info["iterations"] <= steps, (steps, info)
    # A_sp = 0: S_n below the residual saturation everywhere (k_rn = 0)
    c0 = inputs.small_case(5, 4, 1, seed=12)
    u = c0.u.copy(); u[:, 1] = 0.05
    c0 = c0.replace(u=u, u_old=u.copy())
    rp0, ci0, v0 = tpfa.jacobian(c0, c0.u, c0.u_old)
    assert np.all(v0[:, 1, 0] == 0)
    J0 = tpfa.bcsr_to_dense(rp0, ci0, v0)
    M0 = precond.Preconditioner("bf", rp0, ci0, v0, (5, 4, 1), inner="exact")
    _, info = fgmres.fgmres(lambda z: J0 @ z, M0.apply, b, rtol=1e-10)
    assert info["status"] == fgmres.CONVERGED and info["iterations"] == 1


@pytest.mark.parametrize("kind", ["cpr1", "cpr2"])
def test_cpr_exact_on_1d_grid_with_vcycle(kind):
    c, rp, ci, v = _small(40, 1, 1, seed=13)
    M = precond.Preconditioner(kind, rp, ci, v, (40, 1, 1), amg_opts=dict(coarse_max=8))
    J = tpfa.bcsr_to_dense(rp, ci, v)
    b = inputs.random_vector(80, 9)
    _, info = fgmres.fgmres(lambda z: J @ z, M.apply, b, rtol=1e-10)
    assert info["status"] == fgmres.CONVERGED and info["iterations"] == 1


# ----------------------------------------------------------------- FGMRES


def test_fgmres_first_cycle_is_least_squares_minimiser():
    c, rp, ci, v = _small(5, 4, 2, seed=14)
    J = tpfa.bcsr_to_dense(rp, ci, v)
    M = precond.Preconditioner("bf", rp, ci, v, (5, 4, 2))
    Minv = np.column_stack([M.apply(e) for e in np.eye(2 * c.N)])
    b = inputs.random_vector(2 * c.N, 10)
    A = J @ Minv
    for k in range(1, 8):
        x, info = fgmres.fgmres(lambda z: J @ z, lambda r: Minv @ r, b, rtol=1e-30, maxit=k)
        K = np.column_stack([np.linalg.matrix_power(A, i) @ b for i in range(k)])
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
        xe = Minv @ (Q @ y)
        assert info["iterations"] == k
        np.testing.assert_allclose(x, xe, rtol=0, atol=1e-10 * np.abs(xe).max())


def test_fgmres_exact_preconditioner_and_small_n():
    c, rp, ci, v = _small(3, 3, 1, seed=15)
    J = tpfa.bcsr_to_dense(rp, ci, v)
    b = inputs.random_vector(18, 11)
    _, info = fgmres.fgmres(lambda z: J @ z, lambda r: np.linalg.solve(J, r), b)
    assert info["iterations"] == 1 and info["status"] == fgmres.CONVERGED
    _, info = fgmres.fgmres(lambda z: J @ z, lambda r: r, b, rtol=1e-10)
    assert info["status"] == fgmres.CONVERGED and info["iterations"] <= 18
    x, info = fgmres.fgmres(lambda z: J @ z, lambda r: r, np.zeros(18))
    assert info["iterations"] == 0 and np.all(x == 0)


# ----------------------------------------------------------------- full solves


@pytest.mark.parametrize("pd", [0.0, 0.1, 1.0])
def test_bf_converges_across_capillarity(pd):
    """Trend check only (iteration counts are not pinned by the paper)."""
    c = inputs.workload_2d_corner(48, 48, 2.0, 8.0, pd, 50.0, 2)
    _, info, _ = newton.solve(c, "bf")
    assert info["status"] == fgmres.CONVERGED and info["relres"] <= 1e-8


# ----------------------------------------------------------------- Newton


def test_newton_update_chop_and_clamp_closed_form():
    """Newton update of Sec. 3 with the build's reading of the paper's
    unspecified variant: saturation increments limited to [-ds_max, ds_max],
    then S_n clamped to [0, 1]; pressures move by the full increment."""
    u = np.array([[1.0, 0.5], [2.0, 0.1], [-1.0, 0.95], [0.0, 0.3], [3.0, 0.6]])
    d = np.array([[0.3, 0.5], [-0.5, -0.15], [0.25, 0.1], [1.5, -0.35], [-2.0, 0.05]])
    # with the chop at 0.2:
    #   0.5 + min(0.5, 0.2) = 0.7;   0.1 - 0.15 = -0.05 -> 0;  0.95 + 0.1 = 1.05 -> 1;
    #   0.3 - min(0.35, 0.2) = 0.1;  0.6 + 0.05 = 0.65
    un = newton.update(u, d.reshape(-1), ds_max=0.2)
    np.testing.assert_array_equal(un[:, 0], [1.3, 1.5, -0.75, 1.5, 1.0])
    np.testing.assert_allclose(un[:, 1], [0.7, 0.0, 1.0, 0.1, 0.65], rtol=0, atol=1e-16)
    # no chop (ds_max = 0): 0.5 + 0.5 = 1;  0.3 - 0.35 = -0.05 -> 0
    un0 = newton.update(u, d.reshape(-1), ds_max=0.0)
    np.testing.assert_allclose(un0[:, 1], [1.0, 0.0, 1.0, 0.0, 0.65], rtol=0, atol=1e-16)
    np.testing.assert_array_equal(un0[:, 0], un[:, 0])
    # the input state is not modified
    assert u[0, 1] == 0.5 and u[3, 1] == 0.3


# ----------------------------------------------------------------- spectra


def test_simulation_conserves_nonwetting_volume():
    """Backward Euler over several steps of the gravity box (wells through
    boundary faces, gravity, linear P_c): the stored nonwetting volume
    changes by dt times the net inflow at each step's converged state,
    sum_i phi_i V (S_K - S_0)_i = -dt sum_k sum_i R_n,i(u_k, u_k), up to the
    Newton tolerance.  With u_old = u the accumulation term vanishes and the
    interior fluxes cancel, so sum_i R_n,i(u, u) is minus the net inflow.  A
    step that kept the wrong u_old, used another dt or stopped short of the
    tolerance breaks the balance."""
    from oracle import simulate
    c = inputs.gravity_box_xz(10, "advection")
    K = 3
    rec, u = simulate.simulate(c, "bf", K * c.dt, dt=c.dt)
    assert rec["status"] == "converged" and len(rec["steps"]) == K
    states = [c.u] + [st["u"] for st in rec["steps"]]
    np.testing.assert_array_equal(states[-1], u)
    V = c.hx * c.hy * c.hz
    poro = np.asarray(c.poro).reshape(-1)
    stored = float(np.sum(poro * V * (states[-1][:, 1] - states[0][:, 1])))
    inflow = 0.0
    for k in range(1, K + 1):
        ck = c.replace(u=states[k], u_old=states[k])
        inflow -= c.dt * float(np.sum(tpfa.residual(ck, ck.u, ck.u_old)[:, 1]))
        # the step itself met the Newton tolerance
        cs = c.replace(u=states[k], u_old=states[k - 1])
        assert np.linalg.norm(tpfa.residual(cs, cs.u, cs.u_old)) <= 1e-6
    bound = K * c.dt * np.sqrt(2 * c.N) * 1e-6
    assert abs(stored) > 100 * bound  # the balance is not trivially zero
    assert abs(stored - inflow) <= bound, (stored, inflow, bound)


def test_spectrum_bf_is_one_and_schur_ratio():
    """Sec. 4.3 study, exact inner solves.  For BF's block upper-triangular M
    (Eq. m_bf) with S~ in place of the Schur complement S = A_pp - A_ps
    A_ss^{-1} A_sp, J M^{-1} has the eigenvalue 1 N times and the N
    eigenvalues of S S~^{-1}; with S itself every eigenvalue is 1 (a
    defective one, so computed eigenvalues scatter by about sqrt(eps))."""
    from oracle import spectra
    c = inputs.oil_water_xz(2, inputs.PC_LINEAR, nx=10, nz=4)
    rp, ci, v = tpfa.jacobian(c, c.u, c.u_old)
    N = c.N
    ev = np.sort_complex(np.linalg.eigvals(
        spectra.preconditioned_matrix("bf", rp, ci, v, (c.nx, c.ny, c.nz))))
    Pm, App, Aps, Asp, Ass = _dense_blocks(rp, ci, v, N)
    S = App - Aps @ np.linalg.solve(Ass, Asp)
    St = blocks.schur_simple(*(blocks.block(rp, ci, v, a, b)
                               for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)])).toarray()
    expect = np.sort_complex(np.concatenate([np.ones(N), np.linalg.eigvals(S @ np.linalg.inv(St))]))
    assert np.max(np.abs(ev - expect)) <= 1e-6
    # CPR with an exact first stage: J M^{-1} = I
    ev1 = np.linalg.eigvals(spectra.preconditioned_matrix("cpr1", rp, ci, v, (c.nx, c.ny, c.nz),
                                                          p1="exact"))
    assert np.max(np.abs(ev1 - 1.0)) <= 1e-8
    s = spectra.summary(ev)
    assert s["n"] == 2 * N and s["min_abs"] > 0.5
