"""Oracle: residual F(u) and exact Jacobian of the fully implicit TPFA
two-phase discretisation (paper Sec. 2, Eqs. balance1/balance2, the TPFA
flux, upwinding, harmonic averaging, and Eq. fully_discrete_system; Newton
linearisation of Sec. 3 with the 2x2 block structure of Eq. jacobian).

Unknowns per cell: (P_w, S_n), point ordered.  Constant densities: the
volume balance is used (densities only enter the gravity potential).

Readings of the paper used here (all also listed in the design notes):
* flux out of cell l through face (l,h) is +T * lambda_up * (Phi_l - Phi_h),
  added to R_l and subtracted from R_h;
* upwinding is face based: up = l iff Phi_l - Phi_h > 0, else h;
* R_w = -(phi V/dt)(S - S_old) + sum flux_w - q_w,
  R_n = +(phi V/dt)(S - S_old) + sum flux_n - q_n;
* relative permeabilities are Brooks-Corey-Burdine,
  k_rw = Sb^((2+3l)/l), k_rn = (1-Sb)^2 (1 - Sb^((2+l)/l));
* effective saturation Sb = (1 - S_n - S_wr)/(1 - S_wr - S_nr), clamped
  to [0,1], derivative zero strictly outside;
* Brooks-Corey P_c = P_d Sb^(-1/l) continued linearly (C1) below s_eps;
* BHP producer: q_a = -WI lambda_a(S)(P_w - p_bh).
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# geometry


def cell_coords(case):
    N = case.N
    i = np.arange(N)
    ix = i % case.nx
    iy = (i // case.nx) % case.ny
    iz = i // (case.nx * case.ny)
    return ix, iy, iz


def faces(case):
    """Interior faces (l, h, d) with l < h, h = l + stride_d."""
    nx, ny, nz = case.nx, case.ny, case.nz
    ix, iy, iz = cell_coords(case)
    i = np.arange(case.N)
    out_l, out_h, out_d = [], [], []
    for d, (coord, n, stride) in enumerate([(ix, nx, 1), (iy, ny, nx), (iz, nz, nx * ny)]):
        m = coord < n - 1
        out_l.append(i[m])
        out_h.append(i[m] + stride)
        out_d.append(np.full(int(m.sum()), d))
    return np.concatenate(out_l), np.concatenate(out_h), np.concatenate(out_d)


def spacing(case):
    return np.array([case.hx, case.hy, case.hz])


def cell_volume(case):
    return case.hx * case.hy * case.hz


def perm(case, d):
    return [case.kx, case.ky, case.kz][d]


def transmissibility(case, fl, fh, fd):
    """T = gamma_d * K_{l,h} / dx_{lh}: face area gamma_d = V/h_d, the
    harmonic face permeability K = (dx_l+dx_h) K_l K_h / (dx_l K_h + dx_h K_l)
    with equal cells, and the centre distance dx_{lh} = h_d."""
    h = spacing(case)[fd]
    V = cell_volume(case)
    gamma = V / h
    kl = np.choose(fd, [case.kx[fl], case.ky[fl], case.kz[fl]])
    kh = np.choose(fd, [case.kx[fh], case.ky[fh], case.kz[fh]])
    dxl = h
    dxh = h
    kface = (dxl + dxh) * kl * kh / (dxl * kh + dxh * kl)
    return gamma * kface / h


def depth(case):
    _, _, iz = cell_coords(case)
    return (iz + 0.5) * case.hz


# ---------------------------------------------------------------------------
# constitutive relations (complex-safe for complex-step differentiation)


def sat_functions(case, sn):
    """Returns dict of k_rw, k_rn, P_c and their derivatives w.r.t. S_n."""
    a = 1.0 - case.swr - case.snr
    s = (1.0 - sn - case.swr) / a
    sr = np.real(s)
    inside = (sr >= 0.0) & (sr <= 1.0)
    sb = np.where(sr < 0.0, 0.0, np.where(sr > 1.0, 1.0, s))
    dsb = np.where(inside, -1.0 / a, 0.0)
    lam = case.bc_lambda
    ew = (2.0 + 3.0 * lam) / lam
    en = (2.0 + lam) / lam
    krw = sb ** ew
    dkrw_dsb = ew * sb ** (ew - 1.0)
    pn = sb ** en
    krn = (1.0 - sb) ** 2 * (1.0 - pn)
    dkrn_dsb = -2.0 * (1.0 - sb) * (1.0 - pn) - (1.0 - sb) ** 2 * en * sb ** (en - 1.0)
    if case.pc_model == 1:  # linear: P_c = P_0 (1 - Sb)
        pc = case.pd * (1.0 - sb)
        dpc_dsb = np.full_like(sb, -case.pd)
    else:  # Brooks-Corey with C1 linear continuation below s_eps
        eps = case.s_eps
        hi = np.real(sb) >= eps
        sbs = np.where(hi, sb, eps)
        pc_hi = case.pd * sbs ** (-1.0 / lam)
        dpc_hi = -(case.pd / lam) * sbs ** (-1.0 / lam - 1.0)
        pc_eps = case.pd * eps ** (-1.0 / lam)
        dpc_eps = -(case.pd / lam) * eps ** (-1.0 / lam - 1.0)
        pc = np.where(hi, pc_hi, pc_eps + dpc_eps * (sb - eps))
        dpc_dsb = np.where(hi, dpc_hi, dpc_eps)
    return dict(lw=krw / case.mu_w, ln=krn / case.mu_n,
                dlw=dkrw_dsb * dsb / case.mu_w, dln=dkrn_dsb * dsb / case.mu_n,
                pc=pc, dpc=dpc_dsb * dsb)


# ---------------------------------------------------------------------------
# residual


def _dirichlet_geometry(case):
    """For each Dirichlet face: cell, T_b = gamma K_i / (h/2), depth of the face."""
    cells = np.asarray(case.dir_cells, np.int64)
    fcode = np.asarray(case.dir_face, np.int64)
    d = fcode // 2
    h = spacing(case)[d]
    gamma = cell_volume(case) / h
    k = np.choose(d, [case.kx[cells], case.ky[cells], case.kz[cells]]) if len(cells) else np.zeros(0)
    T = gamma * k / (0.5 * h)
    zc = depth(case)[cells]
    dz = np.where(fcode == 4, -0.5 * case.hz, np.where(fcode == 5, 0.5 * case.hz, 0.0))
    return cells, T, zc + dz


def residual(case, u, u_old):
    """F(u) as an (N,2) array, columns (water, nonwetting).  Works for complex u."""
    N = case.N
    P = u[:, 0]
    S = u[:, 1]
    sf = sat_functions(case, S)
    V = cell_volume(case)
    D = depth(case)
    g = case.grav
    R = np.zeros((N, 2), dtype=np.result_type(u, np.float64))
    stor = case.poro * V / case.dt * (S - u_old[:, 1])
    R[:, 0] -= stor
    R[:, 1] += stor
    fl, fh, fd = faces(case)
    T = transmissibility(case, fl, fh, fd)
    phw = P - case.rho_w * g * D
    phn = P + sf["pc"] - case.rho_n * g * D
    dw = phw[fl] - phw[fh]
    dn = phn[fl] - phn[fh]
    upw = np.where(np.real(dw) > 0, fl, fh)
    upn = np.where(np.real(dn) > 0, fl, fh)
    Fw = T * sf["lw"][upw] * dw
    Fn = T * sf["ln"][upn] * dn
    np.add.at(R[:, 0], fl, Fw)
    np.add.at(R[:, 0], fh, -Fw)
    np.add.at(R[:, 1], fl, Fn)
    np.add.at(R[:, 1], fh, -Fn)
    # Dirichlet faces: boundary state (P_b, S_b) at the face centre
    if len(case.dir_cells):
        cells, Tb, zb = _dirichlet_geometry(case)
        sfb = sat_functions(case, np.asarray(case.dir_s, np.float64))
        dwb = phw[cells] - (case.dir_p - case.rho_w * g * zb)
        dnb = phn[cells] - (case.dir_p + sfb["pc"] - case.rho_n * g * zb)
        lwb = np.where(np.real(dwb) > 0, sf["lw"][cells], sfb["lw"])
        lnb = np.where(np.real(dnb) > 0, sf["ln"][cells], sfb["ln"])
        np.add.at(R[:, 0], cells, Tb * lwb * dwb)
        np.add.at(R[:, 1], cells, Tb * lnb * dnb)
    # BHP producers
    pc_ = np.asarray(case.prod_cells, np.int64)
    if len(pc_):
        dp = P[pc_] - case.prod_pbh
        np.add.at(R[:, 0], pc_, case.prod_wi * sf["lw"][pc_] * dp)
        np.add.at(R[:, 1], pc_, case.prod_wi * sf["ln"][pc_] * dp)
    R -= case.q
    return R


# ---------------------------------------------------------------------------
# block CSR pattern and Jacobian


def bcsr_pattern(case):
    """row_ptr (N+1), col_idx (nnzb): block row i holds its existing face
    neighbours and itself, columns ascending (-z,-y,-x,self,+x,+y,+z)."""
    N = case.N
    fl, fh, _ = faces(case)
    rows = np.concatenate([np.arange(N), fl, fh])
    cols = np.concatenate([np.arange(N), fh, fl])
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    row_ptr = np.zeros(N + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols.astype(np.int32)


def block_positions(row_ptr, col_idx, r, c):
    """Index into the nnzb block array of blocks (r, c) (must exist)."""
    N = len(row_ptr) - 1
    rows = np.repeat(np.arange(N, dtype=np.int64), np.diff(row_ptr))
    keys = rows * N + col_idx.astype(np.int64)
    q = np.asarray(r, np.int64) * N + np.asarray(c, np.int64)
    pos = np.searchsorted(keys, q)
    assert np.all(keys[pos] == q)
    return pos


def jacobian(case, u, u_old):
    """Exact dF/du with the upwind choice frozen; returns (row_ptr, col_idx,
    vals[nnzb,2,2]) where vals[e][a][b] = dR_a(row)/du_b(col), a,b in
    {0: water/P_w, 1: nonwetting/S_n}."""
    N = case.N
    P = u[:, 0]
    S = u[:, 1]
    sf = sat_functions(case, S)
    V = cell_volume(case)
    D = depth(case)
    g = case.grav
    row_ptr, col_idx = bcsr_pattern(case)
    vals = np.zeros((len(col_idx), 2, 2))
    cells = np.arange(N)
    pdiag = block_positions(row_ptr, col_idx, cells, cells)
    # storage
    c = case.poro * V / case.dt
    np.add.at(vals[:, 0, 1], pdiag, -c)
    np.add.at(vals[:, 1, 1], pdiag, c)
    # faces
    fl, fh, fd = faces(case)
    T = transmissibility(case, fl, fh, fd)
    phw = P - case.rho_w * g * D
    phn = P + sf["pc"] - case.rho_n * g * D
    dw = phw[fl] - phw[fh]
    dn = phn[fl] - phn[fh]
    wl = dw > 0
    nl = dn > 0
    upw = np.where(wl, fl, fh)
    upn = np.where(nl, fl, fh)
    aw = T * sf["lw"][upw]
    an = T * sf["ln"][upn]
    bw = T * sf["dlw"][upw] * dw                 # dF_w/dS_up
    dFn_dSl = np.where(nl, T * sf["dln"][fl] * dn, 0.0) + an * sf["dpc"][fl]
    dFn_dSh = np.where(nl, 0.0, T * sf["dln"][fh] * dn) - an * sf["dpc"][fh]
    dFw_dSl = np.where(wl, bw, 0.0)
    dFw_dSh = np.where(wl, 0.0, bw)
    p_ll = block_positions(row_ptr, col_idx, fl, fl)
    p_lh = block_positions(row_ptr, col_idx, fl, fh)
    p_hl = block_positions(row_ptr, col_idx, fh, fl)
    p_hh = block_positions(row_ptr, col_idx, fh, fh)
    # F is added to row l and subtracted from row h
    for (a, dP, dSl, dSh) in [(0, aw, dFw_dSl, dFw_dSh), (1, an, dFn_dSl, dFn_dSh)]:
        np.add.at(vals[:, a, 0], p_ll, dP)
        np.add.at(vals[:, a, 0], p_lh, -dP)
        np.add.at(vals[:, a, 0], p_hl, -dP)
        np.add.at(vals[:, a, 0], p_hh, dP)
        np.add.at(vals[:, a, 1], p_ll, dSl)
        np.add.at(vals[:, a, 1], p_lh, dSh)
        np.add.at(vals[:, a, 1], p_hl, -dSl)
        np.add.at(vals[:, a, 1], p_hh, -dSh)
    # Dirichlet faces
    if len(case.dir_cells):
        dc, Tb, zb = _dirichlet_geometry(case)
        sfb = sat_functions(case, np.asarray(case.dir_s, np.float64))
        dwb = phw[dc] - (case.dir_p - case.rho_w * g * zb)
        dnb = phn[dc] - (case.dir_p + sfb["pc"] - case.rho_n * g * zb)
        win = dwb > 0
        nin = dnb > 0
        lwb = np.where(win, sf["lw"][dc], sfb["lw"])
        lnb = np.where(nin, sf["ln"][dc], sfb["ln"])
        pd_ = pdiag[dc]
        np.add.at(vals[:, 0, 0], pd_, Tb * lwb)
        np.add.at(vals[:, 1, 0], pd_, Tb * lnb)
        np.add.at(vals[:, 0, 1], pd_, np.where(win, Tb * sf["dlw"][dc] * dwb, 0.0))
        np.add.at(vals[:, 1, 1], pd_, np.where(nin, Tb * sf["dln"][dc] * dnb, 0.0)
                  + Tb * lnb * sf["dpc"][dc])
    # producers
    pc_ = np.asarray(case.prod_cells, np.int64)
    if len(pc_):
        dp = P[pc_] - case.prod_pbh
        pp = pdiag[pc_]
        np.add.at(vals[:, 0, 0], pp, case.prod_wi * sf["lw"][pc_])
        np.add.at(vals[:, 1, 0], pp, case.prod_wi * sf["ln"][pc_])
        np.add.at(vals[:, 0, 1], pp, case.prod_wi * sf["dlw"][pc_] * dp)
        np.add.at(vals[:, 1, 1], pp, case.prod_wi * sf["dln"][pc_] * dp)
    return row_ptr, col_idx, vals


# ---------------------------------------------------------------------------
# helpers


def bcsr_to_dense(row_ptr, col_idx, vals):
    N = len(row_ptr) - 1
    A = np.zeros((2 * N, 2 * N))
    for i in range(N):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            j = col_idx[e]
            A[2 * i:2 * i + 2, 2 * j:2 * j + 2] = vals[e]
    return A


def bcsr_matrix(row_ptr, col_idx, vals):
    """J as a scipy block-sparse matrix (point ordering)."""
    import scipy.sparse as sp
    N = len(row_ptr) - 1
    return sp.bsr_matrix((vals, col_idx, row_ptr), shape=(2 * N, 2 * N))


def bcsr_spmv(row_ptr, col_idx, vals, x):
    """y = J x for point-ordered x (length 2N)."""
    return bcsr_matrix(row_ptr, col_idx, vals) @ x
