"""GPU parity: every step of the HIP path against the CPU oracle, through
the C ABI.

Bars (stated per test):
* integer structure (BCSR pattern, strength graph, C/F splitting, P/R/A_c
  patterns) bit-exact on identical input bits;
* FP64 values within 1e-12 relative to the magnitude of the row;
* full solves: true relative residual <= 1e-8 and iteration counts within
  +-1 of the oracle's.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg, blocks, fgmres, ilu, newton, precond, tpfa
from paper_1611_00127_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1611_00127_amd import driver, tpf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tpf.init()
    return driver, tpf, torch


def _cases():
    c1 = inputs.config_c1()
    return {
        "c1-initial": c1,
        "c1-random": inputs.random_state(c1, 3),
        "3d-random": inputs.small_case(14, 11, 9, seed=4, dirichlet=True, grav=9.81e-3),
        "3d-linear-pc": inputs.small_case(9, 8, 7, seed=5, pc_model=inputs.PC_LINEAR, pd=0.7),
    }


def _row_scale_close(a, b, rp, tol):
    """|a - b| <= tol * max|row| for CSR value arrays (per row scale)."""
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    scale = np.zeros(n)
    np.maximum.at(scale, rows, np.abs(b))
    err = np.abs(a - b)
    ok = err <= tol * np.maximum(scale[rows], 1e-300)
    return bool(np.all(ok)), float(np.max(err / np.maximum(scale[rows], 1e-300))) if len(err) else 0.0


@pytest.mark.parametrize("name", list(_cases()))
def test_assembly_parity(gpu, name):
    driver, tpf, torch = gpu
    c = _cases()[name]
    say(f"[assembly] case={name} N={c.N}")
    g = driver.GpuCase(c)
    g.assemble()
    torch.cuda.synchronize()
    rp, ci, vals = g.bcsr_numpy()
    orp, oci, ov = tpfa.jacobian(c, c.u, c.u_old)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci), "BCSR pattern must be bit-exact"
    # values: 1e-12 relative to the largest entry of the block row
    N = c.N
    brow = np.repeat(np.arange(N), np.diff(orp))
    scale = np.zeros(N)
    np.maximum.at(scale, brow, np.abs(ov).reshape(len(oci), 4).max(axis=1))
    err = np.abs(vals - ov).reshape(len(oci), 4).max(axis=1)
    assert np.all(err <= 1e-12 * scale[brow]), float(np.max(err / scale[brow]))
    R = g.R.cpu().numpy()
    oR = tpfa.residual(c, c.u, c.u_old).reshape(-1)
    assert np.max(np.abs(R - oR)) <= 1e-12 * np.max(np.abs(oR))
    # face-based upwinding: A_pp and A_sp are exactly symmetric on the GPU too
    for (a, b) in [(0, 0), (1, 0)]:
        B = sp.csr_matrix((vals[:, a, b], ci, rp), shape=(N, N))
        assert (B != B.T).nnz == 0
    g.close()


def test_spmv_parity(gpu):
    driver, tpf, torch = gpu
    c = inputs.small_case(20, 17, 6, seed=9)
    say("[spmv] 20x17x6")
    g = driver.GpuCase(c)
    g.assemble()
    x = inputs.random_vector(2 * c.N, 1)
    xd = torch.tensor(x, device="cuda")
    y = torch.empty_like(xd)
    tpf.tpf_spmv(g.J, xd, y)
    rp, ci, vals = g.bcsr_numpy()
    ye = tpfa.bcsr_spmv(rp, ci, vals, x)
    J = tpfa.bcsr_matrix(rp, ci, vals)
    absrow = abs(J) @ np.abs(x)
    assert np.all(np.abs(y.cpu().numpy() - ye) <= 1e-12 * absrow + 1e-300)
    g.close()


def _download_level(tpf, M, h, l):
    A = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, h, l, tpf.TPF_MAT_A))
    n = len(A[0]) - 1
    return sp.csr_matrix((A[2], A[1], A[0]), shape=(n, n))


def _setup(driver, tpf, c, kind, precision=0, **opts):
    g = driver.GpuCase(c)
    g.assemble()
    M = driver.GpuPrecond(kind, precision, **opts)
    M.setup(g)
    return g, M


@pytest.mark.parametrize("nx,ny,nz", [(13, 12, 7), (16, 11, 1), (12, 9, 3)])
def test_schur_parity(gpu, nx, ny, nz):
    """S~ against the oracle: formed on the grid (3D, at least five cells per
    direction) and by the general sparse product (2D, thin 3D)."""
    driver, tpf, torch = gpu
    c = inputs.small_case(nx, ny, nz, seed=6)
    say(f"[schur] {nx}x{ny}x{nz}")
    g, M = _setup(driver, tpf, c, "bf")
    rp, ci, vals = g.bcsr_numpy()
    blk = [blocks.block(rp, ci, vals, a, b) for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)]]
    So = blocks.schur_simple(*blk)
    Sv = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, 1, 0, tpf.TPF_MAT_SCHUR))
    assert np.array_equal(Sv[0], So.indptr) and np.array_equal(Sv[1], So.indices)
    ok, worst = _row_scale_close(Sv[2], So.data, So.indptr, 1e-12)
    assert ok, worst
    M.close(); g.close()


def _check_levels(tpf, M, hier, interp, coarsening="pmis"):
    """Each level's setup from the GPU's own level matrix (identical bits):
    strength graph, C/F (PMIS or CLJP), P (direct, classical or extended+i,
    truncated as the preconditioner's options say), R and A_c."""
    st = M.stats()
    nlev = st.levels[hier]
    assert nlev >= 2
    for l in range(nlev):
        A = _download_level(tpf, M, hier, l)
        _, dinv_p, n = tpf.tpf_precond_level_data(M.M, hier, l)
        dinv = tpf.device_array(dinv_p, n, np.float64)
        od = amg.Level(A).dinv
        assert np.all(np.abs(dinv - od) <= 1e-14 * np.abs(od)), f"dinv level {l}"
        if l == nlev - 1:
            break
        mask = amg.strength(A, 0.25)
        Sg = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, hier, l, tpf.TPF_MAT_S))
        So = amg.strength_matrix(A, mask)
        assert np.array_equal(Sg[0], So.indptr) and np.array_equal(Sg[1], So.indices), f"S level {l}"
        cf_p, _, _ = tpf.tpf_precond_level_data(M.M, hier, l)
        cf = tpf.device_array(cf_p, n, np.int8)
        ocf, _ = amg.coarsen(A, mask, 0x5eed, coarsening)
        assert np.array_equal(cf, ocf), f"C/F level {l}"
        P = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, hier, l, tpf.TPF_MAT_P))
        Po, _ = amg.interpolation(A, mask, ocf, interp, M.opts.trunc_pmax, M.opts.trunc_factor)
        assert np.array_equal(P[0], Po.indptr) and np.array_equal(P[1], Po.indices), f"P level {l}"
        ok, worst = _row_scale_close(P[2], Po.data, Po.indptr, 1e-12)
        assert ok, (l, worst)
        # R is the exact transpose of the GPU's own P (pure data movement)
        R = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, hier, l, tpf.TPF_MAT_R))
        Pg = sp.csr_matrix((P[2], P[1], P[0]), shape=Po.shape)
        Ro = Pg.T.tocsr(); Ro.sort_indices()
        assert np.array_equal(R[0], Ro.indptr) and np.array_equal(R[1], Ro.indices)
        assert np.array_equal(R[2], Ro.data)
        Ac = _download_level(tpf, M, hier, l + 1)
        Aco, _ = amg.galerkin(A, sp.csr_matrix((P[2], P[1], P[0]), shape=Po.shape))
        assert np.array_equal(Ac.indptr, Aco.indptr) and np.array_equal(Ac.indices, Aco.indices)
        ok, worst = _row_scale_close(Ac.data, Aco.data, Aco.indptr, 1e-12)
        assert ok, (l, worst)
    return nlev


@pytest.mark.parametrize("kind,hier,interp", [("bf", 0, "direct"), ("bf", 1, "ext+i"),
                                              ("cpr1", 0, "ext+i"), ("amg", 0, "direct"),
                                              ("cpr2", 1, "direct")])
def test_amg_setup_parity_per_level(gpu, kind, hier, interp):
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.config_c1(), 7, s_lo=0.15, s_hi=0.85)
    say(f"[amg-setup] kind={kind} hier={hier}")
    g, M = _setup(driver, tpf, c, kind, coarse_max=40)
    _check_levels(tpf, M, hier, interp)
    M.close(); g.close()


@pytest.mark.parametrize("route", list(range(9)))
def test_exti_every_kernel_class(gpu, route):
    """Extended+i on the S~ hierarchy of a 3D case with the F rows pushed to
    each kernel class in turn (route r: classes r-1 and up; 8 = one thread per
    row), every level checked against the oracle."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.small_case(16, 14, 10, seed=21), 22, s_lo=0.15, s_hi=0.85)
    say(f"[exti] 16x14x10 route {route}")
    g, M = _setup(driver, tpf, c, "bf", coarse_max=40, exti_route=route)
    nlev = _check_levels(tpf, M, 1, "ext+i")
    say(f"  {nlev} levels")
    M.close(); g.close()


def _gpu_hierarchy_as_oracle(tpf, M, hier, **cycle):
    st = M.stats()
    As, Ps = [], []
    for l in range(st.levels[hier]):
        As.append(_download_level(tpf, M, hier, l))
        if l < st.levels[hier] - 1:
            P = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, hier, l, tpf.TPF_MAT_P))
            Ps.append(sp.csr_matrix((P[2], P[1], P[0]), shape=(len(P[0]) - 1, int(P[1].max()) + 1)))
    # coarse column count from the next level size
    for l, P in enumerate(Ps):
        Ps[l] = sp.csr_matrix((P.data, P.indices, P.indptr), shape=(P.shape[0], As[l + 1].shape[0]))
    return amg.hierarchy_from_levels(As, Ps, dense_max=1024, **cycle)


@pytest.mark.parametrize("kind,hier", [("bf", 0), ("bf", 1), ("amg", 0)])
def test_vcycle_parity(gpu, kind, hier):
    driver, tpf, torch = gpu
    c = inputs.small_case(24, 20, 5, seed=8)
    c = inputs.random_state(c, 9, s_lo=0.15, s_hi=0.85)
    say(f"[vcycle] kind={kind} hier={hier}")
    g, M = _setup(driver, tpf, c, kind, coarse_max=50)
    H = _gpu_hierarchy_as_oracle(tpf, M, hier)
    n = H.levels[0].n
    b = inputs.random_vector(n, 2)
    bd = torch.tensor(b, device="cuda")
    xd = torch.empty_like(bd)
    tpf.tpf_precond_vcycle(M.M, hier, bd, xd)
    x = xd.cpu().numpy()
    xo = H.vcycle(b)
    assert np.max(np.abs(x - xo)) <= 1e-12 * np.max(np.abs(xo)), float(np.max(np.abs(x - xo)) / np.max(np.abs(xo)))
    M.close(); g.close()


SMOOTHERS = {0: "l1jacobi", 1: "chebyshev"}


@pytest.mark.parametrize("smoother,nu1,nu2,degree", [(1, 1, 1, 2), (1, 2, 1, 3), (0, 2, 2, 2),
                                                     (0, 0, 1, 2), (1, 1, 0, 1)])
def test_vcycle_smoother_variants_parity(gpu, smoother, nu1, nu2, degree):
    """V(nu1, nu2) cycles with l1-Jacobi or Chebyshev smoothing (generic
    sweeps) on both BF hierarchies against the oracle's cycle with the same
    options on the GPU's levels: FP64 within 1e-12 of max|x|, FP32 within
    1e-4."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.small_case(24, 20, 5, seed=8), 9, s_lo=0.15, s_hi=0.85)
    opts = dict(smoother=smoother, nu1=nu1, nu2=nu2, cheb_degree=degree)
    say(f"[smoothers] {opts}")
    g, M = _setup(driver, tpf, c, "bf", coarse_max=50, **opts)
    M32 = driver.GpuPrecond("bf", tpf.TPF_FP32, coarse_max=50, **opts)
    M32.setup(g)
    for hier in (0, 1):
        H = _gpu_hierarchy_as_oracle(tpf, M, hier, smoother=SMOOTHERS[smoother], nu1=nu1,
                                     nu2=nu2, cheb_degree=degree)
        assert len(H.levels) >= 3
        b = inputs.random_vector(H.levels[0].n, 20 + hier)
        xo = H.vcycle(b)
        bd = torch.tensor(b, device="cuda")
        for P, tol in ((M, 1e-12), (M32, 1e-4)):
            xd = torch.empty_like(bd)
            tpf.tpf_precond_vcycle(P.M, hier, bd, xd)
            rel = float(np.max(np.abs(xd.cpu().numpy() - xo)) / np.max(np.abs(xo)))
            say(f"  hierarchy {hier} tol {tol:g}: max rel diff {rel:.2e}")
            assert rel <= tol, rel
    M32.close(); M.close(); g.close()


@pytest.mark.parametrize("nu", [1, 2])
def test_chebyshev_bf_solve_parity(gpu, nu):
    """BF with Chebyshev(2) V(nu, nu) cycles on the 32x32x16 member of the 3D
    workload family: relres <= 1e-8, iterations within +-1 of the oracle's
    BF with the same smoother (oracle built from the same Jacobian)."""
    driver, tpf, torch = gpu
    c = inputs.config_c3(32, 32, 16)
    say(f"[chebyshev solve] nu={nu}")
    g, M = _setup(driver, tpf, c, "bf", smoother=1, nu1=nu, nu2=nu)
    b = g.rhs().contiguous()
    x = torch.empty_like(b)
    info = driver.solve(g, M, b, x, rtol=1e-8)
    rp, ci, vals = g.bcsr_numpy()
    J = tpfa.bcsr_matrix(rp, ci, vals)
    Mo = precond.Preconditioner("bf", rp, ci, vals, (c.nx, c.ny, c.nz),
                                amg_opts=dict(smoother="chebyshev", nu1=nu, nu2=nu))
    bn = b.cpu().numpy()
    _, io = fgmres.fgmres(lambda v: J @ v, Mo.apply, bn, rtol=1e-8)
    rel = np.linalg.norm(bn - J @ x.cpu().numpy()) / np.linalg.norm(bn)
    say(f"  gpu its={info.iterations} relres={rel:.2e} oracle its={io['iterations']}")
    assert info.status == tpf.TPF_CONVERGED and rel <= 1e-8
    assert abs(info.iterations - io["iterations"]) <= 1
    M.close(); g.close()


@pytest.mark.parametrize("dims", [(6, 5, 4), (10, 9, 5)])
def test_coarsest_dense_inverse(gpu, dims):
    """One-level hierarchy (max_levels 1): the V-cycle is the coarsest dense
    solve, x = A^{-1} b, checked against a direct solve of the GPU's own
    operator.  120 rows take the LDS-resident inversion, 450 rows the
    global-memory one."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.small_case(*dims, seed=21), 22, s_lo=0.15, s_hi=0.85)
    say(f"[coarsest] {dims}")
    g, M = _setup(driver, tpf, c, "bf", max_levels=1)
    st = M.stats()
    assert st.levels[0] == 1 and st.coarse_dense[0] == 1
    A = _download_level(tpf, M, 0, 0).toarray()
    b = inputs.random_vector(A.shape[0], 23)
    bd = torch.tensor(b, device="cuda")
    xd = torch.empty_like(bd)
    tpf.tpf_precond_vcycle(M.M, 0, bd, xd)
    x = xd.cpu().numpy()
    xo = np.linalg.solve(A, b)
    assert np.max(np.abs(x - xo)) <= 1e-10 * np.max(np.abs(xo))
    M.close(); g.close()


def test_bilu_parity(gpu):
    driver, tpf, torch = gpu
    c = inputs.small_case(15, 13, 6, seed=10)
    c = inputs.random_state(c, 11, s_lo=0.15, s_hi=0.85)
    say("[bilu] 15x13x6")
    g, M = _setup(driver, tpf, c, "cpr1")
    rp, ci, vals = g.bcsr_numpy()
    B = ilu.Bilu0(rp, ci, vals, c.nx, c.ny, c.nz)
    dv = tpf.device_array(tpf.tpf_precond_bilu_dinv(M.M), 4 * c.N, np.float64).reshape(-1, 2, 2)
    assert np.max(np.abs(dv - B.Dinv)) <= 1e-12 * np.max(np.abs(B.Dinv))
    M.close(); g.close()


@pytest.mark.parametrize("nx,ny", [(37, 23), (9, 70)])
def test_bilu_parity_2d(gpu, nx, ny):
    """Pivot blocks of the block ILU(0) on 2D grids (factorised front by front
    with the previous front's pivots in LDS) against the oracle."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.small_case(nx, ny, 1, seed=44), 45, s_lo=0.15, s_hi=0.85)
    say(f"[bilu 2d] {nx}x{ny}")
    g, M = _setup(driver, tpf, c, "cpr1")
    rp, ci, vals = g.bcsr_numpy()
    B = ilu.Bilu0(rp, ci, vals, c.nx, c.ny, c.nz)
    dv = tpf.device_array(tpf.tpf_precond_bilu_dinv(M.M), 4 * c.N, np.float64).reshape(-1, 2, 2)
    assert np.max(np.abs(dv - B.Dinv)) <= 1e-12 * np.max(np.abs(B.Dinv))
    M.close(); g.close()


@pytest.mark.parametrize("kind", ["amg", "cpr1", "cpr2", "bf"])
def test_precond_apply_parity(gpu, kind):
    """z = M^{-1} r: GPU vs the oracle preconditioner built from the GPU's J."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.small_case(22, 19, 4, seed=12), 13, s_lo=0.15, s_hi=0.85)
    say(f"[precond] kind={kind}")
    g, M = _setup(driver, tpf, c, kind)
    rp, ci, vals = g.bcsr_numpy()
    Mo = precond.Preconditioner(kind, rp, ci, vals, (c.nx, c.ny, c.nz))
    st = M.stats()
    hs = {"amg": [Mo.H] if kind == "amg" else None}.get(kind)
    if kind == "bf":
        hs = [Mo.Hs, Mo.Hschur]
    elif kind == "cpr1":
        hs = [Mo.Hp]
    elif kind == "cpr2":
        hs = [Mo.Hp, Mo.Hs]
    for h, Ho in enumerate(hs):
        assert st.levels[h] == len(Ho.levels)
        assert [st.rows[h][l] for l in range(st.levels[h])] == [L.n for L in Ho.levels]
    r = inputs.random_vector(2 * c.N, 14)
    rd = torch.tensor(r, device="cuda")
    zd = torch.empty_like(rd)
    M.apply(rd, zd)
    z = zd.cpu().numpy()
    zo = Mo.apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo)), float(np.max(np.abs(z - zo)) / np.max(np.abs(zo)))
    M.close(); g.close()


@pytest.mark.parametrize("kind,nx,ny", [("cpr1", 37, 23), ("cpr2", 23, 37), ("cpr1", 70, 9)])
def test_precond_apply_parity_2d(gpu, kind, nx, ny):
    """z = M^{-1} r on 2D grids, whose block ILU(0) sweeps keep the previous
    anti-diagonal front in LDS (fronts shorter than the grid's rows, wide and
    tall grids): GPU vs the oracle preconditioner built from the GPU's J."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.small_case(nx, ny, 1, seed=41), 42, s_lo=0.15, s_hi=0.85)
    say(f"[precond 2d] kind={kind} {nx}x{ny}")
    g, M = _setup(driver, tpf, c, kind)
    rp, ci, vals = g.bcsr_numpy()
    Mo = precond.Preconditioner(kind, rp, ci, vals, (c.nx, c.ny, c.nz))
    r = inputs.random_vector(2 * c.N, 43)
    rd = torch.tensor(r, device="cuda")
    zd = torch.empty_like(rd)
    M.apply(rd, zd)
    z = zd.cpu().numpy()
    zo = Mo.apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo)), float(np.max(np.abs(z - zo)) / np.max(np.abs(zo)))
    M.close(); g.close()


@pytest.mark.parametrize("kind", ["amg", "cpr1", "cpr2", "bf"])
def test_solve_parity_c1(gpu, kind):
    """32x32 workload, first Newton Jacobian: relres <= 1e-8, iterations +-1."""
    driver, tpf, torch = gpu
    c = inputs.config_c1()
    say(f"[solve] 32x32 kind={kind}")
    g, M = _setup(driver, tpf, c, kind)
    b = g.rhs().contiguous()
    x = torch.empty_like(b)
    info = driver.solve(g, M, b, x, rtol=1e-8)
    rp, ci, vals = g.bcsr_numpy()
    J = tpfa.bcsr_matrix(rp, ci, vals)
    Mo = precond.Preconditioner(kind, rp, ci, vals, (c.nx, c.ny, c.nz))
    bn = b.cpu().numpy()
    xo, io = fgmres.fgmres(lambda v: J @ v, Mo.apply, bn, rtol=1e-8)
    xs = x.cpu().numpy()
    rel = np.linalg.norm(bn - J @ xs) / np.linalg.norm(bn)
    say(f"  gpu its={info.iterations} relres={info.relres_true:.3e} oracle its={io['iterations']}")
    assert info.status == tpf.TPF_CONVERGED and io["status"] == fgmres.CONVERGED
    assert rel <= 1e-8 and abs(info.relres_true - rel) <= 1e-10
    assert abs(info.iterations - io["iterations"]) <= 1
    M.close(); g.close()


@pytest.mark.parametrize("kind", ["bf", "cpr2", "amg"])
def test_fp32_vcycle_form_reaches_fp64_accuracy(gpu, kind):
    """FP32 hierarchies and V-cycles inside FP64 FGMRES reach the same 1e-8
    true residual; the error against the FP64 oracle solution is reported.
    (Physical first-Newton-Jacobian state of the 3D workload family.)"""
    driver, tpf, torch = gpu
    c = inputs.config_c3(32, 32, 16)
    say(f"[fp32] kind={kind}")
    g, M = _setup(driver, tpf, c, kind, precision=tpf.TPF_FP32)
    b = g.rhs().contiguous()
    x = torch.empty_like(b)
    info = driver.solve(g, M, b, x, rtol=1e-8)
    rp, ci, vals = g.bcsr_numpy()
    J = tpfa.bcsr_matrix(rp, ci, vals)
    bn = b.cpu().numpy()
    xs = x.cpu().numpy()
    assert info.status == tpf.TPF_CONVERGED
    assert np.linalg.norm(bn - J @ xs) <= 1e-8 * np.linalg.norm(bn)
    Mo = precond.Preconditioner(kind, rp, ci, vals, (c.nx, c.ny, c.nz))
    xo, io = fgmres.fgmres(lambda v: J @ v, Mo.apply, bn, rtol=1e-8)
    err = np.linalg.norm(xs - xo) / np.linalg.norm(xo)
    say(f"  fp32 its={info.iterations} oracle(fp64) its={io['iterations']} err={err:.2e}")
    assert io["status"] == fgmres.CONVERGED
    assert err <= 1e-5
    M.close(); g.close()


@pytest.mark.parametrize("kind,precision", [("bf", 0), ("bf", 1), ("cpr2", 0), ("amg", 0)])
def test_graph_replays_match_eager(gpu, kind, precision):
    """V-cycles replayed from recorded HIP graphs equal the eager launches
    bit for bit on every replay (eager work and synchronisations between the
    replays), on the null stream and on a side stream, and after a numeric
    refresh of the hierarchy; a full solve is identical too."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.small_case(20, 16, 8, seed=31), 32, s_lo=0.15, s_hi=0.85)
    say(f"[graphs] {kind} precision {precision}")
    g, M = _setup(driver, tpf, c, kind, precision)
    n = 2 * c.N
    rng = np.random.default_rng(33)
    rs = [torch.tensor(rng.standard_normal(n), device="cuda") for _ in range(3)]
    side = torch.cuda.Stream()

    def applies(stream=None):
        out = []
        for r in rs:
            z = torch.full_like(r, float("nan"))
            M.apply(r, z, stream=stream)
            out.append(z)
        torch.cuda.synchronize()
        return [z.cpu().numpy() for z in out]

    try:
        for refresh in (False, True):
            if refresh:
                g.u.add_(1e-3 * torch.tensor(rng.standard_normal(n), device="cuda"))
                g.assemble()
                M.setup(g, reuse=True)
                torch.cuda.synchronize()
            tpf.tpf_set_graphs(False)
            eager = applies()
            tpf.tpf_set_graphs(True)
            for rep in range(3):
                got = applies(side if rep == 1 else None)
                for k in range(len(rs)):
                    assert np.array_equal(got[k], eager[k]), (refresh, rep, k)
                y = torch.empty_like(rs[0])
                tpf.tpf_spmv(g.J, rs[rep], y)  # eager work between replays
                torch.cuda.synchronize()
        b = g.R.clone()
        xs, its = [], []
        for graphs in (False, True):
            tpf.tpf_set_graphs(graphs)
            x = torch.empty_like(b)
            info = driver.solve(g, M, b, x)
            xs.append(x.cpu().numpy()); its.append(info.iterations)
        assert its[0] == its[1] and np.array_equal(xs[0], xs[1])
    finally:
        tpf.tpf_set_graphs(False)  # the library default
        M.close(); g.close()


def test_solve_edge_cases(gpu):
    driver, tpf, torch = gpu
    c = inputs.config_c1()
    say("[edge] zero rhs, maxit=1, identity preconditioner, NaN rhs")
    g, M = _setup(driver, tpf, c, "bf")
    b = torch.zeros(2 * c.N, dtype=torch.float64, device="cuda")
    x = torch.ones_like(b)
    info = driver.solve(g, M, b, x)
    assert info.status == tpf.TPF_CONVERGED and info.iterations == 0
    assert float(x.abs().max()) == 0.0
    b = g.rhs().contiguous()
    info = driver.solve(g, M, b, x, maxit=1)
    assert info.status == tpf.TPF_MAX_ITERS and info.iterations == 1
    info = driver.solve(g, None, b, x, maxit=5)
    assert info.iterations == 5
    bn = b.clone()
    bn[7] = float("nan")
    info = driver.solve(g, M, bn, x)
    assert info.status == tpf.TPF_NONFINITE
    M.close(); g.close()


def test_reuse_structure_matches_rebuild(gpu):
    """Numeric refresh on the next Newton Jacobian (same pattern) keeps C/F,
    P, R and gives the Galerkin products of the new level operators."""
    driver, tpf, torch = gpu
    c = inputs.config_c3(24, 24, 12)
    say("[reuse] 24x24x12 Newton step 2 with the step-1 hierarchy")
    g, M = _setup(driver, tpf, c, "bf")
    cf0 = tpf.device_array(tpf.tpf_precond_level_data(M.M, 1, 0)[0], c.N, np.int8)
    b = g.rhs().contiguous()
    x = torch.empty_like(b)
    info = driver.solve(g, M, b, x)
    assert info.status == tpf.TPF_CONVERGED
    tpf.tpf_newton_update(g.prob, g.u, x, 0.2)
    g.assemble()
    M.setup(g, reuse=True)
    cf1 = tpf.device_array(tpf.tpf_precond_level_data(M.M, 1, 0)[0], c.N, np.int8)
    assert np.array_equal(cf0, cf1)
    for h in range(2):
        st = M.stats()
        for l in range(st.levels[h] - 1):
            A0 = _download_level(tpf, M, h, l)
            P = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, h, l, tpf.TPF_MAT_P))
            A1 = _download_level(tpf, M, h, l + 1)
            Pm = sp.csr_matrix((P[2], P[1], P[0]), shape=(A0.shape[0], A1.shape[0]))
            A1o, _ = amg.galerkin(A0, Pm)
            assert np.array_equal(A1.indices, A1o.indices)
            ok, worst = _row_scale_close(A1.data, A1o.data, A1o.indptr, 1e-12)
            assert ok, (h, l, worst)
    b = g.rhs().contiguous()
    info = driver.solve(g, M, b, x)
    say(f"  refreshed solve its={info.iterations} relres={info.relres_true:.2e}")
    assert info.status == tpf.TPF_CONVERGED
    M.close(); g.close()


@pytest.mark.parametrize("reuse", [False, True])
def test_newton_sequence_matches_oracle(gpu, reuse):
    """Four Newton Jacobians of one time step (saturation chop 0.2): every
    linear solve reaches 1e-8, and ||F|| along the sequence follows the
    oracle's Newton sequence (rebuild) to 1e-6 relative."""
    driver, tpf, torch = gpu
    c = inputs.config_c3(20, 20, 10)
    say(f"[newton] 20x20x10 reuse={reuse}")
    g = driver.GpuCase(c)
    M = driver.GpuPrecond("bf")
    recs = driver.newton_sequence(g, M, 4, reuse=reuse, ds_max=0.2)
    seq, _ = newton.sequence(c, 4, "bf", ds_max=0.2)
    for r, (fo, io) in zip(recs, seq):
        say(f"  k={r['k']} |F| gpu={r['fnorm']:.6e} oracle={fo:.6e} its={r['iterations']}/{io['iterations']}")
        assert r["status"] == tpf.TPF_CONVERGED and r["relres"] <= 1e-8
        assert abs(r["fnorm"] - fo) <= 1e-6 * fo
    M.close(); g.close()
