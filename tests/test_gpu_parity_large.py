"""GPU parity at the sizes the benchmark runs, through the C ABI.

Two grids of the 3D workload family (sigma 3, K_z/K_x 0.1, layered,
five-spot, CFL 10):

* 64x64x48 (196,608 cells) at the oracle's own Newton iterate 1: every AMG
  level of both BF hierarchies against the oracle (S~ level 1 has more than
  65,536 rows, so its V-cycle takes the D^{-1}b-first CSR smoother, and the
  levels above 4,096 rows take the multi-launch PMIS rounds), one V-cycle in
  FP64 and FP32 (the streamed CSR smoothers, some wavefronts over several
  LDS windows), the full BF solve (iterations within +-1), and CPR1, whose
  block ILU(0) runs the per-front kernels (fronts of up to 2,496 cells).
* AMG on the point-ordered scalar Jacobian of a 220x200 2D case (88,000
  unknowns, 10 entries per row): its CSR level 0 takes the streamed smoothers
  with two lanes per row; one V-cycle in FP64 and FP32.
* 128x128x64 (1,048,576 cells), the benchmark grid itself: residual,
  Jacobian, SpMV, S~, and the strength graph and C/F splitting of S~'s first
  level, element by element; BF solves against the oracle's stored solves
  (tests/golden/c3_oracle_solves.json, written by make_c3_oracle_solves.py
  from the oracle alone).

Each level's setup is checked on the GPU's own level matrix (identical input
bits, so the oracle's threshold and tie decisions see the same numbers);
that matrix was itself checked against the oracle one step earlier.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg, blocks, fgmres, ilu, newton, precond, tpfa
from paper_1611_00127_amd import inputs

from test_gpu_parity import (_check_levels, _download_level, _gpu_hierarchy_as_oracle,
                             _row_scale_close, _setup, say)

pytestmark = pytest.mark.gpu

GRID = (64, 64, 48)
DS_MAX = 0.2
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "c3_oracle_solves.json")


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1611_00127_amd import driver, tpf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tpf.init()
    return driver, tpf, torch


@pytest.fixture(scope="module")
def newton1():
    """The oracle's Newton iterate 1 on the 64x64x48 grid and the oracle's
    BF solve of J x = -F there."""
    c = inputs.config_c3(*GRID)
    say("[large] oracle: Newton step from the initial condition")
    x0, _, _ = newton.solve(c, "bf", rtol=1e-8)
    c1 = c.replace(u=newton.update(c.u, x0, DS_MAX))
    say("[large] oracle: BF solve at Newton iterate 1")
    x1, info1, _ = newton.solve(c1, "bf", rtol=1e-8)
    say(f"[large] oracle: {info1['iterations']} iterations")
    return c1, x1, info1


def _assembly_close(g, c):
    rp, ci, vals = g.bcsr_numpy()
    orp, oci, ov = tpfa.jacobian(c, c.u, c.u_old)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    brow = np.repeat(np.arange(c.N), np.diff(orp))
    scale = np.zeros(c.N)
    np.maximum.at(scale, brow, np.abs(ov).reshape(len(oci), 4).max(axis=1))
    err = np.abs(vals - ov).reshape(len(oci), 4).max(axis=1)
    assert np.all(err <= 1e-12 * scale[brow]), float(np.max(err / scale[brow]))
    R = g.R.cpu().numpy()
    oR = tpfa.residual(c, c.u, c.u_old).reshape(-1)
    assert np.max(np.abs(R - oR)) <= 1e-12 * np.max(np.abs(oR))
    return rp, ci, vals


def test_large_setup_levels(gpu, newton1):
    """Assembly and S~ at Newton iterate 1, then every level of both BF
    hierarchies: strength graph, C/F (bit-exact), P, R, A_c (pattern
    bit-exact, values 1e-12 of the row scale)."""
    driver, tpf, torch = gpu
    c1, _, _ = newton1
    say("[large] assembly + BF setup at Newton iterate 1")
    g, M = _setup(driver, tpf, c1, "bf")
    rp, ci, vals = _assembly_close(g, c1)
    blk = [blocks.block(rp, ci, vals, a, b) for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)]]
    # the upwind coupling is present: A_ps has off-diagonal entries
    assert np.count_nonzero(blk[1].data) > 2 * c1.N
    So = blocks.schur_simple(*blk)
    Sv = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, 1, 0, tpf.TPF_MAT_SCHUR))
    assert np.array_equal(Sv[0], So.indptr) and np.array_equal(Sv[1], So.indices)
    ok, worst = _row_scale_close(Sv[2], So.data, So.indptr, 1e-12)
    assert ok, worst
    st = M.stats()
    rows_s = [int(st.rows[1][l]) for l in range(st.levels[1])]
    say(f"  S~ levels {rows_s}")
    assert rows_s[1] >= 65536, "S~ level 1 must take the large-level CSR smoother"
    for hier, interp in ((1, "ext+i"), (0, "direct")):
        say(f"  levels of hierarchy {hier} ({interp})")
        _check_levels(tpf, M, hier, interp)
    M.close(); g.close()


def _lanes_per_row(A):
    """Lanes per row the library picks from the mean row length: the
    smallest power of two with 8 LPR >= mean."""
    lpr = 1
    while lpr < 64 and 8 * lpr < A.nnz / A.shape[0]:
        lpr *= 2
    return lpr


def _longest_wavefront_range(A):
    """Entries of the longest run of rows one wavefront of the streamed CSR
    smoothers takes: 64 / LPR rows."""
    n = A.shape[0]
    lpr = _lanes_per_row(A)
    r0 = np.arange(0, n, 64 // lpr)
    return int(np.max(A.indptr[np.minimum(r0 + 64 // lpr, n)] - A.indptr[r0]))


@pytest.mark.parametrize("precision", [0, 1])
def test_large_vcycle(gpu, newton1, precision):
    """One V-cycle of each BF hierarchy against the oracle's cycle on the
    GPU's levels: FP64 within 1e-12 of max|x|; FP32 (stored values and
    vectors rounded to 24 bits, coarsest solve in FP64) within 1e-4."""
    driver, tpf, torch = gpu
    c1, _, _ = newton1
    say(f"[large] V-cycles, precision {precision}")
    g, M = _setup(driver, tpf, c1, "bf")
    M32 = driver.GpuPrecond("bf", tpf.TPF_FP32) if precision else None
    if M32 is not None:
        M32.setup(g)
    longest = 0
    for hier in (1, 0):
        H = _gpu_hierarchy_as_oracle(tpf, M, hier)
        for L in H.levels[1:]:
            if L.n >= 65536:
                longest = max(longest, _longest_wavefront_range(L.A))
        n = H.levels[0].n
        b = inputs.random_vector(n, 40 + hier)
        bd = torch.tensor(b, device="cuda")
        xd = torch.empty_like(bd)
        tpf.tpf_precond_vcycle((M32 or M).M, hier, bd, xd)
        x = xd.cpu().numpy()
        xo = H.vcycle(b)
        rel = float(np.max(np.abs(x - xo)) / np.max(np.abs(xo)))
        say(f"  hierarchy {hier}: {len(H.levels)} levels, max rel diff {rel:.2e}")
        assert rel <= (1e-4 if precision else 1e-12), rel
    # some wavefront of the streamed smoothers takes more than one 512-entry window
    assert longest > 512, longest
    if M32 is not None:
        M32.close()
    M.close(); g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_streamed_two_lane_rows(gpu, precision):
    """AMG on the point-ordered scalar Jacobian of a 2D case with 88,000
    unknowns: level 0 is not a stencil layout, has 10 entries per row (2
    lanes, 32 rows per wavefront) and takes the streamed smoothers; one
    V-cycle against the oracle's cycle on the GPU's levels (FP64 within
    1e-12 of max|x|, FP32 within 1e-4)."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.small_case(220, 200, 1, seed=5), 6, s_lo=0.15, s_hi=0.85)
    say(f"[streamed 2-lane] precision {precision}")
    g, M = _setup(driver, tpf, c, "amg")
    M32 = driver.GpuPrecond("amg", tpf.TPF_FP32) if precision else None
    if M32 is not None:
        M32.setup(g)
    H = _gpu_hierarchy_as_oracle(tpf, M, 0)
    A0 = H.levels[0].A
    say(f"  levels {[L.n for L in H.levels]}, level 0: {A0.nnz / A0.shape[0]:.1f} entries per row")
    assert A0.shape[0] >= 65536 and _lanes_per_row(A0) == 2
    assert int(M.stats().l0_diagonals[0]) == 0  # CSR level 0: the streamed kernels run on it
    b = inputs.random_vector(A0.shape[0], 17)
    bd = torch.tensor(b, device="cuda")
    xd = torch.empty_like(bd)
    tpf.tpf_precond_vcycle((M32 or M).M, 0, bd, xd)
    x = xd.cpu().numpy()
    xo = H.vcycle(b)
    rel = float(np.max(np.abs(x - xo)) / np.max(np.abs(xo)))
    say(f"  max rel diff {rel:.2e}")
    assert rel <= (1e-4 if precision else 1e-12), rel
    if M32 is not None:
        M32.close()
    M.close(); g.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_large_bf_solve_vs_oracle(gpu, newton1, precision):
    """BF FGMRES(30) at Newton iterate 1: true relres <= 1e-8; FP64
    iterations within +-1 of the oracle's; both forms within 1e-5 of the
    oracle's FP64 solution."""
    driver, tpf, torch = gpu
    c1, x1, info1 = newton1
    say(f"[large] BF solve, precision {precision}")
    g, M = _setup(driver, tpf, c1, "bf", precision=precision)
    b = g.rhs().contiguous()
    x = torch.empty_like(b)
    info = driver.solve(g, M, b, x, rtol=1e-8)
    rp, ci, vals = g.bcsr_numpy()
    J = tpfa.bcsr_matrix(rp, ci, vals)
    bn = b.cpu().numpy()
    xs = x.cpu().numpy()
    rel = np.linalg.norm(bn - J @ xs) / np.linalg.norm(bn)
    err = np.linalg.norm(xs - x1) / np.linalg.norm(x1)
    say(f"  gpu its={info.iterations} relres={rel:.2e} oracle its={info1['iterations']} "
        f"err vs oracle={err:.2e}")
    assert info.status == tpf.TPF_CONVERGED and rel <= 1e-8
    if precision == 0:
        assert abs(info.iterations - info1["iterations"]) <= 1
    assert err <= 1e-5
    M.close(); g.close()


def test_large_cpr1_bilu_per_front(gpu, newton1):
    """CPR1 on the 64x64x48 grid: the block ILU(0) pivots (fronts of up to
    2,496 cells, the per-front kernels) within 1e-12 of the oracle's, and
    the preconditioner application within 1e-10 of the oracle's Algorithm 1
    on the same Jacobian."""
    driver, tpf, torch = gpu
    c1, _, _ = newton1
    say("[large] CPR1 setup")
    g, M = _setup(driver, tpf, c1, "cpr1")
    rp, ci, vals = g.bcsr_numpy()
    _, _, counts = ilu.wavefronts(*GRID)
    assert counts.max() > 2048
    dinv = tpf.device_array(tpf.tpf_precond_bilu_dinv(M.M), 4 * c1.N,
                            np.float64).reshape(-1, 2, 2)
    odinv = ilu.Bilu0(rp, ci, vals, *GRID).Dinv
    err = np.abs(dinv - odinv).reshape(-1, 4).max(axis=1)
    scale = np.abs(odinv).reshape(-1, 4).max(axis=1)
    assert np.all(err <= 1e-12 * scale), float(np.max(err / scale))
    say("  oracle CPR1 (A_pp hierarchy)")
    Mo = precond.Preconditioner("cpr1", rp, ci, vals, GRID)
    r = inputs.random_vector(2 * c1.N, 44)
    rd = torch.tensor(r, device="cuda")
    zd = torch.empty_like(rd)
    M.apply(rd, zd)
    z = zd.cpu().numpy()
    zo = Mo.apply(r)
    rel = float(np.max(np.abs(z - zo)) / np.max(np.abs(zo)))
    say(f"  apply max rel diff {rel:.2e}")
    assert rel <= 1e-10
    M.close(); g.close()


# ------------------------------------------------------ the benchmark grid


def test_c3_full_grid_assembly_schur_pmis(gpu):
    """128x128x64 at a seeded random state: R, J (1e-12), SpMV (1e-12 of
    |J||x|), S~ (pattern bit-exact, values 1e-12), and on S~'s first level
    the strength graph and the C/F splitting bit-exact."""
    driver, tpf, torch = gpu
    c = inputs.random_state(inputs.config_c3(), 45, s_lo=0.15, s_hi=0.85)
    say("[c3] assembly at 1,048,576 cells")
    g, M = _setup(driver, tpf, c, "bf")
    rp, ci, vals = _assembly_close(g, c)
    x = inputs.random_vector(2 * c.N, 46)
    xd = torch.tensor(x, device="cuda")
    y = torch.empty_like(xd)
    tpf.tpf_spmv(g.J, xd, y)
    J = tpfa.bcsr_matrix(rp, ci, vals)
    absrow = abs(J) @ np.abs(x)
    assert np.all(np.abs(y.cpu().numpy() - J @ x) <= 1e-12 * absrow + 1e-300)
    say("[c3] S~")
    blk = [blocks.block(rp, ci, vals, a, b) for a, b in [(0, 0), (0, 1), (1, 0), (1, 1)]]
    So = blocks.schur_simple(*blk)
    S = _download_level(tpf, M, 1, 0)
    assert np.array_equal(S.indptr, So.indptr) and np.array_equal(S.indices, So.indices)
    ok, worst = _row_scale_close(S.data, So.data, So.indptr, 1e-12)
    assert ok, worst
    say("[c3] strength and PMIS on S~ level 0")
    mask = amg.strength(S, 0.25)
    Sg = tpf.csr_to_numpy(tpf.tpf_precond_matrix(M.M, 1, 0, tpf.TPF_MAT_S))
    So_ = amg.strength_matrix(S, mask)
    assert np.array_equal(Sg[0], So_.indptr) and np.array_equal(Sg[1], So_.indices)
    cf_p, _, n = tpf.tpf_precond_level_data(M.M, 1, 0)
    cf = tpf.device_array(cf_p, n, np.int8)
    ocf, rounds = amg.pmis(S, mask, 0x5eed)
    say(f"  {rounds} PMIS rounds, {int((ocf == amg.C_PT).sum())} C points")
    assert np.array_equal(cf, ocf)
    M.close(); g.close()


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("state,precision", [("initial", 0), ("initial", 1), ("newton1", 0)])
def test_c3_full_grid_solve_vs_stored_oracle(gpu, state, precision):
    """BF solve of the 128x128x64 workload against the oracle's stored solve:
    relres <= 1e-8; FP64 iterations within +-1 of the oracle's; the solution
    at 4,096 stored sample indices within 1e-5 of max|x|.  At Newton iterate
    1 each side takes its own first Newton step from the identical initial
    state (their iterates differ by the 1e-8 solve tolerance), so only the
    iteration count is compared there."""
    driver, tpf, torch = gpu
    gold = _golden()["states"][state]
    c = inputs.config_c3()
    say(f"[c3] BF solve at {state}, precision {precision}")
    g = driver.GpuCase(c)
    if state == "newton1":
        g.u.copy_(driver.newton_states(g, 2, ds_max=DS_MAX)[1])
    g.assemble()
    M = driver.GpuPrecond("bf", precision)
    M.setup(g)
    b = g.rhs().contiguous()
    x = torch.empty_like(b)
    info = driver.solve(g, M, b, x, rtol=1e-8)
    say(f"  gpu its={info.iterations} relres={info.relres_true:.2e} "
        f"oracle its={gold['iterations']}")
    assert info.status == tpf.TPF_CONVERGED and info.relres_true <= 1e-8
    if precision == 0:
        assert abs(info.iterations - gold["iterations"]) <= 1
    if state == "initial":
        idx = np.asarray(gold["sample_index"])
        xs = x.cpu().numpy()[idx]
        dev = float(np.max(np.abs(xs - np.asarray(gold["sample_x"]))) / gold["max_abs_x"])
        say(f"  sampled solution: max deviation {dev:.2e} of max|x|")
        assert dev <= 1e-5
    M.close(); g.close()
