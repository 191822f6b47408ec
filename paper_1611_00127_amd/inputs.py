"""Seeded synthetic inputs for the two-phase TPFA solver and for its oracle.

This module is shared by the GPU path, the CPU oracle, the tests and the
benchmark.  It produces *inputs only*: grids, permeability and porosity
fields, well descriptions, the state at which a Newton Jacobian is taken,
and seeded random vectors.  It contains no discretisation, constitutive,
preconditioner or Krylov arithmetic.

Random fields: log-permeability is a stationary Gaussian field with an
exponential covariance sigma^2 exp(-r), r the anisotropic distance in cell
units scaled by the correlation lengths, sampled by circulant embedding on a
grid padded to twice the size (negative eigenvalues of the embedding are
clipped to zero).  All draws use numpy's PCG64 generator.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# Capillary-pressure model codes (shared with the C ABI).
PC_BROOKS_COREY = 0
PC_LINEAR = 1

# Dirichlet face codes: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z.
FACE_XM, FACE_XP, FACE_YM, FACE_YP, FACE_ZM, FACE_ZP = range(6)


@dataclass
class Case:
    """One linear-solve workload: a grid, rock and fluid data, wells and the
    Newton linearisation state.  Arrays are float64, cell index
    i = ix + nx*(iy + ny*iz)."""

    nx: int
    ny: int
    nz: int
    hx: float = 1.0
    hy: float = 1.0
    hz: float = 1.0
    kx: np.ndarray = None
    ky: np.ndarray = None
    kz: np.ndarray = None
    poro: np.ndarray = None
    mu_w: float = 1.0
    mu_n: float = 10.0
    rho_w: float = 1000.0
    rho_n: float = 700.0
    grav: float = 0.0
    pc_model: int = PC_BROOKS_COREY
    bc_lambda: float = 2.0
    swr: float = 0.1
    snr: float = 0.1
    pd: float = 0.1          # Brooks-Corey entry pressure, or P_0 of the linear model
    s_eps: float = 0.05      # below this effective saturation P_c is continued linearly
    dt: float = 1.0
    # constant source rates per cell, columns (q_w, q_n); rate injectors live here
    q: np.ndarray = None
    # bottom-hole-pressure producers
    prod_cells: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    prod_wi: np.ndarray = field(default_factory=lambda: np.zeros(0))
    prod_pbh: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # Dirichlet boundary faces
    dir_cells: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    dir_face: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    dir_p: np.ndarray = field(default_factory=lambda: np.zeros(0))
    dir_s: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # state: columns (P_w, S_n); u is the linearisation point, u_old the last time level
    u: np.ndarray = None
    u_old: np.ndarray = None
    name: str = ""

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dim(self) -> int:
        return 3 if self.nz > 1 else 2

    def replace(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# random fields


def gaussian_field(shape, corr, sigma, rng) -> np.ndarray:
    """Stationary Gaussian field, zero mean, covariance sigma^2 exp(-r) with
    r = |(dx/lx, dy/ly, dz/lz)| in cell units; shape is (nz, ny, nx) and
    corr is (lz, ly, lx).  Circulant embedding on a 2x padded torus."""
    shape = tuple(int(s) for s in shape)
    pad = tuple(2 * s for s in shape)
    axes = []
    for m, ell in zip(pad, corr):
        d = np.arange(m, dtype=np.float64)
        d = np.minimum(d, m - d)
        axes.append(d / float(ell))
    grids = np.meshgrid(*axes, indexing="ij", sparse=True)
    r2 = sum(g * g for g in grids)
    cov = (sigma * sigma) * np.exp(-np.sqrt(r2))
    lam = np.fft.fftn(cov).real
    np.maximum(lam, 0.0, out=lam)
    m_tot = float(np.prod(pad))
    xi = rng.standard_normal(pad) + 1j * rng.standard_normal(pad)
    f = np.fft.ifftn(np.sqrt(lam / m_tot) * xi) * m_tot
    sl = tuple(slice(0, s) for s in shape)
    return np.ascontiguousarray(f.real[sl])


def peaceman_wi(k_h: float, hx: float, hy: float, hz: float) -> float:
    """Well index of a vertical well, 2*pi*k*h_z/ln(r_o/r_w), r_o = 0.2 h,
    r_w = 0.1 h (an input parameter of a producer, not solver arithmetic)."""
    return 2.0 * np.pi * k_h * hz / np.log(2.0)


# ----------------------------------------------------------------------------
# workloads


def _finish(case: Case, p_init: float, sn_init: float) -> Case:
    N = case.N
    u = np.empty((N, 2))
    u[:, 0] = p_init
    u[:, 1] = sn_init
    case.u_old = u.copy()
    case.u = u.copy()
    return case


def workload_2d_corner(nx, ny, sigma, corr, pd, cfl, seed, name="") -> Case:
    """2D grid, isotropic log-normal permeability, one rate injector of the
    nonwetting phase at cell (0,0) and one BHP producer at the opposite
    corner; state = the initial condition (uniform P_w = 0, S_n = 0.2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    logk = gaussian_field((1, ny, nx), (1.0, corr, corr), sigma, rng).reshape(-1)
    k = np.exp(logk)
    N = nx * ny
    c = Case(nx=nx, ny=ny, nz=1, kx=k.copy(), ky=k.copy(), kz=k.copy(),
             poro=np.full(N, 0.2), pd=pd, name=name)
    q = np.zeros((N, 2))
    q[0, 1] = cfl * 0.2 * 1.0 / c.dt
    c.q = q
    pc = N - 1
    c.prod_cells = np.array([pc], np.int32)
    c.prod_wi = np.array([peaceman_wi(k[pc], 1.0, 1.0, 1.0)])
    c.prod_pbh = np.array([0.0])
    return _finish(c, 0.0, 0.2)


def workload_3d_fivespot(nx, ny, nz, sigma, corr, pd, cfl, seed, name="",
                         kz_ratio=0.1, layer_every=8, layer_boost=3.0) -> Case:
    """3D grid, log-normal permeability with vertical anisotropy and
    channelised layers (iz % layer_every == 0 gets log k + layer_boost);
    injector columns of the nonwetting phase at the four (x,y) corners, a BHP
    producer column at the centre, all layers perforated; injection in a
    column is split in proportion to K_x.  State = the initial condition."""
    rng = np.random.Generator(np.random.PCG64(seed))
    logk = gaussian_field((nz, ny, nx), (corr[2], corr[1], corr[0]), sigma, rng)
    logk[::layer_every, :, :] += layer_boost
    logk = logk.reshape(-1)
    k = np.exp(logk)
    N = nx * ny * nz
    c = Case(nx=nx, ny=ny, nz=nz, kx=k.copy(), ky=k.copy(), kz=kz_ratio * k,
             poro=np.full(N, 0.2), pd=pd, name=name)
    q = np.zeros((N, 2))
    per_cell = cfl * 0.2 * 1.0 / c.dt
    iz = np.arange(nz)
    for (ix, iy) in [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]:
        cells = ix + nx * (iy + ny * iz)
        w = k[cells] / k[cells].mean()
        q[cells, 1] = per_cell * w
    c.q = q
    pcells = (nx // 2) + nx * ((ny // 2) + ny * iz)
    c.prod_cells = pcells.astype(np.int32)
    c.prod_wi = np.array([peaceman_wi(k[i], 1.0, 1.0, 1.0) for i in pcells])
    c.prod_pbh = np.zeros(nz)
    return _finish(c, 0.0, 0.2)


def config_c1() -> Case:
    """32x32 2D, sigma 1, correlation 4 cells, P_d 0.1, CFL 10, seed 1."""
    return workload_2d_corner(32, 32, 1.0, 4.0, 0.1, 10.0, 1, name="2d-32x32")


def config_c2(pd: float) -> Case:
    """512x512 2D, sigma 2, correlation 16 cells, CFL 50, seed 2."""
    return workload_2d_corner(512, 512, 2.0, 16.0, pd, 50.0, 2, name=f"2d-512x512-pd{pd}")


def config_c3(nx=128, ny=128, nz=64, seed=3) -> Case:
    """128x128x64 3D, sigma 3, correlation (16,16,4), P_d 0.5, five-spot, CFL 10."""
    return workload_3d_fivespot(nx, ny, nz, 3.0, (16.0, 16.0, 4.0), 0.5, 10.0, seed,
                                name=f"3d-{nx}x{ny}x{nz}")


# Workloads that follow a Newton sequence (the 8M-cell case and the serving
# stream) run at CFL 1: at CFL 10 the chopped Newton iteration of the 3D
# five-spot stops converging after two or three iterates and the later
# Jacobians belong to unphysical states.
SEQUENCE_CFL = 1.0


def config_c4(nx=256, ny=256, nz=128, cfl=SEQUENCE_CFL) -> Case:
    """256x256x128 3D, same statistics as the 1M-cell case, seed 4."""
    return workload_3d_fivespot(nx, ny, nz, 3.0, (16.0, 16.0, 4.0), 0.5, cfl, 4,
                                name=f"3d-{nx}x{ny}x{nz}-cfl{cfl:g}")


def serving_realization(r: int, master_seed: int = 5):
    """Realisation r of the serving stream: sigma ~ U[1,3], P_d ~ U[0,1],
    grid edge drawn from {32,48,64,96,128} (cubes), seed 1000 + r."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    sig = rng.uniform(1.0, 3.0, 64)
    pds = rng.uniform(0.0, 1.0, 64)
    edges = rng.choice(np.array([32, 48, 64, 96, 128]), 64)
    e = int(edges[r])
    return dict(nx=e, ny=e, nz=e, sigma=float(sig[r]), pd=float(pds[r]), seed=1000 + r)


def serving_case(r: int, edge_override: int | None = None, cfl: float = SEQUENCE_CFL) -> Case:
    d = serving_realization(r)
    e = edge_override or d["nx"]
    return workload_3d_fivespot(e, e, e, d["sigma"], (16.0, 16.0, 4.0), d["pd"], cfl,
                                d["seed"], name=f"serve-r{r}-{e}")


# ----------------------------------------------------------------------------
# multi-step simulations: stand-ins for the paper's 2D experiments
#
# Units: pressure Pa, length m, time day (so viscosities are in Pa day and
# rates in m^3/day); rho g in Pa/m (time does not enter it).

MILLIDARCY = 9.869233e-16        # m^2
CENTIPOISE = 1e-3 / 86400.0      # Pa day
GRAVITY = 9.81                   # m/s^2
# capillary-pressure parameter sets Ex1-Ex3 (the paper's table of P_c
# parameters): linear P_0, Brooks-Corey P_d and lambda
PC_EXAMPLES = {1: dict(p0=1e5, pd=1e6, lam=2.5),
               2: dict(p0=1e4, pd=1e5, lam=0.8),
               3: dict(p0=1e3, pd=2e4, lam=2.5)}


def _xz_case(nx, nz, hx, hy, hz, k, example, pc_model, name):
    N = nx * nz
    ex = PC_EXAMPLES[example]
    c = Case(nx=nx, ny=1, nz=nz, hx=hx, hy=hy, hz=hz, kx=k.copy(), ky=k.copy(), kz=k.copy(),
             poro=np.full(N, 0.2), mu_w=1.0 * CENTIPOISE, mu_n=10.0 * CENTIPOISE,
             rho_w=1000.0, rho_n=700.0, grav=GRAVITY, pc_model=pc_model,
             bc_lambda=ex["lam"] if pc_model == PC_BROOKS_COREY else 2.0, swr=0.0, snr=0.0,
             pd=ex["pd"] if pc_model == PC_BROOKS_COREY else ex["p0"], name=name)
    c.q = np.zeros((N, 2))
    return c


def _finish_xz(c, inlet_cell, rate, outlet_cell):
    """Inlet: a prescribed water inflow `rate` through the left boundary face
    of inlet_cell (a constant water source of that cell); outlet: a
    Dirichlet right face of outlet_cell with P_w = 0, S_w = 0.2; initial
    P_w = 1e5 Pa, S_n = 0.8."""
    c.q[inlet_cell, 0] = rate
    c.dir_cells = np.array([outlet_cell], np.int32)
    c.dir_face = np.array([FACE_XP], np.int32)
    c.dir_p = np.array([0.0])
    c.dir_s = np.array([0.8])
    return _finish(c, 1e5, 0.8)


def oil_water_xz(example, pc_model, nx=100, nz=20, seed=11, sigma=2.0, corr=(16.0, 2.0),
                 mean_mD=100.0) -> Case:
    """Stand-in for the 2D oil-water cross-section of Sec. 4.1: 762 x 15.24 m
    in the xz plane (gravity along z), nx x 1 x nz cells (7.62 x 7.62 x
    0.762 m at 100 x 20), isotropic log-normal permeability around mean_mD
    with correlation lengths corr = (x, z) cells (the SPE10 model-1 slice the
    paper uses is not available); water enters at 50 m^3/day through the left
    face of the bottom-left cell and leaves through the right face of the
    top-right cell (P_w = 0, S_w = 0.2); initial P_w = 1e5 Pa, S_n = 0.8;
    phi 0.2, mu_w 1 cP, mu_n 10 cP, rho_w 1000, rho_n 700, S_wr = S_nr = 0
    (the paper's table of input data); P_c parameters of example 1-3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    logk = gaussian_field((nz, 1, nx), (corr[1], 1.0, corr[0]), sigma, rng).reshape(-1)
    k = mean_mD * MILLIDARCY * np.exp(logk)
    c = _xz_case(nx, nz, 762.0 / nx, 7.62, 15.24 / nz, k, example, pc_model,
                 f"oil-water-xz-{nx}x{nz}-ex{example}-{'bc' if pc_model == 0 else 'lin'}")
    return _finish_xz(c, (nz - 1) * nx, 50.0, nx - 1)


# regime of the gravity box -> (P_c example, time step in days, final time)
GRAVITY_REGIMES = {"diffusion": (1, 10.0, 20.0), "advection": (2, 4.0, 8.0),
                   "strong-advection": (3, 1.0, 2.0)}


def gravity_box_xz(n, regime) -> Case:
    """Stand-in for the 2D problem with gravity of Sec. 4.2: a 20 x 20 m box
    in the xz plane, n x 1 x n cells of unit thickness, homogeneous 100 mD;
    water enters at 5 m^3/day through the left face of the top-left cell,
    the outlet is the right face of the top-right cell (P_w = 0, S_w =
    0.2); initial state as in the oil-water case; linear P_c with P_0 of
    example 1, 2 or 3 for the diffusion-, advection- and strongly
    advection-dominated regimes (the paper names P_0 = 1e4 for the
    advection case); the time step and final time of each regime are in
    GRAVITY_REGIMES."""
    ex, dt, _ = GRAVITY_REGIMES[regime]
    k = np.full(n * n, 100.0 * MILLIDARCY)
    h = 20.0 / n
    c = _xz_case(n, n, h, 1.0, h, k, ex, PC_LINEAR, f"gravity-box-{n}x{n}-{regime}")
    c = _finish_xz(c, 0, 5.0, n - 1)
    c.dt = dt
    return c


# ----------------------------------------------------------------------------
# small cases and random states for parity tests


def small_case(nx, ny, nz, seed=0, sigma=1.0, pd=0.1, pc_model=PC_BROOKS_COREY,
               wells=True, dirichlet=False, grav=0.0) -> Case:
    """Small heterogeneous case with a random state (for parity tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = nx * ny * nz
    if nz > 1:
        logk = gaussian_field((nz, ny, nx), (2.0, 3.0, 3.0), sigma, rng).reshape(-1)
    else:
        logk = gaussian_field((1, ny, nx), (1.0, 3.0, 3.0), sigma, rng).reshape(-1)
    k = np.exp(logk)
    c = Case(nx=nx, ny=ny, nz=nz, kx=k.copy(), ky=1.3 * k, kz=0.2 * k,
             poro=rng.uniform(0.1, 0.3, N), pd=pd, pc_model=pc_model, grav=grav,
             name=f"small-{nx}x{ny}x{nz}-s{seed}")
    c.q = np.zeros((N, 2))
    if wells:
        c.q[0, 1] = 2.0
        c.q[N // 3, 0] = 0.5
        pc = np.array([N - 1, N // 2], np.int32)
        c.prod_cells = pc
        c.prod_wi = np.array([peaceman_wi(k[i], 1, 1, 1) for i in pc])
        c.prod_pbh = np.array([0.0, -0.3])
    if dirichlet:
        cells, faces = [], []
        for iy in range(ny):
            for iz in range(nz):
                cells.append(0 + nx * (iy + ny * iz)); faces.append(FACE_XM)
                cells.append(nx - 1 + nx * (iy + ny * iz)); faces.append(FACE_XP)
        c.dir_cells = np.array(cells, np.int32)
        c.dir_face = np.array(faces, np.int32)
        c.dir_p = rng.normal(0.0, 1.0, len(cells))
        c.dir_s = rng.uniform(0.1, 0.9, len(cells))
    u = np.empty((N, 2))
    u[:, 0] = rng.normal(0.0, 1.0, N)
    u[:, 1] = rng.uniform(0.02, 0.98, N)
    c.u = u
    uo = u.copy()
    uo[:, 1] = np.clip(u[:, 1] + rng.normal(0.0, 0.05, N), 0.0, 1.0)
    c.u_old = uo
    return c


def random_state(case: Case, seed: int, s_lo=0.02, s_hi=0.98, p_scale=1.0) -> Case:
    """Same case, random linearisation state (P ~ N(0, p_scale), S_n ~ U)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = case.N
    u = np.empty((N, 2))
    u[:, 0] = rng.normal(0.0, p_scale, N)
    u[:, 1] = rng.uniform(s_lo, s_hi, N)
    uo = u.copy()
    uo[:, 1] = np.clip(u[:, 1] + rng.normal(0.0, 0.05, N), 0.0, 1.0)
    return case.replace(u=u, u_old=uo)


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)
