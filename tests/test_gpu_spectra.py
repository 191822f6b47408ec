"""Sec. 4.3 eigenvalue study on the GPU: J M^{-1} with exact inner solves
(one-level hierarchies, dense coarsest inverse; CPR's first stage stays block
ILU(0)) formed column by column from the GPU's preconditioner, against the
oracle's dense J M^{-1} built with sparse LU from the same inputs, for the
diffusion- (Ex1) and advection-dominated (Ex2) oil-water stand-in: entries
within 1e-8 of max|.|, and the spectra's extreme moduli within 1e-4."""
import numpy as np
import pytest

from oracle import spectra, tpfa
from paper_1611_00127_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1611_00127_amd import driver, tpf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tpf.init()
    return driver, tpf, torch


@pytest.mark.parametrize("example", [1, 2])
@pytest.mark.parametrize("kind", ["bf", "cpr1", "cpr2"])
def test_preconditioned_spectrum_matches_oracle(gpu, kind, example):
    driver, tpf, torch = gpu
    c = inputs.oil_water_xz(example, inputs.PC_LINEAR, nx=16, nz=4)
    print(f"[spectra] ex{example} {kind}", flush=True)
    g = driver.GpuCase(c)
    g.assemble()
    M = driver.GpuPrecond(kind, **driver.exact_inner_opts(c.N))
    M.setup(g)
    A = driver.preconditioned_matrix(g, M)
    rp, ci, v = tpfa.jacobian(c, c.u, c.u_old)
    Ao = spectra.preconditioned_matrix(kind, rp, ci, v, (c.nx, c.ny, c.nz))
    err = float(np.max(np.abs(A - Ao)) / np.max(np.abs(Ao)))
    s, so = spectra.summary(np.linalg.eigvals(A)), spectra.summary(np.linalg.eigvals(Ao))
    print(f"  max entry diff {err:.1e}; |lambda| in [{s['min_abs']:.4f}, {s['max_abs']:.4f}] "
          f"(oracle [{so['min_abs']:.4f}, {so['max_abs']:.4f}])", flush=True)
    assert err <= 1e-8
    for k in ("min_abs", "max_abs"):
        assert abs(s[k] - so[k]) <= 1e-4 * so[k]
    M.close()
    g.close()
