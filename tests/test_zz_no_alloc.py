"""tpf_solve_noalloc against tpf_solve, through the C ABI.

The allocation-free solve keeps its Krylov workspace in the library's fixed
per-GPU array.  It must give the same iterates as tpf_solve (the same
kernels in the same order: bitwise equal x, equal iteration count and
residuals), on two calls in a row, the second on a smaller system (the
array keeps the first call's contents), and it must request no device
memory: each solve runs on a fresh stream, where the library's block cache
(kept per stream) holds nothing, so any workspace allocation would reach
torch's allocator.
"""
import numpy as np
import pytest

from oracle import tpfa
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


def _fresh_stream_solve(torch, tpf, fn, g, M, b):
    """Runs fn (tpf_solve or tpf_solve_noalloc) on a new stream; returns
    the solution, the solve info and the allocator requests it made."""
    x = torch.full_like(b, np.nan)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    before = tpf.allocator_calls()
    info = fn(g.J, M.M if M is not None else None, b, x, stream=s)
    calls = tpf.allocator_calls() - before
    torch.cuda.synchronize()
    return x, info, calls


CASES = [  # (name, case, preconditioner, precision); the second system is smaller
    ("2d-48x40 bf fp64", lambda: inputs.workload_2d_corner(48, 40, 1.0, 4.0, 0.1, 10.0, 11), "bf", 0),
    ("2d-20x12 bf fp64", lambda: inputs.workload_2d_corner(20, 12, 1.0, 4.0, 0.1, 10.0, 12), "bf", 0),
    ("3d-24x20x8 bf fp32", lambda: inputs.config_c3(24, 20, 8), "bf", 1),
    ("2d-16x16 cpr1 fp64", lambda: inputs.workload_2d_corner(16, 16, 1.0, 4.0, 0.1, 10.0, 13), "cpr1", 0),
]


def test_noalloc_matches_solve_two_calls(gpu):
    """Consecutive calls (the second on a smaller system, then a 3D FP32
    V-cycle case and a CPR1 case): x bitwise equal to tpf_solve's, equal
    iterations and residuals, relres <= 1e-8 against the oracle's own
    Jacobian product, and no allocator request."""
    driver, tpf, torch = gpu
    for name, make, kind, precision in CASES:
        c = make()
        print(f"[noalloc] {name}: {2 * c.N} unknowns", flush=True)
        g = driver.GpuCase(c)
        g.assemble()
        M = driver.GpuPrecond(kind, precision)
        M.setup(g)
        b = g.rhs().contiguous()
        x_ref, i_ref, _ = _fresh_stream_solve(torch, tpf, tpf.tpf_solve, g, M, b)
        x_na, i_na, calls = _fresh_stream_solve(torch, tpf, tpf.tpf_solve_noalloc, g, M, b)
        assert calls == 0, f"{name}: {calls} allocator requests"
        assert i_na.status == tpf.TPF_CONVERGED == i_ref.status
        assert i_na.iterations == i_ref.iterations, (i_na.iterations, i_ref.iterations)
        assert i_na.relres_true == i_ref.relres_true
        assert torch.equal(x_na, x_ref), float((x_na - x_ref).abs().max())
        rp, ci, vals = g.bcsr_numpy()
        J = tpfa.bcsr_matrix(rp, ci, vals)
        bn, xs = b.cpu().numpy(), x_na.cpu().numpy()
        assert np.linalg.norm(bn - J @ xs) <= 1e-8 * np.linalg.norm(bn)
        M.close()
        g.close()


def test_noalloc_unpreconditioned_and_limits(gpu):
    """M = NULL (identity) matches tpf_solve; a system whose workspace
    exceeds the fixed array, and a restart above 64, are rejected with
    TPF_ERR_INVALID_ARG before any device work."""
    driver, tpf, torch = gpu
    c = inputs.workload_2d_corner(12, 10, 1.0, 4.0, 0.1, 10.0, 14)
    g = driver.GpuCase(c)
    g.assemble()
    b = g.rhs().contiguous()
    x_ref, i_ref, _ = _fresh_stream_solve(torch, tpf, tpf.tpf_solve, g, None, b)
    x_na, i_na, calls = _fresh_stream_solve(torch, tpf, tpf.tpf_solve_noalloc, g, None, b)
    assert calls == 0
    assert i_na.iterations == i_ref.iterations and torch.equal(x_na, x_ref)
    x = torch.empty_like(b)
    with pytest.raises(tpf.TpfError) as e:
        tpf.tpf_solve_noalloc(g.J, None, b, x, restart=65)
    assert e.value.code == -1
    g.close()
    big = inputs.workload_2d_corner(512, 288, 1.0, 4.0, 0.1, 10.0, 15)  # 294,912 unknowns
    g = driver.GpuCase(big)
    b = torch.ones(2 * big.N, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    with pytest.raises(tpf.TpfError) as e:
        tpf.tpf_solve_noalloc(g.J, None, b, x)
    assert e.value.code == -1 and "at most" in str(e.value)
    # restart 10 needs about 22 doubles per unknown: it fits
    g.assemble()
    b = g.rhs().contiguous()
    info = tpf.tpf_solve_noalloc(g.J, None, b, x, restart=10, maxit=20)
    info_ref = tpf.tpf_solve(g.J, None, b, (x_ref := torch.empty_like(b)), restart=10, maxit=20)
    assert info.iterations == info_ref.iterations == 20 and torch.equal(x, x_ref)
    g.close()
