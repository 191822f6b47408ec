"""Host-side logic of bench.py (no GPU): the algorithmic byte counts the
roofline divides by, the reduction of rocprofv3 counter runs to HBM bytes
per dispatch, and the single-GPU guard."""
import csv
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _stats(rows, nnz, p_nnz, diags, dense=1):
    L = len(rows)
    pad = lambda v: list(v) + [0] * (25 - len(v))  # noqa: E731
    return SimpleNamespace(levels=[L], rows=[pad(rows)], nnz=[pad(nnz)], p_nnz=[pad(p_nnz)],
                           l0_diagonals=[diags], coarse_dense=[dense])


def test_vcycle_kernel_bytes_by_hand():
    """Level 0 in the 25-diagonal layout, level 1 a large CSR level (its g
    formed by the restriction into it), level 2 a small CSR level, level 3
    the dense coarsest; P read in ELL form with 3 slots."""
    rows = [1_000_000, 400_000, 20_000, 100]
    nnz = [25_000_000, 22_000_000, 900_000, 5_000]
    pnnz = [2_400_000, 950_000, 40_000, 0]
    st = _stats(rows, nnz, pnnz, 25)
    w = 8
    b0 = bench.vcycle_kernel_bytes(st, 0, 0, w, ell_w=3)
    n, nc = rows[0], rows[1]
    assert b0["vcycle_jacobi_guess"] == 3 * w * n
    assert b0["vcycle_pre_residual"] == 25 * w * n + 3 * w * n
    assert b0["vcycle_post_smooth"] == 25 * w * n + 4 * w * n
    # restriction reads R (= P^T: pnnz entries, nc + 1 row pointers), r, writes b_c and,
    # level 1 being a guess level, reads dinv_c and writes g_c
    assert b0["vcycle_restrict"] == 12 * pnnz[0] + 4 * (nc + 1) + w * n + w * nc + 2 * w * nc
    # ELL prolongation: 3 slots of (value, column) per row, x_c gather, dinv, b -> y
    assert b0["vcycle_prolong"] == 12 * 3 * n + w * nc + 3 * w * n
    b1 = bench.vcycle_kernel_bytes(st, 0, 1, w, ell_w=0)
    n1, nc1 = rows[1], rows[2]
    assert "vcycle_jacobi_guess" not in b1  # formed by the restriction into level 1
    assert b1["vcycle_pre_residual"] == 12 * nnz[1] + 4 * (n1 + 1) + 3 * w * n1
    assert b1["vcycle_restrict"] == 12 * pnnz[1] + 4 * (nc1 + 1) + w * n1 + w * nc1
    assert b1["vcycle_prolong"] == 12 * pnnz[1] + 4 * (n1 + 1) + w * nc1 + 3 * w * n1
    assert bench.vcycle_kernel_bytes(st, 0, 3, w) == {"vcycle_coarse": 8 * 100 * 100 + 2 * w * 100}
    assert bench.guess_level(st, 0, 0) and bench.guess_level(st, 0, 1)
    assert not bench.guess_level(st, 0, 2) and not bench.guess_level(st, 0, 3)
    # the kernels rocprofv3 names for the timers
    assert bench.kernel_symbol(st, 0, 0, "vcycle_pre_residual") == "k_dia_pre2<double, 25>"
    assert bench.kernel_symbol(st, 0, 1, "vcycle_post_smooth") == "k_vc_posts<double, 8>"
    assert bench.kernel_symbol(st, 0, 1, "vcycle_pre_residual") == "k_vc_pre_gs<double, 8>"
    assert bench.kernel_symbol(st, 0, 2, "vcycle_post_smooth") == "k_vc_post<double, 8>"
    assert bench.kernel_symbol(st, 0, 2, "vcycle_pre_residual") == "k_vc_pre<double, 8>"
    assert bench.kernel_symbol(st, 0, 0, "vcycle_restrict") == "k_vc_restrict_gs<double, 1>"
    assert bench.kernel_symbol(st, 0, 1, "vcycle_restrict") == "k_csr_spmv"
    assert bench.kernel_symbol(st, 0, 0, "vcycle_prolong", 3) == "k_vc_prolong_ell2<double, 3>"
    # a large level of long rows (80 entries: 16 lanes) keeps the row kernels
    st16 = _stats([1_000_000, 100_000, 100], [25_000_000, 8_000_000, 5_000],
                  [2_400_000, 300_000, 0], 25)
    assert bench.kernel_symbol(st16, 0, 1, "vcycle_pre_residual") == "k_vc_pre_g<double, 16>"
    assert bench.kernel_symbol(st16, 0, 1, "vcycle_post_smooth") == "k_vc_post<double, 16>"
    # launch sizes: two rows per thread in the diagonal kernels, lanes per row in CSR ones
    assert bench.launch_threads(st, 0, 0, "vcycle_post_smooth") == 500_224  # 500,000 rounded up
    assert bench.launch_threads(st, 0, 1, "vcycle_post_smooth") == 400_000 * 8


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        wr = csv.writer(f)
        wr.writerow(header)
        wr.writerows(rows)


def test_reduce_traffic_scales_counters_by_the_copy(tmp_path, monkeypatch):
    """FETCH_SIZE / WRITE_SIZE per dispatch of the listed kernel, scaled by
    what the same counters read for the 512 MiB copy, and the kernel-trace
    durations of the same dispatches."""
    d = tmp_path
    sym, grid = "k_vc_posts<double, 8>", 3_070_720
    name = f"void tpf::(anonymous namespace)::{sym}(int, int const*)"
    copy = "__amd_rocclr_copyBuffer"
    _write_csv(str(d / "pmc_fetch" / "fetch_counter_collection.csv"),
               ["Kernel_Name", "Grid_Size", "Counter_Value"],
               [[copy, 1 << 20, 262144.0], [name, grid, 100000.0], [name, grid, 110000.0],
                [name, 2048, 5.0]])
    _write_csv(str(d / "pmc_write" / "write_counter_collection.csv"),
               ["Kernel_Name", "Grid_Size", "Counter_Value"],
               [[copy, 1 << 20, 524288.0], [name, grid, 3000.0], [name, grid, 3000.0]])
    _write_csv(str(d / "prof" / "bench_kernel_trace.csv"),
               ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp",
                "End_Timestamp"],
               [[name, grid, 1, 1, 1000, 77000], [name, grid, 1, 1, 200000, 275000],
                [name, 2048, 1, 1, 0, 10]])
    alg = 266_497_228
    (d / "traffic_spec.json").write_text(json.dumps(
        {"vcycle_post_smooth[Schur,l1]": [sym, grid, alg, bench.KERNEL_SOURCES["k_vc_posts"]]}))
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(out))
    rec = bench.reduce_traffic(str(d))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    k = rec["kernels"]["vcycle_post_smooth[Schur,l1]"]
    assert k["dispatches"] == 2 and k["trace_dispatches"] == 2
    hbm = 1024 * (2.0 * 105000.0 + 1.0 * 3000.0)
    assert k["hbm_bytes_per_dispatch"] == int(hbm)
    assert k["traffic_over_algorithmic"] == pytest.approx(hbm / alg, abs=1e-4)
    assert k["trace_avg_us"] == pytest.approx(75.5)
    assert k["source_sha256"] == bench.kernel_digest(bench.KERNEL_SOURCES["k_vc_posts"])
    # the stored file feeds the bench line while the kernel's source is unchanged
    assert bench.stored_traffic("vcycle_post_smooth[Schur,l1]", sym) == round(hbm)
    assert bench.stored_traffic("vcycle_post_smooth[Schur,l1]", "k_vc_posts<double, 16>") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
