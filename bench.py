"""Benchmark: time to a 1e-8 relative residual for a Newton Jacobian of the
3D 128x128x64 heterogeneous workload (1,048,576 cells, 2.1M unknowns),
block-factorisation preconditioner (Algorithm 3) with AMG V-cycles on A_ss
and S~, right-preconditioned FGMRES(30).

The headline Jacobian is taken at Newton iterate 1 of the first time step,
where every face has a pressure difference: A_ps carries the upwind
coupling of the saturation equation.  At the initial condition (uniform
pressure) every face is an upwind tie, A_ps is diagonal and most stored
entries of S~ are zero; that state is timed beside it in FP64.

One step = assembly of residual and Jacobian + full preconditioner setup
(block views, S~, two AMG hierarchies) + FGMRES to ||b - Jx|| <= 1e-8 ||b||,
with every input resident in HBM before the timed region.  The FP64 form is
the primary value; the FP32-V-cycle form (hierarchies stored and cycled in
FP32 inside the FP64 FGMRES) is timed the same way and reported beside it.

Prints one JSON line (rank 0, N = 1 GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DS_MAX = 0.2  # Newton saturation chop
METRIC = "time-to-1e-8 solve (FP64 vs FP32 V-cycle), V-cycle HBM GB/s, p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=str, default="128x128x64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-grid", type=str, default="64x64x32",
                    help="grid of the oracle's bounded sample")
    ap.add_argument("--state", choices=["newton1", "initial"], default="newton1",
                    help="linearisation state of the headline Jacobian (the other state is "
                         "timed in FP64 beside it)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="first run a plain device copy of this many MiB (calibrates the "
                         "FETCH_SIZE/WRITE_SIZE counters of a profiler run)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the 256x256x128 Newton sequence (10 Jacobians, rebuild vs reuse, "
                         "FP64 vs FP32, HBM footprint)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay recorded V-cycle graphs instead of launching every kernel")
    ap.add_argument("--serve-full", action="store_true",
                    help="the full stream: 64 realizations x 16 Newton-step requests, "
                         "grids up to 128^3")
    ap.add_argument("--serve-realizations", type=int, default=32,
                    help="realizations of the serving stream (the first R of its 64)")
    ap.add_argument("--serve-requests", type=int, default=8, help="requests per realization")
    ap.add_argument("--serve-max-edge", type=int, default=128,
                    help="grid edges drawn above this are clamped to it (128: none)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0,
                    help="HBM admission budget of the serving engine")
    ap.add_argument("--serve-active", type=int, default=8, help="requests in flight")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="Poisson arrival rate as a fraction of the sequential FP64 throughput")
    ap.add_argument("--study", choices=["c2", "newton", "simulate", "spectra", "amg-variants"],
                    default=None,
                    help="instead of the benchmark line, print one JSON line for a study: "
                         "c2 = first Jacobian of the 512x512 workload for P_d in {0, 0.1, 1} and "
                         "all four preconditioners; newton = 10 consecutive Newton Jacobians of "
                         "the 256x256x128 workload, BF, rebuild vs reuse x FP64 vs FP32; "
                         "simulate = multi-step runs of the 2D stand-ins, all preconditioners; "
                         "spectra = eigenvalues of J M^-1 with exact inner solves; "
                         "amg-variants = the 128x128x64 Jacobian at Newton iterate 1 with the "
                         "paper's AMG components (CLJP, classical interpolation, multicolour "
                         "Gauss-Seidel) against the defaults")
    ap.add_argument("--study-grid", type=str, default=None,
                    help="grid of the study workload (default: 512x512 / 256x256x128)")
    ap.add_argument("--traffic-spec", type=str, default=None,
                    help="write, for the heaviest V-cycle kernels of the FP64 form, the kernel "
                         "symbol, launch size, algorithmic bytes and source functions to this "
                         "JSON file (read by --reduce-traffic)")
    ap.add_argument("--reduce-traffic", type=str, default=None, metavar="DIR",
                    help="no GPU work: reduce the rocprofv3 outputs under DIR (prof/ kernel "
                         "trace, pmc_fetch/ and pmc_write/ counters, traffic_spec.json) to the "
                         "per-kernel HBM traffic file under profiles/")
    return ap.parse_args()


def lanes_per_row(n, nnz):
    """Lanes per row the CSR row kernels use: about eight entries per lane."""
    avg = nnz / n if n else 1.0
    lanes = 1
    while lanes < 64 and 8 * lanes < avg:
        lanes <<= 1
    return lanes


GUESS_ROWS = 65536  # CSR levels from this size (above the coarsest) cycle from g = D^-1 b


def guess_level(st, h, l):
    """Whether level l's pre-smoothing gathers a formed g = D^-1 b: the
    diagonal-layout level 0, and CSR levels of at least GUESS_ROWS rows above
    the coarsest (whose g the restriction into them forms)."""
    if l == int(st.levels[h]) - 1:
        return False
    return bool(l == 0 and int(st.l0_diagonals[h])) or int(st.rows[h][l]) >= GUESS_ROWS


def vcycle_kernel_bytes(st, h, l, w, ell_w=0):
    """Algorithmic bytes per launch of each V-cycle kernel of level l of
    hierarchy h (value width w): every array the kernel must touch, counted
    once -- the operator (diagonal layout: K * n values; CSR: values, int32
    columns, row pointers; P in ELL form: ell_w slots per row) and each dense
    vector.  Keys are the kernel-timer names without the [hierarchy,level]
    suffix."""
    n, nnz = int(st.rows[h][l]), int(st.nnz[h][l])
    last = l == int(st.levels[h]) - 1
    K = int(st.l0_diagonals[h]) if l == 0 else 0
    mat = w * K * n if K else (w + 4) * nnz + 4 * (n + 1)
    if last:
        if st.coarse_dense[h]:
            return {"vcycle_coarse": 8 * n * n + 2 * w * n}  # FP64 inverse, b, x
        return {"vcycle_coarse": mat + 3 * w * n}           # two sweeps: dinv, b, x
    nc, pnnz = int(st.rows[h][l + 1]), int(st.p_nnz[h][l])
    tr = (w + 4) * pnnz
    out = {}
    if l == 0 and guess_level(st, h, 0):
        out["vcycle_jacobi_guess"] = 3 * w * n                 # dinv, b -> g
    out["vcycle_pre_residual"] = mat + 3 * w * n               # g (or dinv), b -> r
    # R, r -> b_c (and dinv_c -> g_c when the coarse level cycles from g_c)
    out["vcycle_restrict"] = (tr + 4 * (nc + 1) + w * n + w * nc
                              + (2 * w * nc if guess_level(st, h, l + 1) else 0))
    ptr = (w + 4) * ell_w * n if ell_w else tr + 4 * (n + 1)
    out["vcycle_prolong"] = ptr + w * nc + 3 * w * n           # x_c, dinv, b -> y
    out["vcycle_post_smooth"] = mat + 4 * w * n                # dinv, b, y -> x
    return out


STREAM_LANES = 8  # large CSR levels with rows of up to this many lanes take the streamed kernels


def kernel_symbol(st, h, l, timer, ell_w=0):
    """Name of the HIP kernel behind a V-cycle timer (as rocprofv3 lists it)."""
    n, nnz = int(st.rows[h][l]), int(st.nnz[h][l])
    K = int(st.l0_diagonals[h]) if l == 0 else 0
    if timer == "vcycle_pre_residual":
        if K:
            return f"k_dia_pre{'2' if n % 2 == 0 else ''}<double, {K}>"
        lpr = lanes_per_row(n, nnz)
        g = ("_gs" if lpr <= STREAM_LANES else "_g") if guess_level(st, h, l) else ""
        return f"k_vc_pre{g}<double, {lpr}>"
    if timer == "vcycle_post_smooth":
        if K:
            return f"k_dia_post{'2' if n % 2 == 0 else ''}<double, {K}>"
        lpr = lanes_per_row(n, nnz)
        s = "s" if guess_level(st, h, l) and lpr <= STREAM_LANES else ""
        return f"k_vc_post{s}<double, {lpr}>"
    if timer == "vcycle_prolong":
        if ell_w:
            return f"k_vc_prolong_ell{'2' if n % 2 == 0 else ''}<double, {ell_w}>"
        return f"k_vc_prolong<double, {lanes_per_row(n, int(st.p_nnz[h][l]))}>"
    if timer == "vcycle_restrict":
        if guess_level(st, h, l + 1):
            nc = int(st.rows[h][l + 1])
            lpr = lanes_per_row(nc, int(st.p_nnz[h][l]))
            kind = "gs" if lpr <= STREAM_LANES else "guess"
            return f"k_vc_restrict_{kind}<double, {lpr}>"
        return "k_csr_spmv"
    if timer == "vcycle_jacobi_guess":
        return "k_jacobi_guess<double>"
    return "k_dense_gemv<double>" if st.coarse_dense[h] else "k_vc_two_sweeps<double>"


HIER_TAGS = {"bf": ["Ass", "Schur"]}
HIER_NAMES = {"Ass": "A_ss", "Schur": "S~"}


def vcycle_table(tpf, st, tags, w=8, ell_w=0):
    """Per level of each hierarchy: rows, nnz, P entries, and for every
    V-cycle kernel its launches, mean time (HIP events) and algorithmic
    GB/s; per hierarchy the V-cycle's bytes and kernel time."""
    out, kernels = [], []
    for h, tag in enumerate(tags):
        levels, tot_b, tot_ms, cycles = [], 0, 0.0, 0
        for l in range(int(st.levels[h])):
            kb = vcycle_kernel_bytes(st, h, l, w, ell_w)
            row = {"level": l, "rows": int(st.rows[h][l]), "nnz": int(st.nnz[h][l]),
                   "p_nnz": int(st.p_nnz[h][l]), "kernels": {}}
            lb, lms = 0, 0.0
            for timer, b in kb.items():
                cnt, ms = tpf.tpf_kernel_stats(f"{timer}[{tag},l{l}]")
                if not cnt:
                    continue
                if l == 0 and timer == "vcycle_pre_residual":
                    cycles = cnt
                avg_us = 1e3 * ms / cnt
                row["kernels"][timer] = {"launches": cnt, "avg_us": round(avg_us, 2),
                                         "bytes": b, "gbs": round(b / (avg_us * 1e3), 1)}
                kernels.append(dict(hier=tag, level=l, timer=timer, launches=cnt, total_ms=ms,
                                    bytes=b, symbol=kernel_symbol(st, h, l, timer, ell_w)))
                lb += b * cnt
                lms += ms
            row["share_of_cycle_bytes"] = lb
            levels.append(row)
            tot_b += lb
            tot_ms += lms
        for row in levels:
            row["share_of_cycle_bytes"] = round(row["share_of_cycle_bytes"] / max(tot_b, 1), 4)
        per_cycle_b = tot_b / max(cycles, 1)
        per_cycle_ms = tot_ms / max(cycles, 1)
        out.append({"hierarchy": HIER_NAMES.get(tag, tag), "levels": levels,
                    "vcycles": cycles, "bytes_per_vcycle": int(per_cycle_b),
                    "kernel_ms_per_vcycle": round(per_cycle_ms, 4),
                    "kernel_gbs": round(per_cycle_b / (per_cycle_ms * 1e6), 1) if cycles else None})
    return out, kernels


def vcycle_wall(torch, tpf, M, h, n, reps=20, fp32=False):
    """Mean wall time of one V-cycle of hierarchy h, from HIP events around
    `reps` back-to-back cycles on the current stream (launch gaps included)."""
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    for _ in range(2):
        tpf.tpf_precond_vcycle(M.M, h, b, x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        tpf.tpf_precond_vcycle(M.M, h, b, x)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


CSRC = os.path.join(ROOT, "paper_1611_00127_amd", "csrc")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "vcycle_hbm_traffic_3d_128x128x64.json")


def kernel_digest(names):
    """sha256 of the source text of the named device functions, each given
    as "file:function" under csrc/ (from the function's name to the first
    closing brace at column 0): identifies the kernel build that a stored
    counter measurement belongs to."""
    import hashlib
    import re
    h = hashlib.sha256()
    for item in names:
        fname, nm = item.split(":")
        text = open(os.path.join(CSRC, fname)).read()
        m = re.search(r"\b" + re.escape(nm) + r"\(", text)
        if not m:
            return None
        start = text.rfind("\n", 0, m.start()) + 1
        end = text.find("\n}\n", m.end())
        if end < 0:
            return None
        h.update(text[start:end + 3].encode())
    return h.hexdigest()


# source functions whose text identifies each V-cycle kernel family's build
STREAM_SOURCES = ["amg.hip:xcd_contiguous_block", "amg.hip:wave_lds_sync",
                  "amg.hip:stream_window", "amg.hip:stream_rows_dot", "amg.hip:stream_first_row"]
KERNEL_SOURCES = {
    "k_vc_post": ["amg.hip:k_vc_post", "linalg_dev.hpp:row_dot"],
    "k_vc_posts": STREAM_SOURCES + ["amg.hip:k_vc_posts"],
    "k_vc_pre_gs": STREAM_SOURCES + ["amg.hip:k_vc_pre_gs"],
    "k_vc_pre_g": ["amg.hip:k_vc_pre_g", "linalg_dev.hpp:row_dot"],
    "k_vc_pre": ["amg.hip:k_vc_pre", "linalg_dev.hpp:row_dot"],
    "k_dia_pre2": ["amg.hip:clampi", "amg.hip:xcd_contiguous_block", "amg.hip:k_dia_pre2"],
    "k_dia_post2": ["amg.hip:clampi", "amg.hip:xcd_contiguous_block", "amg.hip:k_dia_post2"],
}

# rocprofv3 runs whose outputs --reduce-traffic reads; <repo> is the repository
# root and <out> the folder later given to --reduce-traffic
TRAFFIC_COMMANDS = [
    "cd /tmp && export TMPDIR=/tmp",
    "rocprofv3 --kernel-trace --stats --output-format csv -d <out>/prof -o bench -- python3 "
    "<repo>/bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-serve --no-c4",
    "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pmc_fetch -o fetch -- python3 "
    "<repo>/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-serve --no-c4 --copy-probe 512 "
    "--traffic-spec <out>/traffic_spec.json",
    "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/pmc_write -o write -- python3 "
    "<repo>/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-serve --no-c4 --copy-probe 512",
    "python bench.py --reduce-traffic <out>   (writes this file)",
]


def launch_threads(st, h, l, timer):
    """Threads in the launch grid of a V-cycle kernel (256-thread work-groups):
    how rocprofv3 tells one level's dispatches of a kernel from another's."""
    n, nnz = int(st.rows[h][l]), int(st.nnz[h][l])
    K = int(st.l0_diagonals[h]) if l == 0 else 0
    if K and timer in ("vcycle_pre_residual", "vcycle_post_smooth"):
        work = n // 2 if n % 2 == 0 else n
    else:
        work = n * lanes_per_row(n, nnz)
    return -(-work // 256) * 256


def write_traffic_spec(path, st, kern64, top=4):
    """The `top` V-cycle kernels of the FP64 form by summed time whose family
    has listed sources: timer -> [symbol, launch threads, algorithmic bytes,
    source functions]."""
    spec = {}
    for k in sorted(kern64, key=lambda k: -k["total_ms"]):
        fam = k["symbol"].split("<")[0]
        if fam not in KERNEL_SOURCES:
            continue
        h = HIER_TAGS["bf"].index(k["hier"])
        timer = f"{k['timer']}[{k['hier']},l{k['level']}]"
        spec[timer] = [k["symbol"], launch_threads(st, h, k["level"], k["timer"]), k["bytes"],
                       KERNEL_SOURCES[fam]]
        if len(spec) == top:
            break
    with open(path, "w") as f:
        json.dump(spec, f, indent=1)


def reduce_traffic(d):
    """Per-kernel HBM traffic from the rocprofv3 runs of TRAFFIC_COMMANDS:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each listed kernel's
    dispatches at its level's launch size, each scaled by what the counter
    reads for the 512 MiB device copy of the same run, and the kernel-trace
    durations of the same dispatches.  Writes TRAFFIC_JSON."""
    import collections
    import csv

    def counters(path):
        out = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            out[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        return out

    fetch = counters(os.path.join(d, "pmc_fetch", "fetch_counter_collection.csv"))
    write = counters(os.path.join(d, "pmc_write", "write_counter_collection.csv"))

    def copy_kib(c):
        return max(max(v) for k, v in c.items() if k[0] == "__amd_rocclr_copyBuffer")

    moved = 512 * 1024  # KiB read and written by the copy
    fk, wk = copy_kib(fetch), copy_kib(write)
    fs, ws = moved / fk, moved / wk
    trace = collections.defaultdict(list)
    for r in csv.DictReader(open(os.path.join(d, "prof", "bench_kernel_trace.csv"))):
        g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        trace[(r["Kernel_Name"], g)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    spec = json.load(open(os.path.join(d, "traffic_spec.json")))
    out = {"workload": "3d-128x128x64 BF at Newton iterate 1, FP64 V-cycle kernels of the "
                       "heaviest summed time",
           "fetch_scale": round(fs, 6), "write_scale": round(ws, 6),
           "calibration": f"one 512 MiB device-to-device copy (torch copy_ -> "
                          f"__amd_rocclr_copyBuffer) in the same runs: FETCH_SIZE {fk} KiB, "
                          f"WRITE_SIZE {wk} KiB for {moved} KiB moved each way",
           "commands": TRAFFIC_COMMANDS,
           "method": "per kernel: dispatches of that symbol whose grid has the stated number "
                     "of threads (the level's launch); fetch/write = mean FETCH_SIZE / "
                     "WRITE_SIZE (KiB) per dispatch; HBM bytes = 1024 (fetch_scale * fetch + "
                     "write_scale * write); trace_* = durations of the same dispatches in the "
                     "kernel trace",
           "kernels": {}}
    for timer, (sym, grid, alg, dig) in spec.items():
        keys = [k for k in fetch if k[1] == grid and sym in k[0]]
        if len(keys) != 1:
            raise SystemExit(f"{len(keys)} kernels named {sym} with {grid} threads in the "
                             f"counter runs")
        key = keys[0]
        fv, wv = fetch[key], write[key]
        tv = trace.get(key, [])
        f_avg, w_avg = sum(fv) / len(fv), sum(wv) / len(wv)
        hbm = (f_avg * fs + w_avg * ws) * 1024
        out["kernels"][timer] = {
            "symbol": sym, "grid_threads": grid, "digest_of": dig,
            "source_sha256": kernel_digest(dig), "dispatches": len(fv),
            "fetch_kib_per_dispatch": round(f_avg, 2), "write_kib_per_dispatch": round(w_avg, 2),
            "algorithmic_bytes_per_dispatch": alg, "hbm_bytes_per_dispatch": int(hbm),
            "traffic_over_algorithmic": round(hbm / alg, 4), "trace_dispatches": len(tv),
            "trace_avg_us": round(sum(tv) / len(tv) / 1e3, 2) if tv else None,
            "trace_min_us": round(min(tv) / 1e3, 2) if tv else None,
            "trace_max_us": round(max(tv) / 1e3, 2) if tv else None}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


def stored_traffic(timer, symbol):
    """HBM bytes per launch of the kernel behind V-cycle timer `timer` (e.g.
    "vcycle_post_smooth[Schur,l1]") from the committed FETCH_SIZE /
    WRITE_SIZE measurement (scaled by its copy-kernel calibration), or None
    when there is none, it is of another kernel, or the kernel's source has
    changed since."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    rec = json.load(open(TRAFFIC_JSON))
    k = rec["kernels"].get(timer)
    if (k is None or k["symbol"] != symbol
            or k["source_sha256"] != kernel_digest(k["digest_of"])):
        return None
    kib = (k["fetch_kib_per_dispatch"] * rec["fetch_scale"]
           + k["write_kib_per_dispatch"] * rec["write_scale"])
    return int(round(kib * 1024))


def run_form(torch, tpf, driver, g, precision, steps, warmup, timing):
    """Times `steps` full steps (assemble + setup + solve) of one precision."""
    M = driver.GpuPrecond("bf", precision)
    x = torch.empty(2 * g.N, dtype=torch.float64, device="cuda")
    b = g.R  # J x = F: the Newton step is -x (same solve as with -F)
    infos, t_asm, t_set, t_sol = [], [], [], []

    def one_step():
        t0 = time.perf_counter()
        g.assemble()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        M.setup(g)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        info = driver.solve(g, M, b, x, rtol=1e-8, restart=30, maxit=1000)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return info, (t1 - t0, t2 - t1, t3 - t2)

    for _ in range(warmup):
        one_step()
    if timing:
        tpf.tpf_kernel_stats_reset()
        tpf.tpf_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info, (a, s, v) = one_step()
        infos.append(info)
        t_asm.append(a)
        t_set.append(s)
        t_sol.append(v)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    if timing:
        tpf.tpf_kernel_timing(False)
    st = M.stats()
    res = dict(ms_per_step=1e3 * total / steps, assemble_ms=1e3 * float(np.median(t_asm)),
               setup_ms=1e3 * float(np.median(t_set)), solve_ms=1e3 * float(np.median(t_sol)),
               iterations=[int(i.iterations) for i in infos],
               relres_true=max(float(i.relres_true) for i in infos),
               converged=all(i.status == tpf.TPF_CONVERGED for i in infos),
               levels=[int(st.levels[h]) for h in range(st.n_hier)],
               op_complexity=[round(float(st.operator_complexity[h]), 3) for h in range(st.n_hier)],
               l0_nnz=[int(st.nnz[h][0]) for h in range(st.n_hier)],
               l0_rows=[int(st.rows[h][0]) for h in range(st.n_hier)],
               l0_diagonals=[int(st.l0_diagonals[h]) for h in range(st.n_hier)],
               rows_per_level=[[int(st.rows[h][l]) for l in range(st.levels[h])]
                               for h in range(st.n_hier)],
               coarse_dense=[int(st.coarse_dense[h]) for h in range(st.n_hier)],
               precond_mib=st.device_bytes / 2 ** 20)
    return M, x, res


SETUP_PHASES = ("strength", "coarsen", "interp", "transpose", "galerkin", "finish")


def setup_breakdown(torch, tpf, driver, g, precision):
    """One more full BF setup (after a warm-up one) with each phase bracketed
    by HIP events on its stream: block extraction, S~, and per hierarchy
    (per level and summed over the levels) strength graph, coarsening,
    interpolation, transpose, Galerkin product, and finishing the levels (smoother
    diagonals, FP32 copies, level-0 diagonal layout, coarsest inverse).  The
    two hierarchies are built concurrently on two streams, so their phases
    overlap in time.  Also the number of host round trips the setup makes."""
    M = driver.GpuPrecond("bf", precision)
    M.setup(g)
    torch.cuda.synchronize()
    tpf.tpf_kernel_stats_reset()
    tpf.tpf_kernel_timing(True)
    t0 = time.perf_counter()
    M.setup(g)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tpf.tpf_kernel_timing(False)
    out = {"wall_ms_with_timers": round(1e3 * wall, 2),
           "host_round_trips": int(tpf.tpf_kernel_stats("host_syncs")[0])}
    for name in ("setup_blocks", "setup_schur"):
        out[name[6:] + "_ms"] = round(tpf.tpf_kernel_stats(name)[1], 3)
    st = M.stats()
    for h, tag in enumerate(HIER_TAGS["bf"]):
        per_level = []
        for l in range(int(st.levels[h])):
            rec = {ph: round(tpf.tpf_kernel_stats(f"setup_{ph}[{tag},l{l}]")[1], 3)
                   for ph in SETUP_PHASES if ph != "finish"}
            if any(rec.values()):  # the coarsest level has no phases (or only the first two)
                per_level.append(rec)
        rec = {ph + "_ms": round(sum(p[ph] for p in per_level), 3)
               for ph in SETUP_PHASES if ph != "finish"}
        rec["finish_ms"] = round(tpf.tpf_kernel_stats(f"setup_finish[{tag}]")[1], 3)
        rec["per_level_ms"] = per_level
        out[HIER_NAMES[tag]] = rec
    tpf.tpf_kernel_stats_reset()
    M.close()
    return out


def kernel_table(tpf, names):
    out = {}
    for n in names:
        cnt, ms = tpf.tpf_kernel_stats(n)
        if cnt:
            out[n] = (cnt, ms)
    return out


def host_info():
    """CPU model and logical CPU count of the host running the benchmark."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline(grid, state):
    """The oracle (unmodified) on a bounded sample: the same workload family on
    a smaller grid, one full step (assemble + BF setup + FGMRES to 1e-8) at
    the same linearisation state, BLAS limited to one thread.  For the
    Newton-iterate-1 state the oracle first takes its own first Newton step
    (untimed).  Returns the time, the solve record, the sample case and the
    oracle's solution of J x = -F there."""
    from threadpoolctl import threadpool_limits

    from oracle import newton
    from paper_1611_00127_amd import inputs
    nx, ny, nz = (int(v) for v in grid.split("x"))
    c = inputs.config_c3(nx, ny, nz)
    with threadpool_limits(limits=1):
        if state == "newton1":
            x0, _, _ = newton.solve(c, "bf", rtol=1e-8)
            c = c.replace(u=newton.update(c.u, x0, DS_MAX))
        t0 = time.perf_counter()
        x, info, _ = newton.solve(c, "bf", rtol=1e-8)
        dt = time.perf_counter() - t0
    return dt, info, c, x


def errors_vs_oracle(torch, tpf, driver, c, x_or):
    """GPU solves of the sample case (same state as the oracle's) in both
    forms: relative difference of each solution from the oracle's FP64
    solution, and the true relative residuals."""
    g = driver.GpuCase(c)
    g.assemble()
    b = g.rhs().contiguous()
    out = {}
    xo = np.asarray(x_or)
    for precision, name in ((tpf.TPF_FP64, "fp64"), (tpf.TPF_FP32, "fp32_vcycle")):
        M = driver.GpuPrecond("bf", precision)
        M.setup(g)
        x = torch.empty_like(b)
        info = driver.solve(g, M, b, x, rtol=1e-8)
        xs = x.cpu().numpy()
        out[name] = {"rel_err_vs_oracle": float(np.linalg.norm(xs - xo) / np.linalg.norm(xo)),
                     "relres_true": float(info.relres_true), "iterations": int(info.iterations)}
        M.close()
    g.close()
    return out


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=float), q)) if len(v) else None


def serve_stream(torch, tpf, driver, inputs, args):
    """Serving stream: R realizations (sigma, P_d, grid per realization r),
    K Newton-step requests each, arriving interleaved.  The states u_k are
    generated beforehand by FP64 Newton on the GPU (open loop).  Baseline:
    the same requests one at a time, plain FP64 (assembly + full setup +
    FGMRES).  Served: BF with FP32 V-cycles, hierarchy refresh within a
    realization, up to --serve-active requests in flight."""
    R, K, emax = args.serve_realizations, args.serve_requests, args.serve_max_edge
    if args.serve_full:
        R, K, emax = 64, 16, 128
    rng = np.random.Generator(np.random.PCG64(7))
    seqs = []
    for r in range(R):
        e = min(inputs.serving_realization(r)["nx"], emax)
        case = inputs.serving_case(r, edge_override=e)
        g = driver.GpuCase(case)
        states = driver.newton_states(g, K)
        seqs.append((case, g, states))
        log(f"[serve] realization {r}: {e}^3 cells, {K} states")
    order = []  # request i = (r, k); realizations interleaved, k ascending per realization
    nxt = [0] * R
    for r in rng.permutation(np.repeat(np.arange(R), K)):
        order.append((int(r), nxt[r]))
        nxt[r] += 1
    n = len(order)
    xb = {}
    # ---- baseline: one at a time, plain FP64, full setup per request
    lat_b = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r, k in order:
        case, g, states = seqs[r]
        t1 = time.perf_counter()
        g.u.copy_(states[k])
        g.assemble()
        b = g.R  # J x = F, the negated Newton step
        M = driver.GpuPrecond("bf")
        M.setup(g)
        x = torch.empty_like(b)
        info = driver.solve(g, M, b, x)
        M.close()
        torch.cuda.synchronize()
        lat_b.append(1e3 * (time.perf_counter() - t1))
        xb[(r, k)] = x
        assert info.status == tpf.TPF_CONVERGED, (r, k, info.status)
    base_s = time.perf_counter() - t0
    for case, g, states in seqs:
        g.u.copy_(states[0])
    thr_b = n / base_s
    log(f"[serve] baseline: {n} requests in {base_s:.2f} s ({thr_b:.1f} solves/s)")

    budget = int(args.serve_budget_gib * 2 ** 30)

    def run(rate):
        torch.cuda.synchronize()
        base, _ = tpf.allocator_bytes()
        tpf.reset_allocator_peak()
        sv = driver.Server("bf", precision=tpf.TPF_FP32, max_active=args.serve_active,
                           hbm_budget_bytes=budget)
        arr = np.zeros(n) if rate is None else np.cumsum(rng.exponential(1.0 / rate, n))
        xs = [torch.empty(2 * seqs[r][0].N, dtype=torch.float64, device="cuda") for r, _ in order]
        torch.cuda.synchronize()
        lat, its, rel, errs, ref = [None] * n, [0] * n, [0.0] * n, [0.0] * n, [0] * n
        t_setup, t_solve, t_lat = [0.0] * n, [0.0] * n, [0.0] * n
        tick, i, done = {}, 0, 0
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            while i < n and arr[i] <= now:
                r, k = order[i]
                case, g, states = seqs[r]
                tick[sv.submit(r, g, states[k], g.u_old, xs[i])] = i
                i += 1
            st = sv.stats()
            if st.active == 0 and st.queued == 0:
                if i < n:
                    time.sleep(max(0.0, min(arr[i] - (time.perf_counter() - t0), 0.01)))
                continue
            sv.step()
            for t in list(tick):
                res = sv.poll(t)
                if res is None:
                    continue
                j = tick.pop(t)
                lat[j] = 1e3 * (time.perf_counter() - t0 - arr[j])
                its[j] = res.iterations
                rel[j] = res.relres_true
                ref[j] = res.refreshed
                t_setup[j], t_solve[j], t_lat[j] = res.setup_ms, res.solve_ms, res.latency_ms
                assert res.status == tpf.TPF_CONVERGED, (order[j], res.status)
                done += 1
        total = time.perf_counter() - t0
        st = sv.stats()
        drawn = tpf.allocator_bytes()[1] - base
        sv.close()
        torch.cuda.synchronize()
        for j, (r, k) in enumerate(order):
            # served x is the Newton step; the baseline solved J x = F (its negative)
            errs[j] = float(torch.linalg.norm(xs[j] + xb[(r, k)]) / torch.linalg.norm(xb[(r, k)]))
        by_edge = {}
        for e in sorted({seqs[r][0].nx for r, _ in order}):
            le = [lat[j] for j, (r, _) in enumerate(order) if seqs[r][0].nx == e]
            by_edge[str(e)] = {"requests": len(le), "p50_ms": round(pct(le, 50), 2),
                               "p99_ms": round(pct(le, 99), 2)}
        refreshed = sum(1 for j in range(n) if ref[j])
        # where the slowest 1% of requests spent their time (the server's own clocks:
        # waiting = submit to completion minus setup and solve)
        cut = pct(lat, 99)
        slow = [j for j in range(n) if lat[j] >= cut]
        tail = {k: round(float(np.mean([f(j) for j in slow])), 2) for k, f in (
            ("setup_ms", lambda j: t_setup[j]), ("solve_ms", lambda j: t_solve[j]),
            ("waiting_ms", lambda j: t_lat[j] - t_setup[j] - t_solve[j]))}
        tail["requests"] = len(slow)
        tail["p99_setup_ms_all"] = round(pct(t_setup, 99), 2)
        tail["p99_solve_ms_all"] = round(pct(t_solve, 99), 2)
        return {"arrival_rate_per_s": None if rate is None else round(rate, 2),
                "solves_per_s": round(n / total, 2), "wall_s": round(total, 3),
                "p50_latency_ms": round(pct(lat, 50), 2), "p99_latency_ms": round(pct(lat, 99), 2),
                "latency_by_edge": by_edge, "slowest_1pct": tail, "refreshed_requests": refreshed,
                "mean_iterations": round(float(np.mean(its)), 2),
                "max_relres_true": float(np.max(rel)),
                "max_rel_diff_vs_fp64": float(np.max(errs)),
                "peak_bytes": int(st.peak_bytes),
                "peak_bytes_drawn_from_allocator": int(drawn),
                "evictions": int(st.evictions)}

    log("[serve] burst: every request queued at t = 0")
    burst = run(None)
    rate = args.serve_load * thr_b
    log(f"[serve] Poisson arrivals at {rate:.1f}/s")
    pois = run(rate)
    for case, g, states in seqs:
        g.close()
    edges = sorted({min(inputs.serving_realization(r)["nx"], emax) for r in range(R)})
    return {
        "workload": f"{R} realizations x {K} Newton-step requests, edges {edges}, "
                    f"BF FP32 V-cycle, rtol 1e-8",
        "requests": n, "max_active": args.serve_active, "hbm_budget_bytes": budget,
        "baseline_fp64_sequential": {"solves_per_s": round(thr_b, 2), "wall_s": round(base_s, 3),
                                     "p50_latency_ms": round(pct(lat_b, 50), 2),
                                     "p99_latency_ms": round(pct(lat_b, 99), 2)},
        "burst": burst, "poisson": pois,
        "throughput_speedup_vs_baseline": round(burst["solves_per_s"] / thr_b, 3),
    }


def study_c2(torch, tpf, driver, inputs, args):
    """First Newton Jacobian of the 2D 512x512 workload for P_d in {0, 0.1,
    1}: setup and solve time, iterations and true residual of the four
    preconditioners (FP64), each timed after one warm-up."""
    nx, ny = (int(v) for v in (args.study_grid or "512x512").split("x"))
    rows = []
    for pd in (0.0, 0.1, 1.0):
        c = inputs.workload_2d_corner(nx, ny, 2.0, 16.0, pd, 50.0, 2, name=f"2d-{nx}x{ny}-pd{pd}")
        g = driver.GpuCase(c)
        g.assemble()
        b = g.R  # J x = F, the negated Newton step
        x = torch.empty_like(b)
        for kind in ("amg", "cpr1", "cpr2", "bf"):
            M = driver.GpuPrecond(kind)
            rec = None
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                M.setup(g)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                info = driver.solve(g, M, b, x)
                t2 = time.perf_counter()
                st = M.stats()
                rec = {"pd": pd, "kind": kind, "setup_ms": round(1e3 * (t1 - t0), 2),
                       "solve_ms": round(1e3 * (t2 - t1), 2), "iterations": int(info.iterations),
                       "status": int(info.status), "relres_true": float(info.relres_true),
                       "levels": [int(st.levels[h]) for h in range(st.n_hier)],
                       "op_complexity": [round(float(st.operator_complexity[h]), 3)
                                         for h in range(st.n_hier)]}
            log(f"[c2] P_d {pd} {kind}: {rec['iterations']} its, setup {rec['setup_ms']} ms, "
                f"solve {rec['solve_ms']} ms")
            rows.append(rec)
            M.close()
        g.close()
    return {"study": "c2", "workload": f"2d-{nx}x{ny} sigma=2 corr=16 CFL 50, first Newton "
                                      f"Jacobian", "precision": "f64", "results": rows}


def study_newton(torch, tpf, driver, inputs, args):
    """10 consecutive Newton Jacobians of one time step on the 3D 256x256x128
    workload with BF: full setup at every Jacobian (rebuild) or numeric
    refresh of the first hierarchy (reuse), FP64 and FP32 V-cycles; per
    Jacobian ||F||, iterations, setup and solve time; HBM bytes by part."""
    nx, ny, nz = (int(v) for v in (args.study_grid or "256x256x128").split("x"))
    c = inputs.config_c4(nx, ny, nz)
    out = {"study": "newton", "workload": f"3d-{nx}x{ny}x{nz} log-normal sigma=3, CFL "
                                          f"{inputs.SEQUENCE_CFL:g}, BF, 10 Jacobians",
           "cells": c.N, "sequences": []}
    for precision, pname in ((tpf.TPF_FP64, "f64"), (tpf.TPF_FP32, "f32")):
        for reuse in (False, True):
            g = driver.GpuCase(c)
            M = driver.GpuPrecond("bf", precision)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs = driver.newton_sequence(g, M, 10, reuse=reuse, ds_max=0.2)
            torch.cuda.synchronize()
            total = time.perf_counter() - t0
            st = M.stats()
            v = tpf.tpf_jacobian_view(g.J)
            seq = {"precision": pname, "structure": "reuse" if reuse else "rebuild",
                   "total_s": round(total, 3),
                   "jacobians": [{k: (round(val, 3) if isinstance(val, float) else val)
                                  for k, val in r.items()} for r in recs],
                   "hbm_bytes": {"jacobian": int(v.nnzb) * 36 + 4 * (v.n_block_rows + 1),
                                 "preconditioner": int(st.device_bytes),
                                 "hierarchy_A_ss": int(st.hier_bytes[0]),
                                 "hierarchy_S": int(st.hier_bytes[1]),
                                 "krylov_workspace": 8 * (2 * 30 + 2) * 2 * c.N,
                                 "state_vectors": 8 * 2 * c.N * 4}}
            log(f"[newton] {pname} {seq['structure']}: {total:.2f} s, its "
                f"{[r['iterations'] for r in recs]}")
            out["sequences"].append(seq)
            M.close()
            g.close()
    return out


def study_simulate(torch, tpf, driver, inputs, args):
    """Multi-step simulations on the stand-ins of the paper's 2D experiments,
    every preconditioner, FP64: NI, LI, LI/NI, wall time, status ('-' in the
    paper's tables = diverged).  (1) Oil-water cross-section 100x1x20 for
    Ex1-Ex3 with linear and Brooks-Corey P_c, 200 days at dt = 20 days
    (Sec. 4.1 tables); (2) gravity box n x 1 x n, n in {20, 40, 80, 160},
    three regimes (Sec. 4.2 tables); (3) the 80x80 advection regime with
    dt in {1, 2, 4, 8} days to 8 days (Sec. 4.2 time-step table)."""
    kinds = ("amg", "cpr1", "cpr2", "bf")
    rows = []

    def run(tag, case, t_final, dt, extra=None):
        for kind in kinds:
            r = driver.simulate(case, kind, t_final, dt=dt)
            rec = {"experiment": tag, "kind": kind, "NI": r["NI"], "LI": r["LI"],
                   "LI_per_NI": round(r["LI_per_NI"], 2), "time_s": round(r["wall_s"], 3),
                   "status": r["status"], "steps": len(r["steps"])}
            rec.update(extra or {})
            log(f"[simulate] {tag} {kind}: NI {rec['NI']} LI {rec['LI']} LI/NI "
                f"{rec['LI_per_NI']} {rec['time_s']} s {rec['status']}")
            rows.append(rec)

    for ex in (1, 2, 3):
        for pcm, pname in ((inputs.PC_LINEAR, "linear"), (inputs.PC_BROOKS_COREY, "brooks-corey")):
            run(f"oil-water ex{ex} {pname}", inputs.oil_water_xz(ex, pcm), 200.0, 20.0)
    for regime, (_, dt, tf) in inputs.GRAVITY_REGIMES.items():
        for n in (20, 40, 80, 160):
            run(f"gravity {regime} {n}x{n}", inputs.gravity_box_xz(n, regime), tf, dt)
    for dt in (1.0, 2.0, 4.0, 8.0):
        run(f"gravity advection 80x80 dt {dt:g}", inputs.gravity_box_xz(80, "advection"), 8.0,
            dt, {"NI_per_step": None})
        for r in rows[-len(kinds):]:
            r["NI_per_step"] = round(r["NI"] / max(r["steps"], 1), 2)
    return {"study": "simulate", "precision": "f64", "newton_tol": 1e-6, "rtol": 1e-8,
            "results": rows}


def study_spectra(torch, tpf, driver, inputs, args):
    """Eigenvalues of J M^{-1} with exact inner solves (Sec. 4.3) from the GPU
    preconditioners, for the diffusion- (Ex1) and advection-dominated (Ex2)
    oil-water stand-in with linear P_c (50x1x10, the first Jacobian)."""
    rows = []
    nx, nz = (int(v) for v in (args.study_grid or "50x10").split("x"))
    for ex, regime in ((1, "diffusion"), (2, "advection")):
        c = inputs.oil_water_xz(ex, inputs.PC_LINEAR, nx=nx, nz=nz)
        g = driver.GpuCase(c)
        g.assemble()
        for kind in ("cpr1", "cpr2", "bf"):
            M = driver.GpuPrecond(kind, **driver.exact_inner_opts(c.N))
            M.setup(g)
            ev = np.linalg.eigvals(driver.preconditioned_matrix(g, M))
            a = np.abs(ev)
            rec = {"regime": regime, "kind": kind, "n": int(len(ev)),
                   "min_abs": float(a.min()), "max_abs": float(a.max()),
                   "frac_abs_below_0.1": float(np.mean(a < 0.1)),
                   "frac_within_0.5_of_1": float(np.mean(np.abs(ev - 1.0) < 0.5)),
                   "re_range": [float(ev.real.min()), float(ev.real.max())],
                   "max_abs_imag": float(np.abs(ev.imag).max())}
            log(f"[spectra] {regime} {kind}: |lambda| in [{rec['min_abs']:.3g}, "
                f"{rec['max_abs']:.3g}], {100 * rec['frac_abs_below_0.1']:.1f}% below 0.1")
            rows.append(rec)
            M.close()
        g.close()
    return {"study": "spectra", "grid": f"{nx}x1x{nz}", "inner": "exact (dense inverse)",
            "results": rows}


def study_amg_variants(torch, tpf, driver, inputs, args):
    """BF on the 3D workload's Jacobian at Newton iterate 1, FP64, with each
    AMG variant in both hierarchies: setup and solve time (median of three
    after a warm-up), FGMRES iterations, true residual, operator complexity."""
    nx, ny, nz = (int(v) for v in (args.study_grid or "128x128x64").split("x"))
    c = inputs.config_c3(nx, ny, nz)
    g = driver.GpuCase(c)
    g.u.copy_(linearisation_state(torch, driver, g, "newton1"))
    g.assemble()
    b = g.R
    x = torch.empty_like(b)
    variants = [
        ("default: PMIS, ext+i (S~) / direct (A_ss), l1-Jacobi, P rows truncated to 3", {}),
        ("default without interpolation truncation", dict(trunc_pmax=0)),
        ("PMIS, classical, l1-Jacobi", dict(interp=tpf.TPF_INTERP_CLASSICAL)),
        ("PMIS, default interpolation, multicolour GS", dict(smoother=tpf.TPF_SMOOTH_MC_GS)),
        ("CLJP, default interpolation, l1-Jacobi", dict(coarsening=tpf.TPF_COARSEN_CLJP)),
        ("CLJP, classical, multicolour GS (the paper's components)",
         dict(coarsening=tpf.TPF_COARSEN_CLJP, interp=tpf.TPF_INTERP_CLASSICAL,
              smoother=tpf.TPF_SMOOTH_MC_GS)),
    ]
    rows = []
    for name, opts in variants:
        M = driver.GpuPrecond("bf", **opts)
        t_set, t_sol, info = [], [], None
        for rep_ in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M.setup(g)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            info = driver.solve(g, M, b, x, rtol=1e-8)
            t2 = time.perf_counter()
            if rep_:
                t_set.append(t1 - t0)
                t_sol.append(t2 - t1)
        st = M.stats()
        rec = {"variant": name, "iterations": int(info.iterations), "status": int(info.status),
               "relres_true": float(info.relres_true),
               "setup_ms": round(1e3 * float(np.median(t_set)), 2),
               "solve_ms": round(1e3 * float(np.median(t_sol)), 2),
               "levels": [int(st.levels[h]) for h in range(st.n_hier)],
               "op_complexity": [round(float(st.operator_complexity[h]), 3)
                                 for h in range(st.n_hier)]}
        rec["total_ms"] = round(rec["setup_ms"] + rec["solve_ms"], 2)
        log(f"[amg-variants] {name}: {rec['iterations']} its, setup {rec['setup_ms']} ms, "
            f"solve {rec['solve_ms']} ms")
        rows.append(rec)
        M.close()
    g.close()
    return {"study": "amg-variants", "workload": f"3d-{nx}x{ny}x{nz} BF at Newton iterate 1, FP64",
            "results": rows}


def linearisation_state(torch, driver, g, state):
    """Device copy of the state the benchmark Jacobian is taken at: the
    initial condition of the time step, or Newton iterate 1 (one FP64 BF
    Newton step from it, saturation chop DS_MAX), computed on the GPU."""
    if state == "initial":
        return g.u.clone()
    return driver.newton_states(g, 2, ds_max=DS_MAX)[1].clone()


def state_text(state):
    return ("Newton iterate 1 of the first time step" if state == "newton1"
            else "initial condition of the time step (uniform P_w = 0, S_n = 0.2)")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build runs on a single MI355X "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)
    if args.reduce_traffic:
        rec = reduce_traffic(args.reduce_traffic)
        for timer, k in rec["kernels"].items():
            log(f"{timer} {k['symbol']}: {k['traffic_over_algorithmic']}x the algorithmic "
                f"bytes, {k['trace_avg_us']} us")
        return
    import torch

    from paper_1611_00127_amd import driver, inputs, tpf
    tpf.init()
    tpf.tpf_set_graphs(args.graphs)
    if args.study:
        fn = {"c2": study_c2, "newton": study_newton, "simulate": study_simulate,
              "spectra": study_spectra, "amg-variants": study_amg_variants}[args.study]
        print(json.dumps(fn(torch, tpf, driver, inputs, args)), flush=True)
        return
    if args.copy_probe > 0:
        n = args.copy_probe * 2 ** 20 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written")
        del src, dst
    nx, ny, nz = (int(v) for v in args.grid.split("x"))
    log(f"[bench] generating workload {nx}x{ny}x{nz}")
    c = inputs.config_c3(nx, ny, nz)
    g = driver.GpuCase(c)
    states = {st: linearisation_state(torch, driver, g, st) for st in ("newton1", "initial")}
    head, other = args.state, ("initial" if args.state == "newton1" else "newton1")
    g.u.copy_(states[head])
    torch.cuda.synchronize()
    log(f"[bench] FP64 form at {head}")
    M64, x64, r64 = run_form(torch, tpf, driver, g, tpf.TPF_FP64, args.steps, args.warmup, False)
    # one more step per form with every kernel bracketed by HIP events, for the
    # per-level V-cycle table and the roofline (kept out of the timed steps)
    log("[bench] FP64 instrumented step")
    Mi, _, _ = run_form(torch, tpf, driver, g, tpf.TPF_FP64, 1, 0, True)
    st64 = Mi.stats()
    # the cycle's prolongation reads P in ELL form when truncation bounds its rows
    ell_w = int(Mi.opts.trunc_pmax) if 1 <= int(Mi.opts.trunc_pmax) <= 4 else 0
    vc64, kern64 = vcycle_table(tpf, st64, HIER_TAGS["bf"], 8, ell_w)
    ktab = kernel_table(tpf, ["cgs2", "bcsr_spmv", "bf_rhs", "assemble", "precond_apply"])
    walls = []
    for h in range(st64.n_hier):
        ms = vcycle_wall(torch, tpf, Mi, h, int(st64.rows[h][0]))
        walls.append(ms)
        vc64[h]["wall_ms_per_vcycle"] = round(ms, 4)
        vc64[h]["wall_gbs"] = round(vc64[h]["bytes_per_vcycle"] / (ms * 1e6), 1)
    Mi.close()
    log("[bench] FP64 setup phases")
    setup64 = setup_breakdown(torch, tpf, driver, g, tpf.TPF_FP64)
    log("[bench] FP32-V-cycle form")
    M32, x32, r32 = run_form(torch, tpf, driver, g, tpf.TPF_FP32, args.steps, args.warmup, False)
    err = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
    log("[bench] FP32 instrumented step")
    Mi, _, _ = run_form(torch, tpf, driver, g, tpf.TPF_FP32, 1, 0, True)
    vc32, _ = vcycle_table(tpf, Mi.stats(), HIER_TAGS["bf"], 4, ell_w)
    Mi.close()
    tpf.tpf_kernel_stats_reset()
    M64.close()
    M32.close()
    log(f"[bench] FP64 form at {other}")
    g.u.copy_(states[other])
    Mo, _, ro = run_form(torch, tpf, driver, g, tpf.TPF_FP64, max(1, min(args.steps, 5)), 1, False)
    Mo.close()
    ro = {k: ro[k] for k in ("ms_per_step", "assemble_ms", "setup_ms", "solve_ms", "iterations",
                             "relres_true", "converged", "op_complexity")}
    g.close()

    # roofline of the dominant V-cycle kernel: the largest summed time over
    # every level of both hierarchies (FP64 form)
    if args.traffic_spec:
        write_traffic_spec(args.traffic_spec, st64, kern64)
    dom = max(kern64, key=lambda k: k["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    achieved = dom["bytes"] / (avg_ms * 1e-3) / 1e9
    roof = {"kernel": dom["symbol"],
            "timer": f"{dom['timer']}[{dom['hier']},l{dom['level']}]",
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(f"{dom['timer']}[{dom['hier']},l{dom['level']}]",
                                      dom["symbol"]),
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches": dom["launches"],
            "algorithmic_bytes_per_launch": dom["bytes"],
            "share_of_vcycle_kernel_time": round(
                dom["total_ms"] / sum(k["total_ms"] for k in kern64), 4)}
    tot_b = sum(v["bytes_per_vcycle"] for v in vc64)
    tot_ms = sum(walls)
    vgbs = {"fp64_wall_gbs_bf_apply_vcycles": round(tot_b / (tot_ms * 1e6), 1),
            "fp64_kernel_gbs_bf_apply_vcycles": round(
                tot_b / (sum(v["kernel_ms_per_vcycle"] for v in vc64) * 1e6), 1)}

    serving = None
    if not args.no_serve:
        log("[bench] serving stream")
        tpf.tpf_kernel_timing(0)
        serving = serve_stream(torch, tpf, driver, inputs, args)

    c4 = None
    if not args.no_c4:
        log("[bench] 256x256x128 Newton sequence")
        c4 = study_newton(torch, tpf, driver, inputs, args)

    cpu, vs_oracle = None, None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU baseline: oracle on {args.cpu_grid} at {head}")
        dt, info, cs, xo = cpu_baseline(args.cpu_grid, head)
        scale = c.N / cs.N
        cpu = {"value": round(dt * scale * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
               "sample": f"one full step (assemble + BF setup + FGMRES to 1e-8, "
                         f"{info['iterations']} its) of the same workload family on "
                         f"{args.cpu_grid} ({cs.N} cells) at the {state_text(head)} (the "
                         f"oracle's own), one thread, {dt:.1f} s, scaled x{scale:.0f} by "
                         f"cell count",
               "host": host_info()}
        vs_oracle = dict(errors_vs_oracle(torch, tpf, driver, cs, xo), grid=args.cpu_grid,
                         oracle_iterations=int(info["iterations"]))

    out = {
        "metric": METRIC,
        "value": round(r64["ms_per_step"], 2),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3d-{nx}x{ny}x{nz} log-normal sigma=3 kz/kx=0.1 layered, "
                               f"Brooks-Corey lambda=2 Pd=0.5, five-spot, CFL 10, Jacobian at "
                               f"the {state_text(head)}",
                   "cells": c.N, "unknowns": 2 * c.N, "preconditioner": "bf",
                   "krylov": "fgmres(30)", "rtol": 1e-8},
        "fp64": dict(r64, setup_phases=setup64),
        "fp32_vcycle": dict(r32, rel_diff_vs_fp64=err,
                            speedup_vs_fp64=round(r64["ms_per_step"] / r32["ms_per_step"], 3)),
        "errors_vs_fp64_oracle": vs_oracle,
        f"fp64_at_{other}": ro,
        "vcycle_gbs": vgbs,
        "vcycle_levels_fp64": vc64,
        "vcycle_levels_fp32": vc32,
        "roofline": roof,
        "kernels_ms": {k: {"launches": v[0], "total_ms": round(v[1], 3),
                           "avg_us": round(1e3 * v[1] / v[0], 2)} for k, v in ktab.items()},
        "cpu_baseline": cpu,
        "serving": serving,
        "c4_newton_sequence": c4,
        "p99_latency_ms": serving["poisson"]["p99_latency_ms"] if serving else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
