"""Benchmark: time to a 1e-8 relative residual for the first Newton Jacobian
of the 3D 128x128x64 heterogeneous workload (1,048,576 cells, 2.1M
unknowns), block-factorisation preconditioner (Algorithm 3) with AMG
V-cycles on A_ss and S~, right-preconditioned FGMRES(30).

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
    ap.add_argument("--cpu-grid", type=str, default="80x80x40",
                    help="grid of the oracle's bounded sample")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="first run a plain device copy of this many MiB (calibrates the "
                         "FETCH_SIZE/WRITE_SIZE counters of a profiler run)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--graphs", action="store_true",
                    help="replay recorded V-cycle graphs instead of launching every kernel")
    ap.add_argument("--serve-full", action="store_true",
                    help="the full stream: 64 realizations x 16 Newton-step requests, "
                         "grids up to 128^3")
    ap.add_argument("--serve-realizations", type=int, default=8)
    ap.add_argument("--serve-requests", type=int, default=4, help="requests per realization")
    ap.add_argument("--serve-max-edge", type=int, default=64,
                    help="grid edges drawn above this are clamped to it")
    ap.add_argument("--serve-active", type=int, default=8, help="requests in flight")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="Poisson arrival rate as a fraction of the sequential FP64 throughput")
    ap.add_argument("--study", choices=["c2", "newton"], default=None,
                    help="instead of the benchmark line, print one JSON line for a study: "
                         "c2 = first Jacobian of the 512x512 workload for P_d in {0, 0.1, 1} and "
                         "all four preconditioners; newton = 10 consecutive Newton Jacobians of "
                         "the 256x256x128 workload, BF, rebuild vs reuse x FP64 vs FP32")
    ap.add_argument("--study-grid", type=str, default=None,
                    help="grid of the study workload (default: 512x512 / 256x256x128)")
    return ap.parse_args()


def level0_bytes(nnz, n, w, kind, diagonals=0):
    """Algorithmic bytes of one level-0 V-cycle kernel launch, value width w:
    the operator once (diagonal layout: K*n values; CSR: values, int32
    column indices and row pointers) and each dense vector once."""
    mat = w * diagonals * n if diagonals else (w + 4) * nnz + 4 * (n + 1)
    if kind == "pre":      # read b and D^{-1} b (CSR: dinv); write r
        return mat + 3 * w * n
    if kind == "post":     # read b, dinv, y; write x
        return mat + 4 * w * n
    raise ValueError(kind)


AMG_SRC = os.path.join(ROOT, "paper_1611_00127_amd", "csrc", "amg.hip")


def kernel_digest(path=AMG_SRC, names=("clampi", "xcd_contiguous_block", "k_dia_pre2")):
    """sha256 of the source text of the named device functions (each from
    its name to the first closing brace at column 0): identifies the kernel
    build that a stored counter measurement belongs to."""
    import hashlib
    import re
    text = open(path).read()
    h = hashlib.sha256()
    for nm in names:
        m = re.search(r"\b" + re.escape(nm) + r"\(", text)
        if not m:
            return None
        start = text.rfind("\n", 0, m.start()) + 1
        end = text.find("\n}\n", m.end())
        if end < 0:
            return None
        h.update(text[start:end + 3].encode())
    return h.hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE measurement (scaled by its copy-kernel calibration), or None
    when there is none or the kernel's source has changed since."""
    path = os.path.join(ROOT, "profiles", "k_dia_d25_3d_128x128x64_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    k = rec["kernels"].get(kernel)
    if k is None or k["source_sha256"] != kernel_digest(names=tuple(k["digest_of"])):
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


def kernel_table(tpf, names):
    out = {}
    for n in names:
        cnt, ms = tpf.tpf_kernel_stats(n)
        if cnt:
            out[n] = (cnt, ms)
    return out


def cpu_baseline(grid):
    """The oracle (unmodified) on a bounded sample: the same workload family on
    a smaller grid, one full step (assemble + BF setup + FGMRES to 1e-8),
    BLAS limited to one thread; scaled by the cell ratio to the benchmark
    grid (linear-cost assumption)."""
    from threadpoolctl import threadpool_limits

    from oracle import newton
    from paper_1611_00127_amd import inputs
    nx, ny, nz = (int(v) for v in grid.split("x"))
    c = inputs.config_c3(nx, ny, nz)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, info, _ = newton.solve(c, "bf", rtol=1e-8)
        dt = time.perf_counter() - t0
    return dt, info, c.N


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

    def run(rate):
        sv = driver.Server("bf", precision=tpf.TPF_FP32, max_active=args.serve_active)
        arr = np.zeros(n) if rate is None else np.cumsum(rng.exponential(1.0 / rate, n))
        xs = [torch.empty(2 * seqs[r][0].N, dtype=torch.float64, device="cuda") for r, _ in order]
        torch.cuda.synchronize()
        lat, its, rel, errs = [None] * n, [0] * n, [0.0] * n, [0.0] * n
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
                assert res.status == tpf.TPF_CONVERGED, (order[j], res.status)
                done += 1
        total = time.perf_counter() - t0
        st = sv.stats()
        sv.close()
        torch.cuda.synchronize()
        for j, (r, k) in enumerate(order):
            # served x is the Newton step; the baseline solved J x = F (its negative)
            errs[j] = float(torch.linalg.norm(xs[j] + xb[(r, k)]) / torch.linalg.norm(xb[(r, k)]))
        return {"arrival_rate_per_s": None if rate is None else round(rate, 2),
                "solves_per_s": round(n / total, 2), "wall_s": round(total, 3),
                "p50_latency_ms": round(pct(lat, 50), 2), "p99_latency_ms": round(pct(lat, 99), 2),
                "mean_iterations": round(float(np.mean(its)), 2),
                "max_relres_true": float(np.max(rel)),
                "max_rel_diff_vs_fp64": float(np.max(errs)),
                "peak_bytes": int(st.peak_bytes), "evictions": int(st.evictions)}

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
        "requests": n, "max_active": args.serve_active,
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build runs on a single MI355X "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1611_00127_amd import driver, inputs, tpf
    tpf.init()
    tpf.tpf_set_graphs(args.graphs)
    if args.study:
        fn = study_c2 if args.study == "c2" else study_newton
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
    torch.cuda.synchronize()
    log("[bench] FP64 form")
    M64, x64, r64 = run_form(torch, tpf, driver, g, tpf.TPF_FP64, args.steps, args.warmup, False)
    # one more step with every kernel bracketed by HIP events, for the
    # kernel table and the roofline (kept out of the timed steps above)
    log("[bench] FP64 instrumented step")
    Mi, _, _ = run_form(torch, tpf, driver, g, tpf.TPF_FP64, 1, 0, True)
    Mi.close()
    names = []
    for h, tag in enumerate(["Ass", "Schur"]):
        for k in ["vcycle_pre_residual", "vcycle_post_smooth", "vcycle_restrict", "vcycle_prolong"]:
            names.append(f"{k}[{tag},l0]")
    names += ["cgs2", "bcsr_spmv", "bf_rhs", "assemble", "precond_apply"]
    ktab = kernel_table(tpf, names)
    log("[bench] FP32-V-cycle form")
    M32, x32, r32 = run_form(torch, tpf, driver, g, tpf.TPF_FP32, args.steps, args.warmup, False)
    # the two forms must agree at the stated accuracy
    err = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))

    # roofline of the dominant V-cycle kernel (largest summed time)
    vk = {k: v for k, v in ktab.items() if k.startswith("vcycle_")}
    dom = max(vk, key=lambda k: vk[k][1])
    cnt, ms = vk[dom]
    h = 1 if "Schur" in dom else 0
    nnz, n = r64["l0_nnz"][h], r64["l0_rows"][h]
    kind = "pre" if "pre_residual" in dom else "post"
    bytes_per_launch = level0_bytes(nnz, n, 8, kind, r64["l0_diagonals"][h])
    avg_ms = ms / cnt
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    K = r64["l0_diagonals"][h]
    gpu_kernel = (f"k_dia_{kind}{'2' if n % 2 == 0 else ''}<double, {K}>" if K
                  else f"k_vc_{kind}<double, *>")
    roof = {"kernel": gpu_kernel, "timer": dom,
            "layout": f"diagonal, {K} diagonals" if K else "csr",
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(gpu_kernel),
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches": cnt,
            "algorithmic_bytes_per_launch": bytes_per_launch}

    M64.close()
    M32.close()
    g.close()
    serving = None
    if not args.no_serve:
        log("[bench] serving stream")
        tpf.tpf_kernel_timing(0)
        serving = serve_stream(torch, tpf, driver, inputs, args)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU baseline: oracle on {args.cpu_grid}")
        dt, info, ncpu = cpu_baseline(args.cpu_grid)
        scale = c.N / ncpu
        cpu = {"value": round(dt * scale * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
               "sample": f"one full step (assemble + BF setup + FGMRES to 1e-8, "
                         f"{info['iterations']} its) of the same workload on {args.cpu_grid} "
                         f"({ncpu} cells) in {dt:.1f} s, scaled x{scale:.0f} by cell count"}

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
                               f"Brooks-Corey lambda=2 Pd=0.5, five-spot, first Newton Jacobian",
                   "cells": c.N, "unknowns": 2 * c.N, "preconditioner": "bf",
                   "krylov": "fgmres(30)", "rtol": 1e-8},
        "fp64": r64,
        "fp32_vcycle": dict(r32, rel_diff_vs_fp64=err,
                            speedup_vs_fp64=round(r64["ms_per_step"] / r32["ms_per_step"], 3)),
        "roofline": roof,
        "kernels_ms": {k: {"launches": v[0], "total_ms": round(v[1], 3),
                           "avg_us": round(1e3 * v[1] / v[0], 2)} for k, v in ktab.items()},
        "cpu_baseline": cpu,
        "serving": serving,
        "p99_latency_ms": serving["poisson"]["p99_latency_ms"] if serving else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
