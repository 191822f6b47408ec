"""Device-side plumbing around the C ABI: uploads a workload's arrays to
torch CUDA tensors and drives assemble / setup / solve through the binding.
No solver arithmetic happens here."""
from __future__ import annotations

import numpy as np

from . import tpf


class GpuCase:
    """A problem, its Jacobian and its state resident on the GPU."""

    def __init__(self, case, stream=None):
        import torch
        tpf.init()
        self.case = case
        self.stream = stream
        dev = torch.device("cuda")
        f64 = torch.float64
        self.N = case.N
        self.kx = torch.as_tensor(case.kx, dtype=f64, device=dev).contiguous()
        self.ky = torch.as_tensor(case.ky, dtype=f64, device=dev).contiguous()
        self.kz = torch.as_tensor(case.kz, dtype=f64, device=dev).contiguous()
        self.poro = torch.as_tensor(case.poro, dtype=f64, device=dev).contiguous()
        self.q = torch.as_tensor(np.ascontiguousarray(case.q).reshape(-1), dtype=f64, device=dev)
        self.u = torch.as_tensor(np.ascontiguousarray(case.u).reshape(-1), dtype=f64, device=dev).clone()
        self.u_old = torch.as_tensor(np.ascontiguousarray(case.u_old).reshape(-1), dtype=f64,
                                     device=dev).clone()
        self.R = torch.zeros(2 * self.N, dtype=f64, device=dev)
        self.prob = tpf.tpf_problem_create(
            case.nx, case.ny, case.nz, case.hx, case.hy, case.hz, self.kx, self.ky, self.kz,
            self.poro, case.mu_w, case.mu_n, case.rho_w, case.rho_n, case.grav, case.pc_model,
            case.bc_lambda, case.swr, case.snr, case.pd, case.s_eps, q=self.q,
            prod_cells=case.prod_cells, prod_wi=case.prod_wi, prod_pbh=case.prod_pbh,
            dir_cells=case.dir_cells, dir_face=case.dir_face, dir_p=case.dir_p, dir_s=case.dir_s,
            stream=stream)
        self.J = tpf.tpf_jacobian_create(self.prob, stream=stream)

    def assemble(self):
        tpf.tpf_assemble(self.prob, self.u, self.u_old, self.case.dt, self.R, self.J,
                         stream=self.stream)

    def rhs(self):
        return -self.R

    def bcsr_numpy(self):
        v = tpf.tpf_jacobian_view(self.J)
        rp = tpf.device_array(v.row_ptr, v.n_block_rows + 1, np.int32)
        ci = tpf.device_array(v.col_idx, int(v.nnzb), np.int32)
        vals = tpf.device_array(v.vals, 4 * int(v.nnzb), np.float64).reshape(-1, 2, 2)
        return rp, ci, vals

    def close(self):
        if tpf.shutting_down():
            return
        if self.J is not None:
            tpf.tpf_jacobian_destroy(self.J)
            self.J = None
        if self.prob is not None:
            tpf.tpf_problem_destroy(self.prob)
            self.prob = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GpuPrecond:
    def __init__(self, kind, precision=tpf.TPF_FP64, **opts):
        o = tpf.tpf_precond_default_opts(tpf.KINDS[kind] if isinstance(kind, str) else kind)
        o.precision = precision
        for k, v in opts.items():
            setattr(o, k, v)
        self.opts = o
        self.M = tpf.tpf_precond_create(o)

    def setup(self, gcase, reuse=False):
        tpf.tpf_precond_setup(self.M, gcase.J, int(reuse), stream=gcase.stream)

    def apply(self, r, z, stream=None):
        tpf.tpf_precond_apply(self.M, r, z, stream=stream)

    def stats(self):
        return tpf.tpf_precond_stats(self.M)

    def close(self):
        if tpf.shutting_down():
            return
        if self.M is not None:
            tpf.tpf_precond_destroy(self.M)
            self.M = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(gcase, M, b, x, rtol=1e-8, restart=30, maxit=1000):
    return tpf.tpf_solve(gcase.J, M.M if M is not None else None, b, x, rtol=rtol,
                         restart=restart, maxit=maxit, stream=gcase.stream)


def newton_sequence(gcase, M, n_jacobians, reuse=False, ds_max=0.2, rtol=1e-8, restart=30,
                    maxit=1000, on_step=None):
    """Consecutive Newton Jacobians of one time step on the GPU: assemble,
    set up (full, or numeric refresh of the first hierarchy when `reuse`),
    solve J delta = -F, update u (saturation chop ds_max).  Returns a list of
    dicts (||F||, iterations, status, relres, setup_ms, solve_ms)."""
    import time

    import torch
    out = []
    x = torch.empty(2 * gcase.N, dtype=torch.float64, device="cuda")
    for k in range(n_jacobians):
        gcase.assemble()
        fnorm = tpf.tpf_norm2(gcase.R, stream=gcase.stream)
        t0 = time.perf_counter()
        M.setup(gcase, reuse=bool(reuse and k > 0))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # J x = F, so the Newton step is -x
        info = solve(gcase, M, gcase.R, x, rtol=rtol, restart=restart, maxit=maxit)
        t2 = time.perf_counter()
        tpf.tpf_newton_update(gcase.prob, gcase.u, x, ds_max, alpha=-1.0, stream=gcase.stream)
        rec = dict(k=k, fnorm=fnorm, iterations=int(info.iterations), status=int(info.status),
                   relres=float(info.relres_true), setup_ms=1e3 * (t1 - t0),
                   solve_ms=1e3 * (t2 - t1))
        out.append(rec)
        if on_step:
            on_step(rec)
    torch.cuda.synchronize()
    return out


def simulate(case, kind, t_final, dt=None, precision=tpf.TPF_FP64, newton_tol=1e-6,
             max_newton=25, rtol=1e-8, ds_max=0.2, **precond_opts):
    """Backward-Euler time steps on the GPU (Sec. 2, Eq. fully_discrete_system),
    each a Newton loop (Sec. 3) until ||F(u_k)|| <= newton_tol (Sec. 4.1
    solver settings): assemble, norm of F, preconditioner setup, FGMRES on
    J x = F, update with the saturation chop.  A step whose Newton loop has
    not met the tolerance after max_newton solves, or whose linear solve
    fails, ends the run as diverged.  Returns a dict with per-step residual
    norms and Krylov iterations, NI, LI, LI/NI, wall time, status, and the
    final state (device tensor)."""
    import time

    import torch
    dt = case.dt if dt is None else dt
    n_steps = int(round(t_final / dt))
    g = GpuCase(case.replace(dt=dt))
    M = GpuPrecond(kind, precision, **precond_opts)
    x = torch.empty(2 * g.N, dtype=torch.float64, device="cuda")
    steps, status = [], "converged"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_steps):
        g.u_old.copy_(g.u)
        fnorms, its, st = [], [], "diverged"
        while True:
            g.assemble()
            fn = tpf.tpf_norm2(g.R, stream=g.stream)
            fnorms.append(fn)
            if not np.isfinite(fn):
                break
            if fn <= newton_tol:
                st = "converged"
                break
            if len(its) >= max_newton:
                break
            M.setup(g)
            info = solve(g, M, g.R, x, rtol=rtol)  # J x = F: the Newton step is -x
            its.append(int(info.iterations))
            if info.status != tpf.TPF_CONVERGED:
                break
            tpf.tpf_newton_update(g.prob, g.u, x, ds_max, alpha=-1.0, stream=g.stream)
        steps.append(dict(fnorms=fnorms, iterations=its, status=st))
        if st != "converged":
            status = "diverged"
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ni = sum(len(s["iterations"]) for s in steps)
    li = sum(sum(s["iterations"]) for s in steps)
    u = g.u.clone()
    M.close()
    g.close()
    return dict(steps=steps, NI=ni, LI=li, LI_per_NI=li / ni if ni else 0.0, status=status,
                wall_s=wall, u=u)


def exact_inner_opts(n_cells):
    """Preconditioner options whose inner solves are exact: one-level
    hierarchies solved by the dense coarsest inverse (at most 4,096 rows)."""
    if n_cells > 4096:
        raise ValueError("exact inner solves need at most 4,096 cells")
    return dict(max_levels=1, dense_max=max(n_cells, 1), coarse_max=max(n_cells, 1))


def preconditioned_matrix(gcase, M):
    """Dense J M^{-1} of a GPU Jacobian and preconditioner (Sec. 4.3
    eigenvalue study), formed column by column on the device: column j =
    J (M^{-1} e_j), by tpf_precond_apply and tpf_spmv.  Returns a host array."""
    import torch
    n = 2 * gcase.N
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(e)
    cols = torch.empty((n, n), dtype=torch.float64, device="cuda")
    for j in range(n):
        e.zero_()
        e[j] = 1.0
        M.apply(e, z, stream=gcase.stream)
        tpf.tpf_spmv(gcase.J, z, cols[j], stream=gcase.stream)
    torch.cuda.synchronize()
    return cols.T.cpu().numpy()


class Server:
    """Python side of the serving engine (tpf_server_*): keeps the tensors of
    every request alive until its result has been polled."""

    def __init__(self, kind="bf", precision=tpf.TPF_FP32, max_active=8, hbm_budget_bytes=64 << 30,
                 reuse=True, rtol=1e-8, restart=30, maxit=1000):
        tpf.init()
        o = tpf.tpf_server_default_opts()
        o.kind = tpf.KINDS[kind] if isinstance(kind, str) else kind
        o.precision = precision
        o.max_active = max_active
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.reuse = int(bool(reuse))
        o.solve.rtol, o.solve.restart, o.solve.maxit = rtol, restart, maxit
        self.opts = o
        self.sv = tpf.tpf_server_create(o)
        self._held = {}

    def submit(self, sequence, gcase, u, u_old, x, dt=None):
        """Queues the Newton solve of realization `sequence` (problem of gcase)
        at state u; x receives the update.  Tensors must be ready (the caller
        has synchronised the stream that wrote them)."""
        t = tpf.tpf_server_submit(self.sv, sequence, gcase.prob, u, u_old,
                                  gcase.case.dt if dt is None else dt, x)
        self._held[t] = (gcase, u, u_old, x)
        return t

    def step(self):
        return tpf.tpf_server_step(self.sv)

    def poll(self, ticket):
        r = tpf.tpf_server_poll(self.sv, ticket)
        if r is not None:
            self._held.pop(ticket, None)
        return r

    def cancel(self, ticket):
        tpf.tpf_server_cancel(self.sv, ticket)

    def stats(self):
        return tpf.tpf_server_stats(self.sv)

    def drain(self, tickets):
        """Steps until every ticket has a result; returns {ticket: Result}."""
        out = {}
        pending = set(tickets)
        while pending:
            self.step()
            for t in list(pending):
                r = self.poll(t)
                if r is not None:
                    out[t] = r
                    pending.discard(t)
        return out

    def close(self):
        if tpf.shutting_down():
            return
        if self.sv is not None:
            tpf.tpf_server_destroy(self.sv)
            self.sv = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def newton_states(gcase, n_states, kind="bf", ds_max=0.2, rtol=1e-8):
    """The first n_states Newton iterates u_0..u_{n-1} of gcase's time step
    (FP64 solves, full setups), as a list of device tensors; gcase.u is left
    at its initial value."""
    M = GpuPrecond(kind)
    u0 = gcase.u.clone()
    states = [u0.clone()]
    if n_states > 1:
        newton_sequence(gcase, M, n_states - 1, ds_max=ds_max, rtol=rtol,
                        on_step=lambda rec: states.append(gcase.u.clone()))
    gcase.u.copy_(u0)
    M.close()
    import torch
    torch.cuda.synchronize()
    return states
