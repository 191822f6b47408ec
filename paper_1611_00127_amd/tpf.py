"""Thin Python binding of libtpf (include/tpf.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own.  Device arrays are torch CUDA tensors (float64,
contiguous); host arrays are numpy arrays.  Device memory of the library is
drawn from torch's caching allocator.  Importing this module fails loudly
when the HIP library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpf.so")

# ---- constants (mirror include/tpf.h) -------------------------------------
TPF_OK = 0
TPF_PC_BROOKS_COREY, TPF_PC_LINEAR = 0, 1
TPF_PREC_AMG, TPF_PREC_CPR1, TPF_PREC_CPR2, TPF_PREC_BF, TPF_PREC_NONE = 0, 1, 2, 3, 4
TPF_FP64, TPF_FP32 = 0, 1
TPF_SMOOTH_L1_JACOBI, TPF_SMOOTH_CHEBYSHEV, TPF_SMOOTH_MC_GS = 0, 1, 2
TPF_COARSEN_PMIS, TPF_COARSEN_CLJP = 0, 1
TPF_CONVERGED, TPF_MAX_ITERS, TPF_BREAKDOWN, TPF_NONFINITE, TPF_CANCELLED = 0, 1, 2, 3, 4
TPF_ERR_OVER_BUDGET = -5
TPF_MAT_A, TPF_MAT_P, TPF_MAT_R, TPF_MAT_S, TPF_MAT_GS_COLORS = 0, 1, 2, 3, 4
TPF_MAT_APS, TPF_MAT_SCHUR = 10, 11
TPF_MAX_LEVELS = 25
TPF_INTERP_AUTO, TPF_INTERP_DIRECT, TPF_INTERP_EXTI, TPF_INTERP_CLASSICAL = 0, 1, 2, 3
KINDS = {"amg": TPF_PREC_AMG, "cpr1": TPF_PREC_CPR1, "cpr2": TPF_PREC_CPR2, "bf": TPF_PREC_BF,
         "none": TPF_PREC_NONE}

c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
c_int64, c_uint64 = ctypes.c_int64, ctypes.c_uint64
P_int, P_double = ctypes.POINTER(c_int), ctypes.POINTER(c_double)


class ProblemDesc(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int),
                ("hx", c_double), ("hy", c_double), ("hz", c_double),
                ("kx", c_void_p), ("ky", c_void_p), ("kz", c_void_p), ("poro", c_void_p),
                ("mu_w", c_double), ("mu_n", c_double),
                ("rho_w", c_double), ("rho_n", c_double), ("grav", c_double),
                ("pc_model", c_int), ("bc_lambda", c_double), ("swr", c_double), ("snr", c_double),
                ("pd", c_double), ("s_eps", c_double), ("q", c_void_p),
                ("n_prod", c_int), ("prod_cells", P_int), ("prod_wi", P_double), ("prod_pbh", P_double),
                ("n_dir", c_int), ("dir_cells", P_int), ("dir_face", P_int),
                ("dir_p", P_double), ("dir_s", P_double)]


class BcsrView(ctypes.Structure):
    _fields_ = [("n_block_rows", c_int), ("nnzb", c_int64), ("row_ptr", c_void_p),
                ("col_idx", c_void_p), ("vals", c_void_p)]


class CsrView(ctypes.Structure):
    _fields_ = [("n_rows", c_int), ("n_cols", c_int), ("nnz", c_int64), ("row_ptr", c_void_p),
                ("col_idx", c_void_p), ("vals", c_void_p)]


class PrecondOpts(ctypes.Structure):
    _fields_ = [("kind", c_int), ("precision", c_int), ("theta", c_double), ("max_levels", c_int),
                ("coarse_max", c_int), ("dense_max", c_int), ("interp", c_int),
                ("hash_seed", c_uint64), ("exti_route", c_int), ("smoother", c_int),
                ("nu1", c_int), ("nu2", c_int), ("cheb_degree", c_int), ("coarsening", c_int),
                ("trunc_pmax", c_int), ("trunc_factor", c_double)]


class HierStats(ctypes.Structure):
    _fields_ = [("n_hier", c_int), ("levels", c_int * 3),
                ("rows", (c_int64 * TPF_MAX_LEVELS) * 3), ("nnz", (c_int64 * TPF_MAX_LEVELS) * 3),
                ("p_nnz", (c_int64 * TPF_MAX_LEVELS) * 3),
                ("operator_complexity", c_double * 3), ("grid_complexity", c_double * 3),
                ("coarse_dense", c_int * 3), ("l0_diagonals", c_int * 3),
                ("coarse_smooth_sweeps", c_int * 3),
                ("device_bytes", c_size_t), ("hier_bytes", c_size_t * 3)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", c_double), ("restart", c_int), ("maxit", c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", c_int), ("iterations", c_int), ("relres_est", c_double),
                ("relres_true", c_double), ("ms", c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", c_size_t), ("max_active", c_int), ("kind", c_int),
                ("precision", c_int), ("reuse", c_int), ("solve", SolveOpts)]


class Request(ctypes.Structure):
    _fields_ = [("sequence", c_uint64), ("problem", c_void_p), ("u", c_void_p),
                ("u_old", c_void_p), ("dt", c_double), ("x", c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", c_int), ("iterations", c_int), ("relres_est", c_double),
                ("relres_true", c_double), ("setup_ms", c_double), ("solve_ms", c_double),
                ("latency_ms", c_double), ("refreshed", c_int),
                ("reserved_bytes", c_size_t)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("queued", c_int), ("active", c_int), ("resident_sequences", c_int),
                ("submitted", c_int64), ("completed", c_int64), ("bytes_in_use", c_size_t),
                ("peak_bytes", c_size_t), ("evictions", c_int64)]


class TpfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tpf error {code}: {msg}")
        self.code = code


_lib = None
_alloc_cb = None
_free_cb = None
_shutting_down = False
_alloc_calls = 0  # requests the library made to torch's allocator
_held = {}         # pointer -> bytes the library holds from torch's allocator
_held_bytes = 0
_held_peak = 0


def _mark_shutdown():
    # after this point handles are leaked instead of destroyed: the allocator
    # callbacks must not run while the interpreter is being torn down
    global _shutting_down
    _shutting_down = True


import atexit  # noqa: E402

atexit.register(_mark_shutdown)


def shutting_down():
    return _shutting_down

_SIGS = {
    "tpf_status_string": (ctypes.c_char_p, [c_int]),
    "tpf_last_error": (c_int, [ctypes.c_char_p, c_size_t]),
    "tpf_set_allocator": (c_int, [c_void_p, c_void_p, c_void_p]),
    "tpf_memory_in_use": (c_int, [ctypes.POINTER(c_size_t)]),
    "tpf_release_cached_memory": (c_int, []),
    "tpf_problem_create": (c_int, [ctypes.POINTER(ProblemDesc), c_void_p, ctypes.POINTER(c_void_p)]),
    "tpf_problem_destroy": (c_int, [c_void_p]),
    "tpf_problem_cells": (c_int, [c_void_p, ctypes.POINTER(c_int64)]),
    "tpf_jacobian_create": (c_int, [c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "tpf_jacobian_destroy": (c_int, [c_void_p]),
    "tpf_assemble": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "tpf_jacobian_view": (c_int, [c_void_p, ctypes.POINTER(BcsrView)]),
    "tpf_spmv": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "tpf_newton_update": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double, c_void_p]),
    "tpf_norm2": (c_int, [c_void_p, c_int64, ctypes.POINTER(c_double), c_void_p]),
    "tpf_precond_default_opts": (c_int, [c_int, ctypes.POINTER(PrecondOpts)]),
    "tpf_precond_create": (c_int, [ctypes.POINTER(PrecondOpts), ctypes.POINTER(c_void_p)]),
    "tpf_precond_destroy": (c_int, [c_void_p]),
    "tpf_precond_setup": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    "tpf_precond_apply": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "tpf_precond_stats": (c_int, [c_void_p, ctypes.POINTER(HierStats)]),
    "tpf_precond_matrix": (c_int, [c_void_p, c_int, c_int, c_int, ctypes.POINTER(CsrView)]),
    "tpf_precond_level_data": (c_int, [c_void_p, c_int, c_int, ctypes.POINTER(c_void_p),
                                       ctypes.POINTER(c_void_p), ctypes.POINTER(c_int)]),
    "tpf_precond_bilu_dinv": (c_int, [c_void_p, ctypes.POINTER(c_void_p)]),
    "tpf_precond_vcycle": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "tpf_csr_product": (c_int, [ctypes.POINTER(CsrView), ctypes.POINTER(CsrView),
                                ctypes.POINTER(CsrView), c_double, c_double, c_int, c_int,
                                c_void_p, c_void_p, c_void_p, c_int64, ctypes.POINTER(c_int64),
                                c_void_p]),
    "tpf_csr_transpose": (c_int, [ctypes.POINTER(CsrView), c_void_p, c_void_p, c_void_p, c_void_p]),
    "tpf_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveOpts),
                          ctypes.POINTER(SolveInfo), c_void_p]),
    "tpf_solve_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p,
                                  ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), c_void_p]),
    "tpf_server_default_opts": (c_int, [ctypes.POINTER(ServerOpts)]),
    "tpf_server_create": (c_int, [ctypes.POINTER(ServerOpts), ctypes.POINTER(c_void_p)]),
    "tpf_server_submit": (c_int, [c_void_p, ctypes.POINTER(Request), ctypes.POINTER(c_uint64)]),
    "tpf_server_step": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "tpf_server_poll": (c_int, [c_void_p, c_uint64, ctypes.POINTER(Result)]),
    "tpf_server_cancel": (c_int, [c_void_p, c_uint64]),
    "tpf_server_stats": (c_int, [c_void_p, ctypes.POINTER(ServerCounters)]),
    "tpf_server_destroy": (c_int, [c_void_p]),
    "tpf_kernel_timing": (c_int, [c_int]),
    "tpf_set_graphs": (c_int, [c_int]),
    "tpf_kernel_stats": (c_int, [ctypes.c_char_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_double)]),
    "tpf_kernel_stats_reset": (c_int, []),
}


def exported_symbols():
    return sorted(_SIGS)


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libtpf.so (no GPU needed) and declares every signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1611_00127_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != TPF_OK:
        buf = ctypes.create_string_buffer(1024)
        _lib.tpf_last_error(buf, 1024)
        raise TpfError(rc, buf.value.decode(errors="replace"))


def _ptr(t):
    """Device pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def use_torch_allocator():
    """Routes all library device allocations through torch's caching allocator."""
    global _alloc_cb, _free_cb
    import torch
    lib = load()
    ALLOC = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p, c_void_p)
    FREE = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)

    def _a(nbytes, stream, ctx):
        global _alloc_calls, _held_bytes, _held_peak
        _alloc_calls += 1
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:
            return None
        _held[p] = int(nbytes)
        _held_bytes += int(nbytes)
        _held_peak = max(_held_peak, _held_bytes)
        return p

    def _f(p, stream, ctx):
        global _held_bytes
        _held_bytes -= _held.pop(int(p), 0)
        if not _shutting_down:
            torch.cuda.caching_allocator_delete(int(p))

    _alloc_cb, _free_cb = ALLOC(_a), FREE(_f)
    _check(lib.tpf_set_allocator(ctypes.cast(_alloc_cb, c_void_p), ctypes.cast(_free_cb, c_void_p), None))


def allocator_calls():
    """Number of device allocations the library has requested from torch's
    caching allocator in this process (blocks it reuses from its own cache
    are not requests)."""
    return _alloc_calls


def allocator_bytes():
    """(current, peak) device bytes the library holds from torch's caching
    allocator: blocks in use plus the freed blocks it keeps cached."""
    return _held_bytes, _held_peak


def reset_allocator_peak():
    global _held_peak
    _held_peak = _held_bytes


def init(torch_allocator=True):
    """Loads the library for GPU use; raises if HIP/torch has no device.
    Library memory comes from torch's caching allocator, or with
    torch_allocator=False from the device's stream-ordered pool."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the HIP library needs an MI355X (gfx950)")
    load()
    if torch_allocator and _alloc_cb is None:
        use_torch_allocator()
    return _lib


def tpf_release_cached_memory():
    _check(load().tpf_release_cached_memory())


# ---- entry points (same names as the C ABI) --------------------------------

def tpf_status_string(code):
    return load().tpf_status_string(code).decode()


def tpf_memory_in_use():
    v = c_size_t()
    _check(load().tpf_memory_in_use(ctypes.byref(v)))
    return v.value


def tpf_problem_create(nx, ny, nz, hx, hy, hz, kx, ky, kz, poro, mu_w, mu_n, rho_w, rho_n, grav,
                       pc_model, bc_lambda, swr, snr, pd, s_eps, q=None,
                       prod_cells=None, prod_wi=None, prod_pbh=None,
                       dir_cells=None, dir_face=None, dir_p=None, dir_s=None, stream=None):
    lib = init()
    keep = []

    def host(a, dt, ct):
        if a is None or len(a) == 0:
            return None, 0
        arr = np.ascontiguousarray(a, dtype=dt)
        keep.append(arr)
        return arr.ctypes.data_as(ctypes.POINTER(ct)), len(arr)

    pc, npc = host(prod_cells, np.int32, c_int)
    pw, _ = host(prod_wi, np.float64, c_double)
    pb, _ = host(prod_pbh, np.float64, c_double)
    dc, ndc = host(dir_cells, np.int32, c_int)
    df, _ = host(dir_face, np.int32, c_int)
    dpv, _ = host(dir_p, np.float64, c_double)
    dsv, _ = host(dir_s, np.float64, c_double)
    d = ProblemDesc(nx, ny, nz, hx, hy, hz, _ptr(kx), _ptr(ky), _ptr(kz), _ptr(poro),
                    mu_w, mu_n, rho_w, rho_n, grav, pc_model, bc_lambda, swr, snr, pd, s_eps,
                    _ptr(q), npc, pc, pw, pb, ndc, dc, df, dpv, dsv)
    out = c_void_p()
    _check(lib.tpf_problem_create(ctypes.byref(d), _stream(stream), ctypes.byref(out)))
    return out


def tpf_problem_destroy(p):
    _check(load().tpf_problem_destroy(p))


def tpf_jacobian_create(p, stream=None):
    out = c_void_p()
    _check(load().tpf_jacobian_create(p, _stream(stream), ctypes.byref(out)))
    return out


def tpf_jacobian_destroy(J):
    _check(load().tpf_jacobian_destroy(J))


def tpf_assemble(p, u, u_old, dt, residual, J, stream=None):
    _check(load().tpf_assemble(p, _ptr(u), _ptr(u_old), dt, _ptr(residual), J, _stream(stream)))


def tpf_jacobian_view(J):
    v = BcsrView()
    _check(load().tpf_jacobian_view(J, ctypes.byref(v)))
    return v


def tpf_spmv(J, x, y, stream=None):
    _check(load().tpf_spmv(J, _ptr(x), _ptr(y), _stream(stream)))


def tpf_newton_update(p, u, delta, ds_max=0.0, alpha=1.0, stream=None):
    _check(load().tpf_newton_update(p, _ptr(u), _ptr(delta), float(alpha), float(ds_max),
                                    _stream(stream)))


def tpf_norm2(x, stream=None):
    out = c_double()
    _check(load().tpf_norm2(_ptr(x), x.numel(), ctypes.byref(out), _stream(stream)))
    return out.value


def tpf_precond_default_opts(kind):
    o = PrecondOpts()
    _check(load().tpf_precond_default_opts(kind, ctypes.byref(o)))
    return o


def tpf_precond_create(opts):
    out = c_void_p()
    _check(load().tpf_precond_create(ctypes.byref(opts), ctypes.byref(out)))
    return out


def tpf_precond_destroy(M):
    _check(load().tpf_precond_destroy(M))


def tpf_precond_setup(M, J, reuse_structure=0, stream=None):
    _check(load().tpf_precond_setup(M, J, int(reuse_structure), _stream(stream)))


def tpf_precond_apply(M, r, z, stream=None):
    _check(load().tpf_precond_apply(M, _ptr(r), _ptr(z), _stream(stream)))


def tpf_precond_stats(M):
    s = HierStats()
    _check(load().tpf_precond_stats(M, ctypes.byref(s)))
    return s


def tpf_precond_matrix(M, hier, level, which):
    v = CsrView()
    _check(load().tpf_precond_matrix(M, hier, level, which, ctypes.byref(v)))
    return v


def tpf_precond_level_data(M, hier, level):
    cf, dinv, n = c_void_p(), c_void_p(), c_int()
    _check(load().tpf_precond_level_data(M, hier, level, ctypes.byref(cf), ctypes.byref(dinv),
                                         ctypes.byref(n)))
    return cf.value, dinv.value, n.value


def tpf_precond_bilu_dinv(M):
    p = c_void_p()
    _check(load().tpf_precond_bilu_dinv(M, ctypes.byref(p)))
    return p.value


def tpf_precond_vcycle(M, hier, b, x, stream=None):
    _check(load().tpf_precond_vcycle(M, hier, _ptr(b), _ptr(x), _stream(stream)))


def _csr_arg(m):
    """CsrView of a (row_ptr, col_idx, vals, n_cols) tuple of device tensors."""
    rp, ci, v, ncols = m
    return CsrView(len(rp) - 1, int(ncols), len(ci), _ptr(rp).value, _ptr(ci).value,
                   _ptr(v).value)


def tpf_csr_product(A, B, D=None, alpha=1.0, beta=1.0, route=0, pattern=None, stream=None):
    """C = alpha A B (+ beta D).  A, B, D: (row_ptr, col_idx, vals, n_cols) with
    int32 / float64 device tensors.  Returns (row_ptr, col_idx, vals) device
    tensors; with pattern = (row_ptr, col_idx) only the values are computed."""
    import torch
    lib = load()
    a, b = _csr_arg(A), _csr_arg(B)
    d = ctypes.byref(_csr_arg(D)) if D is not None else None
    n = len(A[0]) - 1
    dev = A[0].device
    nnz = c_int64()
    if pattern is not None:
        rp, ci = pattern
        v = torch.empty(max(len(ci), 1), dtype=torch.float64, device=dev)
        _check(lib.tpf_csr_product(ctypes.byref(a), ctypes.byref(b), d, alpha, beta, route, 1,
                                   _ptr(rp), _ptr(ci), _ptr(v), len(ci), ctypes.byref(nnz),
                                   _stream(stream)))
        return rp, ci, v[:len(ci)]
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    _check(lib.tpf_csr_product(ctypes.byref(a), ctypes.byref(b), d, alpha, beta, route, 0,
                               _ptr(rp), None, None, 0, ctypes.byref(nnz), _stream(stream)))
    m = nnz.value
    ci = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    v = torch.empty(max(m, 1), dtype=torch.float64, device=dev)
    _check(lib.tpf_csr_product(ctypes.byref(a), ctypes.byref(b), d, alpha, beta, route, 0,
                               _ptr(rp), _ptr(ci), _ptr(v), m, ctypes.byref(nnz),
                               _stream(stream)))
    return rp, ci[:m], v[:m]


def tpf_csr_transpose(A, stream=None):
    """A^T of A = (row_ptr, col_idx, vals, n_cols) device tensors; returns
    (row_ptr, col_idx, vals) device tensors."""
    import torch
    a = _csr_arg(A)
    dev = A[0].device
    m, nnz = int(A[3]), len(A[1])
    rp = torch.empty(m + 1, dtype=torch.int32, device=dev)
    ci = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    v = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
    _check(load().tpf_csr_transpose(ctypes.byref(a), _ptr(rp), _ptr(ci), _ptr(v), _stream(stream)))
    return rp, ci[:nnz], v[:nnz]


def tpf_solve(J, M, b, x, rtol=1e-8, restart=30, maxit=1000, stream=None):
    o = SolveOpts(rtol, restart, maxit)
    info = SolveInfo()
    _check(load().tpf_solve(J, M, _ptr(b), _ptr(x), ctypes.byref(o), ctypes.byref(info),
                            _stream(stream)))
    return info


def tpf_solve_noalloc(J, M, b, x, rtol=1e-8, restart=30, maxit=1000, stream=None):
    o = SolveOpts(rtol, restart, maxit)
    info = SolveInfo()
    _check(load().tpf_solve_noalloc(J, M, _ptr(b), _ptr(x), ctypes.byref(o), ctypes.byref(info),
                                    _stream(stream)))
    return info


def tpf_server_default_opts():
    o = ServerOpts()
    _check(load().tpf_server_default_opts(ctypes.byref(o)))
    return o


def tpf_server_create(opts):
    h = c_void_p()
    _check(load().tpf_server_create(ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def tpf_server_submit(sv, sequence, problem, u, u_old, dt, x):
    rq = Request(sequence, problem, _ptr(u), _ptr(u_old), dt, _ptr(x))
    t = c_uint64()
    _check(load().tpf_server_submit(sv, ctypes.byref(rq), ctypes.byref(t)))
    return t.value


def tpf_server_step(sv):
    n = c_int()
    _check(load().tpf_server_step(sv, ctypes.byref(n)))
    return n.value


def tpf_server_poll(sv, ticket):
    """The Result of a finished request (released by this call), else None."""
    r = Result()
    rc = load().tpf_server_poll(sv, ticket, ctypes.byref(r))
    if rc < 0:
        _check(rc)
    return r if rc == 1 else None


def tpf_server_cancel(sv, ticket):
    _check(load().tpf_server_cancel(sv, ticket))


def tpf_server_stats(sv):
    c = ServerCounters()
    _check(load().tpf_server_stats(sv, ctypes.byref(c)))
    return c


def tpf_server_destroy(sv):
    _check(load().tpf_server_destroy(sv))


def tpf_kernel_timing(enable):
    _check(load().tpf_kernel_timing(int(bool(enable))))


def tpf_set_graphs(enable):
    _check(load().tpf_set_graphs(int(bool(enable))))


def tpf_kernel_stats(name):
    cnt, ms = c_int64(), c_double()
    _check(load().tpf_kernel_stats(name.encode(), ctypes.byref(cnt), ctypes.byref(ms)))
    return cnt.value, ms.value


def tpf_kernel_stats_reset():
    _check(load().tpf_kernel_stats_reset())


# ---- device <-> host copies of library-owned arrays (marshalling) -----------

def device_array(ptr, count, dtype):
    """Copies `count` elements of a library-owned device array to numpy."""
    import torch
    tdt = {np.int32: torch.int32, np.float64: torch.float64, np.int8: torch.int8,
           np.uint8: torch.uint8, np.float32: torch.float32}[dtype]
    out = torch.empty(count, dtype=tdt)
    if count == 0:
        return out.numpy()
    import ctypes as ct
    hip = _hip_runtime()
    torch.cuda.synchronize()
    rc = hip.hipMemcpy(ct.c_void_p(out.data_ptr()), ct.c_void_p(ptr), ct.c_size_t(count * out.element_size()), 2)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed: {rc}")
    return out.numpy()


_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = c_int
        _hip.hipMemcpy.argtypes = [c_void_p, c_void_p, c_size_t, c_int]
    return _hip


def csr_to_numpy(view):
    """(row_ptr, col_idx, vals or None) numpy copies of a tpf_csr_view."""
    rp = device_array(view.row_ptr, view.n_rows + 1, np.int32)
    ci = device_array(view.col_idx, int(view.nnz), np.int32)
    v = device_array(view.vals, int(view.nnz), np.float64) if view.vals else None
    return rp, ci, v
