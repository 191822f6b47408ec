"""The C-ABI library loads and exports every symbol include/tpf.h declares;
host-side argument checks return the documented codes (no GPU work)."""
import ctypes
import os
import re

import pytest

from paper_1611_00127_amd import tpf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "tpf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpf_[a-z0-9_]+)\s*\(", text)) - {"tpf_alloc_fn", "tpf_free_fn"})


def test_library_exports_every_declared_symbol():
    lib = tpf.load()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == tpf.exported_symbols()


def test_host_side_errors_without_gpu():
    lib = tpf.load()
    o = tpf.tpf_precond_default_opts(tpf.TPF_PREC_BF)
    assert o.theta == 0.25 and o.max_levels == 25 and o.coarse_max == 128
    M = tpf.tpf_precond_create(o)
    # apply before setup is a state error, detected before any device work
    rc = lib.tpf_precond_apply(M, None, None, None)
    assert rc == -1  # null vectors are rejected first
    r = ctypes.c_void_p(8)
    rc = lib.tpf_precond_apply(M, r, r, None)
    assert rc == -7
    buf = ctypes.create_string_buffer(256)
    assert lib.tpf_last_error(buf, 256) == -7
    assert b"not set up" in buf.value
    tpf.tpf_precond_destroy(M)
    bad = tpf.tpf_precond_default_opts(tpf.TPF_PREC_BF)
    bad.max_levels = 99
    with pytest.raises(tpf.TpfError) as e:
        tpf.tpf_precond_create(bad)
    assert e.value.code == -1
    assert tpf.tpf_status_string(-4) == "singular pivot"


def test_amg_variant_options_host_checks():
    """The options of the paper's AMG components (classical interpolation,
    multicolour Gauss-Seidel, CLJP) are accepted, their defaults are PMIS /
    l1-Jacobi / the automatic interpolation, and out-of-range values are
    rejected before any device work."""
    o = tpf.tpf_precond_default_opts(tpf.TPF_PREC_BF)
    assert o.coarsening == tpf.TPF_COARSEN_PMIS and o.smoother == tpf.TPF_SMOOTH_L1_JACOBI
    assert o.interp == tpf.TPF_INTERP_AUTO and o.nu1 == 1 and o.nu2 == 1
    good = dict(interp=tpf.TPF_INTERP_CLASSICAL, smoother=tpf.TPF_SMOOTH_MC_GS,
                coarsening=tpf.TPF_COARSEN_CLJP)
    o2 = tpf.tpf_precond_default_opts(tpf.TPF_PREC_BF)
    for k, v in good.items():
        setattr(o2, k, v)
    tpf.tpf_precond_destroy(tpf.tpf_precond_create(o2))
    for field, bad_value in (("interp", 4), ("smoother", 3), ("coarsening", 2), ("coarsening", -1)):
        b = tpf.tpf_precond_default_opts(tpf.TPF_PREC_BF)
        setattr(b, field, bad_value)
        with pytest.raises(tpf.TpfError) as e:
            tpf.tpf_precond_create(b)
        assert e.value.code == -1, (field, bad_value)


def test_noalloc_solve_host_checks():
    """tpf_solve_noalloc rejects null arguments and restarts outside
    [1, 64] before any device work."""
    lib = tpf.load()
    o = tpf.SolveOpts(1e-8, 30, 1000)
    info = tpf.SolveInfo()
    assert lib.tpf_solve_noalloc(None, None, None, None, ctypes.byref(o), ctypes.byref(info),
                                 None) == -1
    p = ctypes.c_void_p(8)
    o.restart = 0
    assert lib.tpf_solve_noalloc(p, None, p, p, ctypes.byref(o), ctypes.byref(info), None) == -1
    buf = ctypes.create_string_buffer(256)
    lib.tpf_last_error(buf, 256)
    assert b"restart" in buf.value


def test_server_host_side_checks():
    lib = tpf.load()
    o = tpf.tpf_server_default_opts()
    assert o.kind == tpf.TPF_PREC_BF and o.precision == tpf.TPF_FP32 and o.reuse == 1
    assert o.max_active == 8 and o.hbm_budget_bytes == 64 << 30
    assert o.solve.rtol == 1e-8 and o.solve.restart == 30
    bad = tpf.tpf_server_default_opts()
    bad.max_active = 0
    h = ctypes.c_void_p()
    assert lib.tpf_server_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad = tpf.tpf_server_default_opts()
    bad.solve.restart = 65
    assert lib.tpf_server_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    t = ctypes.c_uint64()
    assert lib.tpf_server_submit(None, None, ctypes.byref(t)) == -1
    assert lib.tpf_server_poll(None, 1, None) == -1
