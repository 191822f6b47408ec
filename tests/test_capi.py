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
