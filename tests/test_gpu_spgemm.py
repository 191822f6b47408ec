"""GPU parity of the sparse product kernels (tpf_csr_product, the SpGEMM
behind the Galerkin products of Sec. 3.2 and S~ of Sec. 3.4) against the
oracle's symbolic pattern and scipy's product placed on it.

Every kernel class is driven: the automatic choice by product count, and
each forced floor (route r: rows start at class r - 1), on rows with 0 to
~20,000 products, empty rows, long runs of one column (sums spanning many
threads and wavefronts), an added matrix D, 64-bit keys (many columns) and the
numeric refresh on a known pattern.  Bars: pattern bit-exact; values within
1e-12 of the row's largest magnitude (sums in a different order).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import blocks

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_1611_00127_amd import tpf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tpf.init()
    return tpf, torch


def _random_csr(rng, lengths, ncols, window=None):
    """CSR with the given row lengths, distinct sorted columns (from
    [0, window) when given) and values in [0.5, 1.5)."""
    rows, cols = [], []
    for i, m in enumerate(lengths):
        hi = window if window else ncols
        m = min(m, hi)
        c = np.sort(rng.choice(hi, size=m, replace=False)) if m else np.zeros(0, np.int64)
        rows.append(np.full(m, i)); cols.append(c)
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    M = sp.csr_matrix((0.5 + rng.random(len(r)), (r, c)), shape=(len(lengths), ncols))
    M.sort_indices()
    return M


def _dev(torch, M):
    return (torch.tensor(M.indptr, dtype=torch.int32, device="cuda"),
            torch.tensor(M.indices, dtype=torch.int32, device="cuda"),
            torch.tensor(M.data, dtype=torch.float64, device="cuda"), M.shape[1])


def _expected(A, B, D, alpha, beta):
    pat = blocks.symbolic_product(A, B)
    val = alpha * (A @ B)
    if D is not None:
        pat = (pat + blocks.ones_like_pattern(D)).tocsr()
        pat.sort_indices()
        val = val + beta * D
    return blocks.place_on_pattern(pat, val)


def _check(tpf, torch, A, B, D=None, alpha=1.0, beta=1.0, route=0, label=""):
    E = _expected(A, B, D, alpha, beta)
    out = tpf.tpf_csr_product(_dev(torch, A), _dev(torch, B),
                              _dev(torch, D) if D is not None else None, alpha, beta, route)
    rp, ci, v = (t.cpu().numpy() for t in out)
    assert np.array_equal(rp, E.indptr), f"{label} row pointers"
    assert np.array_equal(ci, E.indices), f"{label} columns"
    rows = np.repeat(np.arange(E.shape[0]), np.diff(E.indptr))
    scale = np.zeros(E.shape[0])
    np.maximum.at(scale, rows, np.abs(E.data))
    err = np.abs(v - E.data) / np.maximum(scale[rows], 1e-300) if len(v) else np.zeros(1)
    say(f"  {label}: nnz {len(ci)}, worst {err.max():.2e}")
    assert err.max() <= 1e-12, label
    return out, E


def _mixed(rng, ncols_b=3000, window=None, max_la=2100):
    """B: rows of 0..21 entries plus 8 rows of 2,500; A: rows of 0 to max_la
    entries over the short B rows (up to ~14,000 products; rows longer than
    2,048 entries go past the register-sorted classes), and 6 rows of 10
    entries that take all 8 long B rows (~20,000 products, past the LDS-sorted
    class)."""
    nb = 4000
    lb = np.array([0, 1, 2, 3, 5, 8, 13, 21])[np.arange(nb) % 8]
    long_rows = np.arange(0, nb, 500)
    lb[long_rows] = 2500
    B = _random_csr(rng, lb, ncols_b, window)
    short = np.setdiff1d(np.arange(nb), long_rows)
    la_set = [x for x in [0, 1, 2, 5, 9, 17, 33, 70, 140, 300, 700, 1300, 2100] if x <= max_la]
    la = [la_set[i % len(la_set)] for i in range(600)]
    rng.shuffle(la)
    rows, cols = [], []
    for i, m in enumerate(la):
        c = np.sort(rng.choice(short, size=m, replace=False))
        rows.append(np.full(m, i)); cols.append(c)
    for r in range(6):
        i = 100 * r + 7
        c = np.sort(np.concatenate([long_rows, rng.choice(short, size=2, replace=False)]))
        rows[i] = np.full(len(c), i); cols[i] = c
    r = np.concatenate(rows); c = np.concatenate(cols)
    A = sp.csr_matrix((0.5 + rng.random(len(r)), (r, c)), shape=(600, nb))
    A.sort_indices()
    return A, B


@pytest.mark.parametrize("route", list(range(10)))
def test_product_every_class(gpu, route):
    tpf, torch = gpu
    rng = np.random.default_rng(11)
    # the per-row merge costs (outputs x A's row length) per thread: shorter
    # A rows when every row is forced there
    A, B = _mixed(rng, max_la=300 if route == 9 else 2100)
    say(f"[spgemm] mixed rows, route {route}")
    _check(tpf, torch, A, B, route=route, label=f"route {route}")


@pytest.mark.parametrize("route", [0, 5, 6, 7, 8])
def test_product_long_runs(gpu, route):
    """Products concentrated on 5 columns: runs of up to ~5,000 equal
    columns, spanning threads and wavefronts."""
    tpf, torch = gpu
    rng = np.random.default_rng(12)
    A, B = _mixed(rng, window=5)
    say(f"[spgemm] long runs, route {route}")
    _check(tpf, torch, A, B, route=route, label=f"long runs route {route}")


@pytest.mark.parametrize("route", [0, 6, 9])
def test_product_with_added_matrix(gpu, route):
    """C = -A B + D on the union pattern (the S~ form)."""
    tpf, torch = gpu
    rng = np.random.default_rng(13)
    A, B = _mixed(rng, max_la=300 if route == 9 else 2100)
    ld = np.array([0, 1, 4, 30, 100])[np.arange(A.shape[0]) % 5]
    D = _random_csr(rng, ld, B.shape[1])
    say(f"[spgemm] with D, route {route}")
    _check(tpf, torch, A, B, D, alpha=-1.0, beta=1.0, route=route, label=f"D route {route}")


@pytest.mark.parametrize("route", [0, 4, 5, 6, 7])
def test_product_wide_keys(gpu, route):
    """8,388,613 columns: the 512-, 1024-, 2048- and 8192-product classes take
    64-bit (column, index) keys."""
    tpf, torch = gpu
    rng = np.random.default_rng(14)
    A, B = _mixed(rng, ncols_b=(1 << 23) + 5)
    say(f"[spgemm] 2^23+5 columns, route {route}")
    _check(tpf, torch, A, B, route=route, label=f"wide route {route}")


@pytest.mark.parametrize("route", [0, 2])
def test_product_wide_keys_small_rows(gpu, route):
    """67,108,869 columns: even the smallest classes (lane groups of 16,
    four rows per wavefront) take 64-bit keys."""
    tpf, torch = gpu
    rng = np.random.default_rng(17)
    nb, ncols = 500, (1 << 26) + 5
    B = _random_csr(rng, np.arange(nb) % 6, ncols)
    A = _random_csr(rng, np.arange(300) % 31, nb)
    say(f"[spgemm] 2^26+5 columns, small rows, route {route}")
    _check(tpf, torch, A, B, route=route, label=f"wide small route {route}")


def test_product_refresh_and_edges(gpu):
    tpf, torch = gpu
    rng = np.random.default_rng(15)
    A, B = _mixed(rng)
    ld = np.array([0, 3, 50])[np.arange(A.shape[0]) % 3]
    D = _random_csr(rng, ld, B.shape[1])
    (rp, ci, _), E = _check(tpf, torch, A, B, D, alpha=-1.0, beta=1.0, label="pattern")
    # numeric refresh: new values on the same patterns
    A2, B2, D2 = A.copy(), B.copy(), D.copy()
    A2.data = 0.5 + rng.random(A.nnz); B2.data = 0.5 + rng.random(B.nnz)
    D2.data = 0.5 + rng.random(D.nnz)
    _, _, v2 = tpf.tpf_csr_product(_dev(torch, A2), _dev(torch, B2), _dev(torch, D2), -1.0, 1.0,
                                   pattern=(rp, ci))
    E2 = _expected(A2, B2, D2, -1.0, 1.0)
    assert np.array_equal(E2.indices, ci.cpu().numpy())
    v2 = v2.cpu().numpy()
    assert np.max(np.abs(v2 - E2.data) / np.abs(E2.data).max()) <= 1e-12
    # no entries at all, and a matrix with no rows
    Z = sp.csr_matrix((A.shape[0], A.shape[1]))
    _check(tpf, torch, Z, B, label="empty A")
    _check(tpf, torch, sp.csr_matrix((0, A.shape[1])), B, label="no rows")
    # malformed input is refused before any product kernel runs
    bad = B.copy()
    s, e = bad.indptr[5], bad.indptr[6]
    assert e - s >= 2
    bad.indices[s], bad.indices[s + 1] = bad.indices[s + 1], bad.indices[s]
    with pytest.raises(tpf.TpfError):
        tpf.tpf_csr_product(_dev(torch, A), _dev(torch, bad))
    with pytest.raises(tpf.TpfError):
        tpf.tpf_csr_product(_dev(torch, A), _dev(torch, B), route=10)


def test_transpose_every_row_class(gpu):
    """Transposes whose rows span every sorting path: up to 16 entries (a
    lane group per row), up to 1,024 (a wavefront), up to 4,096 (a
    work-group) and beyond (one thread), against scipy's transpose."""
    tpf, torch = gpu
    rng = np.random.default_rng(16)
    n, m = 6000, 3000
    # column 0 in every row (6,000 entries in its transposed row), column 1 in
    # every third (2,000), column 2 in every twelfth (500), plus 0-7 others
    rows, cols = [], []
    for i in range(n):
        extra = rng.choice(np.arange(3, m), size=rng.integers(0, 8), replace=False)
        c = np.unique(np.concatenate([[0], [1] if i % 3 == 0 else [], [2] if i % 12 == 0 else [],
                                      extra]).astype(np.int64))
        rows.append(np.full(len(c), i)); cols.append(c)
    r = np.concatenate(rows); c = np.concatenate(cols)
    A = sp.csr_matrix((0.5 + rng.random(len(r)), (r, c)), shape=(n, m))
    A.sort_indices()
    T = A.T.tocsr(); T.sort_indices()
    lens = np.diff(T.indptr)
    say(f"[transpose] row lengths of A^T: max {lens.max()}, >16: {(lens > 16).sum()}, "
        f">1024: {(lens > 1024).sum()}, >4096: {(lens > 4096).sum()}")
    assert (lens <= 16).any() and (lens > 1024).any() and (lens > 4096).any()
    rp, ci, v = (t.cpu().numpy() for t in tpf.tpf_csr_transpose(_dev(torch, A)))
    assert np.array_equal(rp, T.indptr) and np.array_equal(ci, T.indices)
    assert np.array_equal(v, T.data)
