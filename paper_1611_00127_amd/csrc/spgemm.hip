// Sparse matrix-matrix product and transpose with symbolic (cancellation-
// free) patterns and sorted rows, used for the Galerkin product A_c = R(AP)
// and for the approximate Schur complement S~ = A_pp - (A_ps D^{-1}) A_sp.
//
// Product rows are formed by merging the sorted rows B_k, k in A_i: one
// thread per output row advances a cursor into every B_k and emits the
// columns in increasing order, accumulating each value over k in A's column
// order.  The result is deterministic (no atomics on values) and its
// pattern never depends on values.
#include <climits>

#include "tpf_internal.hpp"

namespace tpf {

namespace {

template <bool FILL>
__global__ void __launch_bounds__(128) k_spgemm_merge(
    int nrows, const int* __restrict__ arp, const int* __restrict__ aci,
    const double* __restrict__ av, const int* __restrict__ brp, const int* __restrict__ bci,
    const double* __restrict__ bv, const int* __restrict__ drp, const int* __restrict__ dci,
    const double* __restrict__ dv, double alpha, double beta, int2* __restrict__ cur,
    int* __restrict__ cnt, const int* __restrict__ crp, int* __restrict__ cci,
    double* __restrict__ cv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  int a0 = arp[i], a1 = arp[i + 1];
  for (int e = a0; e < a1; ++e) {
    int k = aci[e];
    cur[e] = make_int2(brp[k], brp[k + 1]);
  }
  int dp = 0, de = 0;
  if (drp) {
    dp = drp[i];
    de = drp[i + 1];
  }
  int out = FILL ? crp[i] : 0;
  int count = 0;
  while (true) {
    int m = INT_MAX;
    for (int e = a0; e < a1; ++e) {
      int2 c = cur[e];
      if (c.x < c.y) {
        int col = bci[c.x];
        m = col < m ? col : m;
      }
    }
    if (dp < de) {
      int col = dci[dp];
      m = col < m ? col : m;
    }
    if (m == INT_MAX) break;
    double sum = 0.0;
    for (int e = a0; e < a1; ++e) {
      int2 c = cur[e];
      if (c.x < c.y && bci[c.x] == m) {
        if (FILL) sum += av[e] * bv[c.x];
        cur[e].x = c.x + 1;
      }
    }
    if (FILL) {
      double val = alpha * sum;
      if (dp < de && dci[dp] == m) val = beta * dv[dp] + val;
      cci[out + count] = m;
      cv[out + count] = val;
    }
    if (dp < de && dci[dp] == m) ++dp;
    ++count;
  }
  if (!FILL) cnt[i] = count;
}

__global__ void k_col_count(int nrows, const int* __restrict__ rp, const int* __restrict__ ci,
                            int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) atomicAdd(&cnt[ci[e]], 1);
}

__global__ void k_transpose_fill(int nrows, const int* __restrict__ rp, const int* __restrict__ ci,
                                 const double* __restrict__ v, int* __restrict__ cursor,
                                 int* __restrict__ tci, double* __restrict__ tv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    int pos = atomicAdd(&cursor[ci[e]], 1);
    tci[pos] = i;
    if (v) tv[pos] = v[e];
  }
}

// insertion sort of each row by column (rows of a transpose are short)
__global__ void k_sort_rows(int nrows, const int* __restrict__ rp, int* __restrict__ ci,
                            double* __restrict__ v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  int a = rp[i], b = rp[i + 1];
  for (int e = a + 1; e < b; ++e) {
    int key = ci[e];
    double val = v ? v[e] : 0.0;
    int f = e - 1;
    while (f >= a && ci[f] > key) {
      ci[f + 1] = ci[f];
      if (v) v[f + 1] = v[f];
      --f;
    }
    ci[f + 1] = key;
    if (v) v[f + 1] = val;
  }
}

}  // namespace

void spgemm(const CsrRef<double>& A, const CsrRef<double>& B, Csr<double>& C, hipStream_t s,
            const CsrRef<double>* D, double alpha, double beta, bool reuse) {
  TPF_REQUIRE(A.ncols == B.nrows, TPF_ERR_INVALID_ARG, "spgemm: inner dimensions differ (%d vs %d)",
              A.ncols, B.nrows);
  if (D)
    TPF_REQUIRE(D->nrows == A.nrows && D->ncols == B.ncols, TPF_ERR_INVALID_ARG,
                "spgemm: added matrix has the wrong shape");
  int n = A.nrows;
  Buf<int2> cur(A.nnz > 0 ? A.nnz : 1, s);
  const int* drp = D ? D->rp : nullptr;
  const int* dci = D ? D->ci : nullptr;
  const double* dv = D ? D->v : nullptr;
  if (!reuse) {
    C.nrows = n;
    C.ncols = B.ncols;
    C.rp.alloc(n + 1, s);
    Buf<int> cnt(n > 0 ? n : 1, s);
    if (n > 0) {
      k_spgemm_merge<false><<<grid_for(n, 128), 128, 0, s>>>(
          n, A.rp, A.ci, A.v, B.rp, B.ci, B.v, drp, dci, dv, alpha, beta, cur.p, cnt.p, nullptr,
          nullptr, nullptr);
      TPF_CHECK_LAUNCH();
    }
    C.nnz = scan_exclusive(cnt.p, C.rp.p, n, s);
    C.ci.alloc(C.nnz > 0 ? C.nnz : 1, s);
    C.v.alloc(C.nnz > 0 ? C.nnz : 1, s);
  } else {
    TPF_REQUIRE(C.nrows == n && C.ncols == B.ncols && C.rp.p, TPF_ERR_STATE,
                "spgemm reuse: product pattern missing");
  }
  if (n > 0) {
    k_spgemm_merge<true><<<grid_for(n, 128), 128, 0, s>>>(n, A.rp, A.ci, A.v, B.rp, B.ci, B.v, drp,
                                                          dci, dv, alpha, beta, cur.p, nullptr,
                                                          C.rp.p, C.ci.p, C.v.p);
    TPF_CHECK_LAUNCH();
  }
}

void transpose(const CsrRef<double>& A, Csr<double>& C, hipStream_t s) {
  int m = A.ncols;
  C.nrows = m;
  C.ncols = A.nrows;
  C.nnz = A.nnz;
  Buf<int> cnt(m > 0 ? m : 1, s);
  fill_int(cnt.p, 0, m, s);
  if (A.nrows > 0) {
    k_col_count<<<grid_for(A.nrows, 256), 256, 0, s>>>(A.nrows, A.rp, A.ci, cnt.p);
    TPF_CHECK_LAUNCH();
  }
  C.rp.alloc(m + 1, s);
  int64_t tot = scan_exclusive(cnt.p, C.rp.p, m, s);
  TPF_REQUIRE(tot == A.nnz, TPF_ERR_INVALID_ARG, "transpose: column indices out of range");
  C.ci.alloc(A.nnz > 0 ? A.nnz : 1, s);
  if (A.v)
    C.v.alloc(A.nnz > 0 ? A.nnz : 1, s);
  else
    C.v.release();
  copy(cnt.p, C.rp.p, m, s);  // cursors start at the row starts
  if (A.nrows > 0) {
    k_transpose_fill<<<grid_for(A.nrows, 256), 256, 0, s>>>(A.nrows, A.rp, A.ci, A.v, cnt.p,
                                                           C.ci.p, C.v.p);
    TPF_CHECK_LAUNCH();
  }
  if (m > 0) {
    k_sort_rows<<<grid_for(m, 128), 128, 0, s>>>(m, C.rp.p, C.ci.p, C.v.p);
    TPF_CHECK_LAUNCH();
  }
}

}  // namespace tpf
