// Dense-vector and CSR primitives: scans, fills, casts, deterministic
// reductions and CSR row kernels (one group of LPR lanes per row, LPR a
// power of two chosen from the mean row length so that a row is read with
// consecutive lanes).
#include "linalg_dev.hpp"
#include "tpf_internal.hpp"

namespace tpf {

// ---------------------------------------------------------------- scans
namespace {
constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

template <class T, class In>
__global__ void __launch_bounds__(kScanBlock) k_scan_tile(const In* in, T* out, T* block_sums,
                                                          int64_t n) {
  __shared__ T sh[kScanBlock / 64 + 1];
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  T v[kScanItems];
  T local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? T(in[i]) : T(0);
    local += v[k];
  }
  T total;
  T excl = block_exclusive_scan<T, kScanBlock>(local, sh, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = excl;
    excl += v[k];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

template <class T>
__global__ void k_scan_add(T* out, const T* offsets, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * kScanTile + threadIdx.x;
  T off = offsets[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k, i += kScanBlock)
    if (i < n) out[i] += off;
}

// exclusive scan of n values; out has n entries (total returned separately)
template <class T, class In>
void scan_rec(const In* in, T* out, int64_t n, hipStream_t s) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  Buf<T> sums(nb, s);
  k_scan_tile<T, In><<<unsigned(nb), kScanBlock, 0, s>>>(in, out, sums.p, n);
  TPF_CHECK_LAUNCH();
  if (nb > 1) {
    Buf<T> offs(nb, s);
    scan_rec<T, T>(sums.p, offs.p, nb, s);
    k_scan_add<T><<<unsigned(nb), kScanBlock, 0, s>>>(out, offs.p, n);
    TPF_CHECK_LAUNCH();
  }
}
}  // namespace

namespace {
// total = tmp[n-1] + in[n-1] into out[n] and *tot; optionally out[i] = tmp[i]
// narrowed (out != tmp)
template <class T, class In, class Out>
__global__ void k_scan_finish(const T* __restrict__ tmp, const In* __restrict__ in, int64_t n,
                              Out* __restrict__ out, bool narrow, int64_t* __restrict__ tot) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (narrow)
    for (; i < n; i += int64_t(gridDim.x) * blockDim.x) out[i] = Out(tmp[i]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int64_t t = int64_t(tmp[n - 1]) + int64_t(in[n - 1]);
    out[n] = Out(t);
    *tot = t;
  }
}

// reads the 64-bit total written by k_scan_finish (one round trip)
int64_t read_total(const int64_t* tot, hipStream_t s) { return read_scalar(tot, s); }

// Short inputs (the coarse levels): the whole scan in one work-group, tile
// by tile with a running carry, in place of the tile / block-sum / add /
// finish launches.  out[n] and *tot receive the total.
constexpr int kScanOneBlock = 1024;
constexpr int64_t kScanOneMax = 16384;
template <class In, class Out>
__global__ void __launch_bounds__(kScanOneBlock) k_scan_one(const In* __restrict__ in,
                                                            Out* __restrict__ out, int64_t n,
                                                            int64_t* __restrict__ tot) {
  __shared__ int64_t sh[kScanOneBlock / 64 + 1];
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += int64_t(kScanOneBlock) * kScanItems) {
    const int64_t i0 = base + int64_t(threadIdx.x) * kScanItems;
    int64_t v[kScanItems];
    int64_t local = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = i0 + k < n ? int64_t(in[i0 + k]) : 0;
      local += v[k];
    }
    int64_t total;
    int64_t excl = block_exclusive_scan<int64_t, kScanOneBlock>(local, sh, total) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (i0 + k < n) out[i0 + k] = Out(excl);
      excl += v[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) {
    out[n] = Out(carry);
    *tot = carry;
  }
}
}  // namespace

int64_t scan_exclusive(const int* in, int* out, int64_t n, hipStream_t s) {
  // totals are accumulated in 64-bit to detect overflow of the int32 output
  if (n == 0) {
    fill_int(out, 0, 1, s);
    return 0;
  }
  if (n <= kScanOneMax) {
    Buf<int64_t> tot(1, s);
    k_scan_one<int, int><<<1, kScanOneBlock, 0, s>>>(in, out, n, tot.p);
    TPF_CHECK_LAUNCH();
    const int64_t total = read_total(tot.p, s);
    TPF_REQUIRE(total < (int64_t(1) << 31), TPF_ERR_INVALID_ARG,
                "index count %lld exceeds the int32 range", (long long)total);
    return total;
  }
  Buf<int64_t> tmp(n + 1, s);
  scan_rec<int64_t, int>(in, tmp.p, n, s);
  unsigned g = grid_for(n, 256);
  k_scan_finish<int64_t, int, int><<<g > 4096 ? 4096 : g, 256, 0, s>>>(tmp.p, in, n, out, true,
                                                                         tmp.p + n);
  TPF_CHECK_LAUNCH();
  int64_t total = read_total(tmp.p + n, s);
  TPF_REQUIRE(total < (int64_t(1) << 31), TPF_ERR_INVALID_ARG,
              "index count %lld exceeds the int32 range", (long long)total);
  return total;
}

void scan_exclusive_async(const int* in, int* out, int64_t n, hipStream_t s) {
  if (n == 0) {
    fill_int(out, 0, 1, s);
    return;
  }
  if (n <= kScanOneMax) {
    Buf<int64_t> tot(1, s);
    k_scan_one<int, int><<<1, kScanOneBlock, 0, s>>>(in, out, n, tot.p);
    TPF_CHECK_LAUNCH();
    return;
  }
  Buf<int64_t> tmp(n + 1, s);
  scan_rec<int64_t, int>(in, tmp.p, n, s);
  unsigned g = grid_for(n, 256);
  k_scan_finish<int64_t, int, int><<<g > 4096 ? 4096 : g, 256, 0, s>>>(tmp.p, in, n, out, true,
                                                                         tmp.p + n);
  TPF_CHECK_LAUNCH();
}

int64_t scan_exclusive_wide(const int* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n == 0) {
    fill(out, int64_t(0), 1, s);
    return 0;
  }
  Buf<int64_t> tot(1, s);
  if (n <= kScanOneMax) {
    k_scan_one<int, int64_t><<<1, kScanOneBlock, 0, s>>>(in, out, n, tot.p);
  } else {
    scan_rec<int64_t, int>(in, out, n, s);
    k_scan_finish<int64_t, int, int64_t><<<1, 64, 0, s>>>(out, in, n, out, false, tot.p);
  }
  TPF_CHECK_LAUNCH();
  return read_total(tot.p, s);
}

int64_t scan_exclusive64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n == 0) {
    fill(out, int64_t(0), 1, s);
    return 0;
  }
  Buf<int64_t> tot(1, s);
  if (n <= kScanOneMax) {
    k_scan_one<int64_t, int64_t><<<1, kScanOneBlock, 0, s>>>(in, out, n, tot.p);
  } else {
    scan_rec<int64_t, int64_t>(in, out, n, s);
    k_scan_finish<int64_t, int64_t, int64_t><<<1, 64, 0, s>>>(out, in, n, out, false, tot.p);
  }
  TPF_CHECK_LAUNCH();
  return read_total(tot.p, s);
}

// ---------------------------------------------------------------- fills / copies / casts
template <class T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

template <class A, class B>
__global__ void k_cast(B* dst, const A* src, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = B(src[i]);
}

static unsigned stream_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return unsigned(g);
}

void fill_int(int* p, int v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill<int><<<stream_grid(n), 256, 0, s>>>(p, v, n);
  TPF_CHECK_LAUNCH();
}

template <class T>
void fill(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill<T><<<stream_grid(n), 256, 0, s>>>(p, v, n);
  TPF_CHECK_LAUNCH();
}
template void fill<double>(double*, double, int64_t, hipStream_t);
template void fill<float>(float*, float, int64_t, hipStream_t);
template void fill<int8_t>(int8_t*, int8_t, int64_t, hipStream_t);
template void fill<int64_t>(int64_t*, int64_t, int64_t, hipStream_t);

template <class T>
void copy(T* dst, const T* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast<T, T><<<stream_grid(n), 256, 0, s>>>(dst, src, n);
  TPF_CHECK_LAUNCH();
}
template void copy<double>(double*, const double*, int64_t, hipStream_t);
template void copy<float>(float*, const float*, int64_t, hipStream_t);
template void copy<int>(int*, const int*, int64_t, hipStream_t);

template <class A, class B>
void cast(B* dst, const A* src, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast<A, B><<<stream_grid(n), 256, 0, s>>>(dst, src, n);
  TPF_CHECK_LAUNCH();
}
template void cast<double, float>(float*, const double*, int64_t, hipStream_t);
template void cast<float, double>(double*, const float*, int64_t, hipStream_t);
template void cast<int64_t, int>(int*, const int64_t*, int64_t, hipStream_t);

// ---------------------------------------------------------------- reductions
namespace {
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

__global__ void __launch_bounds__(kRedThreads) k_dot_partial(const double* x, const double* y,
                                                             int64_t n, double* part) {
  __shared__ double sh[kRedThreads / 64];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kRedThreads)
    acc += x[i] * y[i];
  acc = block_sum<kRedThreads>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kRedThreads) k_sum_final(const double* part, int m, double* out,
                                                           int sqrt_flag) {
  __shared__ double sh[kRedThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += kRedThreads) acc += part[i];
  acc = block_sum<kRedThreads>(acc, sh);
  if (threadIdx.x == 0) *out = sqrt_flag ? sqrt(acc) : acc;
}
}  // namespace

void dot_device(const double* x, const double* y, int64_t n, double* out, hipStream_t s) {
  Buf<double> part(kRedBlocks, s);
  k_dot_partial<<<kRedBlocks, kRedThreads, 0, s>>>(x, y, n, part.p);
  TPF_CHECK_LAUNCH();
  k_sum_final<<<1, kRedThreads, 0, s>>>(part.p, kRedBlocks, out, 0);
  TPF_CHECK_LAUNCH();
}

void nrm2_device(const double* x, int64_t n, double* out, double* part, hipStream_t s) {
  k_dot_partial<<<kRedBlocks, kRedThreads, 0, s>>>(x, x, n, part);
  TPF_CHECK_LAUNCH();
  k_sum_final<<<1, kRedThreads, 0, s>>>(part, kRedBlocks, out, 1);
  TPF_CHECK_LAUNCH();
}

double nrm2_host(const double* x, int64_t n, hipStream_t s) {
  Buf<double> part(kRedBlocks + 1, s);
  k_dot_partial<<<kRedBlocks, kRedThreads, 0, s>>>(x, x, n, part.p);
  TPF_CHECK_LAUNCH();
  k_sum_final<<<1, kRedThreads, 0, s>>>(part.p, kRedBlocks, part.p + kRedBlocks, 1);
  TPF_CHECK_LAUNCH();
  return read_scalar(part.p + kRedBlocks, s);
}

// ---------------------------------------------------------------- staged rows
namespace {
template <int LPR>
__global__ void __launch_bounds__(256) k_pack_rows(int n, const int64_t* __restrict__ toff,
                                                   const int* __restrict__ crp,
                                                   const int* __restrict__ tci,
                                                   const double* __restrict__ tv,
                                                   int* __restrict__ cci, double* __restrict__ cv) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  if (i >= n) return;
  int64_t src = toff[i];
  int c0 = crp[i], len = crp[i + 1] - c0;
  for (int t = lane; t < len; t += LPR) {
    cci[c0 + t] = tci[src + t];
    cv[c0 + t] = tv[src + t];
  }
}
}  // namespace

void pack_rows(int n, const int64_t* toff, const int* crp, int64_t nnz, const int* tci,
               const double* tv, int* cci, double* cv, hipStream_t s) {
  if (n <= 0) return;
  // a plain copy: about one entry per lane (staged rows are far apart, so
  // short rows with one lane each would read a cache line per entry)
  int lpr = 1;
  while (lpr < 64 && int64_t(lpr) * n < nnz) lpr <<= 1;
  DISPATCH_LPR(lpr, LL, {
    k_pack_rows<LL><<<grid_for(int64_t(n) * lpr, 256), 256, 0, s>>>(n, toff, crp, tci, tv, cci,
                                                                     cv);
  });
  TPF_CHECK_LAUNCH();
}

// ---------------------------------------------------------------- CSR row kernels
namespace {
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_csr_spmv(int nrows, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ v,
                                                  const T* __restrict__ x, T* __restrict__ y) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR);
  int lane = int(gid % LPR);
  if (row >= nrows) return;
  T sum = row_dot<T, LPR>(row, lane, rp, ci, v, [&](int j) { return x[j]; });
  if (lane == 0) y[row] = sum;
}

template <class T, int LPR>
__global__ void __launch_bounds__(256) k_csr_residual(int nrows, const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const T* __restrict__ v,
                                                      const T* __restrict__ x,
                                                      const T* __restrict__ b, T* __restrict__ y) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR);
  int lane = int(gid % LPR);
  if (row >= nrows) return;
  T sum = row_dot<T, LPR>(row, lane, rp, ci, v, [&](int j) { return x[j]; });
  if (lane == 0) y[row] = b[row] - sum;
}
}  // namespace

template <class T>
void csr_spmv(const CsrRef<T>& A, const T* x, T* y, hipStream_t s, const char* tname) {
  if (A.nrows == 0) return;
  int lpr = lanes_per_row(A.nrows, A.nnz);
  TimedScope ts(tname, s);
  DISPATCH_LPR(lpr, L, {
    k_csr_spmv<T, L><<<grid_for(int64_t(A.nrows) * L, 256), 256, 0, s>>>(A.nrows, A.rp, A.ci,
                                                                          A.v, x, y);
  });
  TPF_CHECK_LAUNCH();
}
template void csr_spmv<double>(const CsrRef<double>&, const double*, double*, hipStream_t, const char*);
template void csr_spmv<float>(const CsrRef<float>&, const float*, float*, hipStream_t, const char*);

template <class T>
void csr_residual(const CsrRef<T>& A, const T* x, const T* b, T* y, hipStream_t s) {
  if (A.nrows == 0) return;
  int lpr = lanes_per_row(A.nrows, A.nnz);
  DISPATCH_LPR(lpr, L, {
    k_csr_residual<T, L><<<grid_for(int64_t(A.nrows) * L, 256), 256, 0, s>>>(
        A.nrows, A.rp, A.ci, A.v, x, b, y);
  });
  TPF_CHECK_LAUNCH();
}
template void csr_residual<double>(const CsrRef<double>&, const double*, const double*, double*,
                                   hipStream_t);
template void csr_residual<float>(const CsrRef<float>&, const float*, const float*, float*,
                                  hipStream_t);

}  // namespace tpf
