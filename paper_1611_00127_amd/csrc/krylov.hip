// Right-preconditioned flexible GMRES(m) (paper Sec. 3, Eq. precon-system:
// J M^{-1} c^ = q, c = M^{-1} c^) with classical Gram-Schmidt applied twice
// and Givens rotations.  x_0 = 0; a cycle stops when |g_{j+1}| <= rtol ||b||
// or h_{j+1,j} = 0; convergence is declared on the true residual.
//
// One Arnoldi step streams the basis three times:
//   pass 1  h  = V^T w
//   pass 2  w -= V h,  h' = V^T w      (V read once for both)
//   pass 3  w -= V h', ||w||^2
// Partial sums go to a fixed grid of blocks and are reduced in a fixed order,
// so every run is bitwise reproducible.  The rotation update runs on the
// device; the host reads the residual estimate once per step.
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include "krylov.hpp"
#include "linalg_dev.hpp"

namespace tpf {

namespace {
constexpr int kKBlock = 256;

constexpr int kKGridMax = 2048;  // blocks of the streaming passes (partial sums per block)

int krylov_grid(int64_t n) {
  int64_t g = (n + kKBlock * 4 - 1) / (kKBlock * 4);
  if (g > kKGridMax) g = kKGridMax;
  if (g < 1) g = 1;
  return int(g);
}

// Work-groups of a grid-stride pass of `kernel` over n entries: at most as
// many as the device holds resident at once (the larger bases take more
// registers per thread, and a second, partial round of work-groups would
// leave most compute units idle at the end), and at most krylov_grid(n).
template <class K>
int resident_grid(K kernel, int64_t n) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> fit;  // (device, kernel) -> work-groups
  int dev = 0;
  TPF_HIP(hipGetDevice(&dev));
  const auto key = std::make_pair(dev, reinterpret_cast<const void*>(kernel));
  int g = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = fit.find(key);
    if (it != fit.end()) {
      g = it->second;
    } else {
      int per_cu = 0, cus = 0;
      TPF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kKBlock, 0));
      TPF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      g = per_cu > 0 && cus > 0 ? per_cu * cus : kKGridMax;
      fit[key] = g;
    }
  }
  const int cap = krylov_grid(n);
  return g < cap ? g : cap;
}

// block-wise reduction of KMAX running sums into part[k][block] (one row of
// gridDim.x partial sums per basis vector, read contiguously by the reduction)
template <int KMAX>
__device__ inline void reduce_store(double* acc, int nk, double* part) {
  __shared__ double sh[kKBlock / 64][KMAX];
  int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < nk) {
      double v = wave_sum(acc[k]);
      if (lane == 0) sh[wid][k] = v;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nk; k += kKBlock) {
    double t = 0.0;
    for (int w = 0; w < kKBlock / 64; ++w) t += sh[w][k];
    part[int64_t(k) * gridDim.x + blockIdx.x] = t;
  }
}

// Block sums of per-lane running sums: lane q of each group of L lanes holds
// the sums of basis vectors q*KH .. q*KH+KH-1; part[k][block] gets vector k's.
template <int KH, int L>
__device__ inline void reduce_store_lanes(const double* acc, int nk, double* part) {
  __shared__ double sh[kKBlock / 64][L * KH];
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
#pragma unroll
  for (int u = 0; u < KH; ++u) {
    if (u >= nk) break;  // no lane holds vector u or beyond (the same for every lane)
    double t = acc[u];
    if constexpr (L == 1) {
      t = wave_sum(t);
    } else {
#pragma unroll
      for (int off = 32; off >= L; off >>= 1) t += __shfl_down(t, off, 64);
    }
    if (lane < L) sh[wid][lane * KH + u] = t;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nk; k += kKBlock) {
    double t = 0.0;
    for (int ww = 0; ww < kKBlock / 64; ++ww) t += sh[ww][k];
    part[int64_t(k) * gridDim.x + blockIdx.x] = t;
  }
}

// pass 1: part = V^T w  (nk vectors).  L lanes per pair of entries, lane q
// holding basis vectors q*KH .. q*KH+KH-1 (fewer registers per lane for the
// larger bases).
template <int KMAX, int L>
__global__ void __launch_bounds__(kKBlock) k_cgs_dots(int64_t n, int nk, const double* __restrict__ V,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ part) {
  constexpr int KH = (KMAX + L - 1) / L;
  // entries in pairs (n is even and every basis vector 16-byte aligned)
  const int q = threadIdx.x % L, k0 = q * KH;
  double acc[KH];
#pragma unroll
  for (int u = 0; u < KH; ++u) acc[u] = 0.0;
  const int64_t n2 = n / 2;
  const double2* V2 = reinterpret_cast<const double2*>(V);
  const double2* w2 = reinterpret_cast<const double2*>(w);
  for (int64_t p = (int64_t(blockIdx.x) * kKBlock + threadIdx.x) / L; p < n2;
       p += int64_t(gridDim.x) * (kKBlock / L)) {
    const double2 wi = w2[p];
#pragma unroll
    for (int u = 0; u < KH; ++u)
      if (k0 + u < nk) {
        const double2 v = V2[(k0 + u) * n2 + p];
        acc[u] += v.x * wi.x;
        acc[u] += v.y * wi.y;
      }
  }
  reduce_store_lanes<KH, L>(acc, nk, part);
}

// pass 2: w -= V h; part = V^T w.  L lanes per pair of entries, lane q
// holding basis vectors q*KH .. q*KH+KH-1: each lane sums h_k v_k over its
// part, the L lanes add their sums (a butterfly: the same value in every
// lane), the first lane writes w, and each lane accumulates its part of the
// dot products.
template <int KMAX, int L>
__global__ void __launch_bounds__(kKBlock) k_cgs_axpy_dots(int64_t n, int nk,
                                                           const double* __restrict__ V,
                                                           const double* __restrict__ h,
                                                           double* __restrict__ w,
                                                           double* __restrict__ part) {
  constexpr int KH = (KMAX + L - 1) / L;
  __shared__ double hs[L * KH];
  for (int k = threadIdx.x; k < L * KH; k += kKBlock) hs[k] = k < nk ? h[k] : 0.0;
  __syncthreads();
  const int q = threadIdx.x % L, k0 = q * KH;
  double acc[KH];
#pragma unroll
  for (int u = 0; u < KH; ++u) acc[u] = 0.0;
  const int64_t n2 = n / 2;  // entries in pairs, as in k_cgs_dots
  const double2* V2 = reinterpret_cast<const double2*>(V);
  double2* w2 = reinterpret_cast<double2*>(w);
  for (int64_t p = (int64_t(blockIdx.x) * kKBlock + threadIdx.x) / L; p < n2;
       p += int64_t(gridDim.x) * (kKBlock / L)) {
    double2 v[KH];
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int u = 0; u < KH; ++u) {
      v[u] = make_double2(0.0, 0.0);
      if (k0 + u < nk) {
        v[u] = V2[int64_t(k0 + u) * n2 + p];
        sx += hs[k0 + u] * v[u].x;
        sy += hs[k0 + u] * v[u].y;
      }
    }
#pragma unroll
    for (int off = 1; off < L; off <<= 1) {
      sx += __shfl_xor(sx, off, 64);
      sy += __shfl_xor(sy, off, 64);
    }
    double2 wi = w2[p];
    wi.x -= sx;
    wi.y -= sy;
    if (q == 0) w2[p] = wi;
#pragma unroll
    for (int u = 0; u < KH; ++u)
      if (k0 + u < nk) {
        acc[u] += v[u].x * wi.x;
        acc[u] += v[u].y * wi.y;
      }
  }
  reduce_store_lanes<KH, L>(acc, nk, part);
}

// pass 3: w -= V h; part = ||w||^2
template <int KMAX>
__global__ void __launch_bounds__(kKBlock) k_cgs_axpy_norm(int64_t n, int nk,
                                                           const double* __restrict__ V,
                                                           const double* __restrict__ h,
                                                           double* __restrict__ w,
                                                           double* __restrict__ part) {
  __shared__ double hs[KMAX];
  for (int k = threadIdx.x; k < nk; k += kKBlock) hs[k] = h[k];
  __syncthreads();
  double acc[1] = {0.0};
  const int64_t n2 = n / 2;  // entries in pairs, as in k_cgs_dots
  const double2* V2 = reinterpret_cast<const double2*>(V);
  double2* w2 = reinterpret_cast<double2*>(w);
  for (int64_t p = int64_t(blockIdx.x) * kKBlock + threadIdx.x; p < n2;
       p += int64_t(gridDim.x) * kKBlock) {
    double2 wi = w2[p];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < nk) {
        const double2 v = V2[k * n2 + p];
        wi.x -= hs[k] * v.x;
        wi.y -= hs[k] * v.y;
      }
    w2[p] = wi;
    acc[0] += wi.x * wi.x;
    acc[0] += wi.y * wi.y;
  }
  reduce_store<1>(acc, 1, part);
}

// out[k] = sum of the nb partial sums of row k (one work-group per row,
// fixed order)
constexpr int kRedBlock = 256;
__device__ inline double sum_parts(int nb, const double* __restrict__ row) {
  __shared__ double sh[kRedBlock / 64];
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedBlock) t += row[b];
  return block_sum<kRedBlock>(t, sh);
}

__global__ void __launch_bounds__(kRedBlock) k_reduce_parts(int nb,
                                                            const double* __restrict__ part,
                                                            double* __restrict__ out) {
  const int k = blockIdx.x;
  const double t = sum_parts(nb, part + int64_t(k) * nb);
  if (threadIdx.x == 0) out[k] = t;
}

struct GState {
  double est;     // |g_{j+1}|
  double hn;      // h_{j+1,j}
  double d;       // rotation radius (0 => breakdown)
  double inv_hn;  // 1/h_{j+1,j} (0 if h_{j+1,j} == 0)
};

// Givens update of column j (single thread): h = h1 + h2, apply previous
// rotations, form the new one, update g.
__global__ void __launch_bounds__(kRedBlock) k_givens(int j, int m, const double* __restrict__ h1,
                                                      const double* __restrict__ h2,
                                                      const double* __restrict__ nrm2_part,
                                                      int nparts, double* __restrict__ H,
                                                      double* __restrict__ cs,
                                                      double* __restrict__ sn,
                                                      double* __restrict__ g,
                                                      GState* __restrict__ st) {
  const double ss = sum_parts(nparts, nrm2_part);
  if (threadIdx.x != 0) return;
  double hn = sqrt(ss);
  double* col = H + int64_t(j) * (m + 1);
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    double a = col[i], c = col[i + 1];
    col[i] = cs[i] * a + sn[i] * c;
    col[i + 1] = -sn[i] * a + cs[i] * c;
  }
  double d = hypot(col[j], col[j + 1]);
  GState s;
  s.hn = hn;
  s.d = d;
  s.inv_hn = hn != 0.0 ? 1.0 / hn : 0.0;
  if (d == 0.0 || !isfinite(d)) {
    s.est = fabs(g[j]);
    *st = s;
    return;
  }
  cs[j] = col[j] / d;
  sn[j] = col[j + 1] / d;
  col[j] = d;
  col[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  s.est = fabs(g[j + 1]);
  *st = s;
}

__global__ void k_scale(int64_t n, const double* __restrict__ x, const GState* __restrict__ st,
                        double* __restrict__ y) {
  double a = st->inv_hn;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    y[i] = x[i] * a;
}

__global__ void k_scale_by(int64_t n, const double* __restrict__ x, double a,
                           double* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    y[i] = x[i] * a;
}

// back substitution H(0:k,0:k) y = g(0:k) (single thread)
__global__ void k_trisolve(int k, int m, const double* __restrict__ H, const double* __restrict__ g,
                           double* __restrict__ y) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double t = 0.0;
    for (int l = i + 1; l < k; ++l) t += H[int64_t(l) * (m + 1) + i] * y[l];
    y[i] = (g[i] - t) / H[int64_t(i) * (m + 1) + i];
  }
}

// x += Z(:,0:k) y
__global__ void k_update_x(int64_t n, int k, const double* __restrict__ Z,
                           const double* __restrict__ y, double* __restrict__ x) {
  __shared__ double ys[kMaxRestart];
  for (int l = threadIdx.x; l < k; l += blockDim.x) ys[l] = y[l];
  __syncthreads();
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    double t = x[i];
    for (int l = 0; l < k; ++l) t += Z[l * n + i] * ys[l];
    x[i] = t;
  }
}

// register arrays sized to the basis length in steps of four up to 24 (the
// pass-2 kernel holds KMAX basis values and KMAX sums per thread, so the
// step sets its occupancy)
#define DISPATCH_K(nk, KM, ...)                                  \
  if (nk <= 8) { constexpr int KM = 8; __VA_ARGS__ }             \
  else if (nk <= 12) { constexpr int KM = 12; __VA_ARGS__ }      \
  else if (nk <= 16) { constexpr int KM = 16; __VA_ARGS__ }      \
  else if (nk <= 20) { constexpr int KM = 20; __VA_ARGS__ }      \
  else if (nk <= 24) { constexpr int KM = 24; __VA_ARGS__ }      \
  else if (nk <= 32) { constexpr int KM = 32; __VA_ARGS__ }      \
  else { constexpr int KM = 64; __VA_ARGS__ }

unsigned vec_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return unsigned(g);
}

}  // namespace

// ---------------------------------------------------------------- resumable solver
template <class F>
void Fgmres::for_each_array(int64_t nn, int mm, F&& f) {
  f(V, size_t(mm + 1) * nn);
  f(Z, size_t(mm) * nn);
  f(H, size_t(mm + 1) * mm);
  f(cs, size_t(mm));
  f(sn, size_t(mm));
  f(g, size_t(mm + 1));
  f(h1, size_t(kMaxRestart + 1));
  f(h2, size_t(kMaxRestart + 1));
  f(part, size_t(kKGridMax) * 64);
  f(y, size_t(mm));
  f(r, size_t(nn));
  f(st_dev, size_t(4));
  f(scal, size_t(2));
}

namespace {
constexpr size_t kAlignDoubles = 32;  // 256 bytes
size_t align_up(size_t c) { return (c + kAlignDoubles - 1) / kAlignDoubles * kAlignDoubles; }
}  // namespace

size_t Fgmres::workspace_doubles(int64_t nn, int mm) {
  Fgmres probe;
  size_t total = 0;
  probe.for_each_array(nn, mm, [&](Buf<double>&, size_t c) { total += align_up(c); });
  return total;
}

size_t Fgmres::workspace_footprint(int64_t nn, int mm) {
  Fgmres probe;
  size_t total = 0;
  probe.for_each_array(nn, mm, [&](Buf<double>&, size_t c) { total += alloc_footprint(c * sizeof(double)); });
  return total;
}

void Fgmres::alloc(int64_t nn, int mm, hipStream_t st) {
  if (n == nn && m == mm && V.p) return;
  n = nn;
  m = mm;
  for_each_array(n, m, [&](Buf<double>& b, size_t c) { b.alloc(c, st); });
}

void Fgmres::bind(double* base, int64_t nn, int mm) {
  n = nn;
  m = mm;
  size_t off = 0;
  for_each_array(n, m, [&](Buf<double>& b, size_t c) {
    b.wrap(base + off, c);
    off += align_up(c);
  });
  bound = true;
}

void Fgmres::begin(const tpf_jacobian* J_, tpf_precond* M_, const double* b_, double* x_,
                   const tpf_solve_opts& o_, hipStream_t st, void* host_slot) {
  TPF_REQUIRE(J_ && b_ && x_, TPF_ERR_INVALID_ARG, "null argument");
  TPF_REQUIRE(o_.restart >= 1 && o_.restart <= kMaxRestart, TPF_ERR_INVALID_ARG,
              "restart must be in [1, %d]", kMaxRestart);
  TPF_REQUIRE(o_.maxit >= 1 && o_.rtol > 0, TPF_ERR_INVALID_ARG, "maxit >= 1 and rtol > 0 required");
  if (M_) {
    TPF_REQUIRE(M_->ready, TPF_ERR_STATE, "preconditioner not set up");
    TPF_REQUIRE(M_->o.kind == TPF_PREC_NONE || M_->J == J_, TPF_ERR_STATE,
                "preconditioner was set up for another Jacobian");
  }
  J = J_;
  M = M_;
  b = b_;
  x = x_;
  o = o_;
  s = st;
  TPF_REQUIRE(host_slot, TPF_ERR_INVALID_ARG, "null host slot");
  host = host_slot;
  if (bound)  // n even: the streaming passes read pairs
    TPF_REQUIRE(n == 2 * int64_t(J->nb) && m == o.restart, TPF_ERR_INVALID_ARG,
                "bound workspace is for %lld unknowns and restart %d", (long long)n, m);
  else
    alloc(2 * int64_t(J->nb), o.restart, s);
  total = 0;
  est = 1.0;
  spec_j = -1;
  ev_pending = false;
  status = -1;
  relres = 0.0;
  t0 = std::chrono::steady_clock::now();
  fill(x, 0.0, n, s);
  nrm2_device(b, n, scal.p, part.p, s);
  TPF_HIP(hipMemcpyAsync(host, scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
  phase = kInit;
}

void Fgmres::launch_cycle_start(const double* rsrc, double beta) {
  spec_j = -1;
  spec_est = beta / beta0;
  k_scale_by<<<vec_grid(n), 256, 0, s>>>(n, rsrc, 1.0 / beta, V.p);
  TPF_CHECK_LAUNCH();
  fill(g.p, 0.0, m + 1, s);
  fill(g.p, beta, 1, s);
  j = 0;
  breakdown = false;
  launch_step();
}

// z_col = M^{-1} v_col
void Fgmres::apply_precond(int col) {
  TimedScope ts("precond_apply", s);
  int rc = tpf_precond_apply(M, V.p + int64_t(col) * n, Z.p + int64_t(col) * n, s);
  if (rc != TPF_OK) {
    char msg[1024];
    tpf_last_error(msg, sizeof msg);
    fail(rc, "%s", msg);
  }
}

void Fgmres::launch_step() {
  double* vj = V.p + int64_t(j) * n;
  double* zj = Z.p + int64_t(j) * n;
  double* wv = V.p + int64_t(j + 1) * n;
  if (M && M->o.kind != TPF_PREC_NONE) {
    if (spec_j != j) apply_precond(j);
    spec_j = -1;
  } else {
    copy(zj, vj, n, s);
  }
  bcsr_apply(J, zj, nullptr, wv, s);
  int nk = j + 1;
  {
    TimedScope ts("cgs2", s);
    DISPATCH_K(nk, KM, {
      // lanes per entry: pass 1 holds KM / L1 sums per lane, pass 2 also
      // KM / L2 basis values
      constexpr int L1 = KM <= 16 ? 1 : 2, L2 = KM <= 12 ? 1 : (KM <= 20 ? 2 : 4);
      const int g1 = resident_grid(k_cgs_dots<KM, L1>, n),
                g2 = resident_grid(k_cgs_axpy_dots<KM, L2>, n);
      g_norm = resident_grid(k_cgs_axpy_norm<KM>, n);
      k_cgs_dots<KM, L1><<<g1, kKBlock, 0, s>>>(n, nk, V.p, wv, part.p);
      TPF_CHECK_LAUNCH();
      k_reduce_parts<<<nk, kRedBlock, 0, s>>>(g1, part.p, h1.p);
      TPF_CHECK_LAUNCH();
      k_cgs_axpy_dots<KM, L2><<<g2, kKBlock, 0, s>>>(n, nk, V.p, h1.p, wv, part.p);
      TPF_CHECK_LAUNCH();
      k_reduce_parts<<<nk, kRedBlock, 0, s>>>(g2, part.p, h2.p);
      TPF_CHECK_LAUNCH();
      k_cgs_axpy_norm<KM><<<g_norm, kKBlock, 0, s>>>(n, nk, V.p, h2.p, wv, part.p);
      TPF_CHECK_LAUNCH();
    });
  }
  GState* gs = reinterpret_cast<GState*>(st_dev.p);
  k_givens<<<1, kRedBlock, 0, s>>>(j, m, h1.p, h2.p, part.p, g_norm, H.p, cs.p, sn.p, g.p, gs);
  TPF_CHECK_LAUNCH();
  k_scale<<<vec_grid(n), 256, 0, s>>>(n, wv, gs, wv);
  TPF_CHECK_LAUNCH();
  TPF_HIP(hipMemcpyAsync(host, gs, sizeof(GState), hipMemcpyDeviceToHost, s));
  phase = kStep;
  // the next step's preconditioning behind the scalars, unless this step
  // may end the cycle (last column, iteration cap, estimate near the
  // tolerance: the factor leaves room for two steps of fast convergence)
  if (speculate && M && M->o.kind != TPF_PREC_NONE && j + 1 < m && total + 1 < o.maxit &&
      spec_est > 50.0 * o.rtol) {
    if (!ready) ready = thread_event(2);
    TPF_HIP(hipEventRecord(ready, s));
    ev_pending = true;
    apply_precond(j + 1);
    spec_j = j + 1;
  }
}

void Fgmres::launch_cycle_end() {
  if (k > 0) {
    k_trisolve<<<1, 64, 0, s>>>(k, m, H.p, g.p, y.p);
    TPF_CHECK_LAUNCH();
    k_update_x<<<vec_grid(n), 256, 0, s>>>(n, k, Z.p, y.p, x);
    TPF_CHECK_LAUNCH();
  }
  bcsr_apply(J, x, b, r.p, s);
  nrm2_device(r.p, n, scal.p, part.p, s);
  TPF_HIP(hipMemcpyAsync(host, scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
  phase = kCycleEnd;
}

void Fgmres::finish(int st_code, double rel) {
  status = st_code;
  relres = rel;
  phase = kDone;
  ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

bool Fgmres::complete() {
  switch (phase) {
    case kInit: {
      beta0 = *reinterpret_cast<double*>(host);
      if (beta0 == 0.0) {
        finish(TPF_CONVERGED, 0.0);
        est = 0.0;
        return true;
      }
      if (!std::isfinite(beta0)) {
        finish(TPF_NONFINITE, NAN);
        est = NAN;
        return true;
      }
      launch_cycle_start(b, beta0);
      return false;
    }
    case kStep: {
      GState gst = *reinterpret_cast<GState*>(host);
      ++total;
      bool end = false;
      if (gst.d == 0.0 || !std::isfinite(gst.d)) {
        breakdown = true;
        k = j;
        end = true;
      } else {
        k = j + 1;
        est = gst.est / beta0;
        spec_est = est;
        end = gst.est <= o.rtol * beta0 || gst.hn == 0.0 || total >= o.maxit || j + 1 >= m;
      }
      if (end) {
        launch_cycle_end();
      } else {
        ++j;
        launch_step();
      }
      return false;
    }
    case kCycleEnd: {
      double rn = *reinterpret_cast<double*>(host);
      if (!std::isfinite(rn)) {
        finish(TPF_NONFINITE, NAN);
        return true;
      }
      if (rn <= o.rtol * beta0) {
        finish(TPF_CONVERGED, rn / beta0);
        return true;
      }
      if (breakdown) {
        finish(TPF_BREAKDOWN, rn / beta0);
        return true;
      }
      if (total >= o.maxit) {
        finish(TPF_MAX_ITERS, rn / beta0);
        return true;
      }
      launch_cycle_start(r.p, rn);
      return false;
    }
    default:
      return true;
  }
}

void Fgmres::info(tpf_solve_info* out) const {
  out->status = status;
  out->iterations = total;
  out->relres_est = est;
  out->relres_true = relres;
  out->ms = ms;
}

}  // namespace tpf

using namespace tpf;

extern "C" int tpf_solve(const tpf_jacobian* J, tpf_precond* M, const double* b, double* x,
                         const tpf_solve_opts* o, tpf_solve_info* info, void* stream) {
  return guarded([&] {
    TPF_REQUIRE(J && b && x && o && info, TPF_ERR_INVALID_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Fgmres f;  // workspace drawn from (and returned to) the installed allocator
    f.speculate = true;
    f.begin(J, M, b, x, *o, s, host_scratch().get<double>(8));
    bool done = false;
    while (!done) {
      if (f.ev_pending)
        TPF_HIP(hipEventSynchronize(f.ready));
      else
        TPF_HIP(hipStreamSynchronize(s));
      f.ev_pending = false;
      done = f.complete();
    }
    TPF_HIP(hipStreamSynchronize(s));
    f.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - f.t0).count();
    f.info(info);
  });
}

// ------------------------------------------------------------ allocation-free solve
// The workspace of tpf_solve_noalloc lives in one file-scope device array per
// GPU.  In host code `scratch` names a host-side stand-in, not the device
// copy: its device address is looked up once per device and only that
// address is passed to kernels.
namespace tpf {
namespace {
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kScratchDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchDevices] = {};

// device address of the current device's scratch array (looked up on the
// first call on that device, with it current)
double* scratch_on_current_device() {
  int dev = -1;
  TPF_HIP(hipGetDevice(&dev));
  TPF_REQUIRE(dev >= 0 && dev < kScratchDevices, TPF_ERR_INVALID_ARG,
              "device %d is beyond the %d devices the allocation-free solve supports", dev,
              kScratchDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    TPF_REQUIRE(e == hipSuccess && p, TPF_ERR_HIP,
                "hipGetSymbolAddress(scratch) on device %d -> %s", dev, hipGetErrorString(e));
    TPF_REQUIRE(reinterpret_cast<uintptr_t>(p) % 256 == 0, TPF_ERR_HIP,
                "scratch array is not 256-byte aligned on device %d", dev);
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace
}  // namespace tpf

extern "C" int tpf_solve_noalloc(const tpf_jacobian* J, tpf_precond* M, const double* b,
                                 double* x, const tpf_solve_opts* o, tpf_solve_info* info,
                                 void* stream) {
  return guarded([&] {
    TPF_REQUIRE(J && b && x && o && info, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(o->restart >= 1 && o->restart <= kMaxRestart, TPF_ERR_INVALID_ARG,
                "restart must be in [1, %d]", kMaxRestart);
    TPF_REQUIRE(!graphs_enabled(), TPF_ERR_STATE,
                "V-cycle graphs are instantiated on first use: disable them (tpf_set_graphs(0)) "
                "for the allocation-free solve");
    const int64_t n = 2 * int64_t(J->nb);
    const size_t need = Fgmres::workspace_doubles(n, o->restart) * sizeof(double);
    TPF_REQUIRE(need <= kScratchBytes, TPF_ERR_INVALID_ARG,
                "tpf_solve_noalloc: %lld unknowns at restart %d need %zu bytes of workspace; "
                "the allocation-free solve holds at most %zu bytes (use tpf_solve)",
                (long long)n, o->restart, need, kScratchBytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Fgmres f;  // workspace views the scratch array; nothing is allocated
    f.bind(scratch_on_current_device(), n, o->restart);
    f.speculate = false;
    // pageable and per thread (it outlives a copy still queued when an error
    // ends the call); every read follows a stream synchronisation
    alignas(64) static thread_local double host_slot[8];
    f.begin(J, M, b, x, *o, s, host_slot);
    bool done = false;
    while (!done) {
      TPF_HIP(hipStreamSynchronize(s));
      done = f.complete();
    }
    TPF_HIP(hipStreamSynchronize(s));
    f.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - f.t0).count();
    f.info(info);
  });
}
