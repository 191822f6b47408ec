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

#include "linalg_dev.hpp"
#include "precond.hpp"

namespace tpf {

namespace {
constexpr int kKBlock = 256;
constexpr int kMaxRestart = 64;

int krylov_grid(int64_t n) {
  int64_t g = (n + kKBlock * 4 - 1) / (kKBlock * 4);
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return int(g);
}

// block-wise reduction of KMAX running sums into part[block][k]
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
    part[int64_t(blockIdx.x) * KMAX + k] = t;
  }
}

// pass 1: part = V^T w  (nk vectors)
template <int KMAX>
__global__ void __launch_bounds__(kKBlock) k_cgs_dots(int64_t n, int nk, const double* __restrict__ V,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ part) {
  double acc[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) acc[k] = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kKBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kKBlock) {
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < nk) acc[k] += V[k * n + i] * wi;
  }
  reduce_store<KMAX>(acc, nk, part);
}

// pass 2: w -= V h; part = V^T w
template <int KMAX>
__global__ void __launch_bounds__(kKBlock) k_cgs_axpy_dots(int64_t n, int nk,
                                                           const double* __restrict__ V,
                                                           const double* __restrict__ h,
                                                           double* __restrict__ w,
                                                           double* __restrict__ part) {
  __shared__ double hs[KMAX];
  for (int k = threadIdx.x; k < nk; k += kKBlock) hs[k] = h[k];
  __syncthreads();
  double acc[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) acc[k] = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kKBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kKBlock) {
    double v[KMAX];
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < nk) {
        v[k] = V[k * n + i];
        wi -= hs[k] * v[k];
      }
    w[i] = wi;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < nk) acc[k] += v[k] * wi;
  }
  reduce_store<KMAX>(acc, nk, part);
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
  for (int64_t i = int64_t(blockIdx.x) * kKBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kKBlock) {
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < nk) wi -= hs[k] * V[k * n + i];
    w[i] = wi;
    acc[0] += wi * wi;
  }
  reduce_store<1>(acc, 1, part);
}

// out[k] = sum_b part[b][k]: one wavefront per column k, lanes stride over
// the blocks, fixed reduction tree (deterministic)
__global__ void __launch_bounds__(64) k_reduce_parts(int nb, int kstride,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ out) {
  int k = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) t += part[int64_t(b) * kstride + k];
  t = wave_sum(t);
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
__global__ void __launch_bounds__(64) k_givens(int j, int m, const double* __restrict__ h1,
                                               const double* __restrict__ h2,
                                               const double* __restrict__ nrm2_part, int nparts,
                                               double* __restrict__ H, double* __restrict__ cs,
                                               double* __restrict__ sn, double* __restrict__ g,
                                               GState* __restrict__ st) {
  double ss = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 64) ss += nrm2_part[b];
  ss = wave_sum(ss);
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

#define DISPATCH_K(nk, KM, ...)                                  \
  if (nk <= 8) { constexpr int KM = 8; __VA_ARGS__ }             \
  else if (nk <= 16) { constexpr int KM = 16; __VA_ARGS__ }      \
  else if (nk <= 32) { constexpr int KM = 32; __VA_ARGS__ }      \
  else { constexpr int KM = 64; __VA_ARGS__ }

struct Workspace {
  Buf<double> V, Z, H, cs, sn, g, h1, h2, part, y, r;
  Buf<GState> st;
  int64_t n = 0;
  int m = 0;
};

void ensure_ws(Workspace& w, int64_t n, int m, hipStream_t s) {
  if (w.n == n && w.m == m) return;
  w.V.alloc(size_t(m + 1) * n, s);
  w.Z.alloc(size_t(m) * n, s);
  w.H.alloc(size_t(m + 1) * m, s);
  w.cs.alloc(m, s);
  w.sn.alloc(m, s);
  w.g.alloc(m + 1, s);
  w.h1.alloc(kMaxRestart + 1, s);
  w.h2.alloc(kMaxRestart + 1, s);
  w.part.alloc(size_t(1024) * 64, s);
  w.y.alloc(m, s);
  w.r.alloc(n, s);
  w.st.alloc(1, s);
  w.n = n;
  w.m = m;
}

unsigned vec_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return unsigned(g);
}

}  // namespace

}  // namespace tpf

using namespace tpf;

extern "C" int tpf_solve(const tpf_jacobian* J, tpf_precond* M, const double* b, double* x,
                         const tpf_solve_opts* o, tpf_solve_info* info, void* stream) {
  return guarded([&] {
    TPF_REQUIRE(J && b && x && o && info, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(o->restart >= 1 && o->restart <= kMaxRestart, TPF_ERR_INVALID_ARG,
                "restart must be in [1, %d]", kMaxRestart);
    TPF_REQUIRE(o->maxit >= 1 && o->rtol > 0, TPF_ERR_INVALID_ARG, "maxit >= 1 and rtol > 0 required");
    if (M) {
      TPF_REQUIRE(M->ready, TPF_ERR_STATE, "preconditioner not set up");
      TPF_REQUIRE(M->o.kind == TPF_PREC_NONE || M->J == J, TPF_ERR_STATE,
                  "preconditioner was set up for another Jacobian");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto t0 = std::chrono::steady_clock::now();
    int64_t n = 2 * int64_t(J->nb);
    int m = o->restart;
    Workspace w;  // per call: drawn from (and returned to) the installed allocator
    ensure_ws(w, n, m, s);
    fill(x, 0.0, n, s);
    std::memset(info, 0, sizeof(*info));
    double beta0 = nrm2_host(b, n, s);
    auto finish = [&](int status, double rel_true, double est, int its) {
      info->status = status;
      info->relres_true = rel_true;
      info->relres_est = est;
      info->iterations = its;
      TPF_HIP(hipStreamSynchronize(s));
      info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    if (beta0 == 0.0) {
      finish(TPF_CONVERGED, 0.0, 0.0, 0);
      return;
    }
    if (!std::isfinite(beta0)) {
      finish(TPF_NONFINITE, NAN, NAN, 0);
      return;
    }
    int G = krylov_grid(n);
    int total = 0;
    double est = 1.0;
    const double* rsrc = b;  // residual of x_0 = 0
    while (true) {
      double beta = nrm2_host(rsrc, n, s);
      k_scale_by<<<vec_grid(n), 256, 0, s>>>(n, rsrc, 1.0 / beta, w.V.p);
      TPF_CHECK_LAUNCH();
      fill(w.g.p, 0.0, m + 1, s);
      fill(w.g.p, beta, 1, s);
      int k = 0;
      bool breakdown = false;
      for (int j = 0; j < m; ++j) {
        double* vj = w.V.p + int64_t(j) * n;
        double* zj = w.Z.p + int64_t(j) * n;
        double* wv = w.V.p + int64_t(j + 1) * n;
        if (M && M->o.kind != TPF_PREC_NONE) {
          TimedScope ts("precond_apply", s);
          int rc = tpf_precond_apply(M, vj, zj, s);
          if (rc != TPF_OK) {
            char msg[1024];
            tpf_last_error(msg, sizeof msg);
            fail(rc, "%s", msg);
          }
        } else {
          copy(zj, vj, n, s);
        }
        bcsr_apply(J, zj, nullptr, wv, s);
        int nk = j + 1;
        {
          TimedScope ts("cgs2", s);
          DISPATCH_K(nk, KM, {
            k_cgs_dots<KM><<<G, kKBlock, 0, s>>>(n, nk, w.V.p, wv, w.part.p);
            TPF_CHECK_LAUNCH();
            k_reduce_parts<<<nk, 64, 0, s>>>(G, KM, w.part.p, w.h1.p);
            TPF_CHECK_LAUNCH();
            k_cgs_axpy_dots<KM><<<G, kKBlock, 0, s>>>(n, nk, w.V.p, w.h1.p, wv, w.part.p);
            TPF_CHECK_LAUNCH();
            k_reduce_parts<<<nk, 64, 0, s>>>(G, KM, w.part.p, w.h2.p);
            TPF_CHECK_LAUNCH();
            k_cgs_axpy_norm<KM><<<G, kKBlock, 0, s>>>(n, nk, w.V.p, w.h2.p, wv, w.part.p);
            TPF_CHECK_LAUNCH();
          });
        }
        k_givens<<<1, 64, 0, s>>>(j, m, w.h1.p, w.h2.p, w.part.p, G, w.H.p, w.cs.p, w.sn.p, w.g.p,
                                  w.st.p);
        TPF_CHECK_LAUNCH();
        k_scale<<<vec_grid(n), 256, 0, s>>>(n, wv, w.st.p, wv);
        TPF_CHECK_LAUNCH();
        GState* hst = host_scratch().get<GState>(1);
        TPF_HIP(hipMemcpyAsync(hst, w.st.p, sizeof(GState), hipMemcpyDeviceToHost, s));
        TPF_HIP(hipStreamSynchronize(s));
        GState g = *hst;
        ++total;
        if (g.d == 0.0 || !std::isfinite(g.d)) {
          breakdown = true;
          k = j;
          break;
        }
        k = j + 1;
        est = g.est / beta0;
        if (g.est <= o->rtol * beta0 || g.hn == 0.0 || total >= o->maxit) break;
      }
      if (k > 0) {
        k_trisolve<<<1, 64, 0, s>>>(k, m, w.H.p, w.g.p, w.y.p);
        TPF_CHECK_LAUNCH();
        k_update_x<<<vec_grid(n), 256, 0, s>>>(n, k, w.Z.p, w.y.p, x);
        TPF_CHECK_LAUNCH();
      }
      bcsr_apply(J, x, b, w.r.p, s);
      double rn = nrm2_host(w.r.p, n, s);
      rsrc = w.r.p;
      if (!std::isfinite(rn)) {
        finish(TPF_NONFINITE, NAN, est, total);
        return;
      }
      if (rn <= o->rtol * beta0) {
        finish(TPF_CONVERGED, rn / beta0, est, total);
        return;
      }
      if (breakdown) {
        finish(TPF_BREAKDOWN, rn / beta0, est, total);
        return;
      }
      if (total >= o->maxit) {
        finish(TPF_MAX_ITERS, rn / beta0, est, total);
        return;
      }
    }
  });
}
