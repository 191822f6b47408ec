// The paper's preconditioners (Sec. 3.2-3.4):
//   AMG   one V-cycle on the point-ordered scalar J (black box, Sec. 3.2);
//   CPR1  Algorithm 1 / Eq. m_comb: u = P_1^{-1} r, r' = r - J u,
//         z = u + R_p^T V(A_pp; R_p r');
//   CPR2  Algorithm 2 / Eq. m_add: as CPR1 plus R_s^T V(A_ss; R_s r');
//   BF    Algorithm 3 / Eq. m_bf: s = V(A_ss; R_s r), t = R_p r - A_ps s,
//         p = V(S~; t), z = (p, s), with S~ = A_pp - A_ps diag(A_ss)^{-1} A_sp
//         (Eq. SIMPLE-Schur, trailing factor A_sp as in the exact Schur
//         complement).
// P_1 is block ILU(0) (Sec. 3.3) in the lexicographic point order; on the
// 5/7-point block stencil only the pivot blocks change,
// D_i = A_ii - sum_{k<i} A_ik D_k^{-1} A_ki, and M = (D+L)D^{-1}(D+U).  The
// factorisation and both triangular solves proceed by anti-diagonal
// wavefronts ix+iy+iz = const, whose cells are mutually independent.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <exception>
#include <thread>
#include <type_traits>

#include "linalg_dev.hpp"
#include "precond.hpp"

namespace tpf {

namespace {

__global__ void k_extract_blocks(int64_t nnzb, const double* __restrict__ jv,
                                 double* __restrict__ app, double* __restrict__ aps,
                                 double* __restrict__ asp, double* __restrict__ ass) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nnzb) return;
  double4 b = reinterpret_cast<const double4*>(jv)[e];
  app[e] = b.x;
  aps[e] = b.y;
  asp[e] = b.z;
  ass[e] = b.w;
}

// point-ordered scalar matrix: rows 2i+a, columns 2j+b, 4 entries per block
__global__ void k_scalarize_pattern(int nb, const int* __restrict__ rp, const int* __restrict__ ci,
                                    int* __restrict__ srp, int* __restrict__ sci) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nb) return;
  int r0 = rp[i];
  if (i == nb) {
    srp[2 * nb] = 4 * r0;
    return;
  }
  int len = rp[i + 1] - r0;
  srp[2 * i] = 4 * r0;
  srp[2 * i + 1] = 4 * r0 + 2 * len;
  for (int a = 0; a < 2; ++a) {
    int o = 4 * r0 + a * 2 * len;
    for (int k = 0; k < len; ++k) {
      int j = ci[r0 + k];
      sci[o + 2 * k] = 2 * j;
      sci[o + 2 * k + 1] = 2 * j + 1;
    }
  }
}

__global__ void k_scalarize_values(int nb, const int* __restrict__ rp, const double* __restrict__ jv,
                                   double* __restrict__ sv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int r0 = rp[i], len = rp[i + 1] - r0;
  for (int a = 0; a < 2; ++a) {
    int o = 4 * r0 + a * 2 * len;
    for (int k = 0; k < len; ++k) {
      sv[o + 2 * k] = jv[4 * int64_t(r0 + k) + 2 * a];
      sv[o + 2 * k + 1] = jv[4 * int64_t(r0 + k) + 2 * a + 1];
    }
  }
}

__global__ void k_diag_inv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, double* __restrict__ dinv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] == i) d = v[e];
  dinv[i] = 1.0 / d;
}

__global__ void k_scale_cols(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ v, const double* __restrict__ dinv,
                             double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) out[e] = v[e] * dinv[ci[e]];
}

// ---------------------------------------------------------------- S~ on the grid
// On the 3D grid every block row couples a cell to its in-grid face
// neighbours (offsets kN1, ascending in the cell numbering), so
// S~ = A_pp - A_ps diag(A_ss)^{-1} A_sp couples it to the in-grid cells
// within two face steps (kN2, ascending when every direction has at least
// five cells).  Entry (i, i + t) sums Y_{i,a} (A_sp)_{i+a,b} over the pairs
// a + b = t in ascending a, with Y = A_ps diag(A_ss)^{-1}: the terms and
// the pattern of the general sparse product, formed in one pass without
// sorting.
struct Off3 {
  int x, y, z;
};
__device__ constexpr Off3 kN1[7] = {{0, 0, -1}, {0, -1, 0}, {-1, 0, 0}, {0, 0, 0},
                                    {1, 0, 0},  {0, 1, 0},  {0, 0, 1}};
__device__ constexpr Off3 kN2[25] = {
    {0, 0, -2},  {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {1, 0, -1}, {0, 1, -1}, {0, -2, 0},
    {-1, -1, 0}, {0, -1, 0},  {1, -1, 0},  {-2, 0, 0}, {-1, 0, 0}, {0, 0, 0},  {1, 0, 0},
    {2, 0, 0},   {-1, 1, 0},  {0, 1, 0},   {1, 1, 0},  {0, 2, 0},  {0, -1, 1}, {-1, 0, 1},
    {0, 0, 1},   {1, 0, 1},   {0, 1, 1},   {0, 0, 2}};

__device__ inline bool in_grid(int x, int y, int z, int nx, int ny, int nz) {
  return x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
}

__global__ void __launch_bounds__(256) k_schur_count(int nx, int ny, int nz,
                                                     int* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t sxy = int64_t(nx) * ny;
  if (i >= sxy * nz) return;
  const int x = int(i % nx), y = int((i / nx) % ny), z = int(i / sxy);
  int c = 0;
#pragma unroll
  for (int t = 0; t < 25; ++t) c += in_grid(x + kN2[t].x, y + kN2[t].y, z + kN2[t].z, nx, ny, nz);
  cnt[i] = c;
}

// Rows of S~ at srp (from k_schur_count); rp: the block pattern's rows.  One
// wavefront per work-group takes kSchurRows consecutive rows, stages their
// entries in LDS and writes the (contiguous) range coalesced.
constexpr int kSchurRows = 64;
__global__ void __launch_bounds__(kSchurRows) k_schur_fill(int nx, int ny, int nz,
                                                    const int* __restrict__ rp,
                                                    const double* __restrict__ app,
                                                    const double* __restrict__ aps,
                                                    const double* __restrict__ asp,
                                                    const double* __restrict__ dinv,
                                                    const int* __restrict__ srp,
                                                    int* __restrict__ sci,
                                                    double* __restrict__ sv) {
  __shared__ int lc[kSchurRows * 25];
  __shared__ double lv[kSchurRows * 25];
  const int64_t sxy = int64_t(nx) * ny, n = sxy * nz;
  const int64_t i0 = int64_t(blockIdx.x) * kSchurRows;
  const int64_t i1 = i0 + kSchurRows < n ? i0 + kSchurRows : n;
  const int64_t i = i0 + threadIdx.x < i1 ? i0 + threadIdx.x : i1 - 1;  // clamped: valid row
  const int base = srp[i0];
  const int x = int(i % nx), y = int((i / nx) % ny), z = int(i / sxy);
  auto lin = [&](int dx, int dy, int dz) { return int64_t(dx) + int64_t(nx) * dy + sxy * dz; };
  // Every load below is issued unconditionally at a position clamped into
  // its row (which holds at least the diagonal), so all are in flight
  // before the first wait; entries of out-of-grid neighbours are zeroed.
  bool in1[7];
  int before[7], cnt = 0;
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    in1[a] = in_grid(x + kN1[a].x, y + kN1[a].y, z + kN1[a].z, nx, ny, nz);
    before[a] = cnt;
    cnt += in1[a];
  }
  int64_t nbr[7];
  int rs[7];
  const int r0 = rp[i];
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    nbr[a] = in1[a] ? i + lin(kN1[a].x, kN1[a].y, kN1[a].z) : i;
    rs[a] = rp[nbr[a]];
  }
  // row i of Y and A_pp by neighbour
  double yv[7], pv[7];
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    const int e = r0 + before[a] - (in1[a] ? 0 : (before[a] == cnt ? 1 : 0));
    const double ya = aps[e] * dinv[nbr[a]];
    const double pa = app[e];
    yv[a] = in1[a] ? ya : 0.0;
    pv[a] = in1[a] ? pa : 0.0;
  }
  // rows of A_sp of the neighbours, by neighbour of the neighbour
  double m[7][7];
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    const int xa = x + kN1[a].x, ya = y + kN1[a].y, za = z + kN1[a].z;
    int c = 0;
#pragma unroll
    for (int b = 0; b < 7; ++b) {
      const bool in = in1[a] && in_grid(xa + kN1[b].x, ya + kN1[b].y, za + kN1[b].z, nx, ny, nz);
      // position of entry b in row nbr[a], or of the row's first entry
      const double v = asp[rs[a] + (in ? c : 0)];
      m[a][b] = in ? v : 0.0;
      c += in;
    }
  }
  const bool mine = i0 + threadIdx.x < i1;
  int o = srp[i] - base;
#pragma unroll
  for (int t = 0; t < 25; ++t) {
    const Off3 T = kN2[t];
    if (!in_grid(x + T.x, y + T.y, z + T.z, nx, ny, nz)) continue;
    double acc = 0.0, d = 0.0;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
#pragma unroll
      for (int b = 0; b < 7; ++b)
        if (kN1[a].x + kN1[b].x == T.x && kN1[a].y + kN1[b].y == T.y &&
            kN1[a].z + kN1[b].z == T.z)
          acc += yv[a] * m[a][b];
      if (kN1[a].x == T.x && kN1[a].y == T.y && kN1[a].z == T.z) d = pv[a];
    }
    if (mine) {
      lc[o] = int(i + lin(T.x, T.y, T.z));
      lv[o] = d - acc;
    }
    ++o;
  }
  __syncthreads();
  const int cnt_all = srp[i1] - base;
  for (int q = threadIdx.x; q < cnt_all; q += kSchurRows) {
    sci[base + q] = lc[q];
    sv[base + q] = lv[q];
  }
}

template <class T>
__global__ void k_gather(int n, const double* __restrict__ r, int comp, T* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = T(r[2 * i + comp]);
}

template <class T>
__global__ void k_scatter2(int n, const T* __restrict__ p, const T* __restrict__ s,
                           double* __restrict__ z) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) reinterpret_cast<double2*>(z)[i] = make_double2(double(p[i]), double(s[i]));
}

template <class T>
__global__ void k_add_comp(int n, double* __restrict__ z, int comp, const T* __restrict__ v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[2 * i + comp] += double(v[i]);
}

// out = component comp of r, and g = dinv .* out (the first level's Jacobi
// guess of the V-cycle that takes out as its right-hand side)
template <class T>
__global__ void k_gather_guess(int n, const double* __restrict__ r, int comp,
                               const T* __restrict__ dinv, T* __restrict__ out,
                               T* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const T v = T(r[2 * i + comp]);
    out[i] = v;
    g[i] = dinv[i] * v;
  }
}

// t_i = r_{p,i} - sum_j (A_ps)_ij s_j   (Algorithm 3, step 3); with g, also
// g_i = dinv_i t_i (the S~ cycle's first Jacobi guess)
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_bf_rhs(int n, const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const double* __restrict__ aps,
                                                const double* __restrict__ r,
                                                const T* __restrict__ s, T* __restrict__ t,
                                                const T* __restrict__ dinv, T* __restrict__ g) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  double sum = row_dot<double, LPR>(row, lane, rp, ci, aps, [&](int j) { return double(s[j]); });
  if (lane == 0) {
    const T tv = T(r[2 * row] - sum);
    t[row] = tv;
    if (g) g[row] = dinv[row] * tv;
  }
}

// ---------------------------------------------------------------- block ILU(0)
struct Grid3 {
  int nx, ny, nz;
};

__device__ inline int len2d(int m, int nx, int ny) {
  int lo = m - nx + 1 > 0 ? m - nx + 1 : 0;
  int hi = m < ny - 1 ? m : ny - 1;
  return hi >= lo ? hi - lo + 1 : 0;
}

// position of cell i in the wavefront ordering (fronts ascending, index
// ascending inside a front)
__global__ void k_front_place(Grid3 g, const int* __restrict__ fptr, int* __restrict__ cells) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t N = int64_t(g.nx) * g.ny * g.nz;
  if (i >= N) return;
  int ix = int(i % g.nx), iy = int((i / g.nx) % g.ny), iz = int(i / (int64_t(g.nx) * g.ny));
  int L = ix + iy + iz;
  int64_t pos = fptr[L];
  for (int z = 0; z < iz; ++z) pos += len2d(L - z, g.nx, g.ny);
  int m = L - iz;
  int lo = m - g.nx + 1 > 0 ? m - g.nx + 1 : 0;
  pos += iy - lo;
  cells[pos] = int(i);
}

__device__ inline void mm2(const double* a, const double* b, double* c) {
  c[0] = a[0] * b[0] + a[1] * b[2];
  c[1] = a[0] * b[1] + a[1] * b[3];
  c[2] = a[2] * b[0] + a[3] * b[2];
  c[3] = a[2] * b[1] + a[3] * b[3];
}

__device__ inline void bilu_factor_cell(int i, const int* __restrict__ rp,
                                        const int* __restrict__ ci, const double* __restrict__ jv,
                                        double* __restrict__ dinv, int* __restrict__ flag) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double d[4] = {0.0, 0.0, 0.0, 0.0};
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    int k = ci[e];
    if (k == i) {
      for (int q = 0; q < 4; ++q) d[q] = jv[4 * int64_t(e) + q];
    } else if (k < i) {
      int f = rp[k];
      while (ci[f] != i) ++f;  // A_ki exists: the pattern is symmetric
      double tmp[4], c[4];
      mm2(jv + 4 * int64_t(e), dinv + 4 * int64_t(k), tmp);
      mm2(tmp, jv + 4 * int64_t(f), c);
      for (int q = 0; q < 4; ++q) acc[q] += c[q];
    }
  }
  for (int q = 0; q < 4; ++q) d[q] = d[q] - acc[q];
  double det = d[0] * d[3] - d[1] * d[2];
  if (det == 0.0 || !isfinite(det)) *flag = 1;
  double* o = dinv + 4 * int64_t(i);
  o[0] = d[3] / det;
  o[1] = -d[1] / det;
  o[2] = -d[2] / det;
  o[3] = d[0] / det;
}

__global__ void k_bilu_factor(int cnt, const int* __restrict__ cells, const int* __restrict__ rp,
                              const int* __restrict__ ci, const double* __restrict__ jv,
                              double* __restrict__ dinv, int* __restrict__ flag) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  bilu_factor_cell(cells[t], rp, ci, jv, dinv, flag);
}

// forward: w_i = D_i^{-1} (r_i - sum_{k<i} A_ik w_k)
template <class T>
__device__ inline void bilu_fwd_cell(int i, const int* __restrict__ rp, const int* __restrict__ ci,
                                     const T* __restrict__ jv, const T* __restrict__ dinv,
                                     const double* __restrict__ r, T* __restrict__ w) {
  T a0 = 0, a1 = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    int k = ci[e];
    if (k >= i) break;
    const T* b = jv + 4 * int64_t(e);
    T w0 = w[2 * k], w1 = w[2 * k + 1];
    a0 += b[0] * w0 + b[1] * w1;
    a1 += b[2] * w0 + b[3] * w1;
  }
  T x0 = T(r[2 * i]) - a0, x1 = T(r[2 * i + 1]) - a1;
  const T* di = dinv + 4 * int64_t(i);
  w[2 * i] = di[0] * x0 + di[1] * x1;
  w[2 * i + 1] = di[2] * x0 + di[3] * x1;
}

// backward: z_i = w_i - D_i^{-1} sum_{j>i} A_ij z_j
template <class T>
__device__ inline void bilu_bwd_cell(int i, const int* __restrict__ rp, const int* __restrict__ ci,
                                     const T* __restrict__ jv, const T* __restrict__ dinv,
                                     const T* __restrict__ w, T* __restrict__ z) {
  T a0 = 0, a1 = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    int j = ci[e];
    if (j <= i) continue;
    const T* b = jv + 4 * int64_t(e);
    T z0 = z[2 * j], z1 = z[2 * j + 1];
    a0 += b[0] * z0 + b[1] * z1;
    a1 += b[2] * z0 + b[3] * z1;
  }
  const T* di = dinv + 4 * int64_t(i);
  z[2 * i] = w[2 * i] - (di[0] * a0 + di[1] * a1);
  z[2 * i + 1] = w[2 * i + 1] - (di[2] * a0 + di[3] * a1);
}

// one launch per wavefront (large fronts)
template <class T>
__global__ void k_bilu_fwd(int cnt, const int* __restrict__ cells, const int* __restrict__ rp,
                           const int* __restrict__ ci, const T* __restrict__ jv,
                           const T* __restrict__ dinv, const double* __restrict__ r,
                           T* __restrict__ w) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) bilu_fwd_cell<T>(cells[t], rp, ci, jv, dinv, r, w);
}

template <class T>
__global__ void k_bilu_bwd(int cnt, const int* __restrict__ cells, const int* __restrict__ rp,
                           const int* __restrict__ ci, const T* __restrict__ jv,
                           const T* __restrict__ dinv, const T* __restrict__ w,
                           T* __restrict__ z) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) bilu_bwd_cell<T>(cells[t], rp, ci, jv, dinv, w, z);
}

// Whole sweeps in one work-group (fronts of at most kFrontWg cells, as on
// 2D grids): the fronts are taken in order with a barrier between them, in
// place of one launch per front.  FWD: forward sweep, else backward.
constexpr int kFrontWg = 2048;
template <class T, bool FWD>
__global__ void __launch_bounds__(1024) k_bilu_sweep_wg(int nf, const int* __restrict__ fptr,
                                                        const int* __restrict__ cells,
                                                        const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const T* __restrict__ jv,
                                                        const T* __restrict__ dinv,
                                                        const double* __restrict__ r,
                                                        T* __restrict__ w, T* __restrict__ z) {
  for (int q = 0; q < nf; ++q) {
    const int f = FWD ? q : nf - 1 - q;
    for (int t = fptr[f] + threadIdx.x; t < fptr[f + 1]; t += blockDim.x) {
      if (FWD)
        bilu_fwd_cell<T>(cells[t], rp, ci, jv, dinv, r, w);
      else
        bilu_bwd_cell<T>(cells[t], rp, ci, jv, dinv, w, z);
    }
    __syncthreads();
  }
}

// Row start of cell (x, y) in the 5-point block pattern of a 2D grid: full
// rows below (3 nx - 2 entries each, plus the south and north couplings that
// exist), then the cells to its left.
__device__ inline int64_t rp_5pt(int x, int y, int nx, int ny) {
  return int64_t(y) * (3 * nx - 2) + int64_t(nx) * (y > 0 ? y - 1 : 0) +
         int64_t(nx) * (y < ny - 1 ? y : ny - 1) + int64_t(x) * (1 + (y > 0) + (y < ny - 1)) +
         (x > 0 ? x - 1 : 0) + (x < nx - 1 ? x : nx - 1);
}

// Sweeps on 2D grids of at most kFront2d rows (fronts of at most that many
// cells): thread t takes the cell of row y = lo + t of each front; the
// previous front's results come from LDS (slot y, two buffers by front
// parity) instead of global memory.  A cell's row start follows from the
// 5-point pattern in closed form, so its blocks are loaded with no
// dependent load, two fronts ahead (fronts alternate between two register
// sets), and stay in flight across the LDS-only barriers: a front costs a
// barrier and one LDS exchange.  The work-group has as many threads as the
// longest front (rounded to wavefronts).  Same terms in the same order as the cell
// functions above.  FWD: forward sweep, else backward.
constexpr int kFront2d = 1024;
template <class T>
struct Bilu2dCell {
  T b0[4], b1[4], d[4], v[2];  // lower (FWD) / upper (BWD) blocks, D^{-1}, r (FWD) or w (BWD)
  bool has0, has1, live;
  int y;
  int64_t i;
};

template <class T, bool FWD>
__device__ inline void bilu_2d_load(int nx, int ny, int L, const T* __restrict__ jv,
                                    const T* __restrict__ dinv, const double* __restrict__ r,
                                    const T* __restrict__ w, Bilu2dCell<T>& c) {
  const int lo = L - nx + 1 > 0 ? L - nx + 1 : 0, hi = L < ny - 1 ? L : ny - 1;
  c.y = lo + int(threadIdx.x);
  c.live = c.y <= hi;
  const int y = c.live ? c.y : 0, x = c.live ? L - y : 0;
  c.i = int64_t(y) * nx + x;
  const int64_t rp_i = rp_5pt(x, y, nx, ny);
  // row entries: south (y > 0), west (x > 0), self, east (x < nx-1), north (y < ny-1)
  const int64_t self = rp_i + (y > 0) + (x > 0);
  int64_t e0, e1;
  if (FWD) {
    c.has0 = c.live && y > 0;  // south, column i - nx
    c.has1 = c.live && x > 0;  // west, column i - 1
    e0 = rp_i;
    e1 = rp_i + (y > 0);
  } else {
    c.has0 = c.live && x < nx - 1;  // east, column i + 1
    c.has1 = c.live && y < ny - 1;  // north, column i + nx
    e0 = self + 1;
    e1 = self + 1 + (x < nx - 1);
  }
  e0 = c.has0 ? e0 : self;
  e1 = c.has1 ? e1 : self;
  // only the front's cells load (one CU's memory pipe carries every front)
  if (c.live) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c.b0[q] = jv[4 * e0 + q];
      c.b1[q] = jv[4 * e1 + q];
      c.d[q] = dinv[4 * c.i + q];
    }
    if (FWD) {
      c.v[0] = T(r[2 * c.i]);
      c.v[1] = T(r[2 * c.i + 1]);
    } else {
      c.v[0] = w[2 * c.i];
      c.v[1] = w[2 * c.i + 1];
    }
  }
}

// one front: the previous front's results from buf[(q + 1) & 1], this
// front's into buf[q & 1].  Branch-free (missing couplings add zero, slots
// clamped), so the loads of later fronts keep their own wait counts.
template <class T, bool FWD>
__device__ inline void bilu_2d_step(const Bilu2dCell<T>& c, T (*buf)[kFront2d][2], int q,
                                    T* __restrict__ w, T* __restrict__ z) {
  const int y = c.y < kFront2d ? c.y : kFront2d - 1;
  const T(*prev)[2] = buf[(q + 1) & 1];
  const int s0 = FWD ? (y > 0 ? y - 1 : 0) : y;             // FWD south, BWD east
  const int s1 = FWD ? y : (y + 1 < kFront2d ? y + 1 : y);  // FWD west, BWD north
  const T u0 = prev[s0][0], u1 = prev[s0][1], v0 = prev[s1][0], v1 = prev[s1][1];
  T a0 = 0, a1 = 0;
  a0 += c.has0 ? c.b0[0] * u0 + c.b0[1] * u1 : T(0);
  a1 += c.has0 ? c.b0[2] * u0 + c.b0[3] * u1 : T(0);
  a0 += c.has1 ? c.b1[0] * v0 + c.b1[1] * v1 : T(0);
  a1 += c.has1 ? c.b1[2] * v0 + c.b1[3] * v1 : T(0);
  T o0, o1;
  if (FWD) {
    const T x0 = c.v[0] - a0, x1 = c.v[1] - a1;
    o0 = c.d[0] * x0 + c.d[1] * x1;
    o1 = c.d[2] * x0 + c.d[3] * x1;
  } else {
    o0 = c.v[0] - (c.d[0] * a0 + c.d[1] * a1);
    o1 = c.v[1] - (c.d[2] * a0 + c.d[3] * a1);
  }
  if (c.live) {
    T* out = FWD ? w : z;
    out[2 * c.i] = o0;
    out[2 * c.i + 1] = o1;
    buf[q & 1][y][0] = o0;
    buf[q & 1][y][1] = o1;
  }
}

// LDS-only release/acquire around the barrier: global loads stay in flight
// across it (no thread reads another's global writes inside the sweep)
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <class T, bool FWD>
__global__ void __launch_bounds__(kFront2d) k_bilu_sweep_2d(int nx, int ny,
                                                            const T* __restrict__ jv,
                                                            const T* __restrict__ dinv,
                                                            const double* __restrict__ r,
                                                            T* __restrict__ w, T* __restrict__ z) {
  __shared__ T buf[2][kFront2d][2];
  const int nf = nx + ny - 1;
  auto front = [&](int q) { return FWD ? q : nf - 1 - q; };
  // fronts past the last are loaded as no cells (live false), so the loop
  // body has no branch around its loads
  auto load = [&](int q, Bilu2dCell<T>& c) {
    bilu_2d_load<T, FWD>(nx, ny, q < nf ? front(q) : (FWD ? nf : -1), jv, dinv, r, w, c);
  };
  Bilu2dCell<T> ca, cb;  // fronts q (even) and q + 1
  load(0, ca);
  load(1, cb);
  for (int q = 0; q < nf; q += 2) {
    bilu_2d_step<T, FWD>(ca, buf, q, w, z);
    load(q + 2, ca);
    lds_barrier();
    bilu_2d_step<T, FWD>(cb, buf, q + 1, w, z);
    load(q + 3, cb);
    lds_barrier();
  }
}

// The factorisation on the same fronts: D_i = A_ii - A_is D_s^{-1} A_si -
// A_iw D_w^{-1} A_wi (s, w: the south and west neighbours, on the previous
// front, whose D^{-1} come from LDS), the terms in bilu_factor_cell's order.
struct Bilu2dFac {
  double as[4], aw[4], ad[4], sa[4], wa[4];  // A_is, A_iw, A_ii, A_si, A_wi
  bool hs, hw, live;
  int y;
  int64_t i;
};

__device__ inline void bilu_2d_fac_load(int nx, int ny, int L, const double* __restrict__ jv,
                                        Bilu2dFac& c) {
  const int lo = L - nx + 1 > 0 ? L - nx + 1 : 0, hi = L < ny - 1 ? L : ny - 1;
  c.y = lo + int(threadIdx.x);
  c.live = c.y <= hi;
  const int y = c.live ? c.y : 0, x = c.live ? L - y : 0;
  c.i = int64_t(y) * nx + x;
  c.hs = c.live && y > 0;
  c.hw = c.live && x > 0;
  const int64_t r0 = rp_5pt(x, y, nx, ny);
  const int64_t ed = r0 + (y > 0) + (x > 0);
  // south cell (x, y - 1): its north entry is its last; west cell (x - 1, y):
  // its east entry follows its diagonal
  const int64_t es = c.hs ? r0 : ed;
  const int64_t ew = c.hw ? r0 + (y > 0) : ed;
  const int64_t fs = c.hs ? rp_5pt(x, y - 1, nx, ny) + (y - 1 > 0) + (x > 0) + (x < nx - 1) + 1 : ed;
  const int64_t fw = c.hw ? rp_5pt(x - 1, y, nx, ny) + (y > 0) + (x - 1 > 0) + 1 : ed;
  if (c.live) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c.as[q] = jv[4 * es + q];
      c.aw[q] = jv[4 * ew + q];
      c.ad[q] = jv[4 * ed + q];
      c.sa[q] = jv[4 * fs + q];
      c.wa[q] = jv[4 * fw + q];
    }
  }
}

__device__ inline void bilu_2d_fac_step(const Bilu2dFac& c, double (*buf)[kFront2d][4], int q,
                                        double* __restrict__ dinv, int* __restrict__ flag) {
  const int y = c.y < kFront2d ? c.y : kFront2d - 1;
  const double(*prev)[4] = buf[(q + 1) & 1];
  const int ss = y > 0 ? y - 1 : 0;
  double ds[4], dw[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ds[t] = prev[ss][t];
    dw[t] = prev[y][t];
  }
  double tmp[4], cs_[4], cw_[4];
  mm2(c.as, ds, tmp);
  mm2(tmp, c.sa, cs_);
  mm2(c.aw, dw, tmp);
  mm2(tmp, c.wa, cw_);
  double d[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    double acc = 0.0;
    acc += c.hs ? cs_[t] : 0.0;
    acc += c.hw ? cw_[t] : 0.0;
    d[t] = c.ad[t] - acc;
  }
  const double det = d[0] * d[3] - d[1] * d[2];
  const double o[4] = {d[3] / det, -d[1] / det, -d[2] / det, d[0] / det};
  if (c.live) {
    if (det == 0.0 || !isfinite(det)) *flag = 1;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      dinv[4 * c.i + t] = o[t];
      buf[q & 1][y][t] = o[t];
    }
  }
}

__global__ void __launch_bounds__(kFront2d) k_bilu_factor_2d(int nx, int ny,
                                                             const double* __restrict__ jv,
                                                             double* __restrict__ dinv,
                                                             int* __restrict__ flag) {
  __shared__ double buf[2][kFront2d][4];
  const int nf = nx + ny - 1;
  auto load = [&](int q, Bilu2dFac& c) { bilu_2d_fac_load(nx, ny, q < nf ? q : nf, jv, c); };
  Bilu2dFac ca, cb;  // fronts q (even) and q + 1
  load(0, ca);
  load(1, cb);
  for (int q = 0; q < nf; q += 2) {
    bilu_2d_fac_step(ca, buf, q, dinv, flag);
    load(q + 2, ca);
    lds_barrier();
    bilu_2d_fac_step(cb, buf, q + 1, dinv, flag);
    load(q + 3, cb);
    lds_barrier();
  }
}

__global__ void __launch_bounds__(1024) k_bilu_factor_wg(int nf, const int* __restrict__ fptr,
                                                         const int* __restrict__ cells,
                                                         const int* __restrict__ rp,
                                                         const int* __restrict__ ci,
                                                         const double* __restrict__ jv,
                                                         double* __restrict__ dinv,
                                                         int* __restrict__ flag) {
  for (int f = 0; f < nf; ++f) {
    for (int t = fptr[f] + threadIdx.x; t < fptr[f + 1]; t += blockDim.x)
      bilu_factor_cell(cells[t], rp, ci, jv, dinv, flag);
    __syncthreads();
  }
}

template <class T>
__global__ void k_to_double(int64_t n, const T* __restrict__ a, double* __restrict__ b) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = double(a[i]);
}

Csr<double> block_copy(const tpf_precond* M, const double* vals, hipStream_t s) {
  Csr<double> A;
  A.nrows = A.ncols = M->N;
  A.nnz = M->J->nnzb;
  A.rp.alloc(M->N + 1, s);
  A.ci.alloc(A.nnz, s);
  A.v.alloc(A.nnz, s);
  copy(A.rp.p, M->brp.p, M->N + 1, s);
  copy(A.ci.p, M->bci.p, A.nnz, s);
  copy(A.v.p, vals, A.nnz, s);
  return A;
}

// interpolation per operator: AUTO uses extended+i for the pressure-like
// operators (S~, A_pp) and direct interpolation for A_ss and the scalar J
// offsets of the stencil |dx|+|dy|+|dz| <= radius on the grid, ascending;
// empty when two offsets coincide (very thin grids)
std::vector<int> stencil_offsets(const Phys& ph, int radius) {
  std::vector<int> off;
  int rz = ph.nz > 1 ? radius : 0, ry = ph.ny > 1 ? radius : 0, rx = ph.nx > 1 ? radius : 0;
  for (int dz = -rz; dz <= rz; ++dz)
    for (int dy = -ry; dy <= ry; ++dy)
      for (int dx = -rx; dx <= rx; ++dx)
        if (std::abs(dx) + std::abs(dy) + std::abs(dz) <= radius)
          off.push_back(dx + ph.nx * (dy + ph.ny * dz));
  std::sort(off.begin(), off.end());
  for (size_t k = 1; k < off.size(); ++k)
    if (off[k] == off[k - 1]) return {};
  if (radius >= 2 && (ph.nx < 5 || (ph.ny > 1 && ph.ny < 5) || (ph.nz > 1 && ph.nz < 5))) return {};
  return off;
}

// In-grid cells at each offset (dx,dy,dz) with |dx|+|dy|+|dz| <= radius, summed.
int64_t stencil_entries(const Phys& ph, int radius) {
  int64_t t = 0;
  for (int dz = -radius; dz <= radius; ++dz)
    for (int dy = -radius; dy <= radius; ++dy)
      for (int dx = -radius; dx <= radius; ++dx)
        if (std::abs(dx) + std::abs(dy) + std::abs(dz) <= radius)
          t += int64_t(std::max(ph.nx - std::abs(dx), 0)) * std::max(ph.ny - std::abs(dy), 0) *
               std::max(ph.nz - std::abs(dz), 0);
  return t;
}

// S~ by the grid kernels: a 3D grid of at least five cells per direction
// whose block pattern is the face-neighbour stencil
bool schur_on_grid_ok(const Phys& ph, int64_t nnzb) {
  return ph.nx >= 5 && ph.ny >= 5 && ph.nz >= 5 && nnzb == stencil_entries(ph, 1) &&
         stencil_entries(ph, 2) <= INT_MAX;
}

// S~ = A_pp - A_ps diag(A_ss)^{-1} A_sp on the grid; with pattern_given the
// rows and columns of S are those of an earlier call and only the values
// (and the same columns) are rewritten.
void schur_on_grid(tpf_precond* M, const Phys& ph, Csr<double>& S, bool pattern_given,
                   hipStream_t s) {
  const int64_t N = ph.N;
  if (!pattern_given) {
    S.nrows = S.ncols = int(N);
    S.nnz = stencil_entries(ph, 2);
    S.rp.alloc(N + 1, s);
    Buf<int> cnt(N, s);
    k_schur_count<<<grid_for(N, 256), 256, 0, s>>>(ph.nx, ph.ny, ph.nz, cnt.p);
    TPF_CHECK_LAUNCH();
    scan_exclusive_async(cnt.p, S.rp.p, N, s);  // the counts add up to S.nnz
    S.ci.alloc(S.nnz, s);
    S.v.alloc(S.nnz, s);
  }
  k_schur_fill<<<grid_for(N, kSchurRows), kSchurRows, 0, s>>>(ph.nx, ph.ny, ph.nz, M->brp.p, M->app_v.p,
                                                M->aps_v.p, M->asp_v.p, M->ass_dinv.p, S.rp.p,
                                                S.ci.p, S.v.p);
  TPF_CHECK_LAUNCH();
}

AmgOpts amg_opts(const tpf_precond_opts& o, bool pressure_like) {
  AmgOpts a;
  a.ext_i = o.interp == TPF_INTERP_EXTI || (o.interp == TPF_INTERP_AUTO && pressure_like);
  a.classical = o.interp == TPF_INTERP_CLASSICAL;
  a.cljp = o.coarsening == TPF_COARSEN_CLJP;
  a.exti_first = o.exti_route > 0 ? o.exti_route - 1 : 0;
  a.theta = o.theta;
  a.max_levels = o.max_levels;
  a.coarse_max = o.coarse_max;
  a.dense_max = o.dense_max;
  a.seed = o.hash_seed;
  a.fp32 = o.precision == TPF_FP32;
  a.smoother = o.smoother;
  a.nu1 = o.nu1;
  a.nu2 = o.nu2;
  a.cheb_degree = o.cheb_degree;
  a.trunc_pmax = o.trunc_pmax;
  a.trunc_factor = o.trunc_factor;
  return a;
}

void bilu_setup(tpf_precond* M, bool reuse, hipStream_t s) {
  const tpf_jacobian* J = M->J;
  const Phys& ph = J->prob->ph;
  int N = M->N;
  if (!reuse || M->front_ptr.empty()) {
    int nf = ph.nx + ph.ny + ph.nz - 2;
    std::vector<int> ptr(nf + 1, 0);
    for (int L = 0; L < nf; ++L) {
      int64_t c = 0;
      for (int z = 0; z < ph.nz; ++z) {
        int m = L - z;
        if (m < 0) break;
        int lo = std::max(0, m - ph.nx + 1), hi = std::min(ph.ny - 1, m);
        if (hi >= lo) c += hi - lo + 1;
      }
      ptr[L + 1] = int(ptr[L] + c);
    }
    TPF_REQUIRE(ptr[nf] == N, TPF_ERR_INVALID_ARG, "wavefront ordering does not cover the grid");
    M->front_ptr = ptr;
    M->front_max = 0;
    for (int L = 0; L < nf; ++L) M->front_max = std::max(M->front_max, ptr[L + 1] - ptr[L]);
    M->front_ptr_dev.alloc(nf + 1, s);
    TPF_HIP(hipMemcpyAsync(M->front_ptr_dev.p, ptr.data(), (nf + 1) * sizeof(int),
                           hipMemcpyHostToDevice, s));
    M->front_cells.alloc(N, s);
    k_front_place<<<grid_for(N, 256), 256, 0, s>>>(Grid3{ph.nx, ph.ny, ph.nz}, M->front_ptr_dev.p,
                                                   M->front_cells.p);
    TPF_CHECK_LAUNCH();
    note_host_sync();
    TPF_HIP(hipStreamSynchronize(s));
    M->bilu_dinv.alloc(4 * int64_t(N), s);
  }
  Buf<int> flag(1, s);
  fill_int(flag.p, 0, 1, s);
  int nf = int(M->front_ptr.size()) - 1;
  if (ph.nz == 1 && ph.ny <= kFront2d && int64_t(ph.nx) * ph.ny == N) {
    const int longest = std::min(ph.nx, ph.ny);  // cells of the longest front
    const int threads = (longest + kWave - 1) / kWave * kWave;
    k_bilu_factor_2d<<<1, threads, 0, s>>>(ph.nx, ph.ny, J->v.p, M->bilu_dinv.p, flag.p);
    TPF_CHECK_LAUNCH();
  } else if (M->front_max <= kFrontWg) {
    k_bilu_factor_wg<<<1, 1024, 0, s>>>(nf, M->front_ptr_dev.p, M->front_cells.p, J->rp.p,
                                        J->ci.p, J->v.p, M->bilu_dinv.p, flag.p);
    TPF_CHECK_LAUNCH();
  } else {
    for (int f = 0; f < nf; ++f) {
      int a = M->front_ptr[f], cnt = M->front_ptr[f + 1] - a;
      k_bilu_factor<<<grid_for(cnt, 256), 256, 0, s>>>(cnt, M->front_cells.p + a, J->rp.p,
                                                       J->ci.p, J->v.p, M->bilu_dinv.p, flag.p);
      TPF_CHECK_LAUNCH();
    }
  }
  int fl = read_scalar(flag.p, s);
  TPF_REQUIRE(fl == 0, TPF_ERR_SINGULAR, "zero pivot block in block ILU(0)");
  if (M->o.precision == TPF_FP32) {
    M->bilu_dinv32.ensure(4 * int64_t(N), s);
    cast<double, float>(M->bilu_dinv32.p, M->bilu_dinv.p, 4 * int64_t(N), s);
    M->jv32.ensure(4 * J->nnzb, s);
    cast<double, float>(M->jv32.p, J->v.p, 4 * J->nnzb, s);
  }
}

template <class T>
void bilu_apply(tpf_precond* M, const double* r, T* w, T* z, hipStream_t s) {
  const tpf_jacobian* J = M->J;
  const T* jv;
  const T* dinv;
  if constexpr (std::is_same<T, float>::value) {
    jv = M->jv32.p;
    dinv = M->bilu_dinv32.p;
  } else {
    jv = J->v.p;
    dinv = M->bilu_dinv.p;
  }
  int nf = int(M->front_ptr.size()) - 1;
  TimedScope ts("bilu_solve", s);
  const Phys& ph = J->prob->ph;
  if (ph.nz == 1 && ph.ny <= kFront2d && ph.nx >= 1 && int64_t(ph.nx) * ph.ny == ph.N) {
    const int longest = std::min(ph.nx, ph.ny);  // cells of the longest front
    const int threads = (longest + kWave - 1) / kWave * kWave;
    k_bilu_sweep_2d<T, true><<<1, threads, 0, s>>>(ph.nx, ph.ny, jv, dinv, r, w, z);
    TPF_CHECK_LAUNCH();
    k_bilu_sweep_2d<T, false><<<1, threads, 0, s>>>(ph.nx, ph.ny, jv, dinv, r, w, z);
    TPF_CHECK_LAUNCH();
    return;
  }
  if (M->front_max <= kFrontWg) {
    k_bilu_sweep_wg<T, true><<<1, 1024, 0, s>>>(nf, M->front_ptr_dev.p, M->front_cells.p, J->rp.p,
                                               J->ci.p, jv, dinv, r, w, z);
    TPF_CHECK_LAUNCH();
    k_bilu_sweep_wg<T, false><<<1, 1024, 0, s>>>(nf, M->front_ptr_dev.p, M->front_cells.p,
                                                J->rp.p, J->ci.p, jv, dinv, r, w, z);
    TPF_CHECK_LAUNCH();
    return;
  }
  for (int f = 0; f < nf; ++f) {
    int a = M->front_ptr[f], cnt = M->front_ptr[f + 1] - a;
    k_bilu_fwd<T><<<grid_for(cnt, 256), 256, 0, s>>>(cnt, M->front_cells.p + a, J->rp.p, J->ci.p,
                                                     jv, dinv, r, w);
  }
  TPF_CHECK_LAUNCH();
  for (int f = nf - 1; f >= 0; --f) {
    int a = M->front_ptr[f], cnt = M->front_ptr[f + 1] - a;
    k_bilu_bwd<T><<<grid_for(cnt, 256), 256, 0, s>>>(cnt, M->front_cells.p + a, J->rp.p, J->ci.p,
                                                     jv, dinv, w, z);
  }
  TPF_CHECK_LAUNCH();
}

template <class T>
T* wsel(Buf<double>& d, Buf<float>& f) {
  if constexpr (std::is_same<T, float>::value)
    return f.p;
  else
    return d.p;
}

template <class T>
void apply_t(tpf_precond* M, const double* r, double* z, hipStream_t s) {
  int N = M->N;
  unsigned g = grid_for(N, 256);
  T* v1 = wsel<T>(M->w1, M->f1);
  T* v2 = wsel<T>(M->w2, M->f2);
  T* v3 = wsel<T>(M->w3, M->f3);
  T* v4 = wsel<T>(M->w4, M->f4);
  switch (M->o.kind) {
    case TPF_PREC_AMG: {
      if constexpr (std::is_same<T, float>::value) {
        cast<double, float>(M->fr.p, r, 2 * int64_t(N), s);
        M->H[0]->vcycle<float>(M->fr.p, M->fu.p, s);
        cast<float, double>(z, M->fu.p, 2 * int64_t(N), s);
      } else {
        // fixed buffers, so the recorded V-cycle graph is reused
        copy(M->r2.p, r, 2 * int64_t(N), s);
        M->H[0]->vcycle<double>(M->r2.p, M->u2.p, s);
        copy(z, M->u2.p, 2 * int64_t(N), s);
      }
      break;
    }
    case TPF_PREC_CPR1:
    case TPF_PREC_CPR2: {
      T* uw = wsel<T>(M->r2, M->fr);  // forward sweep result
      T* uz = wsel<T>(M->u2, M->fu);
      bilu_apply<T>(M, r, uw, uz, s);
      // u (FP64) lives in z
      if constexpr (std::is_same<T, float>::value) {
        k_to_double<float><<<grid_for(2 * int64_t(N), 256), 256, 0, s>>>(2 * int64_t(N), uz, z);
      } else {
        copy(z, uz, 2 * int64_t(N), s);
      }
      TPF_CHECK_LAUNCH();
      // R_p (r - J u) (and R_s (r - J u) for CPR2), straight from J's blocks
      bcsr_residual_split<T>(M->J, z, r, v1, M->o.kind == TPF_PREC_CPR2 ? v3 : nullptr, s);
      M->H[0]->vcycle<T>(v1, v2, s);
      if (M->o.kind == TPF_PREC_CPR2) {
        M->H[1]->vcycle<T>(v3, v4, s);
        k_add_comp<T><<<g, 256, 0, s>>>(N, z, 1, v4);
        TPF_CHECK_LAUNCH();
      }
      k_add_comp<T><<<g, 256, 0, s>>>(N, z, 0, v2);
      TPF_CHECK_LAUNCH();
      break;
    }
    case TPF_PREC_BF: {
      // each cycle's first Jacobi guess is formed with its right-hand side
      // when the cycle starts from one
      T* g0 = M->H[0]->guess_buffer<T>();
      T* g1 = M->H[1]->guess_buffer<T>();
      if (g0)
        k_gather_guess<T><<<g, 256, 0, s>>>(N, r, 1, M->H[0]->level0_dinv<T>(), v1, g0);
      else
        k_gather<T><<<g, 256, 0, s>>>(N, r, 1, v1);
      TPF_CHECK_LAUNCH();
      M->H[0]->vcycle<T>(v1, v2, s, g0 != nullptr);  // s = V(A_ss; R_s r)
      int lpr = lanes_per_row(N, M->J->nnzb);
      {
        TimedScope ts("bf_rhs", s);
        const T* d1 = g1 ? M->H[1]->level0_dinv<T>() : nullptr;
        DISPATCH_LPR(lpr, L, {
          k_bf_rhs<T, L><<<grid_for(int64_t(N) * L, 256), 256, 0, s>>>(
              N, M->brp.p, M->bci.p, M->aps_v.p, r, v2, v3, d1, g1);
        });
        TPF_CHECK_LAUNCH();
      }
      M->H[1]->vcycle<T>(v3, v4, s, g1 != nullptr);  // p = V(S~; t)
      k_scatter2<T><<<g, 256, 0, s>>>(N, v4, v2, z);
      TPF_CHECK_LAUNCH();
      break;
    }
    default:
      copy(z, r, 2 * int64_t(N), s);
  }
}

}  // namespace

}  // namespace tpf

using namespace tpf;

size_t tpf_precond::bytes() const {
  size_t b = brp.bytes() + bci.bytes() + app_v.bytes() + aps_v.bytes() + asp_v.bytes() +
             ass_v.bytes() + y_v.bytes() + ass_dinv.bytes() + schur.bytes() + bilu_dinv.bytes() +
             bilu_dinv32.bytes() + jv32.bytes() + front_cells.bytes() + w1.bytes() + w2.bytes() +
             w3.bytes() + w4.bytes() + u2.bytes() + r2.bytes() + f1.bytes() + f2.bytes() +
             f3.bytes() + f4.bytes() + fu.bytes() + fr.bytes();
  for (int h = 0; h < 2; ++h)
    if (H[h]) b += H[h]->bytes();
  return b;
}

tpf_precond::~tpf_precond() {
  H[0].reset();  // hierarchy buffers are released before their stream goes
  H[1].reset();
  if (aux_ev) (void)hipEventDestroy(aux_ev);
  if (aux) {
    (void)hipStreamSynchronize(aux);
    tpf::forget_stream(aux);
    (void)hipStreamDestroy(aux);
  }
}

namespace {
// Runs a(aux) on a second host thread, with its own stream that first waits
// for everything queued on s, and b(s) on this thread; returns when both are
// done (a's stream drained) and rethrows the first failure.
template <class A, class B>
void run_pair(tpf_precond* M, hipStream_t s, A&& a, B&& b) {
  if (!M->aux) {
    TPF_HIP(hipStreamCreateWithFlags(&M->aux, hipStreamNonBlocking));
    TPF_HIP(hipEventCreateWithFlags(&M->aux_ev, hipEventDisableTiming));
  }
  TPF_HIP(hipEventRecord(M->aux_ev, s));
  TPF_HIP(hipStreamWaitEvent(M->aux, M->aux_ev, 0));
  int dev = 0;
  TPF_HIP(hipGetDevice(&dev));
  hipStream_t aux = M->aux;
  std::exception_ptr err_a, err_b;
  std::thread worker([&] {
    try {
      TPF_HIP(hipSetDevice(dev));
      a(aux);
      TPF_HIP(hipStreamSynchronize(aux));
    } catch (...) {
      err_a = std::current_exception();
      (void)hipStreamSynchronize(aux);
    }
  });
  try {
    b(s);
  } catch (...) {
    err_b = std::current_exception();
  }
  worker.join();
  if (err_b) std::rethrow_exception(err_b);
  if (err_a) std::rethrow_exception(err_a);
}
}  // namespace

extern "C" {

int tpf_precond_default_opts(int kind, tpf_precond_opts* o) {
  return guarded([&] {
    TPF_REQUIRE(o, TPF_ERR_INVALID_ARG, "null argument");
    o->kind = kind;
    o->precision = TPF_FP64;
    o->theta = 0.25;
    o->max_levels = 25;
    o->coarse_max = 128;
    o->dense_max = 1024;
    o->interp = TPF_INTERP_AUTO;
    o->hash_seed = 0x5eed;
    o->exti_route = 0;
    o->smoother = TPF_SMOOTH_L1_JACOBI;
    o->nu1 = 1;
    o->nu2 = 1;
    o->cheb_degree = 2;
    o->coarsening = TPF_COARSEN_PMIS;
    o->trunc_pmax = 3;
    o->trunc_factor = 0.0;
  });
}

int tpf_precond_create(const tpf_precond_opts* o, tpf_precond** out) {
  return guarded([&] {
    TPF_REQUIRE(o && out, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(o->kind >= TPF_PREC_AMG && o->kind <= TPF_PREC_NONE, TPF_ERR_INVALID_ARG,
                "unknown preconditioner kind %d", o->kind);
    TPF_REQUIRE(o->precision == TPF_FP64 || o->precision == TPF_FP32, TPF_ERR_INVALID_ARG,
                "unknown precision");
    TPF_REQUIRE(o->max_levels >= 1 && o->max_levels <= TPF_MAX_LEVELS, TPF_ERR_INVALID_ARG,
                "max_levels must be in [1, %d]", TPF_MAX_LEVELS);
    TPF_REQUIRE(o->coarse_max >= 1 && o->dense_max >= 1 && o->dense_max <= 4096,
                TPF_ERR_INVALID_ARG, "coarse_max >= 1 and 1 <= dense_max <= 4096 required");
    TPF_REQUIRE(o->theta > 0 && o->theta < 1, TPF_ERR_INVALID_ARG, "theta must be in (0,1)");
    TPF_REQUIRE(o->interp >= TPF_INTERP_AUTO && o->interp <= TPF_INTERP_CLASSICAL, TPF_ERR_INVALID_ARG,
                "unknown interpolation");
    TPF_REQUIRE(o->exti_route >= 0 && o->exti_route <= 8, TPF_ERR_INVALID_ARG,
                "exti_route must be in [0, 8]");
    TPF_REQUIRE(o->smoother == TPF_SMOOTH_L1_JACOBI || o->smoother == TPF_SMOOTH_CHEBYSHEV ||
                    o->smoother == TPF_SMOOTH_MC_GS,
                TPF_ERR_INVALID_ARG, "unknown smoother %d", o->smoother);
    TPF_REQUIRE(o->nu1 >= 0 && o->nu1 <= 4 && o->nu2 >= 0 && o->nu2 <= 4 && o->nu1 + o->nu2 >= 1,
                TPF_ERR_INVALID_ARG, "nu1, nu2 must be in [0, 4] with nu1 + nu2 >= 1");
    TPF_REQUIRE(o->cheb_degree >= 1 && o->cheb_degree <= 8, TPF_ERR_INVALID_ARG,
                "cheb_degree must be in [1, 8]");
    TPF_REQUIRE(o->coarsening == TPF_COARSEN_PMIS || o->coarsening == TPF_COARSEN_CLJP,
                TPF_ERR_INVALID_ARG, "unknown coarsening %d", o->coarsening);
    TPF_REQUIRE(o->trunc_pmax >= 0 && o->trunc_pmax <= 64, TPF_ERR_INVALID_ARG,
                "trunc_pmax must be in [0, 64]");
    TPF_REQUIRE(o->trunc_factor >= 0.0 && o->trunc_factor < 1.0, TPF_ERR_INVALID_ARG,
                "trunc_factor must be in [0, 1)");
    auto* M = new tpf_precond();
    M->o = *o;
    *out = M;
  });
}

int tpf_precond_destroy(tpf_precond* M) {
  return guarded([&] { delete M; });
}



int tpf_precond_setup(tpf_precond* M, const tpf_jacobian* J, int reuse, void* stream) {
  return guarded([&] {
    TPF_REQUIRE(M && J, TPF_ERR_INVALID_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool re = reuse && M->ready && M->J && M->N == J->nb && M->J->nnzb == J->nnzb;
    TPF_REQUIRE(!reuse || re, TPF_ERR_STATE,
                "reuse_structure requires a previous setup on a Jacobian with the same pattern");
    M->ready = false;
    M->J = J;
    M->s = s;
    int N = J->nb;
    M->N = N;
    int kind = M->o.kind;
    if (kind == TPF_PREC_NONE) {
      M->n_hier = 0;
      M->ready = true;
      return;
    }
    int64_t nnzb = J->nnzb;
    AmgOpts ao_p = amg_opts(M->o, true);
    AmgOpts ao_s = amg_opts(M->o, false);
    if (!re) {
      M->brp.alloc(N + 1, s);
      M->bci.alloc(nnzb, s);
      copy(M->brp.p, J->rp.p, N + 1, s);
      copy(M->bci.p, J->ci.p, nnzb, s);
      for (auto* b : {&M->app_v, &M->aps_v, &M->asp_v, &M->ass_v}) b->alloc(nnzb, s);
      for (auto* b : {&M->w1, &M->w2, &M->w3, &M->w4}) b->alloc(N, s);
      M->u2.alloc(2 * int64_t(N), s);
      M->r2.alloc(2 * int64_t(N), s);
      if (M->o.precision == TPF_FP32) {
        for (auto* b : {&M->f1, &M->f2, &M->f3, &M->f4}) b->alloc(N, s);
        M->fu.alloc(2 * int64_t(N), s);
        M->fr.alloc(2 * int64_t(N), s);
      }
    }
    {
      TimedScope ts("setup_blocks", s);
      k_extract_blocks<<<grid_for(nnzb, 256), 256, 0, s>>>(nnzb, J->v.p, M->app_v.p, M->aps_v.p,
                                                           M->asp_v.p, M->ass_v.p);
      TPF_CHECK_LAUNCH();
    }
    if (kind == TPF_PREC_AMG) {
      M->n_hier = 1;
      if (!re) {
        Csr<double> Js;
        Js.nrows = Js.ncols = 2 * N;
        Js.nnz = 4 * nnzb;
        Js.rp.alloc(2 * int64_t(N) + 1, s);
        Js.ci.alloc(Js.nnz, s);
        Js.v.alloc(Js.nnz, s);
        k_scalarize_pattern<<<grid_for(N + 1, 256), 256, 0, s>>>(N, J->rp.p, J->ci.p, Js.rp.p,
                                                                 Js.ci.p);
        TPF_CHECK_LAUNCH();
        k_scalarize_values<<<grid_for(N, 256), 256, 0, s>>>(N, J->rp.p, J->v.p, Js.v.p);
        TPF_CHECK_LAUNCH();
        M->H[0] = std::make_unique<Hierarchy>();
        M->H[0]->tag = "J";
        M->H[0]->build(std::move(Js), ao_s, s);
      } else {
        k_scalarize_values<<<grid_for(N, 256), 256, 0, s>>>(N, J->rp.p, J->v.p,
                                                            M->H[0]->A0().v.p);
        TPF_CHECK_LAUNCH();
        M->H[0]->refresh(s);
      }
    } else if (kind == TPF_PREC_CPR1 || kind == TPF_PREC_CPR2) {
      M->n_hier = kind == TPF_PREC_CPR2 ? 2 : 1;
      const double* src[2] = {M->app_v.p, M->ass_v.p};
      auto hier = [&](int h, hipStream_t hs) {
        if (!re) {
          auto H = std::make_unique<Hierarchy>();
          H->tag = h == 0 ? "App" : "Ass";
          H->stencil = stencil_offsets(J->prob->ph, 1);
          H->build(block_copy(M, src[h], hs), h == 0 ? ao_p : ao_s, hs);
          M->H[h] = std::move(H);
        } else {
          copy(M->H[h]->A0().v.p, src[h], nnzb, hs);
          M->H[h]->refresh(hs);
        }
      };
      // the A_pp hierarchy on a second stream; block ILU(0) and A_ss here
      run_pair(
          M, s, [&](hipStream_t as) { hier(0, as); },
          [&](hipStream_t ms) {
            bilu_setup(M, re, ms);
            if (M->n_hier == 2) hier(1, ms);
          });
    } else {  // BF
      M->n_hier = 2;
      M->ass_dinv.ensure(N, s);
      k_diag_inv<<<grid_for(N, 256), 256, 0, s>>>(N, M->brp.p, M->bci.p, M->ass_v.p,
                                                  M->ass_dinv.p);
      TPF_CHECK_LAUNCH();
      const Phys& ph = J->prob->ph;
      const bool on_grid = schur_on_grid_ok(ph, nnzb);
      if (!on_grid) {  // Y = A_ps diag(A_ss)^{-1} for the general sparse product
        M->y_v.ensure(nnzb, s);
        k_scale_cols<<<grid_for(N, 256), 256, 0, s>>>(N, M->brp.p, M->bci.p, M->aps_v.p,
                                                      M->ass_dinv.p, M->y_v.p);
        TPF_CHECK_LAUNCH();
      }
      CsrRef<double> Y{N, N, nnzb, M->brp.p, M->bci.p, M->y_v.p};
      CsrRef<double> Asp{N, N, nnzb, M->brp.p, M->bci.p, M->asp_v.p};
      CsrRef<double> App{N, N, nnzb, M->brp.p, M->bci.p, M->app_v.p};
      // the A_ss hierarchy on a second stream, S~ and its hierarchy here
      run_pair(
          M, s,
          [&](hipStream_t as) {
            if (!re) {
              auto H = std::make_unique<Hierarchy>();
              H->tag = "Ass";
              H->stencil = stencil_offsets(J->prob->ph, 1);
              H->build(block_copy(M, M->ass_v.p, as), ao_s, as);
              M->H[0] = std::move(H);
            } else {
              copy(M->H[0]->A0().v.p, M->ass_v.p, nnzb, as);
              M->H[0]->refresh(as);
            }
          },
          [&](hipStream_t ms) {
            if (!re) {
              Csr<double> S;
              {
                TimedScope ts("setup_schur", ms);
                if (on_grid)
                  schur_on_grid(M, ph, S, false, ms);
                else
                  spgemm(Y, Asp, S, ms, &App, -1.0, 1.0, false);
              }
              auto H = std::make_unique<Hierarchy>();
              H->tag = "Schur";
              H->stencil = stencil_offsets(J->prob->ph, 2);
              H->build(std::move(S), ao_p, ms);
              M->H[1] = std::move(H);
            } else {
              if (on_grid)
                schur_on_grid(M, ph, M->H[1]->A0(), true, ms);
              else
                spgemm(Y, Asp, M->H[1]->A0(), ms, &App, -1.0, 1.0);  // same pattern, in full
              M->H[1]->refresh(ms);
            }
          });
    }
    note_host_sync();
    TPF_HIP(hipStreamSynchronize(s));
    M->ready = true;
  });
}

int tpf_precond_apply(tpf_precond* M, const double* r, double* z, void* stream) {
  return guarded([&] {
    TPF_REQUIRE(M && r && z, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(M->ready, TPF_ERR_STATE, "preconditioner not set up");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (M->o.precision == TPF_FP32 && M->o.kind != TPF_PREC_NONE)
      apply_t<float>(M, r, z, s);
    else
      apply_t<double>(M, r, z, s);
  });
}

int tpf_precond_stats(const tpf_precond* M, tpf_hier_stats* out) {
  return guarded([&] {
    TPF_REQUIRE(M && out, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(M->ready, TPF_ERR_STATE, "preconditioner not set up");
    std::memset(out, 0, sizeof(*out));
    out->n_hier = M->n_hier;
    for (int h = 0; h < M->n_hier; ++h) {
      const Hierarchy& H = *M->H[h];
      out->levels[h] = H.levels();
      double nnz0 = 0, rows0 = 0, snnz = 0, srows = 0;
      for (int l = 0; l < H.levels(); ++l) {
        out->rows[h][l] = H.lv[l]->A.nrows;
        out->nnz[h][l] = H.lv[l]->A.nnz;
        out->p_nnz[h][l] = l + 1 < H.levels() ? H.lv[l]->P.nnz : 0;
        if (l == 0) {
          nnz0 = double(H.lv[l]->A.nnz);
          rows0 = double(H.lv[l]->A.nrows);
        }
        snnz += double(H.lv[l]->A.nnz);
        srows += double(H.lv[l]->A.nrows);
      }
      out->operator_complexity[h] = snnz / nnz0;
      out->grid_complexity[h] = srows / rows0;
      out->coarse_dense[h] = H.coarse_dense;
      out->l0_diagonals[h] = H.dia0.ok ? H.dia0.K : 0;
      out->coarse_smooth_sweeps[h] = H.coarse_dense ? 0 : 2;
    }
    out->device_bytes = M->bytes();
    for (int h = 0; h < M->n_hier; ++h) out->hier_bytes[h] = M->H[h]->bytes();
  });
}

int tpf_precond_matrix(const tpf_precond* M, int hier, int level, int which, tpf_csr_view* out) {
  return guarded([&] {
    TPF_REQUIRE(M && out, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(M->ready, TPF_ERR_STATE, "preconditioner not set up");
    std::memset(out, 0, sizeof(*out));
    if (which == TPF_MAT_APS) {
      TPF_REQUIRE(M->n_hier > 0, TPF_ERR_INVALID_ARG, "no block views for this kind");
      out->n_rows = out->n_cols = M->N;
      out->nnz = M->J->nnzb;
      out->row_ptr = M->brp.p;
      out->col_idx = M->bci.p;
      out->vals = M->aps_v.p;
      return;
    }
    if (which == TPF_MAT_SCHUR) {
      TPF_REQUIRE(M->o.kind == TPF_PREC_BF, TPF_ERR_INVALID_ARG, "S~ exists only for BF");
      hier = 1;
      level = 0;
      which = TPF_MAT_A;
    }
    TPF_REQUIRE(hier >= 0 && hier < M->n_hier, TPF_ERR_INVALID_ARG, "hierarchy index out of range");
    const Hierarchy& H = *M->H[hier];
    TPF_REQUIRE(level >= 0 && level < H.levels(), TPF_ERR_INVALID_ARG, "level out of range");
    const Level& L = *H.lv[level];
    if (which == TPF_MAT_GS_COLORS) {
      TPF_REQUIRE(L.gs_rows.p != nullptr, TPF_ERR_INVALID_ARG,
                  "no Gauss-Seidel colouring on this level");
      out->n_rows = int(L.gs_ptr.size()) - 1;
      out->n_cols = L.A.nrows;
      out->nnz = L.A.nrows;
      out->row_ptr = L.gs_ptr_dev.p;
      out->col_idx = L.gs_rows.p;
      out->vals = nullptr;
      return;
    }
    const Csr<double>* C = nullptr;
    switch (which) {
      case TPF_MAT_A: C = &L.A; break;
      case TPF_MAT_P: C = &L.P; break;
      case TPF_MAT_R: C = &L.R; break;
      case TPF_MAT_S: C = &L.S; break;
      default: fail(TPF_ERR_INVALID_ARG, "unknown matrix selector %d", which);
    }
    TPF_REQUIRE(C->rp.p != nullptr, TPF_ERR_INVALID_ARG, "matrix not present on this level");
    out->n_rows = C->nrows;
    out->n_cols = C->ncols;
    out->nnz = C->nnz;
    out->row_ptr = C->rp.p;
    out->col_idx = C->ci.p;
    out->vals = which == TPF_MAT_S ? nullptr : C->v.p;
  });
}

int tpf_precond_level_data(const tpf_precond* M, int hier, int level, const int8_t** cf,
                           const double** dinv, int* n) {
  return guarded([&] {
    TPF_REQUIRE(M, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(M->ready, TPF_ERR_STATE, "preconditioner not set up");
    TPF_REQUIRE(hier >= 0 && hier < M->n_hier, TPF_ERR_INVALID_ARG, "hierarchy index out of range");
    const Hierarchy& H = *M->H[hier];
    TPF_REQUIRE(level >= 0 && level < H.levels(), TPF_ERR_INVALID_ARG, "level out of range");
    const Level& L = *H.lv[level];
    if (cf) *cf = L.cf.p;
    if (dinv) *dinv = L.dinv.p;
    if (n) *n = L.A.nrows;
  });
}

int tpf_precond_bilu_dinv(const tpf_precond* M, const double** dinv) {
  return guarded([&] {
    TPF_REQUIRE(M && dinv, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(M->ready && M->bilu_dinv.p, TPF_ERR_STATE, "no block ILU(0) factors");
    *dinv = M->bilu_dinv.p;
  });
}

int tpf_precond_vcycle(tpf_precond* M, int hier, const double* b, double* x, void* stream) {
  return guarded([&] {
    TPF_REQUIRE(M && b && x, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(M->ready, TPF_ERR_STATE, "preconditioner not set up");
    TPF_REQUIRE(hier >= 0 && hier < M->n_hier, TPF_ERR_INVALID_ARG, "hierarchy index out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Hierarchy& H = *M->H[hier];
    if (M->o.precision == TPF_FP32) {
      int n = H.lv[0]->A.nrows;
      Buf<float> fb(n, s), fx(n, s);
      cast<double, float>(fb.p, b, n, s);
      H.vcycle<float>(fb.p, fx.p, s);
      cast<float, double>(x, fx.p, n, s);
      TPF_HIP(hipStreamSynchronize(s));
    } else {
      H.vcycle<double>(b, x, s);
    }
  });
}

}  // extern "C"
