// Problem description, face transmissibilities, Jacobian pattern and the
// fully implicit TPFA residual/Jacobian assembly (paper Sec. 2 and Sec. 3,
// Eqs. balance1/balance2, the TPFA flux with upwinding and harmonic face
// permeability, Eq. fully_discrete_system, Eq. jacobian).
//
// Assembly is in gather form: one thread per cell evaluates the constitutive
// relations of the cell and of each face neighbour and writes its residual
// pair and its whole block row.  Every face quantity is computed from the
// face's (lower, higher) orientation, so the two cells of a face derive it
// from identical operations on identical inputs: fluxes are exactly
// antisymmetric and the A_pp / A_sp blocks exactly symmetric, with no atomics.
#include <algorithm>
#include <cmath>
#include <map>

#include "linalg_dev.hpp"
#include "problem.hpp"

namespace tpf {

// ------------------------------------------------------------ constitutive
// Effective saturation Sb = (1 - S_n - S_wr)/(1 - S_wr - S_nr), clamped to
// [0,1] (derivative 0 strictly outside); Brooks-Corey-Burdine relative
// permeabilities k_rw = Sb^((2+3l)/l), k_rn = (1-Sb)^2 (1 - Sb^((2+l)/l));
// capillary pressure Brooks-Corey P_d Sb^(-1/l) with a C1 linear extension
// below s_eps, or linear P_0 (1 - Sb).  Derivatives are w.r.t. S_n.
struct Sat {
  double lw, ln, dlw, dln, pc, dpc;
};

__device__ inline Sat sat_eval(double sn, const Phys& ph) {
  double s = (1.0 - sn - ph.swr) / ph.span;
  bool inside = (s >= 0.0) && (s <= 1.0);
  double sb = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  double dsb = inside ? -1.0 / ph.span : 0.0;
  double krw = pow(sb, ph.ew);
  double dkrw = ph.ew * pow(sb, ph.ew - 1.0);
  double pn = pow(sb, ph.en);
  double omsb = 1.0 - sb;
  double krn = omsb * omsb * (1.0 - pn);
  double dkrn = -2.0 * omsb * (1.0 - pn) - omsb * omsb * ph.en * pow(sb, ph.en - 1.0);
  double pc, dpc;
  if (ph.pc_model == TPF_PC_LINEAR) {
    pc = ph.pd * (1.0 - sb);
    dpc = -ph.pd;
  } else if (sb >= ph.s_eps) {
    pc = ph.pd * pow(sb, -1.0 / ph.lam);
    dpc = -(ph.pd / ph.lam) * pow(sb, -1.0 / ph.lam - 1.0);
  } else {
    pc = ph.pc_eps + ph.dpc_eps * (sb - ph.s_eps);
    dpc = ph.dpc_eps;
  }
  Sat r;
  r.lw = krw / ph.mu_w;
  r.ln = krn / ph.mu_n;
  r.dlw = dkrw * dsb / ph.mu_w;
  r.dln = dkrn * dsb / ph.mu_n;
  r.pc = pc;
  r.dpc = dpc * dsb;
  return r;
}

__device__ inline double cell_depth(int iz, const Phys& ph) { return (iz + 0.5) * ph.hz; }

// ------------------------------------------------------------ transmissibility
// T = gamma_d * K_face / h_d, gamma_d = V / h_d (face area), harmonic
// K_face = (dx_l + dx_h) K_l K_h / (dx_l K_h + dx_h K_l) with equal cells.
__global__ void k_face_trans(Phys ph, const double* __restrict__ kx, const double* __restrict__ ky,
                             const double* __restrict__ kz, double* __restrict__ Tx,
                             double* __restrict__ Ty, double* __restrict__ Tz) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  int ix = int(i % ph.nx);
  int iy = int((i / ph.nx) % ph.ny);
  int iz = int(i / (int64_t(ph.nx) * ph.ny));
  const double* K[3] = {kx, ky, kz};
  double* T[3] = {Tx, Ty, Tz};
  int coord[3] = {ix, iy, iz};
  int nd[3] = {ph.nx, ph.ny, ph.nz};
  int64_t stride[3] = {1, ph.nx, int64_t(ph.nx) * ph.ny};
  double hd[3] = {ph.hx, ph.hy, ph.hz};
  for (int d = 0; d < 3; ++d) {
    double t = 0.0;
    if (coord[d] < nd[d] - 1) {
      double h = hd[d];
      double gamma = ph.V / h;
      double kl = K[d][i], kh = K[d][i + stride[d]];
      double kface = (h + h) * kl * kh / (h * kh + h * kl);
      t = gamma * kface / h;
    }
    T[d][i] = t;
  }
}

// ------------------------------------------------------------ pattern
__device__ inline int cell_neighbours(int64_t i, const Phys& ph, int64_t nb[7], int& self_pos) {
  int ix = int(i % ph.nx);
  int iy = int((i / ph.nx) % ph.ny);
  int iz = int(i / (int64_t(ph.nx) * ph.ny));
  int64_t sxy = int64_t(ph.nx) * ph.ny;
  int c = 0;
  if (iz > 0) nb[c++] = i - sxy;
  if (iy > 0) nb[c++] = i - ph.nx;
  if (ix > 0) nb[c++] = i - 1;
  self_pos = c;
  nb[c++] = i;
  if (ix < ph.nx - 1) nb[c++] = i + 1;
  if (iy < ph.ny - 1) nb[c++] = i + ph.nx;
  if (iz < ph.nz - 1) nb[c++] = i + sxy;
  return c;
}

__global__ void k_pattern_count(Phys ph, int* cnt) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  int64_t nb[7];
  int sp;
  cnt[i] = cell_neighbours(i, ph, nb, sp);
}

__global__ void k_pattern_fill(Phys ph, const int* rp, int* ci) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  int64_t nb[7];
  int sp;
  int c = cell_neighbours(i, ph, nb, sp);
  int base = rp[i];
  for (int k = 0; k < c; ++k) ci[base + k] = int(nb[k]);
}

// ------------------------------------------------------------ assembly
// Face between cells l < h with transmissibility T: water and nonwetting
// fluxes out of l and their derivatives (upwind frozen).
struct FaceTerms {
  double Fw, Fn;          // fluxes out of l
  double aw, an;          // dF/dP_l = -dF/dP_h
  double dFw_dSl, dFw_dSh, dFn_dSl, dFn_dSh;
};

__device__ inline FaceTerms face_terms(double T, double Pl, double Ph, const Sat& sl, const Sat& sh,
                                       double zl, double zh, const Phys& ph) {
  double g = ph.grav;
  double phwl = Pl - ph.rho_w * g * zl, phwh = Ph - ph.rho_w * g * zh;
  double phnl = Pl + sl.pc - ph.rho_n * g * zl, phnh = Ph + sh.pc - ph.rho_n * g * zh;
  double dw = phwl - phwh;
  double dn = phnl - phnh;
  bool wl = dw > 0.0;
  bool nl = dn > 0.0;
  FaceTerms f;
  f.aw = T * (wl ? sl.lw : sh.lw);
  f.an = T * (nl ? sl.ln : sh.ln);
  f.Fw = f.aw * dw;
  f.Fn = f.an * dn;
  double bw = T * (wl ? sl.dlw : sh.dlw) * dw;
  f.dFw_dSl = wl ? bw : 0.0;
  f.dFw_dSh = wl ? 0.0 : bw;
  f.dFn_dSl = (nl ? T * sl.dln * dn : 0.0) + f.an * sl.dpc;
  f.dFn_dSh = (nl ? 0.0 : T * sh.dln * dn) - f.an * sh.dpc;
  return f;
}

__global__ void __launch_bounds__(256) k_assemble(Phys ph, double dt, const double* __restrict__ u,
                                                  const double* __restrict__ uold,
                                                  const double* __restrict__ poro,
                                                  const double* __restrict__ q,
                                                  const double* __restrict__ Tx,
                                                  const double* __restrict__ Ty,
                                                  const double* __restrict__ Tz,
                                                  const int* __restrict__ rp,
                                                  double* __restrict__ R, double* __restrict__ Jv) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ph.N) return;
  int ix = int(i % ph.nx);
  int iy = int((i / ph.nx) % ph.ny);
  int iz = int(i / (int64_t(ph.nx) * ph.ny));
  int64_t sxy = int64_t(ph.nx) * ph.ny;
  double Pi = u[2 * i], Si = u[2 * i + 1];
  Sat si = sat_eval(Si, ph);
  double zi = cell_depth(iz, ph);
  double stc = poro[i] * ph.V / dt;
  double st = stc * (Si - uold[2 * i + 1]);
  double Rw = -st, Rn = st;
  double d00 = 0.0, d01 = -stc, d10 = 0.0, d11 = stc;
  double* out = Jv + 4 * int64_t(rp[i]);
  int slot = 0;
  // neighbours in ascending column order: -z, -y, -x, (self), +x, +y, +z
  const int64_t offs[6] = {-sxy, -int64_t(ph.nx), -1, 1, int64_t(ph.nx), sxy};
  const bool has[6] = {iz > 0, iy > 0, ix > 0, ix < ph.nx - 1, iy < ph.ny - 1, iz < ph.nz - 1};
  const int dz[6] = {-1, 0, 0, 0, 0, 1};
  for (int k = 0; k < 6; ++k) {
    if (k == 3) slot++;  // diagonal block position
    if (!has[k]) continue;
    int64_t j = i + offs[k];
    double Pj = u[2 * j], Sj = u[2 * j + 1];
    Sat sj = sat_eval(Sj, ph);
    double zj = cell_depth(iz + dz[k], ph);
    double T;
    bool i_low = k >= 3;  // neighbour above in index: i is the face's lower cell
    if (k == 0) T = Tz[j];
    else if (k == 1) T = Ty[j];
    else if (k == 2) T = Tx[j];
    else if (k == 3) T = Tx[i];
    else if (k == 4) T = Ty[i];
    else T = Tz[i];
    double b00, b01, b10, b11;
    if (i_low) {
      FaceTerms f = face_terms(T, Pi, Pj, si, sj, zi, zj, ph);
      Rw += f.Fw;
      Rn += f.Fn;
      d00 += f.aw;
      d10 += f.an;
      d01 += f.dFw_dSl;
      d11 += f.dFn_dSl;
      b00 = -f.aw;
      b01 = f.dFw_dSh;
      b10 = -f.an;
      b11 = f.dFn_dSh;
    } else {
      FaceTerms f = face_terms(T, Pj, Pi, sj, si, zj, zi, ph);
      Rw -= f.Fw;
      Rn -= f.Fn;
      d00 += f.aw;
      d10 += f.an;
      d01 -= f.dFw_dSh;
      d11 -= f.dFn_dSh;
      b00 = -f.aw;
      b01 = -f.dFw_dSl;
      b10 = -f.an;
      b11 = -f.dFn_dSl;
    }
    double* blk = out + 4 * slot;
    blk[0] = b00;
    blk[1] = b01;
    blk[2] = b10;
    blk[3] = b11;
    slot++;
  }
  // the diagonal block sits after the existing lower neighbours
  int nlow = (iz > 0) + (iy > 0) + (ix > 0);
  double* dblk = out + 4 * nlow;
  dblk[0] = d00;
  dblk[1] = d01;
  dblk[2] = d10;
  dblk[3] = d11;
  if (q) {
    Rw -= q[2 * i];
    Rn -= q[2 * i + 1];
  }
  if (R) {
    R[2 * i] = Rw;
    R[2 * i + 1] = Rn;
  }
}

// BHP producers (at most one per cell): q_a = -WI lambda_a(S)(P_w - p_bh).
__global__ void k_assemble_producers(Phys ph, int n, const int* __restrict__ cell,
                                     const double* __restrict__ wi,
                                     const double* __restrict__ pbh, const double* __restrict__ u,
                                     const int* __restrict__ rp, double* __restrict__ R,
                                     double* __restrict__ Jv) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int64_t i = cell[k];
  int ix = int(i % ph.nx);
  int iy = int((i / ph.nx) % ph.ny);
  int iz = int(i / (int64_t(ph.nx) * ph.ny));
  Sat s = sat_eval(u[2 * i + 1], ph);
  double dp = u[2 * i] - pbh[k];
  double w = wi[k];
  if (R) {
    R[2 * i] += w * s.lw * dp;
    R[2 * i + 1] += w * s.ln * dp;
  }
  int nlow = (iz > 0) + (iy > 0) + (ix > 0);
  double* d = Jv + 4 * (int64_t(rp[i]) + nlow);
  d[0] += w * s.lw;
  d[2] += w * s.ln;
  d[1] += w * s.dlw * dp;
  d[3] += w * s.dln * dp;
}

// Dirichlet faces, grouped by cell: T_b = gamma K / (h/2), boundary state
// (P_b, S_b) at the face centre, upwind against the boundary state.
__global__ void k_assemble_dirichlet(Phys ph, int ncell, const int* __restrict__ dcell,
                                     const int* __restrict__ dptr, const int* __restrict__ dface,
                                     const double* __restrict__ dp_b,
                                     const double* __restrict__ ds_b,
                                     const double* __restrict__ kx, const double* __restrict__ ky,
                                     const double* __restrict__ kz, const double* __restrict__ u,
                                     const int* __restrict__ rp, double* __restrict__ R,
                                     double* __restrict__ Jv) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ncell) return;
  int64_t i = dcell[k];
  int ix = int(i % ph.nx);
  int iy = int((i / ph.nx) % ph.ny);
  int iz = int(i / (int64_t(ph.nx) * ph.ny));
  double Pi = u[2 * i];
  Sat si = sat_eval(u[2 * i + 1], ph);
  double zi = cell_depth(iz, ph);
  double g = ph.grav;
  double phw = Pi - ph.rho_w * g * zi;
  double phn = Pi + si.pc - ph.rho_n * g * zi;
  double rw = 0.0, rn = 0.0, a00 = 0.0, a01 = 0.0, a10 = 0.0, a11 = 0.0;
  for (int f = dptr[k]; f < dptr[k + 1]; ++f) {
    int fc = dface[f];
    int d = fc >> 1;
    double h = d == 0 ? ph.hx : (d == 1 ? ph.hy : ph.hz);
    double kk = d == 0 ? kx[i] : (d == 1 ? ky[i] : kz[i]);
    double gamma = ph.V / h;
    double Tb = gamma * kk / (0.5 * h);
    double zb = zi + (fc == 4 ? -0.5 * ph.hz : (fc == 5 ? 0.5 * ph.hz : 0.0));
    Sat sb = sat_eval(ds_b[f], ph);
    double dwb = phw - (dp_b[f] - ph.rho_w * g * zb);
    double dnb = phn - (dp_b[f] + sb.pc - ph.rho_n * g * zb);
    bool win = dwb > 0.0, nin = dnb > 0.0;
    double lwb = win ? si.lw : sb.lw;
    double lnb = nin ? si.ln : sb.ln;
    rw += Tb * lwb * dwb;
    rn += Tb * lnb * dnb;
    a00 += Tb * lwb;
    a10 += Tb * lnb;
    a01 += win ? Tb * si.dlw * dwb : 0.0;
    a11 += (nin ? Tb * si.dln * dnb : 0.0) + Tb * lnb * si.dpc;
  }
  if (R) {
    R[2 * i] += rw;
    R[2 * i + 1] += rn;
  }
  int nlow = (iz > 0) + (iy > 0) + (ix > 0);
  double* dd = Jv + 4 * (int64_t(rp[i]) + nlow);
  dd[0] += a00;
  dd[1] += a01;
  dd[2] += a10;
  dd[3] += a11;
}

__global__ void k_newton_update(int64_t N, double* u, const double* du, double alpha,
                                double ds_max) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  u[2 * i] += alpha * du[2 * i];
  double d = alpha * du[2 * i + 1];
  if (ds_max > 0.0) d = d < -ds_max ? -ds_max : (d > ds_max ? ds_max : d);
  double s = u[2 * i + 1] + d;
  u[2 * i + 1] = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
}

// ------------------------------------------------------------ BCSR SpMV
// y_i = sum_e B_e x_{col(e)} (or b_i minus it): eight lanes per block row,
// lane k taking blocks k, k + 8, ... so that a wavefront reads eight rows'
// blocks as one contiguous stretch; the lanes' partial sums are combined by
// an xor butterfly.
constexpr int kBcsrLanes = 8;
__global__ void __launch_bounds__(256) k_bcsr_spmv(int nb, const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ y) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / kBcsrLanes), lane = int(gid % kBcsrLanes);
  double y0 = 0.0, y1 = 0.0;
  if (i < nb) {
    for (int e = rp[i] + lane; e < rp[i + 1]; e += kBcsrLanes) {
      int j = ci[e];
      double2 xj = reinterpret_cast<const double2*>(x)[j];
      const double2* blk = reinterpret_cast<const double2*>(v + 4 * int64_t(e));
      double2 r0 = blk[0], r1 = blk[1];
      y0 += r0.x * xj.x + r0.y * xj.y;
      y1 += r1.x * xj.x + r1.y * xj.y;
    }
  }
  y0 = group_sum<kBcsrLanes>(y0);
  y1 = group_sum<kBcsrLanes>(y1);
  if (i < nb && lane == 0) {
    if (b) {
      y0 = b[2 * i] - y0;
      y1 = b[2 * i + 1] - y1;
    }
    reinterpret_cast<double2*>(y)[i] = make_double2(y0, y1);
  }
}

// r = b - J x split by component: the pressure rows into rp, the saturation
// rows into rs (either may be omitted, and then its half of every block is
// not read); outputs in T.
template <class T, bool P, bool S>
__global__ void __launch_bounds__(256) k_bcsr_residual_split(int nb, const int* __restrict__ rp,
                                                             const int* __restrict__ ci,
                                                             const double* __restrict__ v,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ b,
                                                             T* __restrict__ out_p,
                                                             T* __restrict__ out_s) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / kBcsrLanes), lane = int(gid % kBcsrLanes);
  double y0 = 0.0, y1 = 0.0;
  if (i < nb) {
    for (int e = rp[i] + lane; e < rp[i + 1]; e += kBcsrLanes) {
      int j = ci[e];
      double2 xj = reinterpret_cast<const double2*>(x)[j];
      const double2* blk = reinterpret_cast<const double2*>(v + 4 * int64_t(e));
      if (P) {
        double2 r0 = blk[0];
        y0 += r0.x * xj.x + r0.y * xj.y;
      }
      if (S) {
        double2 r1 = blk[1];
        y1 += r1.x * xj.x + r1.y * xj.y;
      }
    }
  }
  if (P) y0 = group_sum<kBcsrLanes>(y0);
  if (S) y1 = group_sum<kBcsrLanes>(y1);
  if (i < nb && lane == 0) {
    if (P) out_p[i] = T(b[2 * i] - y0);
    if (S) out_s[i] = T(b[2 * i + 1] - y1);
  }
}

template <class T>
void bcsr_residual_split(const tpf_jacobian* J, const double* x, const double* b, T* out_p,
                         T* out_s, hipStream_t s) {
  TimedScope ts("bcsr_spmv", s);
  unsigned g = grid_for(int64_t(J->nb) * kBcsrLanes, 256);
  if (out_p && out_s)
    k_bcsr_residual_split<T, true, true><<<g, 256, 0, s>>>(J->nb, J->rp.p, J->ci.p, J->v.p, x, b,
                                                           out_p, out_s);
  else if (out_p)
    k_bcsr_residual_split<T, true, false><<<g, 256, 0, s>>>(J->nb, J->rp.p, J->ci.p, J->v.p, x, b,
                                                            out_p, nullptr);
  else
    k_bcsr_residual_split<T, false, true><<<g, 256, 0, s>>>(J->nb, J->rp.p, J->ci.p, J->v.p, x, b,
                                                            nullptr, out_s);
  TPF_CHECK_LAUNCH();
}
template void bcsr_residual_split<double>(const tpf_jacobian*, const double*, const double*,
                                          double*, double*, hipStream_t);
template void bcsr_residual_split<float>(const tpf_jacobian*, const double*, const double*,
                                         float*, float*, hipStream_t);

void bcsr_apply(const tpf_jacobian* J, const double* x, const double* b, double* y,
                hipStream_t s) {
  TimedScope ts("bcsr_spmv", s);
  k_bcsr_spmv<<<grid_for(int64_t(J->nb) * kBcsrLanes, 256), 256, 0, s>>>(J->nb, J->rp.p, J->ci.p,
                                                                         J->v.p, x, b, y);
  TPF_CHECK_LAUNCH();
}

// ------------------------------------------------------------ host side
static Phys make_phys(const tpf_problem_desc* d) {
  Phys ph{};
  ph.nx = d->nx;
  ph.ny = d->ny;
  ph.nz = d->nz;
  ph.N = int64_t(d->nx) * d->ny * d->nz;
  ph.hx = d->hx;
  ph.hy = d->hy;
  ph.hz = d->hz;
  ph.V = d->hx * d->hy * d->hz;
  ph.mu_w = d->mu_w;
  ph.mu_n = d->mu_n;
  ph.rho_w = d->rho_w;
  ph.rho_n = d->rho_n;
  ph.grav = d->grav;
  ph.pc_model = d->pc_model;
  ph.lam = d->bc_lambda;
  ph.swr = d->swr;
  ph.snr = d->snr;
  ph.pd = d->pd;
  ph.s_eps = d->s_eps;
  ph.span = 1.0 - d->swr - d->snr;
  ph.ew = (2.0 + 3.0 * ph.lam) / ph.lam;
  ph.en = (2.0 + ph.lam) / ph.lam;
  ph.pc_eps = ph.pd * std::pow(ph.s_eps, -1.0 / ph.lam);
  ph.dpc_eps = -(ph.pd / ph.lam) * std::pow(ph.s_eps, -1.0 / ph.lam - 1.0);
  return ph;
}

}  // namespace tpf

using namespace tpf;

extern "C" {

int tpf_problem_create(const tpf_problem_desc* d, void* stream, tpf_problem** out) {
  return guarded([&] {
    TPF_REQUIRE(d && out, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(d->nx >= 1 && d->ny >= 1 && d->nz >= 1, TPF_ERR_INVALID_ARG, "grid sizes must be >= 1");
    int64_t N = int64_t(d->nx) * d->ny * d->nz;
    TPF_REQUIRE(N < (int64_t(1) << 30), TPF_ERR_INVALID_ARG, "too many cells");
    TPF_REQUIRE(d->hx > 0 && d->hy > 0 && d->hz > 0, TPF_ERR_INVALID_ARG, "cell sizes must be > 0");
    TPF_REQUIRE(d->kx && d->ky && d->kz && d->poro, TPF_ERR_INVALID_ARG, "permeability/porosity required");
    TPF_REQUIRE(d->mu_w > 0 && d->mu_n > 0, TPF_ERR_INVALID_ARG, "viscosities must be > 0");
    TPF_REQUIRE(d->pc_model == TPF_PC_BROOKS_COREY || d->pc_model == TPF_PC_LINEAR,
                TPF_ERR_INVALID_ARG, "unknown capillary model");
    TPF_REQUIRE(d->bc_lambda > 0, TPF_ERR_INVALID_ARG, "lambda must be > 0");
    TPF_REQUIRE(d->swr >= 0 && d->snr >= 0 && d->swr + d->snr < 1, TPF_ERR_INVALID_ARG,
                "residual saturations must satisfy swr + snr < 1");
    TPF_REQUIRE(d->pc_model != TPF_PC_BROOKS_COREY || d->s_eps > 0, TPF_ERR_INVALID_ARG,
                "s_eps must be > 0 for Brooks-Corey");
    TPF_REQUIRE(d->n_prod >= 0 && d->n_dir >= 0, TPF_ERR_INVALID_ARG, "negative well/face count");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto* p = new tpf_problem();
    try {
      p->s = s;
      p->ph = make_phys(d);
      p->kx.alloc(N, s);
      p->ky.alloc(N, s);
      p->kz.alloc(N, s);
      p->poro.alloc(N, s);
      copy(p->kx.p, d->kx, N, s);
      copy(p->ky.p, d->ky, N, s);
      copy(p->kz.p, d->kz, N, s);
      copy(p->poro.p, d->poro, N, s);
      if (d->q) {
        p->q.alloc(2 * N, s);
        copy(p->q.p, d->q, 2 * N, s);
      }
      p->Tx.alloc(N, s);
      p->Ty.alloc(N, s);
      p->Tz.alloc(N, s);
      k_face_trans<<<grid_for(N, 256), 256, 0, s>>>(p->ph, p->kx.p, p->ky.p, p->kz.p, p->Tx.p,
                                                     p->Ty.p, p->Tz.p);
      TPF_CHECK_LAUNCH();
      // producers: validate, one per cell
      if (d->n_prod > 0) {
        TPF_REQUIRE(d->prod_cells && d->prod_wi && d->prod_pbh, TPF_ERR_INVALID_ARG,
                    "producer arrays required");
        std::vector<int> cells(d->prod_cells, d->prod_cells + d->n_prod);
        std::vector<int> sorted = cells;
        std::sort(sorted.begin(), sorted.end());
        for (size_t k = 0; k < sorted.size(); ++k) {
          TPF_REQUIRE(sorted[k] >= 0 && sorted[k] < N, TPF_ERR_INVALID_ARG, "producer cell out of range");
          TPF_REQUIRE(k == 0 || sorted[k] != sorted[k - 1], TPF_ERR_INVALID_ARG,
                      "at most one producer per cell");
        }
        p->n_prod = d->n_prod;
        p->prod_cell.alloc(d->n_prod, s);
        p->prod_wi.alloc(d->n_prod, s);
        p->prod_pbh.alloc(d->n_prod, s);
        TPF_HIP(hipMemcpyAsync(p->prod_cell.p, d->prod_cells, d->n_prod * sizeof(int), hipMemcpyHostToDevice, s));
        TPF_HIP(hipMemcpyAsync(p->prod_wi.p, d->prod_wi, d->n_prod * sizeof(double), hipMemcpyHostToDevice, s));
        TPF_HIP(hipMemcpyAsync(p->prod_pbh.p, d->prod_pbh, d->n_prod * sizeof(double), hipMemcpyHostToDevice, s));
      }
      if (d->n_dir > 0) {
        TPF_REQUIRE(d->dir_cells && d->dir_face && d->dir_p && d->dir_s, TPF_ERR_INVALID_ARG,
                    "Dirichlet arrays required");
        std::vector<int> idx(d->n_dir);
        for (int k = 0; k < d->n_dir; ++k) {
          int c = d->dir_cells[k], f = d->dir_face[k];
          TPF_REQUIRE(c >= 0 && c < N && f >= 0 && f < 6, TPF_ERR_INVALID_ARG, "bad Dirichlet face");
          int ix = int(c % d->nx), iy = int((c / d->nx) % d->ny), iz = int(c / (int64_t(d->nx) * d->ny));
          bool onb = (f == 0 && ix == 0) || (f == 1 && ix == d->nx - 1) || (f == 2 && iy == 0) ||
                     (f == 3 && iy == d->ny - 1) || (f == 4 && iz == 0) || (f == 5 && iz == d->nz - 1);
          TPF_REQUIRE(onb, TPF_ERR_INVALID_ARG, "Dirichlet face %d of cell %d is not a domain face", f, c);
          idx[k] = k;
        }
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int a, int b) { return d->dir_cells[a] < d->dir_cells[b]; });
        std::vector<int> ucell, ptr, face;
        std::vector<double> pb, sb;
        for (int k : idx) {
          int c = d->dir_cells[k];
          if (ucell.empty() || ucell.back() != c) {
            ucell.push_back(c);
            ptr.push_back(int(face.size()));
          }
          face.push_back(d->dir_face[k]);
          pb.push_back(d->dir_p[k]);
          sb.push_back(d->dir_s[k]);
        }
        ptr.push_back(int(face.size()));
        p->n_dir_cells = int(ucell.size());
        p->dir_cell.alloc(ucell.size(), s);
        p->dir_ptr.alloc(ptr.size(), s);
        p->dir_face.alloc(face.size(), s);
        p->dir_p.alloc(pb.size(), s);
        p->dir_s.alloc(sb.size(), s);
        TPF_HIP(hipMemcpyAsync(p->dir_cell.p, ucell.data(), ucell.size() * sizeof(int), hipMemcpyHostToDevice, s));
        TPF_HIP(hipMemcpyAsync(p->dir_ptr.p, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice, s));
        TPF_HIP(hipMemcpyAsync(p->dir_face.p, face.data(), face.size() * sizeof(int), hipMemcpyHostToDevice, s));
        TPF_HIP(hipMemcpyAsync(p->dir_p.p, pb.data(), pb.size() * sizeof(double), hipMemcpyHostToDevice, s));
        TPF_HIP(hipMemcpyAsync(p->dir_s.p, sb.data(), sb.size() * sizeof(double), hipMemcpyHostToDevice, s));
      }
      TPF_HIP(hipStreamSynchronize(s));  // host vectors above go out of scope
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

int tpf_problem_destroy(tpf_problem* p) {
  return guarded([&] { delete p; });
}

int tpf_problem_cells(const tpf_problem* p, int64_t* n) {
  return guarded([&] {
    TPF_REQUIRE(p && n, TPF_ERR_INVALID_ARG, "null argument");
    *n = p->ph.N;
  });
}

int tpf_jacobian_create(tpf_problem* p, void* stream, tpf_jacobian** out) {
  return guarded([&] {
    TPF_REQUIRE(p && out, TPF_ERR_INVALID_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto* J = new tpf_jacobian();
    try {
      int64_t N = p->ph.N;
      J->nb = int(N);
      J->prob = p;
      J->rp.alloc(N + 1, s);
      Buf<int> cnt(N, s);
      k_pattern_count<<<grid_for(N, 256), 256, 0, s>>>(p->ph, cnt.p);
      TPF_CHECK_LAUNCH();
      J->nnzb = scan_exclusive(cnt.p, J->rp.p, N, s);
      J->ci.alloc(J->nnzb, s);
      J->v.alloc(4 * J->nnzb, s);
      k_pattern_fill<<<grid_for(N, 256), 256, 0, s>>>(p->ph, J->rp.p, J->ci.p);
      TPF_CHECK_LAUNCH();
      fill(J->v.p, 0.0, 4 * J->nnzb, s);
      TPF_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete J;
      throw;
    }
    *out = J;
  });
}

int tpf_jacobian_destroy(tpf_jacobian* J) {
  return guarded([&] { delete J; });
}

int tpf_assemble(tpf_problem* p, const double* u, const double* u_old, double dt, double* R,
                 tpf_jacobian* J, void* stream) {
  return guarded([&] {
    TPF_REQUIRE(p && u && u_old && J, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(J->prob == p, TPF_ERR_INVALID_ARG, "Jacobian belongs to another problem");
    TPF_REQUIRE(dt > 0, TPF_ERR_INVALID_ARG, "dt must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t N = p->ph.N;
    {
      TimedScope ts("assemble", s);
      k_assemble<<<grid_for(N, 256), 256, 0, s>>>(p->ph, dt, u, u_old, p->poro.p, p->q.p, p->Tx.p,
                                                   p->Ty.p, p->Tz.p, J->rp.p, R, J->v.p);
      TPF_CHECK_LAUNCH();
    }
    if (p->n_prod > 0) {
      k_assemble_producers<<<grid_for(p->n_prod, 64), 64, 0, s>>>(
          p->ph, p->n_prod, p->prod_cell.p, p->prod_wi.p, p->prod_pbh.p, u, J->rp.p, R, J->v.p);
      TPF_CHECK_LAUNCH();
    }
    if (p->n_dir_cells > 0) {
      k_assemble_dirichlet<<<grid_for(p->n_dir_cells, 64), 64, 0, s>>>(
          p->ph, p->n_dir_cells, p->dir_cell.p, p->dir_ptr.p, p->dir_face.p, p->dir_p.p,
          p->dir_s.p, p->kx.p, p->ky.p, p->kz.p, u, J->rp.p, R, J->v.p);
      TPF_CHECK_LAUNCH();
    }
    J->version++;
  });
}

int tpf_jacobian_view(const tpf_jacobian* J, tpf_bcsr_view* out) {
  return guarded([&] {
    TPF_REQUIRE(J && out, TPF_ERR_INVALID_ARG, "null argument");
    out->n_block_rows = J->nb;
    out->nnzb = J->nnzb;
    out->row_ptr = J->rp.p;
    out->col_idx = J->ci.p;
    out->vals = J->v.p;
  });
}

int tpf_spmv(const tpf_jacobian* J, const double* x, double* y, void* stream) {
  return guarded([&] {
    TPF_REQUIRE(J && x && y, TPF_ERR_INVALID_ARG, "null argument");
    bcsr_apply(J, x, nullptr, y, static_cast<hipStream_t>(stream));
  });
}

int tpf_newton_update(tpf_problem* p, double* u, const double* du, double alpha, double ds_max,
                      void* stream) {
  return guarded([&] {
    TPF_REQUIRE(p && u && du, TPF_ERR_INVALID_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_newton_update<<<grid_for(p->ph.N, 256), 256, 0, s>>>(p->ph.N, u, du, alpha, ds_max);
    TPF_CHECK_LAUNCH();
  });
}

int tpf_norm2(const double* x, int64_t n, double* out, void* stream) {
  return guarded([&] {
    TPF_REQUIRE(out && n >= 0 && (n == 0 || x), TPF_ERR_INVALID_ARG, "null argument");
    *out = n == 0 ? 0.0 : nrm2_host(x, n, static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
