// Problem and Jacobian handles.
#pragma once

#include "tpf_internal.hpp"

namespace tpf {

// Grid, fluid and rock constants of one problem, passed to kernels by value.
struct Phys {
  int nx, ny, nz;
  int64_t N;
  double hx, hy, hz, V;
  double mu_w, mu_n, rho_w, rho_n, grav;
  int pc_model;
  double lam, swr, snr, pd, s_eps;
  double span;              // 1 - swr - snr
  double ew, en;            // Burdine exponents (2+3l)/l and (2+l)/l
  double pc_eps, dpc_eps;   // Brooks-Corey value and slope at s_eps
};

}  // namespace tpf

struct tpf_problem {
  tpf::Phys ph{};
  hipStream_t s = nullptr;
  tpf::Buf<double> kx, ky, kz, poro, q;
  tpf::Buf<double> Tx, Ty, Tz;  // transmissibility of the face (i, i + stride_d); 0 if none
  int n_prod = 0;
  tpf::Buf<int> prod_cell;
  tpf::Buf<double> prod_wi, prod_pbh;
  int n_dir_cells = 0;
  tpf::Buf<int> dir_cell, dir_ptr, dir_face;
  tpf::Buf<double> dir_p, dir_s;
};

struct tpf_jacobian {
  tpf_problem* prob = nullptr;
  int nb = 0;          // block rows (cells)
  int64_t nnzb = 0;
  tpf::Buf<int> rp, ci;
  tpf::Buf<double> v;  // 4 * nnzb, row-major 2x2 blocks
  uint64_t version = 0;
};

namespace tpf {
// y = J x, or y = b - J x when b != nullptr
void bcsr_apply(const tpf_jacobian* J, const double* x, const double* b, double* y, hipStream_t s);
// r = b - J x by component: pressure rows to out_p, saturation rows to out_s (either may be null)
template <class T>
void bcsr_residual_split(const tpf_jacobian* J, const double* x, const double* b, T* out_p,
                         T* out_s, hipStream_t s);
}  // namespace tpf
