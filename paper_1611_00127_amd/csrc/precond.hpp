// Preconditioner handle: block views of J, S~, block ILU(0) and the AMG
// hierarchies of the paper's four preconditioners.
#pragma once

#include "amg.hpp"
#include "problem.hpp"

struct tpf_precond {
  tpf_precond_opts o{};
  bool ready = false;
  const tpf_jacobian* J = nullptr;
  int N = 0;
  hipStream_t s = nullptr;
  // field blocks on J's block pattern (shared pattern buffers)
  tpf::Buf<int> brp, bci;
  tpf::Buf<double> app_v, aps_v, asp_v, ass_v, y_v, ass_dinv;
  tpf::Csr<double> schur;
  // AMG hierarchies: AMG {J_scalar}; CPR1 {A_pp}; CPR2 {A_pp, A_ss}; BF {A_ss, S~}
  std::unique_ptr<tpf::Hierarchy> H[2];
  int n_hier = 0;
  // block ILU(0) (CPR)
  tpf::Buf<double> bilu_dinv;     // 4N inverse pivot blocks
  tpf::Buf<float> bilu_dinv32, jv32;
  tpf::Buf<int> front_cells;      // cells ordered by wavefront ix+iy+iz
  std::vector<int> front_ptr;     // host copy, nfronts + 1
  tpf::Buf<int> front_ptr_dev;    // device copy
  int front_max = 0;              // cells in the largest front
  // workspaces
  tpf::Buf<double> w1, w2, w3, w4, u2, r2;   // N or 2N
  tpf::Buf<float> f1, f2, f3, f4, fu, fr;
  // second stream (and host thread) for building two hierarchies at once
  hipStream_t aux = nullptr;
  hipEvent_t aux_ev = nullptr;
  size_t bytes() const;
  ~tpf_precond();
};
