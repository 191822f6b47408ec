// Classical AMG hierarchy built and applied on the device.
#pragma once

#include <memory>

#include "tpf_internal.hpp"

namespace tpf {

struct AmgOpts {
  double theta = 0.25;
  int max_levels = 25;
  int coarse_max = 256;
  int dense_max = 1024;
  uint64_t seed = 0x5eed;
  bool fp32 = false;
  bool ext_i = false;   // extended+i instead of direct interpolation
  bool classical = false;  // classical (modified Ruge-Stueben) instead of direct
  bool cljp = false;       // CLJP coarsening instead of PMIS
  int exti_first = 0;   // extended+i rows start the kernel-class search here (tests)
  int smoother = 0;     // 0 l1-Jacobi, 1 Chebyshev on D^{-1} A, 2 multicolour Gauss-Seidel
  int nu1 = 1, nu2 = 1; // pre- and post-smoothing steps
  int cheb_degree = 2;
  int cheb_eig_iters = 10;  // power steps estimating the top eigenvalue of D^{-1} A
  // interpolation truncation: at most trunc_pmax entries per row of P (0: no
  // limit), none below trunc_factor times the row's largest magnitude
  int trunc_pmax = 0;
  double trunc_factor = 0.0;
  bool truncates() const { return trunc_pmax > 0 || trunc_factor > 0.0; }
  // V(1,1) l1-Jacobi runs the fused smoother kernels; anything else the
  // generic sweeps
  bool fused_cycle() const { return smoother == 0 && nu1 == 1 && nu2 == 1; }
};

struct Level {
  Csr<double> A;        // level operator
  Buf<double> dinv;     // inverse l1-Jacobi diagonal (0 where the l1 row sum is 0)
  Buf<uint8_t> mask;    // strength mask over A's entries
  Csr<double> S;        // strength graph (pattern only)
  Buf<int8_t> cf;       // 1 = C, 2 = F
  Csr<double> P, R, T;  // interpolation, restriction, and the Galerkin intermediate
                        // R*A (level 0) or A*P while the product runs (empty after)
  // FP32 copies of the values (patterns shared)
  Buf<float> Av32, Pv32, Rv32, dinv32;
  // P in ELL form for the cycle's prolongation when truncation bounds its
  // rows: slot k of row i at k * n + i (column -1 and value 0 past the
  // row's end), pe_w slots; FP64 or FP32 values as the cycle runs
  int pe_w = 0;
  Buf<int> pe_ci;
  Buf<double> pe_v;
  Buf<float> pe_v32;
  // A for the streamed smoothers (large levels whose rows take at most 8
  // lanes): inside each 512-entry window of a wavefront's rows the entries
  // are in ascending column order; entry k holds column | p << 23, p its
  // position in the window in CSR order, and the value from that position;
  // FP64 or FP32 values as the cycle runs; one zero entry past the end
  Buf<int> sw_ci;
  Buf<double> sw_v;
  Buf<float> sw_v32;
  // R in the same window-sorted form, for the streamed restriction into a
  // coarse level that forms its guess there
  Buf<int> rw_ci;
  Buf<double> rw_v;
  Buf<float> rw_v32;
  // generic smoothing sweeps: two iterates and the Chebyshev direction, and
  // the Chebyshev interval [cheb_lo, cheb_hi] of D^{-1} A
  Buf<double> xa, xb, dd;
  Buf<float> xa32, xb32, dd32;
  double cheb_lo = 0.0, cheb_hi = 0.0;
  // multicolour Gauss-Seidel: the points sorted by colour (order inside a
  // colour unspecified), colour c's at gs_rows[gs_ptr[c] .. gs_ptr[c+1]),
  // gs_ptr on the host and on the device, and 1/a_ii (0 where a_ii = 0)
  Buf<int> gs_rows, gs_ptr_dev;
  std::vector<int> gs_ptr;
  Buf<double> gsd;
  Buf<float> gsd32;
  // workspace: r, y always; b, x on levels >= 1
  Buf<double> r, y, b, x;
  Buf<float> r32, y32, b32, x32;
  int64_t pmis_rounds = 0;
  // kernel-timer labels of this level (persistent storage for TimedScope)
  std::string t_pre, t_guess, t_restrict, t_prolong, t_post, t_coarse;
};

// Level-0 operator in diagonal (stencil) layout: value of row i on diagonal
// k at v[k * n + i], column i + off[k]; entries outside the grid are zero.
constexpr int kMaxDiag = 32;
struct Dia {
  int K = 0;
  int n = 0;
  int off[kMaxDiag] = {};
  Buf<double> v;
  Buf<float> v32;
  bool ok = false;
  size_t bytes() const { return v.bytes() + v32.bytes(); }
};

struct Hierarchy {
  AmgOpts o;
  std::vector<std::unique_ptr<Level>> lv;
  bool coarse_dense = false;
  Buf<double> Ainv;     // dense inverse of the coarsest operator (row-major)
  hipStream_t s = nullptr;
  std::string tag = "A";  // operator name used in kernel-timer labels
  std::vector<int> stencil;  // level-0 diagonal offsets (empty: CSR only)
  Dia dia0;

  // V-cycle graphs, one per value type: recorded on a private stream the
  // first time a (b, x) pair is seen, replayed on the caller's stream after,
  // dropped whenever the levels change.
  struct VGraph {
    const void* b = nullptr;
    void* x = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  VGraph vg[4];  // FP64 / FP32, each with and without a formed level-0 guess
  hipStream_t cap_s = nullptr;
  void drop_graphs();
  ~Hierarchy();

  // Full setup from the level-0 operator.
  void build(Csr<double>&& A0, const AmgOpts& opts, hipStream_t st);
  // Numeric refresh after lv[0]->A values changed (same pattern): keeps C/F, P, R.
  void refresh(hipStream_t st);
  Csr<double>& A0() { return lv[0]->A; }
  // g_ready: the caller formed g = D^-1 b of level 0 in guess_buffer()
  template <class T>
  void vcycle(const T* b, T* x, hipStream_t st, bool g_ready = false);
  // level 0's buffer for g = D^-1 b when the cycle starts from it (else null),
  // and level 0's inverse l1 diagonal
  template <class T>
  T* guess_buffer();
  template <class T>
  const T* level0_dinv() const;
  size_t bytes() const;
  int levels() const { return int(lv.size()); }

 private:
  void finish_levels(hipStream_t st);
  bool streamed_level(int l, int n, int lpr) const;
  bool streamed_restriction(int l) const;
  void coarse_setup(hipStream_t st);
  void chebyshev_setup(Level& L, hipStream_t st);
  void gs_setup(Level& L, hipStream_t st);
  template <class T>
  const T* smooth(Level& L, const T* b, const T* x0, T* out, T* spare0, T* spare1, int steps,
                  bool post, hipStream_t st);
  // g_ready: the caller's restriction already put D^{-1} b in the level's y
  template <class T>
  void vcycle_level(int l, const T* b, T* x, hipStream_t st, bool g_ready = false);
};

}  // namespace tpf
