// Resumable right-preconditioned FGMRES(m) (paper Sec. 3).  A solve is a
// sequence of asynchronous device phases, each ending in a small
// device->host copy of the scalars the next decision needs:
//
//   begin()     set up and queue the first phase (||b||) on the stream
//   complete()  once that stream has drained: read the scalars, decide, and
//               queue the next phase; returns true when the solve is over
//
// A caller that drives one solve loops sync/complete; a scheduler drives
// many solves, each on its own stream, and interleaves their phases.
#pragma once

#include <chrono>

#include "precond.hpp"
#include "tpf_internal.hpp"

namespace tpf {

constexpr int kMaxRestart = 64;

struct Fgmres {
  enum Phase { kIdle, kInit, kStep, kCycleEnd, kDone };

  // workspace (kept across solves of the same size)
  int64_t n = 0;
  int m = 0;
  Buf<double> V, Z, H, cs, sn, g, h1, h2, part, y, r, st_dev, scal;
  bool bound = false;  // workspace placed by bind()
  void* host = nullptr;  // 64-byte host slot owned by the caller (pinned, or pageable)

  // solve state
  const tpf_jacobian* J = nullptr;
  tpf_precond* M = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  tpf_solve_opts o{};
  hipStream_t s = nullptr;
  Phase phase = kIdle;
  int g_norm = 1;  // work-groups of the last step's norm pass (its partial sums)
  int j = 0, k = 0, total = 0;
  bool breakdown = false;
  double beta0 = 0.0, est = 1.0, relres = 0.0, ms = 0.0;
  int status = -1;
  std::chrono::steady_clock::time_point t0;

  // Speculative preconditioning (a caller driving one solve sets it before
  // begin()): after step j's scalars are queued, M^{-1} v_{j+1} is queued
  // behind them while the estimate of the last decision is far from the
  // tolerance, so the GPU does not idle while the host decides.  The
  // scalars are then marked by `ready` (ev_pending): wait on it, not on the
  // stream.  The results are those of the plain sequence.
  bool speculate = false;
  int spec_j = -1;          // Z column already holding M^{-1} v for that step
  double spec_est = 0.0;    // relative residual estimate of the last decision
  bool ev_pending = false;
  hipEvent_t ready = nullptr;

  // Workspace of an FGMRES(m) solve of n unknowns, in doubles, each array
  // starting on a 256-byte boundary: the size bind() needs, and an upper
  // bound of what alloc() draws from the allocator.
  static size_t workspace_doubles(int64_t n, int m);
  // Device bytes alloc() draws for that workspace (allocated sizes).
  static size_t workspace_footprint(int64_t n, int m);
  // Places the workspace in caller-held device memory (base: 256-byte
  // aligned, at least workspace_doubles(n, m) doubles) instead of drawing it
  // from the allocator; begin() then allocates nothing and requires the same
  // n and m.  The memory must outlive the solve.
  void bind(double* base, int64_t n, int m);

  void begin(const tpf_jacobian* J, tpf_precond* M, const double* b, double* x,
             const tpf_solve_opts& o, hipStream_t s, void* host_slot);
  bool complete();
  bool done() const { return phase == kDone; }
  void info(tpf_solve_info* out) const;
  void finish(int status, double relres);

 private:
  void alloc(int64_t n, int m, hipStream_t s);
  // calls f(buffer, element count) for every workspace array, in layout order
  template <class F> void for_each_array(int64_t n, int m, F&& f);
  void launch_cycle_start(const double* r, double beta);
  void launch_step();
  void launch_cycle_end();
  void apply_precond(int col);
};

}  // namespace tpf
