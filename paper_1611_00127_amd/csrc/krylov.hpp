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
  void* host = nullptr;  // pinned 64-byte slot owned by the caller

  // solve state
  const tpf_jacobian* J = nullptr;
  tpf_precond* M = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  tpf_solve_opts o{};
  hipStream_t s = nullptr;
  Phase phase = kIdle;
  int G = 1;
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

  void begin(const tpf_jacobian* J, tpf_precond* M, const double* b, double* x,
             const tpf_solve_opts& o, hipStream_t s, void* host_slot);
  bool complete();
  bool done() const { return phase == kDone; }
  void info(tpf_solve_info* out) const;
  void finish(int status, double relres);

 private:
  void alloc(int64_t n, int m, hipStream_t s);
  void launch_cycle_start(const double* r, double beta);
  void launch_step();
  void launch_cycle_end();
  void apply_precond(int col);
};

}  // namespace tpf
