// Serving engine: continuous batching of independent Newton-step solves on
// one GPU.  Each request is one linear solve of Sec. 3 (assemble J(u_k) and
// F(u_k), set up or refresh the preconditioner, right-preconditioned FGMRES
// on J x = -F).  Requests of different sequences run concurrently, each on a
// stream of its own slot, and advance one solver phase per server step, so
// the kernels of many solves overlap on the device.
//
// Threads, streams and memory:
//   - the calling thread admits requests and advances the running solves;
//     a setup thread does each admitted request's assembly and
//     preconditioner setup (host-synchronous work) meanwhile, on one setup
//     stream, so everything a resident sequence owns is allocated and freed
//     on that stream; the request's slot stream waits for it by an event;
//   - the FGMRES workspace of a request is allocated and released on its
//     slot stream, after the host has seen the request's last phase finish;
//   - resident data of a sequence is only touched by one request at a time.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "krylov.hpp"
#include "precond.hpp"
#include "problem.hpp"

namespace tpf {
namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

void check_rc(int rc) {
  if (rc == TPF_OK) return;
  char msg[1024];
  tpf_last_error(msg, sizeof msg);
  fail(rc, "%s", msg);
}

__global__ void k_negate(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    y[i] = -x[i];
}

// device bytes of an FGMRES(m) workspace for 2N unknowns: the arrays Fgmres
// allocates, at their allocated sizes
size_t krylov_bytes(int64_t cells, int m) { return Fgmres::workspace_footprint(2 * cells, m); }

}  // namespace

struct Resident {
  uint64_t seq = 0;
  tpf_problem* prob = nullptr;
  int64_t cells = 0;
  tpf_jacobian* J = nullptr;
  tpf_precond* M = nullptr;
  Buf<double> rhs;
  bool built = false;  // preconditioner structure exists
  bool busy = false;
  std::atomic<size_t> bytes{0};
  std::atomic<size_t> setup_extra{0};  // held beyond its own bytes during its last setup
  std::atomic<hipStream_t> aux{nullptr};  // the preconditioner's second setup stream
  uint64_t last_use = 0;
  ~Resident() {
    if (M) tpf_precond_destroy(M);
    if (J) tpf_jacobian_destroy(J);
  }
  // device bytes this sequence holds (Jacobian, preconditioner, right-hand
  // side), at allocated sizes
  size_t measure() const {
    size_t b = rhs.bytes();
    if (J) b += J->rp.bytes() + J->ci.bytes() + J->v.bytes();
    if (M) b += M->bytes();
    return b;
  }
};

struct Pending {
  uint64_t ticket = 0;
  tpf_request rq{};
  Clock::time_point submit;
};

enum SlotState { kFree, kSetup, kReady, kFailed };

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  void* host = nullptr;  // pinned readback slot
  std::atomic<int> state{kFree};
  std::unique_ptr<Fgmres> f;
  Pending req;
  Resident* res = nullptr;
  int64_t cells = 0;
  bool fresh = false;
  bool cancel = false;
  bool started = false;  // first phase seen by the calling thread
  double setup_ms = 0.0;
  int refreshed = 0;
  size_t ws_bytes = 0;   // reserved while in setup, the FGMRES workspace after
  size_t admitted = 0;   // bytes of the budget reserved at admission
  int err_code = TPF_OK;
  std::string err_msg;
  bool busy() const { return state.load(std::memory_order_acquire) != kFree; }
};

}  // namespace tpf

using namespace tpf;

struct tpf_server {
  tpf_server_opts o{};
  hipStream_t setup_s = nullptr;
  hipEvent_t setup_ev = nullptr;
  void* host_block = nullptr;
  int device = 0;
  std::vector<std::unique_ptr<Slot>> slots;
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Resident>> res;
  std::unordered_map<uint64_t, tpf_result> results;
  uint64_t next_ticket = 1;
  uint64_t tick = 0;
  int64_t submitted = 0, completed = 0, evictions = 0;
  size_t peak = 0;
  // shared with the setup thread
  std::mutex mu;
  std::condition_variable cv_job, cv_done;
  std::deque<Slot*> jobs;
  bool stop = false;
  // (cells, resident bytes, extra bytes held during the setup) of built sequences
  struct Seen {
    int64_t cells;
    size_t resident, extra;
  };
  std::vector<Seen> seen;
  std::thread worker;

  // Device bytes the server holds: every block drawn on its streams (the
  // setup stream, the slot streams, each resident preconditioner's second
  // setup stream), in use or cached for reuse, at allocated sizes.
  size_t held() const {
    size_t b = stream_held(setup_s).first;
    for (auto& sl : slots) b += stream_held(sl->s).first;
    for (auto& kv : res) {
      hipStream_t a = kv.second->aux.load();
      if (a) b += stream_held(a).first;
    }
    return b;
  }
  // bytes reserved for setups not finished yet (their draws so far are also
  // in held(): the sum errs high)
  size_t reserved() const {
    size_t b = 0;
    for (auto& sl : slots)
      if (sl->state.load(std::memory_order_acquire) == kSetup) b += sl->ws_bytes;
    return b;
  }
  size_t in_use() const { return held() + reserved(); }
  void note_peak() { peak = std::max(peak, held()); }

  bool setup_in_flight() {
    std::lock_guard<std::mutex> lk(mu);
    if (!jobs.empty()) return true;
    for (auto& sl : slots)
      if (sl->state.load(std::memory_order_acquire) == kSetup) return true;
    return false;
  }

  // Returns the cached blocks of idle streams to the allocator: free slots,
  // resident sequences not in use, and the setup stream when no setup runs.
  // Each such stream has been synchronised since its blocks were freed.
  void trim_caches() {
    for (auto& sl : slots)
      if (!sl->busy()) release_stream_cache(sl->s);
    for (auto& kv : res) {
      hipStream_t a = kv.second->aux.load();
      if (!kv.second->busy && a) release_stream_cache(a);
    }
    if (!setup_in_flight()) {
      TPF_HIP(hipStreamSynchronize(setup_s));
      release_stream_cache(setup_s);
    }
  }

  // Frees device memory until in_use() + need fits the budget: idle caches
  // first, then idle sequences, those with no queued request before the
  // others, least recently used first.  Returns whether it fits.
  bool make_room(size_t need, uint64_t keep,
                 const std::unordered_map<uint64_t, int>& queued = {}) {
    if (in_use() + need <= o.hbm_budget_bytes) return true;
    trim_caches();
    while (in_use() + need > o.hbm_budget_bytes) {
      if (!evict_one(keep, queued)) return false;
      trim_caches();  // the evicted sequence's blocks went to the setup stream's cache
    }
    return true;
  }

  // Resident bytes and setup bytes a new sequence of `cells` cells is
  // expected to need.  Realizations of one grid size differ (their
  // hierarchies follow their permeability fields), so each size keeps the
  // largest footprint built so far, with a 25% margin:
  //   (a) that of the smallest built size at least as large;
  //   (b) else that of the largest smaller size, scaled by 1.25 times the
  //       cell ratio (deeper hierarchies hold a little more per cell);
  //   (c) before any build, and whenever it is smaller, 2 MiB plus 3 KiB per
  //       cell for each (small grids are dominated by fixed costs, large
  //       ones hold about 4 KiB per cell with the FP32 copies).
  std::pair<size_t, size_t> estimate(int64_t cells) {
    std::lock_guard<std::mutex> lk(mu);
    std::map<int64_t, std::pair<double, double>> worst;  // cells -> largest (resident, extra)
    for (auto& ob : seen) {
      auto& w = worst[ob.cells];
      if (double(ob.resident) + double(ob.extra) > w.first + w.second)
        w = {double(ob.resident), double(ob.extra)};
    }
    double br = double(size_t(2) << 20) + 3072.0 * double(cells), bx = 3072.0 * double(cells);
    double f = 0.0, er = 0.0, ex = 0.0;
    auto up = worst.lower_bound(cells);
    if (up != worst.end()) {
      f = 1.25;
      er = up->second.first;
      ex = up->second.second;
    } else if (!worst.empty()) {
      auto lo = std::prev(worst.end());
      f = 1.25 * 1.25 * double(cells) / double(lo->first);
      er = lo->second.first;
      ex = lo->second.second;
    }
    if (f > 0.0 && f * (er + ex) < br + bx) {
      br = f * er;
      bx = f * ex;
    }
    return {size_t(br), size_t(bx)};
  }

  bool evict_one(uint64_t keep, const std::unordered_map<uint64_t, int>& queued = {}) {
    auto waits = [&](const Resident* r) {
      auto q = queued.find(r->seq);
      return q != queued.end() && q->second > 0;
    };
    Resident* victim = nullptr;
    for (auto& kv : res) {
      Resident* r = kv.second.get();
      if (r->busy || r->seq == keep) continue;
      if (!victim || std::make_pair(waits(r), r->last_use) <
                         std::make_pair(waits(victim), victim->last_use))
        victim = r;
    }
    if (!victim) return false;
    res.erase(victim->seq);
    ++evictions;
    return true;
  }

  void finish_request(const Pending& p, int status, int iters, double est, double rel,
                      double setup_ms, double solve_ms, int refreshed, size_t reserved = 0) {
    tpf_result r{};
    r.reserved_bytes = reserved;
    r.status = status;
    r.iterations = iters;
    r.relres_est = est;
    r.relres_true = rel;
    r.setup_ms = setup_ms;
    r.solve_ms = solve_ms;
    r.latency_ms = ms_since(p.submit);
    r.refreshed = refreshed;
    results[p.ticket] = r;
    ++completed;
  }

  bool sequence_busy(uint64_t seq) const {
    auto it = res.find(seq);
    return it != res.end() && it->second->busy;
  }

  Slot* free_slot() {
    for (auto& sl : slots)
      if (!sl->busy()) return sl.get();
    return nullptr;
  }

  // Setup thread: assembly, right-hand side -F, preconditioner setup or
  // refresh on the setup stream, then the first FGMRES phase on the slot
  // stream.  Touches only the slot and its resident sequence.
  void run_setup(Slot& sl) {
    auto t0 = Clock::now();
    Resident* r = sl.res;
    const Pending& p = sl.req;
    const int64_t cells = sl.cells;
    // blocks the setup draws, on the setup stream and the preconditioner's
    // second setup stream (no other thread allocates on either meanwhile)
    hipStream_t aux0 = r->M ? r->M->aux : nullptr;
    reset_stream_held_peak(setup_s);
    if (aux0) reset_stream_held_peak(aux0);
    const size_t held0 = stream_held(setup_s).first + (aux0 ? stream_held(aux0).first : 0);
    const size_t own0 = r->bytes.load();
    try {
      if (!r->J) check_rc(tpf_jacobian_create(r->prob, setup_s, &r->J));
      if (!r->M) {
        tpf_precond_opts po;
        check_rc(tpf_precond_default_opts(o.kind, &po));
        po.precision = o.precision;
        check_rc(tpf_precond_create(&po, &r->M));
      }
      r->rhs.ensure(size_t(2 * cells), setup_s);
      check_rc(tpf_assemble(r->prob, p.rq.u, p.rq.u_old, p.rq.dt, r->rhs.p, r->J, setup_s));
      k_negate<<<std::min(grid_for(2 * cells, 256), 4096u), 256, 0, setup_s>>>(2 * cells, r->rhs.p,
                                                                          r->rhs.p);
      TPF_CHECK_LAUNCH();
      bool reuse = o.reuse && r->built;
      check_rc(tpf_precond_setup(r->M, r->J, reuse ? 1 : 0, setup_s));  // synchronises
      r->built = true;
      sl.refreshed = reuse ? 1 : 0;
      r->bytes.store(r->measure());
      // device memory drawn beyond what the sequence keeps (temporaries, now
      // cached for the setup streams): reserved for its next setup
      const size_t pk = stream_held(setup_s).second + (r->M->aux ? stream_held(r->M->aux).second : 0);
      const size_t grow = pk > held0 ? pk - held0 : 0;
      const size_t kept = r->bytes.load() - std::min(own0, r->bytes.load());
      r->setup_extra.store(grow > kept ? grow - kept : 0);
      r->aux.store(r->M->aux);
      sl.setup_ms = ms_since(t0);
      TPF_HIP(hipEventRecord(setup_ev, setup_s));
      TPF_HIP(hipStreamWaitEvent(sl.s, setup_ev, 0));
      sl.f = std::make_unique<Fgmres>();
      sl.f->begin(r->J, r->M, r->rhs.p, p.rq.x, o.solve, sl.s, sl.host);
      TPF_HIP(hipEventRecord(sl.ev, sl.s));
      sl.err_code = TPF_OK;
    } catch (const Error& e) {
      sl.err_code = e.code;
      sl.err_msg = e.what();
      (void)hipStreamSynchronize(setup_s);
      (void)hipStreamSynchronize(sl.s);
      sl.setup_ms = ms_since(t0);
    }
  }

  void worker_loop() {
    (void)hipSetDevice(device);
    while (true) {
      Slot* sl = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_job.wait(lk, [&] { return stop || !jobs.empty(); });
        if (jobs.empty()) return;  // stop requested and nothing left
        sl = jobs.front();
        jobs.pop_front();
      }
      run_setup(*sl);
      {
        std::lock_guard<std::mutex> lk(mu);
        if (sl->err_code == TPF_OK && sl->fresh)
          seen.push_back({sl->cells, sl->res->bytes.load(), sl->res->setup_extra.load()});
        sl->state.store(sl->err_code == TPF_OK ? kReady : kFailed, std::memory_order_release);
      }
      cv_done.notify_all();
    }
  }

  // Reserves slot sl for request p and hands its setup to the setup thread.
  void start(Slot& sl, const Pending& p, int64_t cells, size_t reserve) {
    Resident* r = nullptr;
    auto it = res.find(p.rq.sequence);
    bool fresh = it == res.end();
    if (fresh) {
      auto nr = std::make_unique<Resident>();
      nr->seq = p.rq.sequence;
      nr->prob = p.rq.problem;
      nr->cells = cells;
      r = nr.get();
      res[p.rq.sequence] = std::move(nr);
    } else {
      r = it->second.get();
    }
    r->busy = true;
    r->last_use = ++tick;
    sl.req = p;
    sl.res = r;
    sl.cells = cells;
    sl.fresh = fresh;
    sl.cancel = false;
    sl.started = false;
    sl.refreshed = 0;
    sl.ws_bytes = reserve;
    sl.admitted = reserve;
    sl.err_code = TPF_OK;
    sl.err_msg.clear();
    {
      std::lock_guard<std::mutex> lk(mu);
      sl.state.store(kSetup, std::memory_order_release);
      jobs.push_back(&sl);
    }
    cv_job.notify_one();
    note_peak();
  }

  void release(Slot& sl) {
    sl.f.reset();  // workspace returned on the slot stream (its work is done)
    if (sl.res) sl.res->busy = false;
    sl.res = nullptr;
    sl.ws_bytes = 0;
    sl.state.store(kFree, std::memory_order_release);
  }

  // Admission, in two passes over the queue in submission order: the first
  // takes requests whose sequence is resident (a workspace and a refresh),
  // the second those that need a build.  A request that does not fit now is
  // passed over, and so are the later requests of its sequence, so a
  // sequence's requests still start in submission order while other
  // sequences go ahead.
  void admit() {
    std::unordered_map<uint64_t, int> queued;  // queued requests per sequence
    for (auto& q : queue) ++queued[q.rq.sequence];
    std::unordered_set<uint64_t> passed;  // sequences passed over in this call
    for (int pass = 0; pass < 2; ++pass) {
      for (auto it = queue.begin(); it != queue.end();) {
        Slot* sl = free_slot();
        if (!sl) return;
        const Pending& p = *it;
        const uint64_t seq = p.rq.sequence;
        auto rit = res.find(seq);
        const bool resident = rit != res.end();
        if (resident != (pass == 0)) {  // the other pass takes it
          ++it;
          continue;
        }
        if (passed.count(seq) || sequence_busy(seq)) {
          passed.insert(seq);  // its later requests wait behind this one
          ++it;
          continue;
        }
        int64_t cells = 0;
        if (resident) {
          cells = rit->second->cells;
          if (rit->second->prob != p.rq.problem) {
            Pending bad = p;
            it = queue.erase(it);
            --queued[seq];
            set_last_error(TPF_ERR_INVALID_ARG, "request names another problem than its sequence");
            finish_request(bad, TPF_ERR_INVALID_ARG, 0, NAN, NAN, 0.0, 0.0, 0);
            continue;
          }
        } else {
          check_rc(tpf_problem_cells(p.rq.problem, &cells));
        }
        const size_t ws = krylov_bytes(cells, o.solve.restart);
        size_t need = ws;
        if (!resident) {
          auto e = estimate(cells);
          need += e.first + e.second;
        } else {
          // a refresh draws about what the sequence's last setup drew beyond its
          // own bytes; 25% more covers a state whose products come out larger
          need += rit->second->setup_extra.load() + rit->second->setup_extra.load() / 4;
        }
        if (need > o.hbm_budget_bytes) {
          Pending bad = p;
          it = queue.erase(it);
          --queued[seq];
          set_last_error(TPF_ERR_OVER_BUDGET, "request does not fit in the HBM budget");
          finish_request(bad, TPF_ERR_OVER_BUDGET, 0, NAN, NAN, 0.0, 0.0, 0, need);
          continue;
        }
        if (!make_room(need, seq, queued)) {
          bool any_active = false;
          for (auto& x : slots) any_active |= x->busy();
          if (any_active) {  // waits for active solves to retire; later ones may fit
            passed.insert(seq);
            ++it;
            continue;
          }
          Pending bad = p;  // cannot fit even with the device to itself
          it = queue.erase(it);
          --queued[seq];
          set_last_error(TPF_ERR_OVER_BUDGET, "request does not fit in the HBM budget");
          finish_request(bad, TPF_ERR_OVER_BUDGET, 0, NAN, NAN, 0.0, 0.0, 0, need);
          continue;
        }
        Pending go = p;
        it = queue.erase(it);
        --queued[seq];
        start(*sl, go, cells, need);
      }
    }
  }

  // Advances every request whose setup has finished by one phase; waits for
  // a setup to finish when nothing else can advance.
  int step() {
    admit();
    {
      std::unique_lock<std::mutex> lk(mu);
      auto runnable = [&] {
        bool setup = false;
        for (auto& sl : slots) {
          int st = sl->state.load(std::memory_order_acquire);
          if (st == kReady || st == kFailed) return true;
          setup |= st == kSetup;
        }
        return !setup;
      };
      cv_done.wait(lk, runnable);
    }
    int done = 0;
    for (auto& slp : slots) {
      Slot& sl = *slp;
      int st = sl.state.load(std::memory_order_acquire);
      if (st == kFailed) {
        set_last_error(sl.err_code, sl.err_msg.c_str());
        Pending p = sl.req;
        uint64_t seq = p.rq.sequence;
        double setup_ms = sl.setup_ms;
        int code = sl.err_code;
        const size_t admitted = sl.admitted;
        release(sl);
        res.erase(seq);  // rebuilt from scratch by the next request
        finish_request(p, code, 0, NAN, NAN, setup_ms, 0.0, 0, admitted);
        ++done;
        continue;
      }
      if (st != kReady) continue;
      if (!sl.started) {
        // the resident size is known now: the workspace replaces the reservation,
        // and idle sequences give way if the estimate was low
        sl.started = true;
        sl.ws_bytes = krylov_bytes(sl.cells, o.solve.restart);
        make_room(0, sl.res->seq);
        note_peak();
      }
      TPF_HIP(hipEventSynchronize(sl.ev));
      Fgmres& f = *sl.f;
      bool fin = false;
      try {
        if (sl.cancel) {
          f.finish(TPF_CANCELLED, NAN);
          fin = true;
        } else {
          fin = f.complete();
        }
      } catch (const Error& e) {
        set_last_error(e.code, e.what());
        TPF_HIP(hipStreamSynchronize(sl.s));
        f.finish(e.code, NAN);
        fin = true;
      }
      if (!fin) {
        TPF_HIP(hipEventRecord(sl.ev, sl.s));
        continue;
      }
      TPF_HIP(hipStreamSynchronize(sl.s));
      finish_request(sl.req, f.status, f.total, f.est, f.relres, sl.setup_ms, ms_since(f.t0),
                     sl.refreshed, sl.admitted);
      release(sl);
      ++done;
    }
    return done;
  }

  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_job.notify_all();
    if (worker.joinable()) worker.join();
  }
};

extern "C" int tpf_server_default_opts(tpf_server_opts* o) {
  return guarded([&] {
    TPF_REQUIRE(o, TPF_ERR_INVALID_ARG, "null argument");
    *o = tpf_server_opts{};
    o->hbm_budget_bytes = size_t(64) << 30;
    o->max_active = 8;
    o->kind = TPF_PREC_BF;
    o->precision = TPF_FP32;
    o->reuse = 1;
    o->solve.rtol = 1e-8;
    o->solve.restart = 30;
    o->solve.maxit = 1000;
  });
}

extern "C" int tpf_server_create(const tpf_server_opts* o, tpf_server** out) {
  return guarded([&] {
    TPF_REQUIRE(o && out, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(o->max_active >= 1 && o->max_active <= 64, TPF_ERR_INVALID_ARG,
                "max_active must be in [1, 64]");
    TPF_REQUIRE(o->kind >= TPF_PREC_AMG && o->kind <= TPF_PREC_NONE, TPF_ERR_INVALID_ARG,
                "unknown preconditioner kind %d", o->kind);
    TPF_REQUIRE(o->solve.restart >= 1 && o->solve.restart <= kMaxRestart && o->solve.maxit >= 1 &&
                    o->solve.rtol > 0,
                TPF_ERR_INVALID_ARG, "invalid solve options");
    auto sv = std::make_unique<tpf_server>();
    sv->o = *o;
    TPF_HIP(hipStreamCreateWithFlags(&sv->setup_s, hipStreamNonBlocking));
    TPF_HIP(hipEventCreateWithFlags(&sv->setup_ev, hipEventDisableTiming));
    TPF_HIP(hipHostMalloc(&sv->host_block, size_t(64) * o->max_active, hipHostMallocDefault));
    for (int i = 0; i < o->max_active; ++i) {
      sv->slots.push_back(std::make_unique<Slot>());
      Slot& sl = *sv->slots.back();
      TPF_HIP(hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking));
      TPF_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
      sl.host = static_cast<char*>(sv->host_block) + 64 * i;
    }
    TPF_HIP(hipGetDevice(&sv->device));
    tpf_server* raw = sv.get();
    sv->worker = std::thread([raw] { raw->worker_loop(); });
    *out = sv.release();
  });
}

extern "C" int tpf_server_submit(tpf_server* sv, const tpf_request* rq, uint64_t* ticket) {
  return guarded([&] {
    TPF_REQUIRE(sv && rq && ticket, TPF_ERR_INVALID_ARG, "null argument");
    TPF_REQUIRE(rq->problem && rq->u && rq->u_old && rq->x, TPF_ERR_INVALID_ARG,
                "request needs problem, u, u_old and x");
    TPF_REQUIRE(rq->dt > 0, TPF_ERR_INVALID_ARG, "dt must be positive");
    Pending p;
    p.ticket = sv->next_ticket++;
    p.rq = *rq;
    p.submit = Clock::now();
    sv->queue.push_back(p);
    ++sv->submitted;
    *ticket = p.ticket;
  });
}

extern "C" int tpf_server_step(tpf_server* sv, int* n_done) {
  return guarded([&] {
    TPF_REQUIRE(sv && n_done, TPF_ERR_INVALID_ARG, "null argument");
    *n_done = sv->step();
  });
}

extern "C" int tpf_server_poll(tpf_server* sv, uint64_t ticket, tpf_result* out) {
  if (!sv || !out) {
    set_last_error(TPF_ERR_INVALID_ARG, "null argument");
    return TPF_ERR_INVALID_ARG;
  }
  auto it = sv->results.find(ticket);
  if (it != sv->results.end()) {
    *out = it->second;
    sv->results.erase(it);
    return 1;
  }
  for (auto& p : sv->queue)
    if (p.ticket == ticket) return 0;
  for (auto& sl : sv->slots)
    if (sl->busy() && sl->req.ticket == ticket) return 0;
  set_last_error(TPF_ERR_INVALID_ARG, "unknown ticket");
  return TPF_ERR_INVALID_ARG;
}

extern "C" int tpf_server_cancel(tpf_server* sv, uint64_t ticket) {
  return guarded([&] {
    TPF_REQUIRE(sv, TPF_ERR_INVALID_ARG, "null argument");
    for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it) {
      if (it->ticket == ticket) {
        Pending p = *it;
        sv->queue.erase(it);
        sv->finish_request(p, TPF_CANCELLED, 0, NAN, NAN, 0.0, 0.0, 0);
        return;
      }
    }
    for (auto& sl : sv->slots) {
      if (sl->busy() && sl->req.ticket == ticket) {
        sl->cancel = true;  // read by the calling thread once the setup is done
        return;
      }
    }
    TPF_REQUIRE(sv->results.count(ticket), TPF_ERR_INVALID_ARG, "unknown ticket");
  });
}

extern "C" int tpf_server_stats(const tpf_server* sv, tpf_server_counters* out) {
  return guarded([&] {
    TPF_REQUIRE(sv && out, TPF_ERR_INVALID_ARG, "null argument");
    *out = tpf_server_counters{};
    out->queued = int(sv->queue.size());
    for (auto& sl : sv->slots) out->active += sl->busy() ? 1 : 0;
    out->resident_sequences = int(sv->res.size());
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->bytes_in_use = sv->held();
    out->peak_bytes = sv->peak;
    out->evictions = sv->evictions;
  });
}

extern "C" int tpf_server_destroy(tpf_server* sv) {
  return guarded([&] {
    if (!sv) return;
    std::unique_ptr<tpf_server> own(sv);
    sv->shutdown();  // the setup thread finishes the setups it holds, then exits
    for (auto& sl : sv->slots) {
      if (sl->s) (void)hipStreamSynchronize(sl->s);
      sl->f.reset();
    }
    if (sv->setup_s) (void)hipStreamSynchronize(sv->setup_s);
    sv->res.clear();
    if (sv->setup_s) (void)hipStreamSynchronize(sv->setup_s);
    for (auto& sl : sv->slots) {
      if (sl->ev) (void)hipEventDestroy(sl->ev);
      if (sl->s) {
        (void)hipStreamSynchronize(sl->s);
        forget_stream(sl->s);
        (void)hipStreamDestroy(sl->s);
      }
    }
    if (sv->setup_ev) (void)hipEventDestroy(sv->setup_ev);
    if (sv->setup_s) {
      forget_stream(sv->setup_s);
      (void)hipStreamDestroy(sv->setup_s);
    }
    if (sv->host_block) (void)hipHostFree(sv->host_block);
  });
}
