// Runtime services: error state, allocator hook, kernel timing registry.
#include <atomic>
#include <cstdarg>
#include <map>
#include <mutex>

#include "tpf_internal.hpp"

namespace tpf {

namespace {
thread_local int g_last_code = TPF_OK;
thread_local char g_last_msg[1024] = "";

tpf_alloc_fn g_alloc = nullptr;
tpf_free_fn g_free = nullptr;
void* g_ctx = nullptr;
// Byte counts at allocated (size-class) sizes, under g_mem_mu: blocks handed
// out, blocks held from the upstream allocator (handed out or cached), and
// the peak of the latter since the last reset.
size_t g_live = 0;
size_t g_held = 0;
size_t g_held_peak = 0;
struct StreamHeld {
  size_t held = 0, peak = 0;
};
std::map<hipStream_t, StreamHeld> g_stream_held;  // blocks drawn per stream
std::mutex g_mem_mu;

bool g_timing = false;
struct TimedRecord {
  hipEvent_t e0, e1;
};
std::mutex g_time_mu;
std::map<std::string, std::vector<TimedRecord>> g_records;
std::atomic<int64_t> g_host_syncs{0};
std::vector<hipEvent_t> g_event_pool;

hipEvent_t get_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  TPF_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

void set_last_error(int code, const char* msg) {
  g_last_code = code;
  std::snprintf(g_last_msg, sizeof(g_last_msg), "%s", msg);
}

void fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error(code, buf);
}

// Without an installed allocator, memory comes from the current device's
// stream-ordered pool (hipMallocAsync / hipFreeAsync), whose release
// threshold is raised to the maximum the first time a device is used.
namespace {
std::mutex g_pool_mu;
std::vector<int> g_pool_ready;
void prepare_pool() {
  int dev = 0;
  TPF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (int(g_pool_ready.size()) <= dev) g_pool_ready.resize(dev + 1, 0);
  if (g_pool_ready[dev]) return;
  hipMemPool_t pool;
  TPF_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = UINT64_MAX;
  TPF_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  g_pool_ready[dev] = 1;
}

void count_held(hipStream_t s, size_t add, size_t sub) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_held = g_held + add - sub;
  if (g_held > g_held_peak) g_held_peak = g_held;
  StreamHeld& h = g_stream_held[s];
  h.held = h.held + add - sub;
  if (h.held > h.peak) h.peak = h.held;
  if (h.held == 0 && h.peak == 0) g_stream_held.erase(s);
}

void* upstream_alloc(size_t bytes, hipStream_t s) {
  void* p = nullptr;
  if (g_alloc) {
    p = g_alloc(bytes, reinterpret_cast<void*>(s), g_ctx);
    if (!p) fail(TPF_ERR_OOM, "allocator returned NULL for %zu bytes", bytes);
  } else {
    prepare_pool();
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(TPF_ERR_OOM, "hipMallocAsync(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
  }
  count_held(s, bytes, 0);
  return p;
}

// bytes: the block's allocated (size-class) size
void upstream_free(void* p, size_t bytes, hipStream_t s) {
  if (g_free)
    g_free(p, reinterpret_cast<void*>(s), g_ctx);
  else
    (void)hipFreeAsync(p, s);
  count_held(s, 0, bytes);
}

// Block cache in front of the upstream allocator: a freed block is kept
// under (stream, size class) and handed to the next allocation of that class
// on the same stream, which stream order makes safe; no callback or host
// round trip per allocation.  Size classes are eight per octave (at most
// 12.5% rounding).  Blocks of a stream the library destroys go back
// upstream first (forget_stream); past kCacheLimit cached bytes, freed
// blocks go straight back.
constexpr size_t kCacheLimit = size_t(16) << 30;
struct BlockCache {
  std::mutex mu;
  std::map<std::pair<hipStream_t, size_t>, std::vector<void*>> free;
  size_t cached = 0;
};
BlockCache& cache() {
  static BlockCache* c = new BlockCache();  // never destroyed (process teardown)
  return *c;
}
size_t size_class(size_t b) {
  if (b <= 512) return 512;
  const int k = 63 - __builtin_clzll(b - 1);  // 2^k < b <= 2^(k+1)
  const size_t step = size_t(1) << (k - 2 > 9 ? k - 2 : 9);
  return (b + step - 1) / step * step;
}
}  // namespace

void* dalloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) return nullptr;
  const size_t cls = size_class(bytes);
  void* p = nullptr;
  {
    BlockCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.free.find({s, cls});
    if (it != c.free.end() && !it->second.empty()) {
      p = it->second.back();
      it->second.pop_back();
      c.cached -= cls;
    }
  }
  if (!p) p = upstream_alloc(cls, s);
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_live += cls;
  return p;
}

size_t alloc_footprint(size_t bytes) { return bytes ? size_class(bytes) : 0; }

void dfree(void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  const size_t cls = size_class(bytes);
  bool kept = false;
  {
    BlockCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.cached + cls <= kCacheLimit) {
      c.free[{s, cls}].push_back(p);
      c.cached += cls;
      kept = true;
    }
  }
  if (!kept) upstream_free(p, cls, s);
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_live -= cls;
}

size_t cached_bytes(hipStream_t s) {
  BlockCache& c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  size_t b = 0;
  for (auto it = c.free.lower_bound({s, 0}); it != c.free.end() && it->first.first == s; ++it)
    b += it->first.second * it->second.size();
  return b;
}

void release_stream_cache(hipStream_t s) {
  std::vector<std::pair<void*, size_t>> back;
  {
    BlockCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto it = c.free.lower_bound({s, 0}); it != c.free.end() && it->first.first == s;) {
      for (void* p : it->second) back.push_back({p, it->first.second});
      c.cached -= it->first.second * it->second.size();
      it = c.free.erase(it);
    }
  }
  for (auto& b : back) upstream_free(b.first, b.second, s);
}

size_t held_bytes() {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  return g_held;
}

size_t held_peak() {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  return g_held_peak;
}

void reset_held_peak() {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_held_peak = g_held;
}

std::pair<size_t, size_t> stream_held(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  auto it = g_stream_held.find(s);
  return it == g_stream_held.end() ? std::pair<size_t, size_t>{0, 0}
                                   : std::pair<size_t, size_t>{it->second.held, it->second.peak};
}

void reset_stream_held_peak(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  auto it = g_stream_held.find(s);
  if (it != g_stream_held.end()) it->second.peak = it->second.held;
}

namespace {
struct Side {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_side_mu;
std::map<hipStream_t, Side>& sides() {
  static auto* m = new std::map<hipStream_t, Side>();  // never destroyed (process teardown)
  return *m;
}
Side& side_of(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_side_mu);
  Side& sd = sides()[s];
  if (!sd.st) {
    TPF_HIP(hipStreamCreateWithFlags(&sd.st, hipStreamNonBlocking));
    TPF_HIP(hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming));
    TPF_HIP(hipEventCreateWithFlags(&sd.join, hipEventDisableTiming));
  }
  return sd;
}
}  // namespace

hipStream_t fork_side(hipStream_t s) {
  Side& sd = side_of(s);
  TPF_HIP(hipEventRecord(sd.fork, s));
  TPF_HIP(hipStreamWaitEvent(sd.st, sd.fork, 0));
  return sd.st;
}

void join_side(hipStream_t s) {
  Side& sd = side_of(s);
  TPF_HIP(hipEventRecord(sd.join, sd.st));
  TPF_HIP(hipStreamWaitEvent(s, sd.join, 0));
}

void forget_stream(hipStream_t s) {
  {
    Side sd;
    {
      std::lock_guard<std::mutex> lk(g_side_mu);
      auto it = sides().find(s);
      if (it != sides().end()) {
        sd = it->second;
        sides().erase(it);
      }
    }
    if (sd.st) {
      (void)hipStreamSynchronize(sd.st);
      (void)hipEventDestroy(sd.fork);
      (void)hipEventDestroy(sd.join);
      (void)hipStreamDestroy(sd.st);
    }
  }
  release_stream_cache(s);
}

void release_cache() {
  struct Back {
    void* p;
    size_t bytes;
    hipStream_t s;
  };
  std::vector<Back> back;
  {
    BlockCache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto& kv : c.free)
      for (void* p : kv.second) back.push_back({p, kv.first.second, kv.first.first});
    c.free.clear();
    c.cached = 0;
  }
  if (back.empty()) return;
  TPF_HIP(hipDeviceSynchronize());  // no queued work may still use the blocks
  for (auto& b : back) upstream_free(b.p, b.bytes, b.s);
}

HostScratch& host_scratch() {
  // never destroyed: pinned memory must not be released during process teardown
  static thread_local HostScratch* hs = new HostScratch();
  return *hs;
}

hipEvent_t thread_event(int k) {
  struct Events {
    hipEvent_t e[4] = {};
  };
  static thread_local Events* ev = new Events();  // kept until the process ends
  TPF_REQUIRE(k >= 0 && k < 4, TPF_ERR_INVALID_ARG, "thread_event: index %d", k);
  if (!ev->e[k]) TPF_HIP(hipEventCreateWithFlags(&ev->e[k], hipEventDisableTiming));
  return ev->e[k];
}

bool timing_enabled() { return g_timing; }

namespace {
std::atomic<bool> g_graphs{false};
}
bool graphs_enabled() { return g_graphs.load(std::memory_order_relaxed); }

void note_host_sync() { g_host_syncs.fetch_add(1, std::memory_order_relaxed); }

TimedScope::TimedScope(const char* n, hipStream_t st) : name(n), s(st) {
  if (!g_timing) return;
  std::lock_guard<std::mutex> lk(g_time_mu);
  e0 = get_event();
  e1 = get_event();
  TPF_HIP(hipEventRecord(e0, s));
}

TimedScope::~TimedScope() {
  if (!e0) return;
  if (hipEventRecord(e1, s) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_time_mu);
  g_records[name].push_back({e0, e1});
}

}  // namespace tpf

using namespace tpf;

extern "C" {

const char* tpf_status_string(int st) {
  switch (st) {
    case TPF_OK: return "ok";
    case TPF_ERR_INVALID_ARG: return "invalid argument";
    case TPF_ERR_OOM: return "out of memory";
    case TPF_ERR_HIP: return "HIP runtime error";
    case TPF_ERR_SINGULAR: return "singular pivot";
    case TPF_ERR_OVER_BUDGET: return "request exceeds the memory budget";
    case TPF_ERR_NOT_IMPLEMENTED: return "not implemented";
    case TPF_ERR_STATE: return "call out of order";
    default: return "unknown status";
  }
}

int tpf_last_error(char* buf, size_t n) {
  if (buf && n) std::snprintf(buf, n, "%s", g_last_msg);
  return g_last_code;
}

int tpf_set_allocator(tpf_alloc_fn a, tpf_free_fn f, void* ctx) {
  if ((a == nullptr) != (f == nullptr)) {
    set_last_error(TPF_ERR_INVALID_ARG, "alloc and free must both be set or both be NULL");
    return TPF_ERR_INVALID_ARG;
  }
  int rc = tpf::guarded([] { tpf::release_cache(); });  // blocks of the previous allocator
  if (rc != TPF_OK) return rc;
  g_alloc = a;
  g_free = f;
  g_ctx = ctx;
  return TPF_OK;
}

int tpf_release_cached_memory(void) {
  return tpf::guarded([] {
    tpf::release_cache();
    if (!tpf::g_alloc) {
      int dev = 0;
      TPF_HIP(hipGetDevice(&dev));
      hipMemPool_t pool;
      TPF_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
      TPF_HIP(hipDeviceSynchronize());
      TPF_HIP(hipMemPoolTrimTo(pool, 0));
    }
  });
}

int tpf_memory_in_use(size_t* bytes) {
  if (!bytes) return TPF_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mem_mu);
  *bytes = g_held;
  return TPF_OK;
}

int tpf_set_graphs(int enable) {
  tpf::g_graphs.store(enable != 0);
  return TPF_OK;
}

int tpf_kernel_timing(int enable) {
  g_timing = enable != 0;
  return TPF_OK;
}

int tpf_kernel_stats(const char* name, int64_t* count, double* total_ms) {
  return guarded([&] {
    TPF_REQUIRE(name && count && total_ms, TPF_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(g_time_mu);
    *count = 0;
    *total_ms = 0.0;
    if (std::strcmp(name, "host_syncs") == 0) {
      *count = g_host_syncs.load();
      return;
    }
    auto it = g_records.find(name);
    if (it == g_records.end()) return;
    for (auto& r : it->second) {
      TPF_HIP(hipEventSynchronize(r.e1));
      float ms = 0.f;
      TPF_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
      *total_ms += ms;
      ++*count;
    }
  });
}

int tpf_kernel_stats_reset(void) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(g_time_mu);
    for (auto& kv : g_records)
      for (auto& r : kv.second) {
        TPF_HIP(hipEventSynchronize(r.e1));
        g_event_pool.push_back(r.e0);
        g_event_pool.push_back(r.e1);
      }
    g_records.clear();
    g_host_syncs.store(0);
  });
}

}  // extern "C"
