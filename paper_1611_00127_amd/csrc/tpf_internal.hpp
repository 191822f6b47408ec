// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tpf.h"

namespace tpf {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const char* fmt, ...);
void set_last_error(int code, const char* msg);

#define TPF_HIP(x)                                                                  \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess)                                                           \
      ::tpf::fail(TPF_ERR_HIP, "%s:%d %s -> %s", __FILE__, __LINE__, #x,            \
                  hipGetErrorString(e_));                                           \
  } while (0)

#define TPF_CHECK_LAUNCH() TPF_HIP(hipGetLastError())

#define TPF_REQUIRE(cond, code, ...)        \
  do {                                      \
    if (!(cond)) ::tpf::fail(code, __VA_ARGS__); \
  } while (0)

// Runs body, converting exceptions to status codes (used by every C entry point).
template <class F>
int guarded(F&& body) {
  try {
    body();
    return TPF_OK;
  } catch (const Error& e) {
    set_last_error(e.code, e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error(TPF_ERR_OOM, "host allocation failed");
    return TPF_ERR_OOM;
  } catch (const std::exception& e) {
    set_last_error(TPF_ERR_INVALID_ARG, e.what());
    return TPF_ERR_INVALID_ARG;
  }
}

// ---------------------------------------------------------------- memory
// Device memory for stream s (cached per stream and size class; see
// runtime.hip).  Buffers are freed on the stream they were allocated on.
void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, size_t bytes, hipStream_t s);
// Returns the blocks cached for stream s to the upstream allocator; call
// after s is synchronised and before it is destroyed.
void forget_stream(hipStream_t s);
// Side stream of stream s, for kernels that may overlap the rest of s's
// work (independent row classes of one product).  fork_side(s) orders the
// side stream after everything queued on s so far and returns it;
// join_side(s) orders s after everything queued on the side stream.  Memory
// the side kernels use must be allocated on s before the fork and freed on
// s after the join.  Created on first use (default priority), destroyed by
// forget_stream(s).
hipStream_t fork_side(hipStream_t s);
void join_side(hipStream_t s);
// Forks the side stream of s when `use` holds (else `side` is s itself);
// join() orders s after the side work, and so does the destructor if join()
// was not reached (an error between the two).
struct SideFork {
  hipStream_t s, side;
  SideFork(hipStream_t s_, bool use) : s(s_), side(use ? fork_side(s_) : s_) {}
  void join() {
    if (side != s) join_side(s);
    side = s;
  }
  ~SideFork() {
    if (side != s) {
      try {
        join_side(s);
      } catch (...) {
      }
    }
  }
  SideFork(const SideFork&) = delete;
  SideFork& operator=(const SideFork&) = delete;
};
// Returns every cached block to the upstream allocator (device idle).
void release_cache();
// Allocated size of a block of `bytes` bytes (its size class).
size_t alloc_footprint(size_t bytes);
// Bytes of freed blocks cached for stream s (allocated sizes).
size_t cached_bytes(hipStream_t s);
// Returns the blocks cached for stream s to the upstream allocator; no work
// queued on s may still use them (s synchronised since they were freed).
void release_stream_cache(hipStream_t s);
// Bytes held from the upstream allocator (blocks in use plus cached ones, at
// allocated sizes), and the peak of that figure since reset_held_peak().
size_t held_bytes();
size_t held_peak();
void reset_held_peak();
// The same for the blocks allocated on stream s: (held, peak since
// reset_stream_held_peak(s)).
std::pair<size_t, size_t> stream_held(hipStream_t s);
void reset_stream_held_peak(hipStream_t s);

// Device array; frees through the installed allocator when it owns its
// memory (alloc), not when it views memory held elsewhere (wrap).
template <class T>
struct Buf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  bool own = true;
  Buf() = default;
  Buf(size_t count, hipStream_t st) { alloc(count, st); }
  ~Buf() { release(); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : p(o.p), n(o.n), s(o.s), own(o.own) { o.p = nullptr; o.n = 0; }
  Buf& operator=(Buf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; s = o.s; own = o.own;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  void alloc(size_t count, hipStream_t st) {
    release();
    s = st;
    n = count;
    own = true;
    p = count ? static_cast<T*>(dalloc(count * sizeof(T), st)) : nullptr;
  }
  // views count elements at ptr without taking ownership
  void wrap(T* ptr, size_t count) {
    release();
    p = ptr;
    n = count;
    own = false;
  }
  // grows (discarding contents) when smaller than count
  void ensure(size_t count, hipStream_t st) { if (n < count || !p) alloc(count < 1 ? 1 : count, st); }
  void release() {
    if (p && own) dfree(p, n * sizeof(T), s);
    p = nullptr;
    n = 0;
    own = true;
  }
  // device bytes the buffer occupies (its allocated size; 0 for a view)
  size_t bytes() const { return p && own ? alloc_footprint(n * sizeof(T)) : 0; }
  T* get() const { return p; }
};

// Pinned host scratch for small device->host reads (one per thread, kept
// until the process ends).
struct HostScratch {
  void* p = nullptr;
  size_t bytes = 0;
  template <class T> T* get(size_t count) {
    size_t need = count * sizeof(T);
    if (need > bytes) {
      if (p) TPF_HIP(hipHostFree(p));
      TPF_HIP(hipHostMalloc(&p, need < 4096 ? 4096 : need, hipHostMallocDefault));
      bytes = need < 4096 ? 4096 : need;
    }
    return static_cast<T*>(p);
  }
};
HostScratch& host_scratch();
// pinned slot for small arrays read back together with a later scalar read
// (bytes 1024..4095 of the calling thread's scratch; read_scalar uses the start)
inline int* host_counts_slot() {
  return reinterpret_cast<int*>(host_scratch().get<char>(4096) + 1024);
}

// Event k (k < 4) of the calling thread, without timing (created on first
// use, kept until the process ends).
hipEvent_t thread_event(int k);

// Host round trips (a stream or event synchronisation the host waits on),
// counted for the setup accounting; read back as tpf_kernel_stats("host_syncs").
void note_host_sync();

template <class T>
T read_scalar(const T* dptr, hipStream_t s) {
  note_host_sync();
  T* h = host_scratch().get<T>(1);
  TPF_HIP(hipMemcpyAsync(h, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  TPF_HIP(hipStreamSynchronize(s));
  return *h;
}

// ---------------------------------------------------------------- sparse
template <class T>
struct Csr {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  Buf<int> rp, ci;
  Buf<T> v;
  size_t bytes() const { return rp.bytes() + ci.bytes() + v.bytes(); }
};

// Non-owning view used by kernels (lets FP32 value copies share a pattern).
template <class T>
struct CsrRef {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  const int* rp = nullptr;
  const int* ci = nullptr;
  const T* v = nullptr;
};
template <class T>
inline CsrRef<T> ref(const Csr<T>& A) {
  return CsrRef<T>{A.nrows, A.ncols, A.nnz, A.rp.p, A.ci.p, A.v.p};
}
template <class T, class U>
inline CsrRef<T> ref_with(const Csr<U>& A, const T* v) {
  return CsrRef<T>{A.nrows, A.ncols, A.nnz, A.rp.p, A.ci.p, v};
}

// ---------------------------------------------------------------- kernel timing
struct TimedScope {
  const char* name;
  hipStream_t s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TimedScope(const char* n, hipStream_t st);
  ~TimedScope();
};
bool timing_enabled();
// V-cycles launched as recorded HIP graphs (default on; off: eager launches)
bool graphs_enabled();

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  return static_cast<unsigned>(g);
}

// ---------------------------------------------------------------- utilities (linalg.hip)
// exclusive scan of n ints into out[0..n], out[n] = total; returns total (synchronises)
int64_t scan_exclusive(const int* in, int* out, int64_t n, hipStream_t s);
// the same without reading the total back (no synchronisation), for counts
// whose total the caller knows fits in int32
void scan_exclusive_async(const int* in, int* out, int64_t n, hipStream_t s);
int64_t scan_exclusive64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
// int counts into 64-bit offsets out[0..n] (no overflow check needed)
int64_t scan_exclusive_wide(const int* in, int64_t* out, int64_t n, hipStream_t s);
// Rows built in a staging area (row i at toff[i]) moved to packed CSR
// storage with row pointers crp (nnz entries in total).
void pack_rows(int n, const int64_t* toff, const int* crp, int64_t nnz, const int* tci,
               const double* tv, int* cci, double* cv, hipStream_t s);
void fill_int(int* p, int v, int64_t n, hipStream_t s);
template <class T> void fill(T* p, T v, int64_t n, hipStream_t s);
template <class T> void copy(T* dst, const T* src, int64_t n, hipStream_t s);
template <class A, class B> void cast(B* dst, const A* src, int64_t n, hipStream_t s);

// deterministic reductions: result written to device memory *out
void dot_device(const double* x, const double* y, int64_t n, double* out, hipStream_t s);
double nrm2_host(const double* x, int64_t n, hipStream_t s);
// *out = ||x||_2 on the device; part: workspace of kNrm2Parts doubles
constexpr int kNrm2Parts = 512;
void nrm2_device(const double* x, int64_t n, double* out, double* part, hipStream_t s);

template <class T>
void csr_spmv(const CsrRef<T>& A, const T* x, T* y, hipStream_t s, const char* tname = "csr_spmv");
// y = b - A x (CSR)
template <class T>
void csr_residual(const CsrRef<T>& A, const T* x, const T* b, T* y, hipStream_t s);

// ---------------------------------------------------------------- spgemm / transpose
// C = alpha * A * B (+ beta * D on the union pattern if D != nullptr).  When
// reuse is true, C's pattern is kept and only values are recomputed.  Rows go
// to the smallest kernel class (by product count) from first_class on.
void spgemm(const CsrRef<double>& A, const CsrRef<double>& B, Csr<double>& C, hipStream_t s,
            const CsrRef<double>* D = nullptr, double alpha = 1.0, double beta = 1.0,
            bool reuse = false, int first_class = 0);
// C = A^T (values copied when A.v != nullptr); rows of C sorted by column.
// A's columns must lie in [0, A.ncols) (not checked; no host round trip).
void transpose(const CsrRef<double>& A, Csr<double>& C, hipStream_t s);

}  // namespace tpf
