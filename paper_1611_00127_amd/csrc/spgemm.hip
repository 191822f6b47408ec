// Sparse matrix-matrix product and transpose with symbolic (cancellation-
// free) patterns and sorted rows, used for the Galerkin product A_c = R(AP)
// and for the approximate Schur complement S~ = A_pp - (A_ps D^{-1}) A_sp.
//
// Output row i has the sorted unique columns of the rows B_k, k in A_i (and
// of D_i when a matrix is added); each value is the sum over k in A's column
// order of A_ik B_kj, so the result is deterministic.  Rows are grouped by
// their product count ub_i:
//   ub_i <= 64 .. 512   one wavefront, ub_i <= 2048 a 256-thread and
//   ub_i <= 8192        a 512-thread work-group (A rows of at most 2048
//                       entries) take the flattened product list: the
//                       (column, product index) keys are sorted by a bitonic
//                       network held in registers (in-lane exchanges,
//                       shuffles across lanes, LDS only across wavefronts),
//                       and each run of equal columns is summed in order;
//   ub_i <= 16384       one work-group sorts the product columns, then sums
//                       over k per output entry;
//   larger              one thread per row merges the sorted B rows with a
//                       cursor each.
// Every row is written once, at an upper-bound offset in a staging area, and
// the rows are packed afterwards.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "linalg_dev.hpp"
#include "tpf_internal.hpp"

namespace tpf {

namespace {

template <bool FILL>
__global__ void __launch_bounds__(128) k_spgemm_merge(
    int nlist, const int* __restrict__ rows, const int* __restrict__ arp, const int* __restrict__ aci,
    const double* __restrict__ av, const int* __restrict__ brp, const int* __restrict__ bci,
    const double* __restrict__ bv, const int* __restrict__ drp, const int* __restrict__ dci,
    const double* __restrict__ dv, double alpha, double beta, int2* __restrict__ cur,
    int* __restrict__ cnt, const int64_t* __restrict__ toff, int* __restrict__ cci,
    double* __restrict__ cv) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlist) return;
  int i = rows[t];
  int a0 = arp[i], a1 = arp[i + 1];
  for (int e = a0; e < a1; ++e) {
    int k = aci[e];
    cur[e] = make_int2(brp[k], brp[k + 1]);
  }
  int dp = 0, de = 0;
  if (drp) {
    dp = drp[i];
    de = drp[i + 1];
  }
  int64_t out = FILL ? toff[i] : 0;
  int count = 0;
  while (true) {
    int m = INT_MAX;
    for (int e = a0; e < a1; ++e) {
      int2 c = cur[e];
      if (c.x < c.y) {
        int col = bci[c.x];
        m = col < m ? col : m;
      }
    }
    if (dp < de) {
      int col = dci[dp];
      m = col < m ? col : m;
    }
    if (m == INT_MAX) break;
    double sum = 0.0;
    for (int e = a0; e < a1; ++e) {
      int2 c = cur[e];
      if (c.x < c.y && bci[c.x] == m) {
        if (FILL) sum += av[e] * bv[c.x];
        cur[e].x = c.x + 1;
      }
    }
    if (FILL) {
      double val = alpha * sum;
      if (dp < de && dci[dp] == m) val = beta * dv[dp] + val;
      cci[out + count] = m;
      cv[out + count] = val;
    }
    if (dp < de && dci[dp] == m) ++dp;
    ++count;
  }
  cnt[i] = count;
}

// ---- row classification and the sort-based product
// ub_i = products of row i (plus D's row), at least A's row length; LPR
// lanes per row
template <int LPR>
__global__ void __launch_bounds__(256) k_spgemm_ub(int nrows, const int* __restrict__ arp,
                                                   const int* __restrict__ aci,
                                                   const int* __restrict__ brp,
                                                   const int* __restrict__ drp,
                                                   int* __restrict__ ub) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  int64_t t = 0;
  int a0 = 0, a1 = 0;
  if (i < nrows) {
    a0 = arp[i];
    a1 = arp[i + 1];
  }
  for (int e = a0 + lane; e < a1; e += LPR) {
    int k = aci[e];
    t += brp[k + 1] - brp[k];
  }
  t = group_sum<LPR>(t);
  if (i < nrows && lane == 0) {
    if (drp) t += drp[i + 1] - drp[i];
    int64_t la = a1 - a0;
    if (la > t) t = la;  // the flattened kernels also hold A's row in LDS
    ub[i] = t > INT_MAX ? INT_MAX : int(t);
  }
}

// appends row i to the list of its size class: the first class whose cap
// holds ub[i] (flattened wavefront / work-group kernels, then the
// sorted-columns work-group), else the last list (per-thread merge)
constexpr int kClasses = 9;
struct Caps {
  int c[kClasses - 1];   // product bound of each class
  int la[kClasses - 1];  // bound on A's row length
};
// smallest class from `first` on whose bounds the row fits
__global__ void k_spgemm_classify(int nrows, const int* __restrict__ ub,
                                  const int* __restrict__ arp, Caps caps, int first,
                                  int* __restrict__ counts, int* __restrict__ lists) {
  block_append_rows<kClasses, 256, kClassifyRows>(
      nrows,
      [&](int i) {
        const int u = ub[i], la = arp[i + 1] - arp[i];
        int c = kClasses - 1;
#pragma unroll
        for (int k = kClasses - 2; k >= 0; --k)
          if (k >= first && u <= caps.c[k] && la <= caps.la[k]) c = k;
        return c;
      },
      nrows, counts, lists);
}

__device__ inline int bsearch_col(const int* __restrict__ c, int lo, int hi, int key) {
  // position in the sorted range [lo, hi) holding key, or -1
  int end = hi;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    int v = c[mid];
    if (v < key) lo = mid + 1;
    else hi = mid;
  }
  return (lo < end && c[lo] == key) ? lo : -1;
}

template <int BLOCK, int CAP, bool FILL>
__global__ void __launch_bounds__(BLOCK) k_spgemm_sorted(
    const int* __restrict__ rows, const int* __restrict__ ub, const int* __restrict__ arp,
    const int* __restrict__ aci, const double* __restrict__ av, const int* __restrict__ brp,
    const int* __restrict__ bci, const double* __restrict__ bv, const int* __restrict__ drp,
    const int* __restrict__ dci, const double* __restrict__ dv, double alpha, double beta,
    int* __restrict__ cnt, const int64_t* __restrict__ toff, int* __restrict__ cci,
    double* __restrict__ cv) {
  __shared__ __attribute__((aligned(16))) int keys[CAP];
  __shared__ int ukeys[CAP];
  __shared__ int sh[BLOCK / 64 + 1];
  int i = rows[blockIdx.x];
  int u = ub[i];
  int p2 = 1;
  while (p2 < u) p2 <<= 1;
  // gather product columns
  int off = 0;
  int a0 = arp[i], a1 = arp[i + 1];
  for (int e = a0; e < a1; ++e) {
    int k = aci[e];
    int b0 = brp[k], b1 = brp[k + 1];
    for (int t = threadIdx.x; t < b1 - b0; t += BLOCK) keys[off + t] = bci[b0 + t];
    off += b1 - b0;
  }
  if (drp) {
    int d0 = drp[i], d1 = drp[i + 1];
    for (int t = threadIdx.x; t < d1 - d0; t += BLOCK) keys[off + t] = dci[d0 + t];
    off += d1 - d0;
  }
  for (int t = off + threadIdx.x; t < p2; t += BLOCK) keys[t] = INT_MAX;
  __syncthreads();
  // bitonic sort, ascending
  for (int k = 2; k <= p2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < p2; t += BLOCK) {
        int q = t ^ j;
        if (q > t) {
          int x = keys[t], y = keys[q];
          bool up = (t & k) == 0;
          if ((x > y) == up) {
            keys[t] = y;
            keys[q] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // unique columns in order
  int64_t o = FILL ? toff[i] : 0;
  int running = 0;
  for (int base = 0; base < p2; base += BLOCK) {
    int t = base + threadIdx.x;
    int flag = 0;
    if (t < p2) {
      int x = keys[t];
      flag = x != INT_MAX && (t == 0 || keys[t - 1] != x);
    }
    int total;
    int excl = block_exclusive_scan<int, BLOCK>(flag, sh, total);
    if (flag) ukeys[running + excl] = keys[t];
    running += total;
  }
  if (threadIdx.x == 0) cnt[i] = running;
  if (!FILL) return;
  __syncthreads();
  for (int t = threadIdx.x; t < running; t += BLOCK) cci[o + t] = ukeys[t];
  if (running <= CAP / 2) {
    // values: scatter A_ik B_kj into an LDS accumulator (aliasing keys), one
    // k at a time in A's column order, so each sum has the sequential order
    double* acc = reinterpret_cast<double*>(keys);
    for (int t = threadIdx.x; t < running; t += BLOCK) acc[t] = 0.0;
    __syncthreads();
    for (int e = a0; e < a1; ++e) {
      int k = aci[e];
      double a = av[e];
      int b0 = brp[k], b1 = brp[k + 1];
      for (int t = threadIdx.x; t < b1 - b0; t += BLOCK) {
        int col = bci[b0 + t];
        int lo = 0, hi = running;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (ukeys[mid] < col) lo = mid + 1;
          else hi = mid;
        }
        acc[lo] += a * bv[b0 + t];
      }
      __syncthreads();
    }
    for (int t = threadIdx.x; t < running; t += BLOCK) acc[t] = alpha * acc[t];
    __syncthreads();
    if (drp) {
      int d0 = drp[i], d1 = drp[i + 1];
      for (int t = threadIdx.x; t < d1 - d0; t += BLOCK) {
        int col = dci[d0 + t];
        int lo = 0, hi = running;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (ukeys[mid] < col) lo = mid + 1;
          else hi = mid;
        }
        acc[lo] = beta * dv[d0 + t] + acc[lo];
      }
      __syncthreads();
    }
    for (int t = threadIdx.x; t < running; t += BLOCK) cv[o + t] = acc[t];
    return;
  }
  // wide rows: each output entry sums over k in order (B_kj by binary search)
  for (int t = threadIdx.x; t < running; t += BLOCK) {
    int col = ukeys[t];
    double sum = 0.0;
    for (int e = a0; e < a1; ++e) {
      int k = aci[e];
      int p = bsearch_col(bci, brp[k], brp[k + 1], col);
      if (p >= 0) sum += av[e] * bv[p];
    }
    double val = alpha * sum;
    if (drp) {
      int p = bsearch_col(dci, drp[i], drp[i + 1], col);
      if (p >= 0) val = beta * dv[p] + val;
    }
    cv[o + t] = val;
  }
}

// Flattened product list (rows with at most CAP products and LACAP entries
// in A's row): product t of row i is (e, p) with e the last entry of A's row
// whose B-row prefix offset is <= t.  Keys (col << bits | t) are
// bitonic-sorted, so equal columns are adjacent in increasing t, i.e. in A's
// column order; each output value is the sum over its run, formed by the
// threads holding the run's pieces (contiguous chunks of the sorted keys) and
// a segmented scan across the threads.  Keys are 32 bits when the column
// count leaves room for log2(CAP) index bits (the caller checks), else 64.
template <class KEY, int CAP>
struct FlatKey {
  static constexpr int kIdxBits = sizeof(KEY) == 8 ? 32 : __builtin_ctz(CAP);
  static constexpr KEY kIdxMask = (KEY(1) << kIdxBits) - 1;
};

// Partial run sums: f = a run starts in the piece, (s, d) = product sum and
// added-matrix term since the last start.
struct RunPart {
  int f;
  double s, d;
};
__device__ inline RunPart run_combine(const RunPart& a, const RunPart& b) {
  return b.f ? b : RunPart{a.f, a.s + b.s, a.d + b.d};
}

// Exclusive segmented scan of RunPart over the block's threads in thread
// order (fixed combination order).  sh: BLOCK / 64 entries.
template <int BLOCK>
__device__ inline RunPart run_scan_exclusive(RunPart x, RunPart* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    RunPart y{__shfl_up(x.f, off, 64), __shfl_up(x.s, off, 64), __shfl_up(x.d, off, 64)};
    if (lane >= off) x = run_combine(y, x);
  }
  RunPart ex{__shfl_up(x.f, 1, 64), __shfl_up(x.s, 1, 64), __shfl_up(x.d, 1, 64)};
  if (lane == 0) ex = RunPart{0, 0.0, 0.0};
  if (BLOCK > 64) {
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    RunPart c{0, 0.0, 0.0};
    for (int w = 0; w < wid; ++w) c = run_combine(c, sh[w]);
    ex = lane == 0 ? c : run_combine(c, ex);
  }
  return ex;
}

template <int BLOCK, int CAP, class KEY, int LACAP = CAP>
__global__ void __launch_bounds__(BLOCK, BLOCK == 64 ? 8 : (BLOCK == 256 ? 4 : 2)) k_spgemm_flat(
    const int* __restrict__ rows, const int* __restrict__ ub, const int* __restrict__ arp,
    const int* __restrict__ aci, const double* __restrict__ av, const int* __restrict__ brp,
    const int* __restrict__ bci, const double* __restrict__ bv, const int* __restrict__ drp,
    const int* __restrict__ dci, const double* __restrict__ dv, double alpha, double beta,
    int* __restrict__ cnt, const int64_t* __restrict__ toff, int* __restrict__ cci,
    double* __restrict__ cv) {
  using FK = FlatKey<KEY, CAP>;
  // LDS: the B-row prefix offsets and row starts of A's entries live until
  // every product is located; the product values then take their place
  // (the sorted keys follow the values and are written after the sort)
  constexpr int kValBytes = CAP * int(sizeof(double));
  static_assert((2 * LACAP + 1) * int(sizeof(int)) <= kValBytes + CAP * int(sizeof(KEY)),
                "offsets must fit in the value and key areas");
  __shared__ __attribute__((aligned(16))) unsigned char lds[kValBytes + CAP * sizeof(KEY)];
  int* offs = reinterpret_cast<int*>(lds);      // LACAP + 1 entries
  int* bst = offs + LACAP + 1;                  // start of B row k_e for each entry e
  double* pv = reinterpret_cast<double*>(lds);  // CAP product values
  KEY* keys = reinterpret_cast<KEY*>(lds + kValBytes);
  __shared__ int sh[BLOCK / 64 + 1];
  __shared__ RunPart rsh[BLOCK / 64];
  int i = rows[blockIdx.x];
  int a0 = arp[i], a1 = arp[i + 1];
  int la = a1 - a0;
  // prefix of B row lengths over A's row (block scan in chunks)
  int run = 0;
  for (int base = 0; base < la; base += BLOCK) {
    int e = base + threadIdx.x;
    int len = 0, b0 = 0;
    if (e < la) {
      int k = aci[a0 + e];
      b0 = brp[k];
      len = brp[k + 1] - b0;
    }
    int total;
    int excl = block_exclusive_scan<int, BLOCK>(len, sh, total);
    if (e < la) {
      offs[e] = run + excl;
      bst[e] = b0;
    }
    run += total;
  }
  if (threadIdx.x == 0) offs[la] = run;
  int nprod = run;
  int nd = drp ? drp[i + 1] - drp[i] : 0;
  int u = nprod + nd;
  int p2 = 1;
  while (p2 < u) p2 <<= 1;
  int top = 1;  // largest power of two below la
  while (2 * top < la) top <<= 1;
  __syncthreads();
  // products: each lane's CAP / BLOCK slots are located in LDS first (the
  // searches of all slots advance together), then all their loads are issued
  // before the first wait: every slot reads a valid position (slots past the
  // B products repeat the last one, or read D's row), values are selected after
  constexpr int PER = CAP / BLOCK;
  // element t of this thread's slot q: wave w holds t in [w * 64 PER, (w + 1) * 64 PER)
  const int lane = threadIdx.x & 63, wbase = (threadIdx.x >> 6) * 64 * PER;
  int ent[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) ent[q] = 0;
  const int tlast = nprod - 1;
  for (int step = top; step > 0; step >>= 1) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = min(wbase + q * 64 + lane, tlast);
      const int c = ent[q] + step;  // largest e with offs[e] <= t
      if (c < la && offs[c] <= t) ent[q] = c;
    }
  }
  const int d0 = nd > 0 ? drp[i] : 0;
  int col[PER];
  double val[PER];
  if (u > 0) {
    double x[PER], a[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = wbase + q * 64 + lane;
      const bool fromb = nprod > 0 && (t < nprod || nd == 0);
      const int tb = min(t, tlast);
      const int idx = fromb ? bst[ent[q]] + (tb - offs[ent[q]]) : d0 + min(max(t - nprod, 0), nd - 1);
      const int* cp = fromb ? bci : dci;
      const double* vp = fromb ? bv : dv;
      col[q] = cp[idx];
      x[q] = vp[idx];
      a[q] = la > 0 ? av[a0 + ent[q]] : 1.0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = wbase + q * 64 + lane;
      val[q] = t < nprod ? a[q] * x[q] : x[q];
    }
  }
  // bitonic network in registers: exchanges inside a lane (distance 64 ..
  // 32 PER) in place, across lanes (distance < 64) through shuffles, across
  // wavefronts (distance >= 64 PER) through LDS
  KEY kr[PER];
  __syncthreads();  // offsets and row starts are dead: values take their place
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = wbase + q * 64 + lane;
    kr[q] = t < u ? (static_cast<KEY>(static_cast<unsigned>(col[q])) << FK::kIdxBits) | KEY(t)
                  : ~KEY(0);
    if (t < u) pv[t] = val[q];
  }
  bitonic_regs<PER>(kr, wbase, lane, p2, keys);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = wbase + q * 64 + lane;
    if (t < p2) keys[t] = kr[q];
  }
  __syncthreads();
  // run sums: thread j takes the sorted elements [j PER, (j + 1) PER)
  const int t0 = threadIdx.x * PER;
  int rc[PER];
  double rv[PER];
  bool rd[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    rc[q] = -1;
    rv[q] = 0.0;
    rd[q] = false;
    if (t0 + q < u) {
      const KEY k = keys[t0 + q];
      const int e = int(k & FK::kIdxMask);
      rc[q] = int(k >> FK::kIdxBits);
      rv[q] = pv[e];
      rd[q] = e >= nprod;
    }
  }
  const int cprev = (t0 > 0 && t0 < u) ? int(keys[t0 - 1] >> FK::kIdxBits) : -1;
  const int cnext = (t0 + PER < u) ? int(keys[t0 + PER] >> FK::kIdxBits) : -1;
  RunPart part{0, 0.0, 0.0};
  int heads = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (t0 + q >= u) break;
    if (rc[q] != (q ? rc[q - 1] : cprev)) {
      part = RunPart{1, 0.0, 0.0};
      ++heads;
    }
    if (rd[q]) part.d += rv[q];
    else part.s += rv[q];
  }
  int count;
  const int hx = block_exclusive_scan<int, BLOCK>(heads, sh, count);
  RunPart acc = run_scan_exclusive<BLOCK>(part, rsh);
  const int64_t o = toff[i];
  int r = hx - 1;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (t0 + q >= u) break;
    if (rc[q] != (q ? rc[q - 1] : cprev)) {
      acc = RunPart{1, 0.0, 0.0};
      ++r;
    }
    if (rd[q]) acc.d += rv[q];
    else acc.s += rv[q];
    if (rc[q] != (q + 1 < PER ? rc[q + 1] : cnext)) {
      cci[o + r] = rc[q];
      cv[o + r] = beta * acc.d + alpha * acc.s;
    }
  }
  if (threadIdx.x == 0) cnt[i] = count;
}

// Bitonic sort of the p2 (a power of two, at most G PER) keys of a G-lane
// group: element t = q G + ll sits in register q of group lane ll.  Exchanges
// at distance >= G stay inside a lane, shorter ones are shuffles within the
// group (groups are G-aligned, so lane ^ j stays in the group).
template <int G, int PER, class KEY>
__device__ inline void bitonic_group(KEY (&kr)[PER], int ll, int p2) {
  for (int kk = 2; kk <= p2; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j >= G) {
        const int qj = j / G;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          if ((q & qj) != 0) continue;
          const int qp = q | qj;
          if (qp >= PER) continue;
          const bool up = ((q * G + ll) & kk) == 0;
          const KEY x = kr[q], y = kr[qp];
          const bool sw = (x > y) == up;
          kr[q] = sw ? y : x;
          kr[qp] = sw ? x : y;
        }
      } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const KEY x = kr[q];
          const KEY y = __shfl_xor(x, j, 64);
          const bool up = ((q * G + ll) & kk) == 0, lower = (ll & j) == 0;
          const KEY mn = x < y ? x : y, mx = x < y ? y : x;
          kr[q] = lower == up ? mn : mx;
        }
      }
    }
}

// Exclusive segmented scan of RunPart over the G lanes of a group.
template <int G>
__device__ inline RunPart run_scan_group(RunPart x, int ll) {
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    RunPart y{__shfl_up(x.f, off, G), __shfl_up(x.s, off, G), __shfl_up(x.d, off, G)};
    if (ll >= off) x = run_combine(y, x);
  }
  RunPart ex{__shfl_up(x.f, 1, G), __shfl_up(x.s, 1, G), __shfl_up(x.d, 1, G)};
  if (ll == 0) ex = RunPart{0, 0.0, 0.0};
  return ex;
}

// The flattened-product row kernel with 64 / G rows per wavefront, a G-lane
// group per row (at most G PER products and G PER entries in A's row): the
// same steps as k_spgemm_flat (located products, loads issued together,
// register bitonic sort, contiguous run-sum chunks with a segmented scan),
// each group on its own LDS slice.  More rows in flight per CU for the many
// short rows of the finest levels.
template <int G, int PER, class KEY>
__global__ void __launch_bounds__(64, 8) k_spgemm_group(
    int nlist, const int* __restrict__ rows, const int* __restrict__ arp,
    const int* __restrict__ aci, const double* __restrict__ av, const int* __restrict__ brp,
    const int* __restrict__ bci, const double* __restrict__ bv, const int* __restrict__ drp,
    const int* __restrict__ dci, const double* __restrict__ dv, double alpha, double beta,
    int* __restrict__ cnt, const int64_t* __restrict__ toff, int* __restrict__ cci,
    double* __restrict__ cv) {
  constexpr int CAP = G * PER, RPW = 64 / G;
  using FK = FlatKey<KEY, CAP>;
  constexpr int kValBytes = CAP * int(sizeof(double));
  constexpr int kSlice = kValBytes + CAP * int(sizeof(KEY));
  static_assert((2 * CAP + 1) * int(sizeof(int)) <= kSlice, "offsets must fit in the slice");
  __shared__ __attribute__((aligned(16))) unsigned char lds[RPW * kSlice];
  const int lane = threadIdx.x, g = lane / G, ll = lane % G;
  unsigned char* mine = lds + g * kSlice;
  int* offs = reinterpret_cast<int*>(mine);      // CAP + 1
  int* bst = offs + CAP + 1;                     // CAP
  double* pv = reinterpret_cast<double*>(mine);  // CAP values (after the offsets are dead)
  KEY* keys = reinterpret_cast<KEY*>(mine + kValBytes);
  const int slot = blockIdx.x * RPW + g;
  const bool live = slot < nlist;
  const int i = live ? rows[slot] : 0;
  const int a0 = live ? arp[i] : 0, a1 = live ? arp[i + 1] : 0;
  const int la = a1 - a0;
  int run = 0;
  for (int base = 0; base < la; base += G) {
    const int e = base + ll;
    int len = 0, b0 = 0;
    if (e < la) {
      const int k = aci[a0 + e];
      b0 = brp[k];
      len = brp[k + 1] - b0;
    }
    int x = len;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
      const int y = __shfl_up(x, off, G);
      if (ll >= off) x += y;
    }
    if (e < la) {
      offs[e] = run + x - len;
      bst[e] = b0;
    }
    run += __shfl(x, G - 1, G);
  }
  if (ll == 0) offs[la] = run;
  const int nprod = run;
  const int nd = live && drp ? drp[i + 1] - drp[i] : 0;
  const int u = nprod + nd;
  int p2 = 1;
  while (p2 < u) p2 <<= 1;
  int top = 1;
  while (2 * top < la) top <<= 1;
  __syncthreads();
  int ent[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) ent[q] = 0;
  const int tlast = nprod - 1;
  for (int step = top; step > 0; step >>= 1) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = min(q * G + ll, tlast);
      const int c = ent[q] + step;
      if (c < la && offs[c] <= t) ent[q] = c;
    }
  }
  const int d0 = nd > 0 ? drp[i] : 0;
  int col[PER];
  double val[PER];
  if (u > 0) {
    double x[PER], a[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int t = q * G + ll;
      const bool fromb = nprod > 0 && (t < nprod || nd == 0);
      const int tb = min(t, tlast);
      const int idx = fromb ? bst[ent[q]] + (tb - offs[ent[q]]) : d0 + min(max(t - nprod, 0), nd - 1);
      const int* cp = fromb ? bci : dci;
      const double* vp = fromb ? bv : dv;
      col[q] = cp[idx];
      x[q] = vp[idx];
      a[q] = la > 0 ? av[a0 + ent[q]] : 1.0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) val[q] = q * G + ll < nprod ? a[q] * x[q] : x[q];
  }
  KEY kr[PER];
  __syncthreads();  // offsets and row starts are dead: values take their place
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = q * G + ll;
    kr[q] = t < u ? (static_cast<KEY>(static_cast<unsigned>(col[q])) << FK::kIdxBits) | KEY(t)
                  : ~KEY(0);
    if (t < u) pv[t] = val[q];
  }
  bitonic_group<G, PER>(kr, ll, p2);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int t = q * G + ll;
    if (t < p2) keys[t] = kr[q];
  }
  __syncthreads();
  // run sums: group lane ll takes the sorted elements [ll PER, (ll + 1) PER)
  const int t0 = ll * PER;
  int rc[PER];
  double rv[PER];
  bool rd[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    rc[q] = -1;
    rv[q] = 0.0;
    rd[q] = false;
    if (t0 + q < u) {
      const KEY k = keys[t0 + q];
      const int e = int(k & FK::kIdxMask);
      rc[q] = int(k >> FK::kIdxBits);
      rv[q] = pv[e];
      rd[q] = e >= nprod;
    }
  }
  const int cprev = (t0 > 0 && t0 < u) ? int(keys[t0 - 1] >> FK::kIdxBits) : -1;
  const int cnext = (t0 + PER < u) ? int(keys[t0 + PER] >> FK::kIdxBits) : -1;
  RunPart part{0, 0.0, 0.0};
  int heads = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (t0 + q >= u) break;
    if (rc[q] != (q ? rc[q - 1] : cprev)) {
      part = RunPart{1, 0.0, 0.0};
      ++heads;
    }
    if (rd[q]) part.d += rv[q];
    else part.s += rv[q];
  }
  int hx = heads;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    const int y = __shfl_up(hx, off, G);
    if (ll >= off) hx += y;
  }
  const int count = __shfl(hx, G - 1, G);
  hx -= heads;
  RunPart acc = run_scan_group<G>(part, ll);
  if (!live) return;
  const int64_t o = toff[i];
  int r = hx - 1;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (t0 + q >= u) break;
    if (rc[q] != (q ? rc[q - 1] : cprev)) {
      acc = RunPart{1, 0.0, 0.0};
      ++r;
    }
    if (rd[q]) acc.d += rv[q];
    else acc.s += rv[q];
    if (rc[q] != (q + 1 < PER ? rc[q + 1] : cnext)) {
      cci[o + r] = rc[q];
      cv[o + r] = beta * acc.d + alpha * acc.s;
    }
  }
  if (ll == 0) cnt[i] = count;
}

// numeric refresh on a known pattern: one wavefront per row
__global__ void __launch_bounds__(64) k_spgemm_values(
    int nrows, const int* __restrict__ arp, const int* __restrict__ aci,
    const double* __restrict__ av, const int* __restrict__ brp, const int* __restrict__ bci,
    const double* __restrict__ bv, const int* __restrict__ drp, const int* __restrict__ dci,
    const double* __restrict__ dv, double alpha, double beta, const int* __restrict__ crp,
    const int* __restrict__ cci, double* __restrict__ cv) {
  int i = blockIdx.x;
  if (i >= nrows) return;
  int a0 = arp[i], a1 = arp[i + 1];
  for (int t = crp[i] + threadIdx.x; t < crp[i + 1]; t += 64) {
    int col = cci[t];
    double sum = 0.0;
    for (int e = a0; e < a1; ++e) {
      int k = aci[e];
      int p = bsearch_col(bci, brp[k], brp[k + 1], col);
      if (p >= 0) sum += av[e] * bv[p];
    }
    double val = alpha * sum;
    if (drp) {
      int p = bsearch_col(dci, drp[i], drp[i + 1], col);
      if (p >= 0) val = beta * dv[p] + val;
    }
    cv[t] = val;
  }
}

__global__ void k_col_count(int nrows, const int* __restrict__ rp, const int* __restrict__ ci,
                            int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) atomicAdd(&cnt[ci[e]], 1);
}

__global__ void k_transpose_fill(int nrows, const int* __restrict__ rp, const int* __restrict__ ci,
                                 const double* __restrict__ v, int* __restrict__ cursor,
                                 int* __restrict__ tci, double* __restrict__ tv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    int pos = atomicAdd(&cursor[ci[e]], 1);
    tci[pos] = i;
    if (v) tv[pos] = v[e];
  }
}

// Ascending bitonic sort of keys[0, p2) (p2 a power of two, padded with
// INT_MAX) carrying vals along when given; all threads of the block take
// part.
template <int NT>
__device__ inline void bitonic_kv(int* keys, double* vals, int p2) {
  for (int k = 2; k <= p2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < p2; t += NT) {
        int q = t ^ j;
        if (q > t) {
          int x = keys[t], y = keys[q];
          bool up = (t & k) == 0;
          if ((x > y) == up) {
            keys[t] = y;
            keys[q] = x;
            if (vals) {
              double vx = vals[t];
              vals[t] = vals[q];
              vals[q] = vx;
            }
          }
        }
      }
      __syncthreads();
    }
}

// Sorts row i of (ci, v) by column with the NT threads of the block: rows of
// at most 64 entries by rank (the columns of a row are distinct, so an
// entry's position is the number of smaller columns), longer rows by a
// bitonic sort in LDS (CAP entries at most).
template <int NT, int CAP>
__device__ inline void sort_row(int a, int len, int* __restrict__ ci, double* __restrict__ v,
                                int* keys, double* vals) {
  for (int j = threadIdx.x; j < len; j += NT) {
    keys[j] = ci[a + j];
    if (v) vals[j] = v[a + j];
  }
  if (len <= 64) {
    __syncthreads();
    for (int j = threadIdx.x; j < len; j += NT) {
      int key = keys[j];
      int rank = 0;
      for (int m = 0; m < len; ++m) rank += keys[m] < key;
      ci[a + rank] = key;
      if (v) v[a + rank] = vals[j];
    }
    return;
  }
  int p2 = 1;
  while (p2 < len) p2 <<= 1;
  for (int j = len + threadIdx.x; j < p2; j += NT) keys[j] = INT_MAX;
  __syncthreads();
  bitonic_kv<NT>(keys, v ? vals : nullptr, p2);
  for (int j = threadIdx.x; j < len; j += NT) {
    ci[a + j] = keys[j];
    if (v) v[a + j] = vals[j];
  }
}

// Rows of at most kShortRow entries: kShortRow lanes per row, 256 / kShortRow
// rows per work-group; each lane takes one entry and finds its rank (the
// columns of a row are distinct) from the group's keys by shuffles, then
// writes it in place (all reads precede the writes in the wavefront).
// Longer rows are left to k_sort_mid_rows.
constexpr int kShortRow = 16;
__global__ void __launch_bounds__(256) k_sort_short_rows(int nrows, const int* __restrict__ rp,
                                                         int* __restrict__ ci,
                                                         double* __restrict__ v) {
  const int g = threadIdx.x / kShortRow, j = threadIdx.x % kShortRow;
  const int i = blockIdx.x * (256 / kShortRow) + g;
  int a = 0, len = 0;
  if (i < nrows) {
    a = rp[i];
    len = rp[i + 1] - a;
  }
  const bool mine = len > 1 && len <= kShortRow;
  int key = INT_MAX;
  double val = 0.0;
  if (mine && j < len) {
    key = ci[a + j];
    if (v) val = v[a + j];
  }
  const int base = threadIdx.x & 63 & ~(kShortRow - 1);
  int rank = 0;
#pragma unroll
  for (int m = 0; m < kShortRow; ++m) rank += __shfl(key, base + m, 64) < key;
  if (mine && j < len) {
    ci[a + rank] = key;
    if (v) v[a + rank] = val;
  }
}

// Rows of more than kShortRow entries, one wavefront per row.  Rows come in
// chunks of 64; a chunk's long rows are found by a ballot over their lengths
// (a queue filled by the short-row kernel would take one same-address atomic
// per work-group there) and dealt to `sub` work-groups in turn, so small
// matrices with many long rows still spread over the chip.  Work-groups
// stride over the (chunk, share) pairs.  Rows longer than kSortCap are
// queued for k_sort_long_rows.
constexpr int kSortCap = 1024;
constexpr int kSortMidGroups = 4096;  // work-groups of k_sort_mid_rows at most
__global__ void __launch_bounds__(64) k_sort_mid_rows(int nrows, int sub, const int* __restrict__ rp,
                                                      int* __restrict__ ci, double* __restrict__ v,
                                                      int* __restrict__ nlong,
                                                      int* __restrict__ long_rows) {
  __shared__ int keys[kSortCap];
  __shared__ double vals[kSortCap];
  const int64_t total = int64_t((nrows + 63) / 64) * sub;
  for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
    const int base = int(g / sub) * 64, share = int(g % sub);
    const int r = base + int(threadIdx.x);
    const int rlen = r < nrows ? rp[r + 1] - rp[r] : 0;
    unsigned long long b = __ballot(rlen > kShortRow);
    for (int k = 0; b; ++k) {
      const int i = base + __ffsll(b) - 1;
      b &= b - 1;
      if (k % sub != share) continue;
      const int a = rp[i], len = rp[i + 1] - a;
      if (len > kSortCap) {
        if (threadIdx.x == 0) long_rows[atomicAdd(nlong, 1)] = i;
      } else {
        sort_row<64, kSortCap>(a, len, ci, v, keys, vals);
      }
      __syncthreads();
    }
  }
}

// The queued long rows, one 256-thread work-group per row (bitonic sort in
// LDS up to kSortLongCap entries, else an insertion sort by one thread).  The
// work-groups stride over the queue, whose length they read.
constexpr int kSortLongCap = 4096;
constexpr int kSortLongGroups = 512;  // two per CU (48 KiB of LDS each)
__global__ void __launch_bounds__(256) k_sort_long_rows(const int* __restrict__ nlong,
                                                         const int* __restrict__ long_rows,
                                                         const int* __restrict__ rp,
                                                         int* __restrict__ ci,
                                                         double* __restrict__ v) {
  __shared__ int keys[kSortLongCap];
  __shared__ double vals[kSortLongCap];
  const int cnt = *nlong;
  for (int q = blockIdx.x; q < cnt; q += gridDim.x) {
    const int i = long_rows[q];
    const int a = rp[i], len = rp[i + 1] - a;
    if (len > kSortLongCap) {
      if (threadIdx.x == 0) {
        for (int e = a + 1; e < a + len; ++e) {
          int key = ci[e];
          double val = v ? v[e] : 0.0;
          int f = e - 1;
          while (f >= a && ci[f] > key) {
            ci[f + 1] = ci[f];
            if (v) v[f + 1] = v[f];
            --f;
          }
          ci[f + 1] = key;
          if (v) v[f + 1] = val;
        }
      }
    } else {
      sort_row<256, kSortLongCap>(a, len, ci, v, keys, vals);
    }
    __syncthreads();
  }
}

// Flags (bad = 1) a CSR matrix whose row pointers are not a non-decreasing
// sequence from 0 to nnz or whose rows are not strictly increasing column
// lists within [0, ncols).
__global__ void k_csr_check(int nrows, int ncols, int64_t nnz, const int* __restrict__ rp,
                            const int* __restrict__ ci, int* __restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  int64_t a = rp[i], b = rp[i + 1];
  bool ok = 0 <= a && a <= b && b <= nnz && (i > 0 || a == 0) && (i < nrows - 1 || b == nnz);
  if (ok)
    for (int64_t e = a; e < b; ++e) {
      int c = ci[e];
      if (c < 0 || c >= ncols || (e > a && ci[e - 1] >= c)) {
        ok = false;
        break;
      }
    }
  if (!ok) atomicOr(bad, 1);
}

}  // namespace

void spgemm(const CsrRef<double>& A, const CsrRef<double>& B, Csr<double>& C, hipStream_t s,
            const CsrRef<double>* D, double alpha, double beta, bool reuse, int first_class) {
  TPF_REQUIRE(A.ncols == B.nrows, TPF_ERR_INVALID_ARG, "spgemm: inner dimensions differ (%d vs %d)",
              A.ncols, B.nrows);
  if (D)
    TPF_REQUIRE(D->nrows == A.nrows && D->ncols == B.ncols, TPF_ERR_INVALID_ARG,
                "spgemm: added matrix has the wrong shape");
  int n = A.nrows;
  const int* drp = D ? D->rp : nullptr;
  const int* dci = D ? D->ci : nullptr;
  const double* dv = D ? D->v : nullptr;
  if (reuse) {
    TPF_REQUIRE(C.nrows == n && C.ncols == B.ncols && C.rp.p, TPF_ERR_STATE,
                "spgemm reuse: product pattern missing");
    if (n > 0) {
      k_spgemm_values<<<n, 64, 0, s>>>(n, A.rp, A.ci, A.v, B.rp, B.ci, B.v, drp, dci, dv, alpha,
                                       beta, C.rp.p, C.ci.p, C.v.p);
      TPF_CHECK_LAUNCH();
    }
    return;
  }
  C.nrows = n;
  C.ncols = B.ncols;
  C.rp.alloc(n + 1, s);
  if (n == 0) {
    C.nnz = scan_exclusive(nullptr, C.rp.p, 0, s);
    C.ci.alloc(1, s);
    C.v.alloc(1, s);
    return;
  }
  // caps ascending: flat<64,CAP> wavefront kernels (CAP 64 .. 1024), flat<256,2048>,
  // flat<512,8192> (A rows of at most 2048), sorted<256,16384>; beyond, the per-thread merge
  const Caps caps{{64, 128, 256, 512, 1024, 2048, 8192, 16384},
                  {64, 128, 256, 512, 1024, 2048, 2048, 16384}};
  Buf<int> ub(n, s), counts(kClasses, s), lists(kClasses * int64_t(n), s), cnt(n, s);
  fill_int(counts.p, 0, kClasses, s);
  {
    const int lpr = lanes_per_row(n, A.nnz);
    DISPATCH_LPR(lpr, LL, {
      k_spgemm_ub<LL><<<grid_for(int64_t(n) * LL, 256), 256, 0, s>>>(n, A.rp, A.ci, B.rp, drp,
                                                                     ub.p);
    });
    TPF_CHECK_LAUNCH();
  }
  k_spgemm_classify<<<grid_for(n, 256 * kClassifyRows), 256, 0, s>>>(n, ub.p, A.rp, caps, first_class, counts.p,
                                                      lists.p);
  TPF_CHECK_LAUNCH();
  // one pass: each row writes its sorted unique entries at its upper-bound
  // offset in a staging area, then the rows are packed
  Buf<int64_t> toff(size_t(n) + 1, s);
  int* hc_pinned = host_counts_slot();
  TPF_HIP(hipMemcpyAsync(hc_pinned, counts.p, kClasses * sizeof(int), hipMemcpyDeviceToHost, s));
  int64_t staged = scan_exclusive_wide(ub.p, toff.p, n, s);  // synchronises: counts arrived
  int hc[kClasses];
  std::memcpy(hc, hc_pinned, sizeof(hc));
  Buf<int> tci(staged > 0 ? size_t(staged) : 1, s);
  Buf<double> tv(staged > 0 ? size_t(staged) : 1, s);
  Buf<int2> cur;
  if (hc[kClasses - 1] > 0) cur.alloc(A.nnz > 0 ? A.nnz : 1, s);
  auto list = [&](int c) { return lists.p + int64_t(c) * n; };
  // The classes of long rows (work-groups of 256 threads and more, and the
  // per-thread merge) have few rows that each take long, leaving most of
  // the chip idle: they run on the side stream, beside the wavefront classes.
  int nshort = 0, nlong = 0;
  for (int c = 0; c < kClasses; ++c) (c < 5 ? nshort : nlong) += hc[c];
  SideFork fork(s, nshort > 0 && nlong > 0);
  const hipStream_t ls = fork.side;
  // 32-bit keys when the column count leaves room for the product index
  auto flat = [&](auto block_tag, auto cap_tag, auto la_tag, int c) {
    constexpr int BL = decltype(block_tag)::value, CP = decltype(cap_tag)::value;
    constexpr int LC = decltype(la_tag)::value;
    if (hc[c] == 0) return;
    const hipStream_t st = c < 5 ? s : ls;
    if (int64_t(B.ncols) < (int64_t(1) << (32 - __builtin_ctz(CP))))
      k_spgemm_flat<BL, CP, uint32_t, LC><<<hc[c], BL, 0, st>>>(
          list(c), ub.p, A.rp, A.ci, A.v, B.rp, B.ci, B.v, drp, dci, dv, alpha, beta, cnt.p, toff.p,
          tci.p, tv.p);
    else
      k_spgemm_flat<BL, CP, uint64_t, LC><<<hc[c], BL, 0, st>>>(
          list(c), ub.p, A.rp, A.ci, A.v, B.rp, B.ci, B.v, drp, dci, dv, alpha, beta, cnt.p, toff.p,
          tci.p, tv.p);
  };
  using W1 = std::integral_constant<int, 64>;
  using W4 = std::integral_constant<int, 256>;
  using W8 = std::integral_constant<int, 512>;
  using C512 = std::integral_constant<int, 512>;
  using C1024 = std::integral_constant<int, 1024>;
  using C2048 = std::integral_constant<int, 2048>;
  using C8192 = std::integral_constant<int, 8192>;
  // the three smallest classes: lane groups, four (16 lanes) or two (32) rows per wavefront
  auto group = [&](auto g_tag, auto per_tag, int c) {
    constexpr int G = decltype(g_tag)::value, PER = decltype(per_tag)::value, CP = G * PER;
    if (hc[c] == 0) return;
    const unsigned grid = grid_for(hc[c], 64 / G);
    if (int64_t(B.ncols) < (int64_t(1) << (32 - __builtin_ctz(CP))))
      k_spgemm_group<G, PER, uint32_t><<<grid, 64, 0, s>>>(
          hc[c], list(c), A.rp, A.ci, A.v, B.rp, B.ci, B.v, drp, dci, dv, alpha, beta, cnt.p,
          toff.p, tci.p, tv.p);
    else
      k_spgemm_group<G, PER, uint64_t><<<grid, 64, 0, s>>>(
          hc[c], list(c), A.rp, A.ci, A.v, B.rp, B.ci, B.v, drp, dci, dv, alpha, beta, cnt.p,
          toff.p, tci.p, tv.p);
  };
  using G16 = std::integral_constant<int, 16>;
  using G32 = std::integral_constant<int, 32>;
  // long-row classes first (side stream), then the wavefront classes
  flat(W8{}, C8192{}, C2048{}, 6);
  if (hc[7] > 0)
    k_spgemm_sorted<256, 16384, true><<<hc[7], 256, 0, ls>>>(list(7), ub.p, A.rp, A.ci, A.v, B.rp,
                                                             B.ci, B.v, drp, dci, dv, alpha, beta,
                                                             cnt.p, toff.p, tci.p, tv.p);
  if (hc[8] > 0)
    k_spgemm_merge<true><<<grid_for(hc[8], 128), 128, 0, ls>>>(
        hc[8], list(8), A.rp, A.ci, A.v, B.rp, B.ci, B.v, drp, dci, dv, alpha, beta, cur.p, cnt.p,
        toff.p, tci.p, tv.p);
  flat(W4{}, C2048{}, C2048{}, 5);
  group(G16{}, std::integral_constant<int, 4>{}, 0);
  group(G16{}, std::integral_constant<int, 8>{}, 1);
  group(G32{}, std::integral_constant<int, 8>{}, 2);
  flat(W1{}, C512{}, C512{}, 3);
  flat(W1{}, C1024{}, C1024{}, 4);
  TPF_CHECK_LAUNCH();
  fork.join();
  C.nnz = scan_exclusive(cnt.p, C.rp.p, n, s);
  C.ci.alloc(C.nnz > 0 ? C.nnz : 1, s);
  C.v.alloc(C.nnz > 0 ? C.nnz : 1, s);
  pack_rows(n, toff.p, C.rp.p, C.nnz, tci.p, tv.p, C.ci.p, C.v.p, s);
}

void transpose(const CsrRef<double>& A, Csr<double>& C, hipStream_t s) {
  int m = A.ncols;
  C.nrows = m;
  C.ncols = A.nrows;
  C.nnz = A.nnz;
  Buf<int> cnt(m > 0 ? m : 1, s);
  fill_int(cnt.p, 0, m, s);
  if (A.nrows > 0) {
    k_col_count<<<grid_for(A.nrows, 256), 256, 0, s>>>(A.nrows, A.rp, A.ci, cnt.p);
    TPF_CHECK_LAUNCH();
  }
  C.rp.alloc(m + 1, s);
  // the counts add up to A.nnz (columns of A lie in [0, m)): no read-back
  scan_exclusive_async(cnt.p, C.rp.p, m, s);
  C.ci.alloc(A.nnz > 0 ? A.nnz : 1, s);
  if (A.v)
    C.v.alloc(A.nnz > 0 ? A.nnz : 1, s);
  else
    C.v.release();
  copy(cnt.p, C.rp.p, m, s);  // cursors start at the row starts
  if (A.nrows > 0) {
    k_transpose_fill<<<grid_for(A.nrows, 256), 256, 0, s>>>(A.nrows, A.rp, A.ci, A.v, cnt.p,
                                                           C.ci.p, C.v.p);
    TPF_CHECK_LAUNCH();
  }
  if (m > 0) {
    Buf<int> nlong(1, s), long_rows(m, s);
    fill_int(nlong.p, 0, 1, s);
    k_sort_short_rows<<<grid_for(m, 256 / kShortRow), 256, 0, s>>>(m, C.rp.p, C.ci.p, C.v.p);
    TPF_CHECK_LAUNCH();
    const int64_t chunks = (int64_t(m) + 63) / 64;
    const int sub = int(std::max<int64_t>(1, std::min<int64_t>(64, kSortMidGroups / chunks)));
    const int mid_grid = int(std::min<int64_t>(chunks * sub, kSortMidGroups));
    k_sort_mid_rows<<<mid_grid, 64, 0, s>>>(m, sub, C.rp.p, C.ci.p, C.v.p, nlong.p, long_rows.p);
    TPF_CHECK_LAUNCH();
    k_sort_long_rows<<<kSortLongGroups, 256, 0, s>>>(nlong.p, long_rows.p, C.rp.p, C.ci.p, C.v.p);
    TPF_CHECK_LAUNCH();
  }
}

// Checks a caller's CSR matrix (see k_csr_check); synchronises the stream.
static void check_csr(const CsrRef<double>& M, const char* name, hipStream_t s) {
  TPF_REQUIRE(M.nrows >= 0 && M.ncols >= 0 && M.nnz >= 0 && M.rp && (M.nnz == 0 || M.ci),
              TPF_ERR_INVALID_ARG, "tpf_csr_product: %s has invalid sizes or pointers", name);
  TPF_REQUIRE(M.nnz <= INT_MAX, TPF_ERR_INVALID_ARG, "tpf_csr_product: %s has more than 2^31 entries",
              name);
  Buf<int> bad(1, s);
  fill_int(bad.p, 0, 1, s);
  if (M.nrows > 0) {
    k_csr_check<<<grid_for(M.nrows, 256), 256, 0, s>>>(M.nrows, M.ncols, M.nnz, M.rp, M.ci, bad.p);
    TPF_CHECK_LAUNCH();
  }
  TPF_REQUIRE(read_scalar(bad.p, s) == 0, TPF_ERR_INVALID_ARG,
              "tpf_csr_product: %s is not a CSR matrix with sorted, in-range columns", name);
}

}  // namespace tpf

extern "C" int tpf_csr_transpose(const tpf_csr_view* A, int* c_row_ptr, int* c_col_idx,
                                 double* c_vals, void* stream) {
  using namespace tpf;
  return guarded([&] {
    TPF_REQUIRE(A && c_row_ptr && (A->nnz == 0 || (c_col_idx && (c_vals || !A->vals))),
                TPF_ERR_INVALID_ARG, "tpf_csr_transpose: null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const CsrRef<double> a{A->n_rows, A->n_cols, A->nnz, A->row_ptr, A->col_idx, A->vals};
    check_csr(a, "A", s);
    Csr<double> C;
    transpose(a, C, s);
    copy(c_row_ptr, C.rp.p, int64_t(a.ncols) + 1, s);
    if (a.nnz > 0) {
      copy(c_col_idx, C.ci.p, a.nnz, s);
      if (a.v) copy(c_vals, C.v.p, a.nnz, s);
    }
    TPF_HIP(hipStreamSynchronize(s));
  });
}

extern "C" int tpf_csr_product(const tpf_csr_view* A, const tpf_csr_view* B,
                               const tpf_csr_view* D, double alpha, double beta, int route,
                               int pattern_given, int* c_row_ptr, int* c_col_idx, double* c_vals,
                               int64_t c_cap, int64_t* c_nnz, void* stream) {
  using namespace tpf;
  return guarded([&] {
    TPF_REQUIRE(A && B && c_row_ptr && c_nnz, TPF_ERR_INVALID_ARG, "tpf_csr_product: null argument");
    TPF_REQUIRE((A->vals || A->nnz == 0) && (B->vals || B->nnz == 0) &&
                    (!D || D->vals || D->nnz == 0),
                TPF_ERR_INVALID_ARG, "tpf_csr_product: values are required");
    TPF_REQUIRE(route >= 0 && route <= kClasses, TPF_ERR_INVALID_ARG,
                "tpf_csr_product: route %d outside [0, %d]", route, kClasses);
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto view = [](const tpf_csr_view* v) {
      return CsrRef<double>{v->n_rows, v->n_cols, v->nnz, v->row_ptr, v->col_idx, v->vals};
    };
    const CsrRef<double> a = view(A), b = view(B);
    CsrRef<double> d;
    check_csr(a, "A", s);
    check_csr(b, "B", s);
    if (D) {
      d = view(D);
      check_csr(d, "D", s);
    }
    TPF_REQUIRE(a.ncols == b.nrows, TPF_ERR_INVALID_ARG,
                "tpf_csr_product: inner dimensions differ (%d vs %d)", a.ncols, b.nrows);
    const int n = a.nrows;
    Csr<double> C;
    if (pattern_given) {
      TPF_REQUIRE(c_col_idx && c_vals, TPF_ERR_INVALID_ARG, "tpf_csr_product: pattern missing");
      const CsrRef<double> cp{n, b.ncols, 0, c_row_ptr, c_col_idx, nullptr};
      int64_t nnz = read_scalar(c_row_ptr + n, s);
      TPF_REQUIRE(nnz >= 0 && nnz <= c_cap, TPF_ERR_INVALID_ARG,
                  "tpf_csr_product: pattern has %lld entries, capacity %lld", (long long)nnz,
                  (long long)c_cap);
      check_csr(CsrRef<double>{cp.nrows, cp.ncols, nnz, cp.rp, cp.ci, nullptr}, "C", s);
      C.nrows = n;
      C.ncols = b.ncols;
      C.nnz = nnz;
      C.rp.alloc(n + 1, s);
      copy(C.rp.p, c_row_ptr, n + 1, s);
      C.ci.alloc(nnz > 0 ? nnz : 1, s);
      copy(C.ci.p, c_col_idx, nnz, s);
      C.v.alloc(nnz > 0 ? nnz : 1, s);
      spgemm(a, b, C, s, D ? &d : nullptr, alpha, beta, true);
      copy(c_vals, C.v.p, nnz, s);
      *c_nnz = nnz;
    } else {
      spgemm(a, b, C, s, D ? &d : nullptr, alpha, beta, false, route > 0 ? route - 1 : 0);
      copy(c_row_ptr, C.rp.p, n + 1, s);
      *c_nnz = C.nnz;
      if (C.nnz <= c_cap && c_col_idx && c_vals) {
        copy(c_col_idx, C.ci.p, C.nnz, s);
        copy(c_vals, C.v.p, C.nnz, s);
      }
    }
    TPF_HIP(hipStreamSynchronize(s));
  });
}
