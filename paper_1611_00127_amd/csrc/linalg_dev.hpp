// Device-side helpers: wavefront (64-lane) and block reductions/scans and
// the CSR row-dot with a power-of-two lane group per row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tpf {

constexpr int kWave = 64;

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  return v;  // valid in lane 0
}

// Sum over a block of BLOCK threads (BLOCK a multiple of 64); fixed order,
// result valid in thread 0.  sh needs BLOCK/64 entries.
template <int BLOCK, class T>
__device__ inline T block_sum(T v, T* sh) {
  v = wave_sum(v);
  int lane = threadIdx.x & (kWave - 1);
  int wid = threadIdx.x / kWave;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T acc = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < BLOCK / kWave; ++w) acc += sh[w];
  }
  __syncthreads();
  return acc;
}

// Exclusive scan over a block; `total` receives the block sum in every
// thread.  sh needs BLOCK/64 + 1 entries.
template <class T, int BLOCK>
__device__ inline T block_exclusive_scan(T v, T* sh, T& total) {
  int lane = threadIdx.x & (kWave - 1);
  int wid = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) sh[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int w = 0; w < BLOCK / kWave; ++w) {
      T t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[BLOCK / kWave] = acc;
  }
  __syncthreads();
  T excl = x - v + sh[wid];
  total = sh[BLOCK / kWave];
  __syncthreads();
  return excl;
}

// Dot of CSR row `row` with gathered values g(col); LPR consecutive lanes
// share the row, each lane summing entries lane, lane + LPR, ... in order
// (loads issued eight entries at a time); result valid in the group's first lane.
template <class T, int LPR, class G>
__device__ inline T row_dot(int row, int lane, const int* __restrict__ rp,
                            const int* __restrict__ ci, const T* __restrict__ v, G g) {
  T sum = T(0);
  const int e1 = rp[row + 1];
  int e = rp[row] + lane;
  // eight entries per lane at a time: every position clamped to the row's
  // last entry, so all loads are valid and issued before the first wait;
  // positions past the row add nothing (the sums keep the entry order)
  constexpr int B = 8;
  for (; e < e1; e += B * LPR) {
    int c[B];
    T a[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int f = min(e + u * LPR, e1 - 1);
      c[u] = ci[f];
      a[u] = v[f];
    }
    T x[B];
#pragma unroll
    for (int u = 0; u < B; ++u) x[u] = g(c[u]);
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (e + u * LPR < e1) sum += a[u] * x[u];
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) sum += __shfl_down(sum, off, LPR);
  return sum;
}

// Sorts rows into lists by class: a work-group of BLOCK threads takes R*BLOCK
// consecutive rows (row base + r * BLOCK + threadIdx.x at step r), class_of(i)
// gives row i's list (< 0: none), and each list receives one atomic per
// work-group.  Same-address atomics serialise, so fewer, larger work-groups
// append faster than one per BLOCK rows.  Launch with
// ceil(n / (R * BLOCK)) work-groups; order inside a list is not specified.
constexpr int kClassifyRows = 8;  // R of the row classifiers
template <int NL, int BLOCK, int R, class ClassOf>
__device__ inline void block_append_rows(int n, ClassOf class_of, int stride, int* counts,
                                         int* lists) {
  __shared__ int wcnt[BLOCK / kWave][NL];
  __shared__ int base[NL];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t i0 = int64_t(blockIdx.x) * (BLOCK * R) + threadIdx.x;
  int cls[R], off[R], run[NL];
#pragma unroll
  for (int c = 0; c < NL; ++c) run[c] = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = i0 + int64_t(r) * BLOCK;
    cls[r] = i < n ? class_of(int(i)) : -1;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    off[r] = 0;
#pragma unroll
    for (int c = 0; c < NL; ++c) {
      const unsigned long long b = __ballot(cls[r] == c);
      if (cls[r] == c) off[r] = run[c] + __popcll(b & below);
      run[c] += __popcll(b);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NL; ++c) wcnt[w][c] = run[c];
  }
  __syncthreads();
  if (threadIdx.x < NL) {
    const int c = threadIdx.x;
    int tot = 0;
    for (int ww = 0; ww < BLOCK / kWave; ++ww) {
      const int t = wcnt[ww][c];
      wcnt[ww][c] = tot;
      tot += t;
    }
    base[c] = tot ? atomicAdd(&counts[c], tot) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (cls[r] >= 0)
      lists[int64_t(cls[r]) * stride + base[cls[r]] + wcnt[w][cls[r]] + off[r]] =
          int(i0 + int64_t(r) * BLOCK);
}

// Sum / max over a group of LPR consecutive lanes (xor butterfly: every lane
// of the group ends with the same bits).
template <int LPR, class T>
__device__ inline T group_sum(T v) {
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LPR);
  return v;
}
template <int LPR>
__device__ inline double group_max(double v) {
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, LPR));
  return v;
}

// Bits of the calling lane's LPR-lane group in a wavefront ballot.
template <int LPR>
__device__ inline unsigned long long group_ballot(bool f) {
  unsigned long long b = __ballot(f);
  if constexpr (LPR == 64) {
    return b;
  } else {
    int base = (threadIdx.x & (kWave - 1)) & ~(LPR - 1);
    return (b >> base) & ((1ull << LPR) - 1ull);
  }
}

// Lanes per row for the CSR row kernels: about eight entries per lane
// (measured against two, four, sixteen: the FP64 step is fastest at eight).
// Ascending bitonic sort of p2 keys (a power of two) held in registers:
// element t = wbase + 64 q + lane sits in register q of lane `lane` of the
// wavefront whose first element is wbase (wbase a multiple of 64 PER).
// Exchanges at distance 64 .. 32 PER stay inside a lane, shorter ones go
// through shuffles and longer ones (several wavefronts) through `lds`, which
// must hold 64 PER entries per wavefront of the block.  All threads of the
// block must call it.
template <int QJ, int PER, class KEY>
__device__ inline void bitonic_in_lane(KEY (&kr)[PER], int base, int kk) {
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if ((q & QJ) == 0 && (q | QJ) < PER) {
      const int qp = q | QJ;
      const bool up = ((base + q * 64) & kk) == 0;
      const KEY x = kr[q], y = kr[qp];
      const bool sw = (x > y) == up;
      kr[q] = sw ? y : x;
      kr[qp] = sw ? x : y;
    }
  }
}

template <int PER, class KEY>
__device__ inline void bitonic_regs(KEY (&kr)[PER], int wbase, int lane, int p2, KEY* lds) {
  for (int kk = 2; kk <= p2; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j >= 64 * PER) {
#pragma unroll
        for (int q = 0; q < PER; ++q) lds[wbase + q * 64 + lane] = kr[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int t = wbase + q * 64 + lane;
          const KEY x = kr[q], y = lds[t ^ j];
          const bool up = (t & kk) == 0, lower = (t & j) == 0;
          const KEY mn = x < y ? x : y, mx = x < y ? y : x;
          kr[q] = lower == up ? mn : mx;
        }
        __syncthreads();
      } else if (j >= 64) {
        switch (j >> 6) {
          case 1: bitonic_in_lane<1>(kr, wbase + lane, kk); break;
          case 2: bitonic_in_lane<2>(kr, wbase + lane, kk); break;
          case 4: bitonic_in_lane<4>(kr, wbase + lane, kk); break;
          default: bitonic_in_lane<8>(kr, wbase + lane, kk); break;
        }
      } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int t = wbase + q * 64 + lane;
          const KEY x = kr[q];
          const KEY y = __shfl_xor(x, j, 64);
          const bool up = (t & kk) == 0, lower = (lane & j) == 0;
          const KEY mn = x < y ? x : y, mx = x < y ? y : x;
          kr[q] = lower == up ? mn : mx;
        }
      }
    }
}

inline int lanes_per_row(int64_t nrows, int64_t nnz) {
  double avg = nrows ? double(nnz) / double(nrows) : 1.0;
  int l = 1;
  while (l < 64 && 8 * l < avg) l <<= 1;
  return l;
}

}  // namespace tpf

#define DISPATCH_LPR(lpr, L, ...)                     \
  switch (lpr) {                                      \
    case 1: { constexpr int L = 1; __VA_ARGS__ } break;   \
    case 2: { constexpr int L = 2; __VA_ARGS__ } break;   \
    case 4: { constexpr int L = 4; __VA_ARGS__ } break;   \
    case 8: { constexpr int L = 8; __VA_ARGS__ } break;   \
    case 16: { constexpr int L = 16; __VA_ARGS__ } break; \
    case 32: { constexpr int L = 32; __VA_ARGS__ } break; \
    default: { constexpr int L = 64; __VA_ARGS__ } break; \
  }
