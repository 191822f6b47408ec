// Classical AMG on the device: strength of connection, PMIS coarsening,
// direct interpolation, Galerkin coarse operators, dense coarsest inverse,
// and the V(1,1) cycle with l1-Jacobi smoothing.  The paper applies one
// AMG V-cycle per inner solve (Sec. 3.2-3.4; solver settings in Sec. 4.1)
// using BoomerAMG; the components here are data-parallel replacements whose
// definitions are:
//   strength  s_i = sign(a_ii) (+1 if a_ii >= 0), m_i = max_{k!=i} -s_i a_ik,
//             j strong for i iff m_i > 0 and -s_i a_ij >= theta m_i;
//   PMIS      w_i = |S^T_i| + (splitmix64(seed ^ i) >> 40) 2^-24; |S^T_i| = 0
//             starts F; per round an undecided i becomes C iff (w_i, i) beats
//             every undecided j in S_i u S^T_i, then undecided j with a new C
//             point in S_j become F;
//   direct interpolation (Stueben): w_ij = -alpha_i a_ij / a~_ii over the
//             strong C neighbours, alpha_i = sum_{k!=i} a_ik^- / sum_{P_i} a_ik^-,
//             a~_ii = a_ii + same-signed off-diagonals; C rows inject;
//   Galerkin  A_c = R (A P), R = P^T, symbolic pattern;
//   smoother  l1-Jacobi d_i = a_ii + s_i sum_{j!=i} |a_ij|.
#include <climits>
#include <cmath>
#include <type_traits>

#include "amg.hpp"
#include "linalg_dev.hpp"

namespace tpf {

namespace {
constexpr int8_t kUndecided = 0, kC = 1, kF = 2;

__device__ inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline double row_diag(int i, int a0, int a1, const int* ci, const double* v) {
  for (int e = a0; e < a1; ++e)
    if (ci[e] == i) return v[e];
  return 0.0;
}

// l1 diagonal d_i = a_ii + s_i sum_{j != i} |a_ij| (s_i = sign a_ii), inverted
// (0 for a zero row sum); LPR lanes per row
template <int LPR>
__global__ void __launch_bounds__(256) k_l1_dinv(int n, const int* __restrict__ rp,
                                                 const int* __restrict__ ci,
                                                 const double* __restrict__ v,
                                                 double* __restrict__ dinv) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  double dg = 0.0, off = 0.0;
  if (i < n)
    for (int e = rp[i] + lane; e < rp[i + 1]; e += LPR) {
      if (ci[e] == i) dg += v[e];
      else off += fabs(v[e]);
    }
  dg = group_sum<LPR>(dg);
  off = group_sum<LPR>(off);
  if (i < n && lane == 0) {
    double s = dg < 0.0 ? -1.0 : 1.0;
    double d = dg + s * off;
    dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
  }
}

// classical strength: j strongly influences i iff -s_i a_ij >= theta max_k(-s_i a_ik)
// (off-diagonal), with a positive maximum; LPR lanes per row
template <int LPR>
__global__ void __launch_bounds__(256) k_strength(int n, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const double* __restrict__ v, double theta,
                                                  uint8_t* __restrict__ mask,
                                                  int* __restrict__ cnt) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  int a0 = 0, a1 = 0;
  if (i < n) {
    a0 = rp[i];
    a1 = rp[i + 1];
  }
  // rows of at most kB entries per lane keep them in registers for both
  // passes (loads at clamped positions, all issued before the first wait)
  constexpr int kB = 8;
  const bool inreg = a1 - a0 <= kB * LPR;
  int cr[kB];
  double vr[kB];
  if (inreg) {
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int e = min(a0 + lane + u * LPR, a1 - 1);
      cr[u] = a1 > a0 ? ci[e] : i;
      vr[u] = a1 > a0 ? v[e] : 0.0;
    }
  }
  double dg = 0.0, mpos = -INFINITY, mneg = -INFINITY;
  if (inreg) {
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      if (a0 + lane + u * LPR >= a1) break;
      if (cr[u] == i) {
        dg += vr[u];
      } else {
        mpos = fmax(mpos, vr[u]);
        mneg = fmax(mneg, -vr[u]);
      }
    }
  } else {
    for (int e = a0 + lane; e < a1; e += LPR) {
      double x = v[e];
      if (ci[e] == i) {
        dg += x;
      } else {
        mpos = fmax(mpos, x);
        mneg = fmax(mneg, -x);
      }
    }
  }
  dg = group_sum<LPR>(dg);
  mpos = group_max<LPR>(mpos);
  mneg = group_max<LPR>(mneg);
  double s = dg < 0.0 ? -1.0 : 1.0;
  double m = dg < 0.0 ? mpos : mneg;  // max of -s a_ij
  double thr = theta * m;
  int c = 0;
  if (inreg) {
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int e = a0 + lane + u * LPR;
      if (e >= a1) break;
      const bool st = cr[u] != i && m > 0.0 && (-s * vr[u]) >= thr;
      mask[e] = st;
      c += st;
    }
  } else {
    for (int e = a0 + lane; e < a1; e += LPR) {
      bool st = ci[e] != i && m > 0.0 && (-s * v[e]) >= thr;
      mask[e] = st;
      c += st;
    }
  }
  c = group_sum<LPR>(c);
  if (i < n && lane == 0) cnt[i] = c;
}

// strong columns of each row, in row order (LPR lanes per row)
template <int LPR>
__global__ void __launch_bounds__(256) k_compact_pattern(int n, const int* __restrict__ rp,
                                                         const int* __restrict__ ci,
                                                         const uint8_t* __restrict__ mask,
                                                         const int* __restrict__ srp,
                                                         int* __restrict__ sci) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  int a0 = 0, a1 = 0, o = 0;
  if (i < n) {
    a0 = rp[i];
    a1 = rp[i + 1];
    o = srp[i];
  }
  for (int base = a0; base < a1; base += LPR) {
    int e = base + lane;
    bool f = e < a1 && mask[e];
    unsigned long long g = group_ballot<LPR>(f);
    if (f) sci[o + __popcll(g & ((1ull << lane) - 1ull))] = ci[e];
    o += __popcll(g);
  }
}

__global__ void k_pmis_init(int n, uint64_t seed, const int* __restrict__ strp,
                            double* __restrict__ w, int8_t* __restrict__ state) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int nst = strp[i + 1] - strp[i];
  uint64_t z = splitmix64(seed ^ uint64_t(i));
  double u = double(z >> 40) * 0x1p-24;
  w[i] = double(nst) + u;
  state[i] = nst == 0 ? kF : kUndecided;
}

__device__ inline bool beats(double wj, int j, double wi, int i) {
  return wj > wi || (wj == wi && j > i);
}

__global__ void k_pmis_select(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                              const int* __restrict__ strp, const int* __restrict__ stci,
                              const double* __restrict__ w, const int8_t* __restrict__ state,
                              uint8_t* __restrict__ newc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] != kUndecided) {
    newc[i] = 0;
    return;
  }
  double wi = w[i];
  bool sel = true;
  for (int e = srp[i]; e < srp[i + 1] && sel; ++e) {
    int j = sci[e];
    if (state[j] == kUndecided && beats(w[j], j, wi, i)) sel = false;
  }
  for (int e = strp[i]; e < strp[i + 1] && sel; ++e) {
    int j = stci[e];
    if (state[j] == kUndecided && beats(w[j], j, wi, i)) sel = false;
  }
  newc[i] = sel;
}

// `undecided` is set to 1 (plain stores, all of the same value) when a point
// stays undecided.  A count would take one same-address atomic per wavefront,
// and those serialise: on a million points they cost more than the round.
__global__ void k_pmis_update(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                              const uint8_t* __restrict__ newc, int8_t* __restrict__ state,
                              int* __restrict__ undecided) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool und = false;
  if (i < n && state[i] == kUndecided) {
    if (newc[i]) {
      state[i] = kC;
    } else {
      bool f = false;
      for (int e = srp[i]; e < srp[i + 1]; ++e)
        if (newc[sci[e]]) {
          f = true;
          break;
        }
      if (f)
        state[i] = kF;
      else
        und = true;
    }
  }
  if (__ballot(und) && (threadIdx.x & 63) == 0) *undecided = 1;
}

// All PMIS rounds of a small level in one work-group (the same select and
// update steps as the two kernels above, with block barriers between them);
// rounds[0] receives the number of rounds, or -1 if n + 1 rounds left
// points undecided.
constexpr int kPmisWg = 1024;
constexpr int kPmisWgMax = 4096;  // levels up to this size use it (on larger ones a
                                  // kernel pair per round and a host check is faster)
__global__ void __launch_bounds__(kPmisWg) k_pmis_block(
    int n, const int* __restrict__ srp, const int* __restrict__ sci,
    const int* __restrict__ strp, const int* __restrict__ stci, const double* __restrict__ w,
    int8_t* __restrict__ state, uint8_t* __restrict__ newc, int* __restrict__ rounds) {
  __shared__ int left;
  int r = 0;
  while (true) {
    if (threadIdx.x == 0) left = 0;
    for (int i = threadIdx.x; i < n; i += kPmisWg) {
      bool sel = state[i] == kUndecided;
      if (sel) {
        const double wi = w[i];
        for (int e = srp[i]; e < srp[i + 1] && sel; ++e) {
          const int j = sci[e];
          if (state[j] == kUndecided && beats(w[j], j, wi, i)) sel = false;
        }
        for (int e = strp[i]; e < strp[i + 1] && sel; ++e) {
          const int j = stci[e];
          if (state[j] == kUndecided && beats(w[j], j, wi, i)) sel = false;
        }
      }
      newc[i] = sel;
    }
    __syncthreads();
    int und = 0;
    for (int i = threadIdx.x; i < n; i += kPmisWg) {
      if (state[i] != kUndecided) continue;
      if (newc[i]) {
        state[i] = kC;
        continue;
      }
      bool f = false;
      for (int e = srp[i]; e < srp[i + 1]; ++e)
        if (newc[sci[e]]) {
          f = true;
          break;
        }
      if (f)
        state[i] = kF;
      else
        ++und;
    }
    if (und) atomicAdd(&left, und);
    __syncthreads();
    ++r;
    const int l = left;
    __syncthreads();
    if (l == 0 || r > n) {
      if (threadIdx.x == 0) rounds[0] = l == 0 ? r : -1;
      return;
    }
  }
}

__global__ void k_is_c(int n, const int8_t* __restrict__ cf, int* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cf[i] == kC;
}

// Direct interpolation, LPR lanes per row (the rows of coarse Galerkin
// operators run to hundreds of entries): number of entries of each P row.
template <int LPR>
__global__ void __launch_bounds__(256) k_interp_count(int n, const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const uint8_t* __restrict__ mask,
                                                      const int8_t* __restrict__ cf,
                                                      int* __restrict__ cnt) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  const bool frow = i < n && cf[i] != kC;
  int a0 = 0, a1 = 0;
  if (frow) {
    a0 = rp[i];
    a1 = rp[i + 1];
  }
  int c = 0;
  for (int e = a0 + lane; e < a1; e += LPR) c += mask[e] && cf[ci[e]] == kC;
  c = group_sum<LPR>(c);
  if (i < n && lane == 0) cnt[i] = frow ? c : 1;
}

// Direct interpolation weights of each row, LPR lanes per row; the strong C
// entries are written in row order (ballot over the group).
template <int LPR>
__global__ void __launch_bounds__(256) k_interp_fill(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const double* __restrict__ v,
                                                     const uint8_t* __restrict__ mask,
                                                     const int8_t* __restrict__ cf,
                                                     const int* __restrict__ cidx,
                                                     const int* __restrict__ prp,
                                                     int* __restrict__ pci,
                                                     double* __restrict__ pv) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  const bool live = i < n;
  const bool crow = live && cf[i] == kC;
  int a0 = 0, a1 = 0, o = 0;
  if (live) {
    o = prp[i];
    if (!crow) {
      a0 = rp[i];
      a1 = rp[i + 1];
    }
  }
  if (crow && lane == 0) {
    pci[o] = cidx[i];
    pv[o] = 1.0;
  }
  double aii = 0.0;
  for (int e = a0 + lane; e < a1; e += LPR)
    if (ci[e] == i) aii += v[e];
  aii = group_sum<LPR>(aii);
  const double s = aii < 0.0 ? -1.0 : 1.0;
  double sn_opp = 0.0, sn_same = 0.0, sp_opp = 0.0;
  for (int e = a0 + lane; e < a1; e += LPR) {
    const int j = ci[e];
    if (j == i) continue;
    const double a = v[e];
    if (s * a < 0.0)
      sn_opp += a;
    else if (s * a > 0.0)
      sn_same += a;
    if (mask[e] && cf[j] == kC) sp_opp += a;
  }
  sn_opp = group_sum<LPR>(sn_opp);
  sn_same = group_sum<LPR>(sn_same);
  sp_opp = group_sum<LPR>(sp_opp);
  const double atil = aii + sn_same;
  const double alpha = sn_opp / sp_opp;
  for (int base = a0; base < a1; base += LPR) {
    const int e = base + lane;
    const bool f = e < a1 && mask[e] && cf[ci[e]] == kC;
    const unsigned long long g = group_ballot<LPR>(f);
    if (f) {
      const int q = o + __popcll(g & ((1ull << lane) - 1ull));
      pci[q] = cidx[ci[e]];
      pv[q] = -alpha * v[e] / atil;
    }
    o += __popcll(g);
  }
}

// ---------------------------------------------------------------- classical
// Position of column `key` in the sorted columns ci[lo..hi), or -1.
__device__ inline int find_col(const int* __restrict__ ci, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int c = ci[mid];
    if (c == key) return mid;
    if (c < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return -1;
}

// Classical (modified Ruge-Stueben) interpolation weights, LPR lanes per
// row; the pattern is direct interpolation's (C n S_i), counted by
// k_interp_count.  For an F row i:
//   1. the strong C entries are written in row order with a_ij as the
//      running numerator (fine column index for now); the diagonal a~_ii
//      starts as a_ii plus the weak off-diagonal entries;
//   2. every strong F neighbour k, in row order: d = sum of the entries of
//      row k whose sign is opposite to a_kk and whose column is in C_i;
//      d = 0 lumps a_ik into a~_ii, else each P entry j gains
//      a_ik a_kj / d when a_kj has that sign;
//   3. w_ij = -numerator / a~_ii, columns renumbered to coarse indices.
// Lane l owns the P entries l, l + LPR, ... in steps 2 and 3.
template <int LPR>
__global__ void __launch_bounds__(256) k_classical_fill(int n, const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const double* __restrict__ v,
                                                        const uint8_t* __restrict__ mask,
                                                        const int8_t* __restrict__ cf,
                                                        const int* __restrict__ cidx,
                                                        const int* __restrict__ prp,
                                                        int* __restrict__ pci,
                                                        double* __restrict__ pv) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  const bool live = i < n;
  const bool crow = live && cf[i] == kC;
  int a0 = 0, a1 = 0, o = 0, np = 0;
  if (live) {
    o = prp[i];
    np = prp[i + 1] - o;
    if (!crow) {
      a0 = rp[i];
      a1 = rp[i + 1];
    }
  }
  if (crow && lane == 0) {
    pci[o] = cidx[i];
    pv[o] = 1.0;
  }
  // step 1
  double dpart = 0.0;
  for (int base = a0; base < a1; base += LPR) {
    const int e = base + lane;
    int j = -1;
    bool f = false;
    if (e < a1) {
      j = ci[e];
      if (j == i)
        dpart += v[e];
      else if (!mask[e])
        dpart += v[e];
      else
        f = cf[j] == kC;
    }
    const unsigned long long g = group_ballot<LPR>(f);
    if (f) {
      const int q = o + __popcll(g & ((1ull << lane) - 1ull));
      pci[q] = j;
      pv[q] = v[e];
    }
    o += __popcll(g);
  }
  double atil = group_sum<LPR>(dpart);
  o -= np;  // back to the row start (C rows: a0 == a1, o unchanged)
  __threadfence_block();  // the group reads the entries its lanes wrote
  // step 2
  for (int base = a0; base < a1; base += LPR) {
    const int e = base + lane;
    const bool sf = e < a1 && mask[e] && ci[e] != i && cf[ci[e]] != kC;
    unsigned long long g = group_ballot<LPR>(sf);
    while (g) {
      const int src = __ffsll(static_cast<long long>(g)) - 1;
      g &= g - 1;
      const int ek = base + src;  // the strong F entry (same in every lane)
      const int k = ci[ek];
      const double aik = v[ek];
      const int k0 = rp[k], k1 = rp[k + 1];
      double akk = 0.0;
      for (int f = k0 + lane; f < k1; f += LPR)
        if (ci[f] == k) akk += v[f];
      akk = group_sum<LPR>(akk);
      const double sk = akk < 0.0 ? -1.0 : 1.0;
      double d = 0.0;
      for (int f = k0 + lane; f < k1; f += LPR) {
        const int m = ci[f];
        const double a = v[f];
        if (sk * a < 0.0 && cf[m] == kC) {
          const int pos = find_col(ci, a0, a1, m);
          if (pos >= 0 && mask[pos]) d += a;
        }
      }
      d = group_sum<LPR>(d);
      if (d == 0.0) {
        atil += aik;
        continue;
      }
      for (int q = o + lane; q < o + np; q += LPR) {
        const int pos = find_col(ci, k0, k1, pci[q]);
        if (pos >= 0 && sk * v[pos] < 0.0) pv[q] += aik * v[pos] / d;
      }
    }
  }
  // step 3
  if (!crow && live)
    for (int q = o + lane; q < o + np; q += LPR) {
      pv[q] = -pv[q] / atil;
      pci[q] = cidx[pci[q]];
    }
}

// ---------------------------------------------------------------- truncation
// Interpolation truncation, one thread per row of P (rows hold a few
// entries).  Entries rank by magnitude rounded to FP32, larger first, the
// lower column first among equal magnitudes; an entry is kept if its rank is
// below pmax (every rank when pmax = 0) and its rounded magnitude reaches
// factor times the row's largest.  The kept positive entries are scaled by
// (sum of the row's positive entries) / (sum of the kept positive ones), the
// negative ones likewise.  Row i's entries sit at [start[i], start[i] +
// len[i]) in ascending column order (len == nullptr: CSR, len = start[i+1] -
// start[i]).  Without out_rp the kept count goes to cnt[i]; with it the kept
// entries are written from out_rp[i] on.
__device__ inline double trunc_key(double w) { return double(float(fabs(w))); }
// (ka, ca) ranks before (kb, cb)
__device__ inline bool trunc_before(double ka, int ca, double kb, int cb) {
  return ka > kb || (ka == kb && ca < cb);
}
constexpr int kTruncTop = 8;  // pmax up to this selects in registers

template <class Off>
__global__ void __launch_bounds__(256) k_truncate(int n, const Off* __restrict__ start,
                                                  const int* __restrict__ len,
                                                  const int* __restrict__ ci,
                                                  const double* __restrict__ v, int pmax,
                                                  double factor, int* __restrict__ cnt,
                                                  const int* __restrict__ out_rp,
                                                  int* __restrict__ out_ci,
                                                  double* __restrict__ out_v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t lo = int64_t(start[i]);
  const int m = len ? len[i] : int(int64_t(start[i + 1]) - lo);
  const int* rci = ci + lo;
  const double* rv = v + lo;
  if (factor <= 0.0 && (pmax <= 0 || m <= pmax)) {
    // nothing to drop: every scale factor would be x / x = 1
    if (!out_rp) {
      cnt[i] = m;
    } else {
      const int q = out_rp[i];
      for (int a = 0; a < m; ++a) {
        out_ci[q + a] = rci[a];
        out_v[q + a] = rv[a];
      }
    }
    return;
  }
  double largest = 0.0;
  for (int a = 0; a < m; ++a) largest = fmax(largest, trunc_key(rv[a]));
  const double thr = factor * largest;
  // the last kept rank: the pmax-th entry of the ranking (none when the row
  // is no longer than pmax)
  const bool ranked = pmax > 0 && m > pmax;
  double last_k = -1.0;
  int last_c = INT_MAX;
  if (ranked && pmax <= kTruncTop) {
    double tk[kTruncTop];
    int tc[kTruncTop];
#pragma unroll
    for (int q = 0; q < kTruncTop; ++q) {
      tk[q] = -1.0;
      tc[q] = INT_MAX;
    }
    for (int a = 0; a < m; ++a) {
      double k = trunc_key(rv[a]);
      int c = rci[a];
      // insertion into the best kTruncTop, best first
#pragma unroll
      for (int q = 0; q < kTruncTop; ++q)
        if (trunc_before(k, c, tk[q], tc[q])) {
          const double tkq = tk[q];
          const int tcq = tc[q];
          tk[q] = k;
          tc[q] = c;
          k = tkq;
          c = tcq;
        }
    }
#pragma unroll
    for (int q = 0; q < kTruncTop; ++q)
      if (q == pmax - 1) {
        last_k = tk[q];
        last_c = tc[q];
      }
  }
  auto kept = [&](int a) {
    const double ka = trunc_key(rv[a]);
    if (!(ka >= thr)) return false;
    if (!ranked) return true;
    if (pmax <= kTruncTop) return !trunc_before(last_k, last_c, ka, rci[a]);
    int rank = 0;
    for (int b = 0; b < m && rank < pmax; ++b)
      rank += trunc_before(trunc_key(rv[b]), rci[b], ka, rci[a]);
    return rank < pmax;
  };
  double pos = 0.0, neg = 0.0, kpos = 0.0, kneg = 0.0;
  int k = 0;
  for (int a = 0; a < m; ++a) {
    const double w = rv[a];
    const bool keep = kept(a);
    k += keep;
    if (w > 0.0) {
      pos += w;
      if (keep) kpos += w;
    } else if (w < 0.0) {
      neg += w;
      if (keep) kneg += w;
    }
  }
  if (!out_rp) {
    cnt[i] = k;
    return;
  }
  const double spos = kpos != 0.0 ? pos / kpos : 1.0, sneg = kneg != 0.0 ? neg / kneg : 1.0;
  int q = out_rp[i];
  for (int a = 0; a < m; ++a) {
    if (!kept(a)) continue;
    const double w = rv[a];
    out_ci[q] = rci[a];
    out_v[q] = w > 0.0 ? w * spos : (w < 0.0 ? w * sneg : w);
    ++q;
  }
}

// ---------------------------------------------------------------- CLJP
// CLJP coarsening (Cleary, Falgout, Henson, Jones).  Edges of the strength
// graph S (i -> j: i depends on j) are alive until a heuristic removes them;
// st2s maps each S^T entry (c, k) to the S entry of edge k -> c.  Weights
// start as in PMIS (k_pmis_init), so points influencing nothing are F.

// st2s[e] for every entry e of S^T row c: the position of c in S row k
__global__ void k_cljp_st2s(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                            const int* __restrict__ strp, const int* __restrict__ stci,
                            int* __restrict__ st2s) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int e = strp[c]; e < strp[c + 1]; ++e) {
    const int k = stci[e];
    st2s[e] = find_col(sci, srp[k], srp[k + 1], c);
  }
}

// D: undecided points whose (w, i) beats every undecided point joined to
// them by an alive edge, either direction
__global__ void k_cljp_select(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                              const int* __restrict__ strp, const int* __restrict__ stci,
                              const int* __restrict__ st2s, const int* __restrict__ alive,
                              const double* __restrict__ w, const int8_t* __restrict__ state,
                              uint8_t* __restrict__ newc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] != kUndecided) {
    newc[i] = 0;
    return;
  }
  const double wi = w[i];
  bool sel = true;
  for (int e = srp[i]; e < srp[i + 1] && sel; ++e) {
    const int j = sci[e];
    if (alive[e] && state[j] == kUndecided && beats(w[j], j, wi, i)) sel = false;
  }
  for (int e = strp[i]; e < strp[i + 1] && sel; ++e) {
    const int j = stci[e];
    const int es = st2s[e];
    if (es >= 0 && alive[es] && state[j] == kUndecided && beats(w[j], j, wi, i)) sel = false;
  }
  newc[i] = sel;
}

// The two heuristics for every c of D (one thread per point).  Edge k -> j
// is removed once whichever c reaches it (atomic exchange), and lowers w_j
// by exactly 1, so the round does not depend on thread order.  Edges into
// c are read here and removed by k_cljp_remove_in afterwards: no other c of
// D touches them (D is independent).
__global__ void k_cljp_heuristics(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                                  const int* __restrict__ strp, const int* __restrict__ stci,
                                  const int* __restrict__ st2s, int* __restrict__ alive,
                                  double* __restrict__ w, const uint8_t* __restrict__ newc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || !newc[c]) return;
  // c's neighbours it depends on are less needed as C points
  for (int e = srp[c]; e < srp[c + 1]; ++e)
    if (atomicExch(&alive[e], 0)) atomicAdd(&w[sci[e]], -1.0);
  // j and k both depend on c, k depends on j: k can take its value from c
  for (int a = strp[c]; a < strp[c + 1]; ++a) {
    if (st2s[a] < 0 || !alive[st2s[a]]) continue;
    const int j = stci[a];
    for (int b = strp[c]; b < strp[c + 1]; ++b) {
      if (b == a || st2s[b] < 0 || !alive[st2s[b]]) continue;
      const int k = stci[b];
      const int pos = find_col(sci, srp[k], srp[k + 1], j);
      if (pos >= 0 && atomicExch(&alive[pos], 0)) atomicAdd(&w[j], -1.0);
    }
  }
}

__global__ void k_cljp_remove_in(int n, const int* __restrict__ strp, const int* __restrict__ st2s,
                                 int* __restrict__ alive, const uint8_t* __restrict__ newc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || !newc[c]) return;
  for (int a = strp[c]; a < strp[c + 1]; ++a)
    if (st2s[a] >= 0) alive[st2s[a]] = 0;
}

// D becomes C, undecided points with w < 1 become F; *undecided is set when
// a point is left
__global__ void k_cljp_state(int n, const uint8_t* __restrict__ newc, const double* __restrict__ w,
                             int8_t* __restrict__ state, int* __restrict__ undecided) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || state[i] != kUndecided) return;
  if (newc[i])
    state[i] = kC;
  else if (w[i] < 1.0)
    state[i] = kF;
  else
    *undecided = 1;
}

// ---------------------------------------------------------------- extended+i
// Interpolation set of an F point i: strong C neighbours of i and of every
// strong F neighbour k, merged in ascending fine index by advancing one
// cursor per list (own row + one per strong F neighbour).  cur holds the
// cursors, indexed like A's entries.
__device__ inline int next_strong_c(int f, int end, const int* __restrict__ ci,
                                    const uint8_t* __restrict__ mask,
                                    const int8_t* __restrict__ cf) {
  while (f < end && !(mask[f] && cf[ci[f]] == kC)) ++f;
  return f;
}

template <bool FILL>
__device__ inline int exti_merge(int i, const int* __restrict__ rp, const int* __restrict__ ci,
                                 const uint8_t* __restrict__ mask, const int8_t* __restrict__ cf,
                                 int2* __restrict__ cur, int* __restrict__ out) {
  int a0 = rp[i], a1 = rp[i + 1];
  int own = next_strong_c(a0, a1, ci, mask, cf);
  for (int e = a0; e < a1; ++e) {
    int k = ci[e];
    if (mask[e] && k != i && cf[k] == kF) {
      int k0 = rp[k], k1 = rp[k + 1];
      cur[e] = make_int2(next_strong_c(k0, k1, ci, mask, cf), k1);
    }
  }
  int count = 0;
  while (true) {
    int m = INT_MAX;
    if (own < a1) m = ci[own];
    for (int e = a0; e < a1; ++e) {
      int k = ci[e];
      if (mask[e] && k != i && cf[k] == kF) {
        int2 c = cur[e];
        if (c.x < c.y) {
          int col = ci[c.x];
          m = col < m ? col : m;
        }
      }
    }
    if (m == INT_MAX) break;
    if (FILL) out[count] = m;
    ++count;
    if (own < a1 && ci[own] == m) own = next_strong_c(own + 1, a1, ci, mask, cf);
    for (int e = a0; e < a1; ++e) {
      int k = ci[e];
      if (mask[e] && k != i && cf[k] == kF) {
        int2 c = cur[e];
        if (c.x < c.y && ci[c.x] == m) cur[e].x = next_strong_c(c.x + 1, c.y, ci, mask, cf);
      }
    }
  }
  return count;
}

// per-thread version for the rows with the largest candidate sets
// position of fine index j in the sorted list c[0..len), or -1
__device__ inline int find_sorted(const int* __restrict__ c, int len, int j) {
  int lo = 0, hi = len - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    int v = c[mid];
    if (v == j) return mid;
    if (v < j) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

// weights: w_ij = -(a_ij + sum_k a_ik abar_kj / d_ik) / a~_ii with
// abar_kl = a_kl if its sign is opposite to a_kk, d_ik = sum over
// l in C^_i u {i} of abar_kl; weak entries outside C^_i and strong F
// neighbours with d_ik = 0 are lumped into a~_ii.
__global__ void k_exti_fill(int nl, const int* __restrict__ rows, const int* __restrict__ rp,
                            const int* __restrict__ ci, const double* __restrict__ v,
                            const uint8_t* __restrict__ mask, const int8_t* __restrict__ cf,
                            const int* __restrict__ cidx, int2* __restrict__ cur,
                            const int64_t* __restrict__ toff, int* __restrict__ cnt,
                            int* __restrict__ pci, double* __restrict__ pv) {
  int tt = blockIdx.x * blockDim.x + threadIdx.x;
  if (tt >= nl) return;
  int i = rows[tt];
  int64_t o = toff[i];
  int* c = pci + o;
  double* w = pv + o;
  int len = exti_merge<true>(i, rp, ci, mask, cf, cur, c);
  cnt[i] = len;
  for (int t = 0; t < len; ++t) w[t] = 0.0;
  int a0 = rp[i], a1 = rp[i + 1];
  double atil = row_diag(i, a0, a1, ci, v);
  for (int e = a0; e < a1; ++e) {
    int j = ci[e];
    if (j == i) continue;
    int t = find_sorted(c, len, j);
    if (t >= 0)
      w[t] += v[e];
    else if (!(mask[e] && cf[j] == kF))
      atil += v[e];
  }
  for (int e = a0; e < a1; ++e) {
    int k = ci[e];
    if (!(mask[e] && k != i && cf[k] == kF)) continue;
    double aik = v[e];
    int k0 = rp[k], k1 = rp[k + 1];
    double sk = row_diag(k, k0, k1, ci, v) < 0.0 ? -1.0 : 1.0;
    double d = 0.0;
    for (int f = k0; f < k1; ++f) {
      int l = ci[f];
      if (sk * v[f] < 0.0 && (l == i || find_sorted(c, len, l) >= 0)) d += v[f];
    }
    if (d == 0.0) {
      atil += aik;
      continue;
    }
    for (int f = k0; f < k1; ++f) {
      if (!(sk * v[f] < 0.0)) continue;
      int l = ci[f];
      int t = find_sorted(c, len, l);
      if (t >= 0)
        w[t] += aik * v[f] / d;
      else if (l == i)
        atil += aik * v[f] / d;
    }
  }
  for (int t = 0; t < len; ++t) {
    w[t] = -w[t] / atil;
    c[t] = cidx[c[t]];
  }
}

// ---- extended+i, one wavefront per F row.  The rows of the strong F
// neighbours are loaded once, flattened over the lanes, into LDS; the
// candidate set C^_i is sorted there and the weights accumulate over the
// neighbours k in row order.  Rows whose bounds exceed the wavefront
// kernels' capacities use the per-thread kernel above.
// Row classes by (strong F neighbours, candidates with duplicates, flattened
// neighbour entries): the flattened wavefront kernel at four sizes (the
// small ones need little LDS, so many rows are in flight), then the wide
// wavefront kernel (neighbour rows from global memory), then one thread per row.
constexpr int kExtK = 64;  // strong F neighbours a flattened-kernel class may hold
struct ExtClass {
  int k, cap, flat;
};
constexpr int kExtFlatN = 6;
constexpr ExtClass kExtFlatClasses[kExtFlatN] = {{16, 64, 128},  {16, 64, 512},  {16, 64, 1024},
                                                 {16, 64, 2048}, {64, 256, 512}, {64, 1024, 2048}};
constexpr int kExtCapWide = 4096;
constexpr int kExtClasses = kExtFlatN + 2;  // + wide wavefront + one thread per row

__device__ inline unsigned long long lanes_below() {
  return (1ull << (threadIdx.x & 63)) - 1ull;
}

// Largest power of two below n (1 when n <= 2): the first step of the
// binary-lifting searches over n sorted offsets.
__device__ inline int lift_top(int n) {
  int top = 1;
  while (2 * top < n) top <<= 1;
  return top;
}

// Segment of B flattened positions q[b]: the largest s < nseg with
// off[s] <= q[b] (off ascending, off[0] = 0); the searches advance together.
template <int B>
__device__ inline void segment_of_batch(const int* off, int nseg, int top, const int (&q)[B],
                                        int (&seg)[B]) {
#pragma unroll
  for (int b = 0; b < B; ++b) seg[b] = 0;
  for (int step = top; step > 0; step >>= 1) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int c = seg[b] + step;
      if (c < nseg && off[c] <= q[b]) seg[b] = c;
    }
  }
}

// Strong C entries of each row: sc_k = #{f in row k : f strong, column C}.
template <int LPR>
__global__ void __launch_bounds__(256) k_strong_c_count(int n, const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const uint8_t* __restrict__ mask,
                                                        const int8_t* __restrict__ cf,
                                                        int* __restrict__ sc) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  int a0 = 0, a1 = 0;
  if (i < n) {
    a0 = rp[i];
    a1 = rp[i + 1];
  }
  int c = 0;
  for (int e = a0 + lane; e < a1; e += LPR) c += mask[e] && cf[ci[e]] == kC;
  c = group_sum<LPR>(c);
  if (i < n && lane == 0) sc[i] = c;
}

// Per F row i: ub = strong C entries of row i and of the rows of its strong
// F neighbours k (duplicates counted: sc_i + sum sc_k), fl = summed length of
// those rows, nk = number of strong F neighbours.  C rows get ub = 1 (their
// injection entry).
template <int LPR>
__global__ void __launch_bounds__(256) k_exti_ub(int n, const int* __restrict__ rp,
                                                 const int* __restrict__ ci,
                                                 const uint8_t* __restrict__ mask,
                                                 const int8_t* __restrict__ cf,
                                                 const int* __restrict__ sc, int* __restrict__ ub,
                                                 int* __restrict__ fl, int* __restrict__ nko) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int i = int(gid / LPR), lane = int(gid % LPR);
  const bool frow = i < n && cf[i] != kC;
  int a0 = 0, a1 = 0;
  if (frow) {
    a0 = rp[i];
    a1 = rp[i + 1];
  }
  int64_t t = 0, flat = 0;
  int nk = 0;
  for (int e = a0 + lane; e < a1; e += LPR) {
    const int k = ci[e];
    if (!mask[e] || k == i || cf[k] != kF) continue;
    t += sc[k];
    flat += rp[k + 1] - rp[k];
    ++nk;
  }
  t = group_sum<LPR>(t);
  flat = group_sum<LPR>(flat);
  nk = group_sum<LPR>(nk);
  if (i < n && lane == 0) {
    if (frow) {
      t += sc[i];
      ub[i] = t > INT_MAX ? INT_MAX : int(t);
      fl[i] = flat > INT_MAX ? INT_MAX : int(flat);
      nko[i] = nk;
    } else {
      ub[i] = 1;
      fl[i] = 0;
      nko[i] = 0;
    }
  }
}

// F rows by their bounds: the first fitting class from `first` on among the
// flattened wavefront kernels, then the wide wavefront kernel, then one
// thread per row
__global__ void k_exti_classify(int n, const int* __restrict__ ub, const int* __restrict__ fl,
                                const int* __restrict__ nk, const int8_t* __restrict__ cf,
                                int first, int* __restrict__ counts, int* __restrict__ lists) {
  block_append_rows<kExtClasses, 256, kClassifyRows>(
      n,
      [&](int i) {
        if (cf[i] == kC) return -1;
        const int u = ub[i], f = fl[i], k0 = nk[i];
        int c = kExtClasses - 1;
        if (first <= kExtFlatN && u <= kExtCapWide) c = kExtFlatN;
#pragma unroll
        for (int k = kExtFlatN - 1; k >= 0; --k)
          if (k >= first && k0 <= kExtFlatClasses[k].k && u <= kExtFlatClasses[k].cap &&
              f <= kExtFlatClasses[k].flat)
            c = k;
        return c;
      },
      n, counts, lists);
}

__device__ inline int lds_find(const int* u, int m, int key) {
  int lo = 0, hi = m;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (u[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return (lo < m && u[lo] == key) ? lo : -1;
}

// Positions of B keys in the sorted u[0, m) (-1 when absent); top is the
// largest power of two <= m (0 when m = 0).  The B searches advance together,
// so their LDS reads overlap.
template <int B>
__device__ inline void lds_find_batch(const int* u, int m, int top, const int (&key)[B],
                                      int (&pos)[B]) {
  int lo[B];
#pragma unroll
  for (int b = 0; b < B; ++b) lo[b] = -1;  // u[lo] < key
  for (int step = top; step > 0; step >>= 1) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int c = lo[b] + step;
      if (c < m && u[c] < key[b]) lo[b] = c;
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int p = lo[b] + 1;
    pos[b] = (p < m && u[p] == key[b]) ? p : -1;
  }
}

// Extended+i weights of one F row (see k_exti_fill for the formula); writes
// the row's sorted coarse columns and weights at toff[i], its length to cnt.
// After the candidates are sorted, every flattened neighbour entry gets its
// candidate index once (or -2 for column i, -1 otherwise); the sums d_ik run
// one neighbour per lane; the weights then accumulate over the neighbours k
// in row order, one neighbour row per step.
template <int KCAP, int CAP, int FCAP>
__global__ void __launch_bounds__(64, CAP <= 64 ? 8 : 4) k_exti_flat(
    const int* __restrict__ rows, const int* __restrict__ rp, const int* __restrict__ ci,
    const double* __restrict__ v, const uint8_t* __restrict__ mask, const int8_t* __restrict__ cf,
    const int* __restrict__ cidx, const int64_t* __restrict__ toff, int* __restrict__ cnt,
    int* __restrict__ pci, double* __restrict__ pv) {
  constexpr int PC = CAP / 64;
  // reads / searches per lane in flight (fewer in the small classes, whose
  // LDS allows more wavefronts per CU when the registers do too)
  constexpr int kBMax = CAP <= 64 ? 4 : 8;
  constexpr int kB = FCAP / 64 < kBMax ? FCAP / 64 : kBMax;
  __shared__ int cand[CAP];
  __shared__ int uniq[CAP];
  __shared__ double w[CAP];
  __shared__ int fcol[FCAP];  // column, then candidate index / -2 (column i) / -1
  __shared__ double fval[FCAP];
  __shared__ int ks[KCAP];
  __shared__ int kst[KCAP];
  __shared__ int ko[KCAP + 1];
  __shared__ double ka[KCAP];
  __shared__ double kdg[KCAP];
  __shared__ double kd[KCAP];
  const int lane = threadIdx.x;
  const int i = rows[blockIdx.x];
  const int a0 = rp[i], a1 = rp[i + 1];
  // row i: strong C columns are candidates; strong F neighbours in row order
  constexpr int RB = KCAP <= 16 ? 2 : 4;  // row entries per lane in flight (clamped reads)
  int len = 0, nk = 0;
  for (int base = a0; base < a1; base += 64 * RB) {
    int k[RB];
    uint8_t m[RB];
    double x[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int e = min(base + b * 64 + lane, a1 - 1);
      k[b] = ci[e];
      m[b] = mask[e];
      x[b] = v[e];
    }
    int8_t c[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) c[b] = cf[k[b]];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const bool mm = base + b * 64 + lane < a1 && m[b] && k[b] != i;
      const bool sc = mm && c[b] == kC, sf = mm && c[b] == kF;
      unsigned long long bal = __ballot(sc);
      if (sc) cand[len + __popcll(bal & lanes_below())] = k[b];
      len += __popcll(bal);
      bal = __ballot(sf);
      if (sf) {
        int p = nk + __popcll(bal & lanes_below());
        ks[p] = k[b];
        ka[p] = x[b];
      }
      nk += __popcll(bal);
    }
  }
  __syncthreads();
  // neighbour rows: start, length, flattened offsets
  int rl = 0;
  if (lane < nk) {
    int k = ks[lane];
    int k0 = rp[k];
    kst[lane] = k0;
    rl = rp[k + 1] - k0;
    kdg[lane] = 0.0;
  }
  int incl = rl;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 0) ko[0] = 0;
  if (lane < nk) ko[lane + 1] = incl;
  const int flat = __shfl(incl, 63, 64);
  __syncthreads();
  {
    constexpr int FB = kB;  // flattened entries per lane in flight (clamped reads, one wait)
    const int top = lift_top(nk);
    for (int q0 = 0; q0 < flat; q0 += 64 * FB) {
      int q[FB], seg[FB];
#pragma unroll
      for (int b = 0; b < FB; ++b) q[b] = min(q0 + b * 64 + lane, flat - 1);
      segment_of_batch<FB>(ko, nk, top, q, seg);
      int col[FB];
      uint8_t m[FB];
      double x[FB];
#pragma unroll
      for (int b = 0; b < FB; ++b) {
        const int f = kst[seg[b]] + (q[b] - ko[seg[b]]);
        col[b] = ci[f];
        m[b] = mask[f];
        x[b] = v[f];
      }
      int8_t c[FB];
#pragma unroll
      for (int b = 0; b < FB; ++b) c[b] = cf[col[b]];
#pragma unroll
      for (int b = 0; b < FB; ++b) {
        const bool in = q0 + b * 64 + lane < flat;
        if (in) {
          fcol[q[b]] = col[b];
          fval[q[b]] = x[b];
          if (col[b] == ks[seg[b]]) kdg[seg[b]] = x[b];
        }
        const bool isc = in && m[b] && c[b] == kC;
        unsigned long long bal = __ballot(isc);
        if (isc) cand[len + __popcll(bal & lanes_below())] = col[b];
        len += __popcll(bal);
      }
    }
  }
  __syncthreads();
  // sorted unique candidates (register bitonic network, one wavefront)
  int p2 = 1;
  while (p2 < len) p2 <<= 1;
  {
    int kr[PC];
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      const int t = q * 64 + lane;
      kr[q] = t < len ? cand[t] : INT_MAX;
    }
    bitonic_regs<PC>(kr, 0, lane, p2, cand);
#pragma unroll
    for (int q = 0; q < PC; ++q) cand[q * 64 + lane] = kr[q];
  }
  __syncthreads();
  int m = 0;
  for (int base = 0; base < p2; base += 64) {
    int t = base + lane;
    bool f = t < len && (t == 0 || cand[t - 1] != cand[t]);
    unsigned long long b = __ballot(f);
    if (f) uniq[m + __popcll(b & lanes_below())] = cand[t];
    m += __popcll(b);
  }
  for (int t = lane; t < m; t += 64) w[t] = 0.0;
  int top = 0;
  if (m > 0) {
    top = 1;
    while (2 * top <= m) top <<= 1;
  }
  __syncthreads();
  // candidate index of every flattened entry (in place of its column)
  for (int q0 = 0; q0 < flat; q0 += 64 * kB) {
    int key[kB], pos[kB];
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const int q = q0 + b * 64 + lane;
      key[b] = q < flat ? fcol[q] : -1;
    }
    lds_find_batch<kB>(uniq, m, top, key, pos);
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const int q = q0 + b * 64 + lane;
      if (q < flat) fcol[q] = key[b] == i ? -2 : pos[b];
    }
  }
  // direct couplings; weak entries outside C^_i go to the diagonal
  double aii = 0.0, lump = 0.0;
  for (int base = a0; base < a1; base += 64 * RB) {
    int key[RB], pos[RB];
    double x[RB];
    bool sfm[RB];
    uint8_t mk[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int e = min(base + b * 64 + lane, a1 - 1);
      key[b] = ci[e];
      x[b] = v[e];
      mk[b] = mask[e];
    }
    int8_t c[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) c[b] = cf[key[b]];
#pragma unroll
    for (int b = 0; b < RB; ++b) sfm[b] = mk[b] && c[b] == kF;
    lds_find_batch<RB>(uniq, m, top, key, pos);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int e = base + b * 64 + lane;
      if (e >= a1) continue;
      const int j = key[b];
      if (j == i)
        aii = x[b];
      else if (pos[b] >= 0)
        w[pos[b]] += x[b];
      else if (!sfm[b])
        lump += x[b];
    }
  }
  aii = wave_sum(aii);
  lump = wave_sum(lump);
  __syncthreads();
  // d_ik: one neighbour row per lane, in row order (eight entries in flight)
  if (lane < nk) {
    const double sk = kdg[lane] < 0.0 ? -1.0 : 1.0;
    const int q1 = ko[lane + 1];
    double d = 0.0;
    for (int q0 = ko[lane]; q0 < q1; q0 += 8) {
      double x[8];
      int c[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        x[b] = fval[min(q0 + b, q1 - 1)];
        c[b] = fcol[min(q0 + b, q1 - 1)];
      }
#pragma unroll
      for (int b = 0; b < 8; ++b)
        if (q0 + b < q1 && sk * x[b] < 0.0 && c[b] != -1) d += x[b];
    }
    kd[lane] = d;
  }
  __syncthreads();
  double extra = 0.0, toi = 0.0;  // extra uniform across lanes, toi per lane
  for (int s = 0; s < nk; ++s) {
    const double aik = ka[s], d = kd[s];
    if (d == 0.0) {
      extra += aik;
      continue;
    }
    const double sk = kdg[s] < 0.0 ? -1.0 : 1.0;
    for (int q = ko[s] + lane; q < ko[s + 1]; q += 64) {
      const double x = fval[q];
      if (!(sk * x < 0.0)) continue;
      const int t = fcol[q];
      if (t >= 0)
        w[t] += aik * x / d;
      else if (t == -2)
        toi += aik * x / d;
    }
    __syncthreads();
  }
  const double atil = __shfl(aii + lump, 0, 64) + extra + __shfl(wave_sum(toi), 0, 64);
  __syncthreads();
  const int64_t o = toff[i];
  for (int t = lane; t < m; t += 64) {
    pci[o + t] = cidx[uniq[t]];
    pv[o + t] = -w[t] / atil;
  }
  if (lane == 0) cnt[i] = m;
}

// appends the columns of entries e in [e0, e1) that pass the filter to buf
// (order preserved), returning the new length (wavefront-wide)
__device__ inline int wave_append_strong_c(int e0, int e1, const int* __restrict__ ci,
                                           const uint8_t* __restrict__ mask,
                                           const int8_t* __restrict__ cf, int* buf, int len) {
  int lane = threadIdx.x & 63;
  for (int base = e0; base < e1; base += 64) {
    int e = base + lane;
    bool f = e < e1 && mask[e] && cf[ci[e]] == kC;
    unsigned long long b = __ballot(f);
    int pos = __popcll(b & ((1ull << lane) - 1ull));
    if (f) buf[len + pos] = ci[e];
    len += __popcll(b);
  }
  return len;
}

// Wide rows (many strong F neighbours or long neighbour rows): the same
// weights with the neighbour rows read from global memory one at a time.
template <int CAP>
__global__ void __launch_bounds__(64) k_exti_wide(
    const int* __restrict__ rows, const int* __restrict__ rp, const int* __restrict__ ci,
    const double* __restrict__ v, const uint8_t* __restrict__ mask, const int8_t* __restrict__ cf,
    const int* __restrict__ cidx, const int64_t* __restrict__ toff, int* __restrict__ cnt,
    int* __restrict__ pci, double* __restrict__ pv) {
  __shared__ int cand[CAP];
  __shared__ int uniq[CAP];
  __shared__ double w[CAP];
  int lane = threadIdx.x;
  int i = rows[blockIdx.x];
  int a0 = rp[i], a1 = rp[i + 1];
  // candidates: strong C neighbours of i and of its strong F neighbours
  int len = wave_append_strong_c(a0, a1, ci, mask, cf, cand, 0);
  for (int e = a0; e < a1; ++e) {
    int k = ci[e];
    if (mask[e] && k != i && cf[k] == kF)
      len = wave_append_strong_c(rp[k], rp[k + 1], ci, mask, cf, cand, len);
  }
  int p2 = 1;
  while (p2 < len) p2 <<= 1;
  for (int t = len + lane; t < p2; t += 64) cand[t] = INT_MAX;
  __syncthreads();
  for (int k = 2; k <= p2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < p2; t += 64) {
        int q = t ^ j;
        if (q > t) {
          int x = cand[t], y = cand[q];
          bool up = (t & k) == 0;
          if ((x > y) == up) {
            cand[t] = y;
            cand[q] = x;
          }
        }
      }
      __syncthreads();
    }
  int m = 0;
  for (int base = 0; base < p2; base += 64) {
    int t = base + lane;
    bool f = t < p2 && cand[t] != INT_MAX && (t == 0 || cand[t - 1] != cand[t]);
    unsigned long long b = __ballot(f);
    int pos = __popcll(b & ((1ull << lane) - 1ull));
    if (f) uniq[m + pos] = cand[t];
    m += __popcll(b);
  }
  for (int t = lane; t < m; t += 64) w[t] = 0.0;
  __syncthreads();
  // direct couplings; weak entries outside C^_i go to the diagonal
  double aii = 0.0, lump = 0.0;
  for (int e = a0 + lane; e < a1; e += 64) {
    int j = ci[e];
    if (j == i) {
      aii = v[e];
      continue;
    }
    int t = lds_find(uniq, m, j);
    if (t >= 0)
      w[t] += v[e];
    else if (!(mask[e] && cf[j] == kF))
      lump += v[e];
  }
  aii = wave_sum(aii);
  lump = wave_sum(lump);
  __syncthreads();
  double extra = 0.0;  // uniform across lanes (computed from wavefront sums)
  for (int e = a0; e < a1; ++e) {
    int k = ci[e];
    if (!(mask[e] && k != i && cf[k] == kF)) continue;
    double aik = v[e];
    int k0 = rp[k], k1 = rp[k + 1];
    double dk = 0.0;
    for (int f = k0 + lane; f < k1; f += 64)
      if (ci[f] == k) dk = v[f];
    dk = __shfl(wave_sum(dk), 0, 64);
    double sk = dk < 0.0 ? -1.0 : 1.0;
    double d = 0.0;
    for (int f = k0 + lane; f < k1; f += 64) {
      int l = ci[f];
      if (sk * v[f] < 0.0 && (l == i || lds_find(uniq, m, l) >= 0)) d += v[f];
    }
    d = __shfl(wave_sum(d), 0, 64);
    if (d == 0.0) {
      extra += aik;
      continue;
    }
    double toi = 0.0;
    for (int f = k0 + lane; f < k1; f += 64) {
      if (!(sk * v[f] < 0.0)) continue;
      int l = ci[f];
      int t = lds_find(uniq, m, l);
      if (t >= 0)
        w[t] += aik * v[f] / d;
      else if (l == i)
        toi += aik * v[f] / d;
    }
    extra += __shfl(wave_sum(toi), 0, 64);
    __syncthreads();
  }
  double atil = __shfl(aii + lump, 0, 64) + extra;
  __syncthreads();
  const int64_t o = toff[i];
  for (int t = lane; t < m; t += 64) {
    pci[o + t] = cidx[uniq[t]];
    pv[o + t] = -w[t] / atil;
  }
  if (lane == 0) cnt[i] = m;
}


__global__ void k_inject_c(int n, const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                           const int64_t* __restrict__ toff, int* __restrict__ cnt,
                           int* __restrict__ pci, double* __restrict__ pv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || cf[i] != kC) return;
  pci[toff[i]] = cidx[i];
  pv[toff[i]] = 1.0;
  cnt[i] = 1;
}

// dense [A | I] for Gauss-Jordan (row-major, n x 2n)
__global__ void k_dense_augment(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, double* __restrict__ M) {
  int i = blockIdx.x;
  for (int c = threadIdx.x; c < 2 * n; c += blockDim.x) M[int64_t(i) * 2 * n + c] = (c - n == i) ? 1.0 : 0.0;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int e = rp[i]; e < rp[i + 1]; ++e) M[int64_t(i) * 2 * n + ci[e]] += v[e];
}

// Gauss-Jordan elimination with partial pivoting (largest |a|, lowest row on
// ties) on [A | I] by one work-group; singular -> *flag = 1.
__global__ void __launch_bounds__(1024) k_gauss_jordan(int n, double* __restrict__ M,
                                                       double* __restrict__ fac,
                                                       int* __restrict__ flag) {
  __shared__ double best_v[1024];
  __shared__ int best_i[1024];
  int w = 2 * n;
  for (int k = 0; k < n; ++k) {
    double bv = -1.0;
    int bi = n;
    for (int r = k + threadIdx.x; r < n; r += blockDim.x) {
      double a = fabs(M[int64_t(r) * w + k]);
      if (a > bv || (a == bv && r < bi)) {
        bv = a;
        bi = r;
      }
    }
    best_v[threadIdx.x] = bv;
    best_i[threadIdx.x] = bi;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) {
        double ov = best_v[threadIdx.x + st];
        int oi = best_i[threadIdx.x + st];
        if (ov > best_v[threadIdx.x] || (ov == best_v[threadIdx.x] && oi < best_i[threadIdx.x])) {
          best_v[threadIdx.x] = ov;
          best_i[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    int p = best_i[0];
    double pv = best_v[0];
    __syncthreads();
    if (!(pv > 0.0)) {
      if (threadIdx.x == 0) *flag = 1;
      return;
    }
    if (p != k)
      for (int c = threadIdx.x; c < w; c += blockDim.x) {
        double t = M[int64_t(k) * w + c];
        M[int64_t(k) * w + c] = M[int64_t(p) * w + c];
        M[int64_t(p) * w + c] = t;
      }
    __syncthreads();
    double piv = M[int64_t(k) * w + k];
    __syncthreads();
    for (int c = threadIdx.x; c < w; c += blockDim.x) M[int64_t(k) * w + c] /= piv;
    for (int r = threadIdx.x; r < n; r += blockDim.x) fac[r] = M[int64_t(r) * w + k];
    __syncthreads();
    // columns <= k of the left block are already reduced (unit vectors);
    // one wavefront per row, lanes along the row
    int lane = threadIdx.x & 63;
    for (int r = threadIdx.x >> 6; r < n; r += blockDim.x >> 6) {
      if (r == k) continue;
      double f = fac[r];
      for (int c = k + 1 + lane; c < w; c += 64) M[int64_t(r) * w + c] -= f * M[int64_t(k) * w + c];
    }
    for (int r = threadIdx.x; r < n; r += blockDim.x)
      if (r != k) M[int64_t(r) * w + k] = 0.0;
    __syncthreads();
  }
}

// Gauss-Jordan inversion in place with the whole matrix in LDS (n <= 128):
// partial pivoting by rows (largest |a|, lowest row on ties), row k
// normalised, every other row eliminated, column k taking the inverse's
// entries; the row interchanges are undone on the columns at the end.
// Reads the CSR operator, writes A^{-1} (row-major n x n); singular ->
// *flag = 1.
constexpr int kGjLds = 128;
__global__ void __launch_bounds__(1024) k_gauss_jordan_lds(int n, const int* __restrict__ rp,
                                                           const int* __restrict__ ci,
                                                           const double* __restrict__ v,
                                                           double* __restrict__ inv,
                                                           int* __restrict__ flag) {
  __shared__ double a[kGjLds * kGjLds];
  __shared__ double fac[kGjLds];
  __shared__ int perm[kGjLds];
  __shared__ int piv_row;
  __shared__ double piv_abs;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  for (int t = tid; t < n * n; t += blockDim.x) a[t] = 0.0;
  __syncthreads();
  for (int r = wid; r < n; r += nw)
    for (int e = rp[r] + lane; e < rp[r + 1]; e += 64) a[r * n + ci[e]] += v[e];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (wid == 0) {
      double bv = -1.0;
      int bi = n;
      for (int r = k + lane; r < n; r += 64) {
        double x = fabs(a[r * n + k]);
        if (x > bv || (x == bv && r < bi)) {
          bv = x;
          bi = r;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(bv, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        piv_row = bi;
        piv_abs = bv;
        perm[k] = bi;
      }
    }
    __syncthreads();
    const int p = piv_row;
    if (!(piv_abs > 0.0)) {
      if (tid == 0) *flag = 1;
      return;
    }
    if (p != k)
      for (int c = tid; c < n; c += blockDim.x) {
        double t = a[k * n + c];
        a[k * n + c] = a[p * n + c];
        a[p * n + c] = t;
      }
    __syncthreads();
    const double pv = a[k * n + k];
    __syncthreads();
    for (int c = tid; c < n; c += blockDim.x) a[k * n + c] = (c == k ? 1.0 : a[k * n + c]) / pv;
    for (int r = tid; r < n; r += blockDim.x) fac[r] = r == k ? 0.0 : a[r * n + k];
    __syncthreads();
    for (int r = wid; r < n; r += nw) {
      if (r == k) continue;
      double f = fac[r];
      for (int c = lane; c < n; c += 64) a[r * n + c] = (c == k ? 0.0 : a[r * n + c]) - f * a[k * n + c];
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    int p = perm[k];
    if (p != k)
      for (int r = tid; r < n; r += blockDim.x) {
        double t = a[r * n + k];
        a[r * n + k] = a[r * n + p];
        a[r * n + p] = t;
      }
    __syncthreads();
  }
  for (int t = tid; t < n * n; t += blockDim.x) inv[t] = a[t];
}

__global__ void k_dense_extract(int n, const double* __restrict__ M, double* __restrict__ Ainv) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * n) return;
  int r = int(t / n), c = int(t % n);
  Ainv[t] = M[int64_t(r) * 2 * n + n + c];
}

// ---------------------------------------------------------------- V-cycle kernels
// r = b - A (D^{-1} b): pre-smoothing from a zero guess fused with the residual
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_pre(int n, const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const T* __restrict__ v,
                                                const T* __restrict__ dinv,
                                                const T* __restrict__ b, T* __restrict__ r) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  T sum = row_dot<T, LPR>(row, lane, rp, ci, v, [&](int j) { return dinv[j] * b[j]; });
  if (lane == 0) r[row] = b[row] - sum;
}

// r = b - A g with g = D^{-1} b formed beforehand (large levels: one gather
// per entry instead of two)
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_pre_g(int n, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ v,
                                                  const T* __restrict__ g,
                                                  const T* __restrict__ b, T* __restrict__ r) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  T sum = row_dot<T, LPR>(row, lane, rp, ci, v, [&](int j) { return g[j]; });
  if (lane == 0) r[row] = b[row] - sum;
}

// y = D^{-1} b + P x_c: prolongation added to the pre-smoothed iterate
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_prolong(int n, const int* __restrict__ prp,
                                                    const int* __restrict__ pci,
                                                    const T* __restrict__ pv,
                                                    const T* __restrict__ dinv,
                                                    const T* __restrict__ b,
                                                    const T* __restrict__ xc, T* __restrict__ y) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  T sum = row_dot<T, LPR>(row, lane, prp, pci, pv, [&](int c) { return xc[c]; });
  if (lane == 0) y[row] = dinv[row] * b[row] + sum;
}

// y = D^{-1} b + P x_c with P in ELL form (W slots per row, column-major):
// the entries are summed in row order, as the CSR kernel does with one lane
template <class T, int W>
__global__ void __launch_bounds__(256) k_vc_prolong_ell(int n, const int* __restrict__ eci,
                                                        const T* __restrict__ ev,
                                                        const T* __restrict__ dinv,
                                                        const T* __restrict__ b,
                                                        const T* __restrict__ xc,
                                                        T* __restrict__ y) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  int c[W];
  T a[W];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    c[k] = eci[int64_t(k) * n + row];
    a[k] = ev[int64_t(k) * n + row];
  }
  T sum = T(0);
#pragma unroll
  for (int k = 0; k < W; ++k)
    if (c[k] >= 0) sum += a[k] * xc[c[k]];
  y[row] = dinv[row] * b[row] + sum;
}

// CSR rows of at most W entries -> ELL slots (see Level::pe_ci)
template <class T>
__global__ void __launch_bounds__(256) k_csr_to_ell(int n, int W, const int* __restrict__ rp,
                                                    const int* __restrict__ ci,
                                                    const double* __restrict__ v,
                                                    int* __restrict__ eci, T* __restrict__ ev) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const int e0 = rp[row], len = rp[row + 1] - e0;
  for (int k = 0; k < W; ++k) {
    eci[int64_t(k) * n + row] = k < len ? ci[e0 + k] : -1;
    ev[int64_t(k) * n + row] = k < len ? T(v[e0 + k]) : T(0);
  }
}

// restriction b_c = R r that also forms the next level's Jacobi guess
// g_c = D_c^{-1} b_c (a large coarse level's pre-smoothing gathers g_c)
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_restrict_guess(int nc, const int* __restrict__ rrp,
                                                           const int* __restrict__ rci,
                                                           const T* __restrict__ rv,
                                                           const T* __restrict__ r,
                                                           const T* __restrict__ dinv_c,
                                                           T* __restrict__ bc, T* __restrict__ gc) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= nc) return;
  T sum = row_dot<T, LPR>(row, lane, rrp, rci, rv, [&](int j) { return r[j]; });
  if (lane == 0) {
    bc[row] = sum;
    gc[row] = dinv_c[row] * sum;
  }
}

// x = y + D^{-1} (b - A y): post-smoothing
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_post(int n, const int* __restrict__ rp,
                                                 const int* __restrict__ ci,
                                                 const T* __restrict__ v,
                                                 const T* __restrict__ dinv,
                                                 const T* __restrict__ b,
                                                 const T* __restrict__ y, T* __restrict__ x) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  T sum = row_dot<T, LPR>(row, lane, rp, ci, v, [&](int j) { return y[j]; });
  if (lane == 0) x[row] = y[row] + dinv[row] * (b[row] - sum);
}

// two l1-Jacobi sweeps from zero: x = D^{-1}b + D^{-1}(b - A D^{-1} b)
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_two_sweeps(int n, const int* __restrict__ rp,
                                                       const int* __restrict__ ci,
                                                       const T* __restrict__ v,
                                                       const T* __restrict__ dinv,
                                                       const T* __restrict__ b,
                                                       T* __restrict__ x) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  T sum = row_dot<T, LPR>(row, lane, rp, ci, v, [&](int j) { return dinv[j] * b[j]; });
  if (lane == 0) {
    T x0 = dinv[row] * b[row];
    x[row] = x0 + dinv[row] * (b[row] - sum);
  }
}

// One sweep of the generic smoothers: r = D^{-1}(b - A x), d <- cd d + cr r
// (d may be null: Jacobi sweeps keep no direction), x_new = x + d.  x == null
// stands for the zero iterate.  l1-Jacobi: cd = 0, cr = 1; Chebyshev: the
// three-term recurrence's coefficients.
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_smooth_sweep(int n, const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const T* __restrict__ v,
                                                      const T* __restrict__ dinv,
                                                      const T* __restrict__ b,
                                                      const T* __restrict__ x, T* __restrict__ d,
                                                      T cd, T cr, T* __restrict__ xn) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  T sum = T(0);
  if (x) sum = row_dot<T, LPR>(row, lane, rp, ci, v, [&](int j) { return x[j]; });
  if (lane == 0) {
    const T r = dinv[row] * (b[row] - sum);
    T dn = cr * r;
    if (d) {
      if (cd != T(0)) dn = cd * d[row] + dn;
      d[row] = dn;
    }
    xn[row] = x ? x[row] + dn : dn;
  }
}

// y = x + P x_c (x == null: the zero iterate)
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_prolong_add(int n, const int* __restrict__ prp,
                                                        const int* __restrict__ pci,
                                                        const T* __restrict__ pv,
                                                        const T* __restrict__ x,
                                                        const T* __restrict__ xc,
                                                        T* __restrict__ y) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  T sum = row_dot<T, LPR>(row, lane, prp, pci, pv, [&](int c) { return xc[c]; });
  if (lane == 0) y[row] = x ? x[row] + sum : sum;
}

// Power iteration for the Chebyshev interval: the start vector (the PMIS
// hash u_i - 1/2), w = D^{-1} A v, v = w / s.
__global__ void k_hash_centered(int n, uint64_t seed, double* __restrict__ v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  v[i] = double(splitmix64(seed ^ uint64_t(i)) >> 40) * 0x1p-24 - 0.5;
}

template <int LPR>
__global__ void __launch_bounds__(256) k_dinv_spmv(int n, const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ dinv,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ w) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int row = int(gid / LPR), lane = int(gid % LPR);
  if (row >= n) return;
  double sum = row_dot<double, LPR>(row, lane, rp, ci, v, [&](int j) { return x[j]; });
  if (lane == 0) w[row] = dinv[row] * sum;
}

__global__ void k_div_scalar(int n, const double* __restrict__ w, double s, double* __restrict__ v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = w[i] / s;
}

// x = Ainv b in FP64 (one wavefront per row)
template <class T>
__global__ void __launch_bounds__(256) k_dense_gemv(int n, const double* __restrict__ Ainv,
                                                    const T* __restrict__ b, T* __restrict__ x) {
  int row = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  int lane = threadIdx.x & (kWave - 1);
  if (row >= n) return;
  double sum = 0.0;
  for (int c = lane; c < n; c += kWave) sum += Ainv[int64_t(row) * n + c] * double(b[c]);
  sum = wave_sum(sum);
  if (lane == 0) x[row] = T(sum);
}

// ---------------------------------------------------------------- level-0 diagonal layout
struct DiagOffs {
  int off[kMaxDiag];  // ascending
};

// Row i's entry at column i + off[k] goes to dv[k n + i] (zero where the row
// has no entry).  A work-group takes kDiaRows consecutive rows: LPR lanes per
// row read the entries (coalesced), place them in an LDS tile by diagonal
// (binary search over the ascending offsets), then the tile is written out
// one diagonal at a time (coalesced).  A work-group whose rows hold an entry
// off the listed diagonals sets *missed to 1 (a plain store: one
// same-address atomic per work-group would serialise over the whole grid);
// the layout is usable when *missed stays 0.
constexpr int kDiaRows = 64;
template <int LPR>
__global__ void __launch_bounds__(256) k_csr_to_dia(int n, const int* __restrict__ rp,
                                                    const int* __restrict__ ci,
                                                    const double* __restrict__ v, int K,
                                                    DiagOffs o, double* __restrict__ dv,
                                                    int* __restrict__ missed) {
  __shared__ double tile[kMaxDiag][kDiaRows];
  __shared__ int off[kMaxDiag];
  __shared__ int sh[256 / 64];
  const int i0 = blockIdx.x * kDiaRows;
  const int rows = min(kDiaRows, n - i0);
  for (int t = threadIdx.x; t < kMaxDiag * kDiaRows; t += 256) tile[t / kDiaRows][t % kDiaRows] = 0.0;
  if (threadIdx.x < kMaxDiag) off[threadIdx.x] = o.off[threadIdx.x];
  __syncthreads();
  int top = 1;
  while (2 * top <= K) top <<= 1;
  int found = 0;
  constexpr int RPP = 256 / LPR;  // rows per pass
  const int g = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  for (int r0 = 0; r0 < rows; r0 += RPP) {
    const int r = r0 + g;
    if (r >= rows) continue;
    const int i = i0 + r;
    const int a0 = rp[i], a1 = rp[i + 1];
    for (int e = a0 + lane; e < a1; e += LPR) {
      const int d = ci[e] - i;
      int lo = -1;  // off[lo] < d
      for (int step = top; step > 0; step >>= 1)
        if (lo + step < K && off[lo + step] < d) lo += step;
      const int k = lo + 1;
      if (k < K && off[k] == d) {
        tile[k][r] = v[e];
        ++found;
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < K * kDiaRows; t += 256) {
    const int k = t / kDiaRows, r = t % kDiaRows;
    if (r < rows) dv[int64_t(k) * n + i0 + r] = tile[k][r];
  }
  const int tot = block_sum<256>(found, sh);
  if (threadIdx.x == 0 && tot != rp[i0 + rows] - rp[i0]) *missed = 1;
}

__device__ inline int clampi(int j, int n) { return j < 0 ? 0 : (j >= n ? n - 1 : j); }

// Work-groups are handed to the eight XCDs round-robin (group b to XCD
// b % 8).  This renumbering gives each XCD a contiguous eighth of the
// groups, so the neighbouring rows a stencil row gathers from sit in the
// same XCD's L2.  It is a bijection on [0, gridDim.x).
__device__ inline int xcd_contiguous_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb / 8, r = nb % 8;
  const int x = b % 8, t = b / 8;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + t;
}

// g = D^{-1} b (the pre-smoothed iterate from a zero guess)
template <class T>
__global__ void __launch_bounds__(256) k_jacobi_guess(int n, const T* __restrict__ dinv,
                                                      const T* __restrict__ b,
                                                      T* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = dinv[i] * b[i];
}

// r = b - A g with g = D^{-1} b
template <class T, int K>
__global__ void __launch_bounds__(256) k_dia_pre(int n, DiagOffs o, const T* __restrict__ v,
                                                 const T* __restrict__ g,
                                                 const T* __restrict__ b, T* __restrict__ r) {
  int i = xcd_contiguous_block() * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T sum = T(0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int j = clampi(i + o.off[k], n);
    sum += v[int64_t(k) * n + i] * g[j];
  }
  r[i] = b[i] - sum;
}

template <class T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };
// clang vector of two T (what the non-temporal builtin accepts)
template <class T> using nt2 = T __attribute__((ext_vector_type(2)));

// Two rows per thread (n even): the diagonals and the row vectors are read
// as pairs.  Same sums, in the same order, as the one-row kernels.
template <class T, int K>
__global__ void __launch_bounds__(256) k_dia_pre2(int n, DiagOffs o, const T* __restrict__ v,
                                                  const T* __restrict__ g,
                                                  const T* __restrict__ b, T* __restrict__ r) {
  using T2 = typename Vec2<T>::type;
  int i = 2 * (xcd_contiguous_block() * blockDim.x + threadIdx.x);
  if (i >= n) return;
  T s0 = T(0), s1 = T(0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // the diagonals are streamed once: non-temporal, so L2 keeps the gathered vector
    nt2<T> a = __builtin_nontemporal_load(reinterpret_cast<const nt2<T>*>(v + int64_t(k) * n + i));
    s0 += a.x * g[clampi(i + o.off[k], n)];
    s1 += a.y * g[clampi(i + 1 + o.off[k], n)];
  }
  T2 bb = *reinterpret_cast<const T2*>(b + i);
  T2 out;
  out.x = bb.x - s0;
  out.y = bb.y - s1;
  *reinterpret_cast<T2*>(r + i) = out;
}

template <class T, int K>
__global__ void __launch_bounds__(256) k_dia_post2(int n, DiagOffs o, const T* __restrict__ v,
                                                   const T* __restrict__ dinv,
                                                   const T* __restrict__ b,
                                                   const T* __restrict__ y, T* __restrict__ x) {
  using T2 = typename Vec2<T>::type;
  int i = 2 * (xcd_contiguous_block() * blockDim.x + threadIdx.x);
  if (i >= n) return;
  T s0 = T(0), s1 = T(0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    nt2<T> a = __builtin_nontemporal_load(reinterpret_cast<const nt2<T>*>(v + int64_t(k) * n + i));
    s0 += a.x * y[clampi(i + o.off[k], n)];
    s1 += a.y * y[clampi(i + 1 + o.off[k], n)];
  }
  T2 yy = *reinterpret_cast<const T2*>(y + i);
  T2 dd = *reinterpret_cast<const T2*>(dinv + i);
  T2 bb = *reinterpret_cast<const T2*>(b + i);
  T2 out;
  out.x = yy.x + dd.x * (bb.x - s0);
  out.y = yy.y + dd.y * (bb.y - s1);
  *reinterpret_cast<T2*>(x + i) = out;
}

// FP32 forms of the two kernels above with four rows per thread (16-byte
// loads of the diagonals and row vectors, as the FP64 forms read); each
// row's terms are summed in the same order.
using nt4f = float __attribute__((ext_vector_type(4)));
template <int K>
__global__ void __launch_bounds__(256) k_dia_pre4f(int n, DiagOffs o, const float* __restrict__ v,
                                                   const float* __restrict__ g,
                                                   const float* __restrict__ b,
                                                   float* __restrict__ r) {
  const int i = 4 * (xcd_contiguous_block() * blockDim.x + threadIdx.x);
  if (i >= n) return;
  float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const nt4f a = __builtin_nontemporal_load(reinterpret_cast<const nt4f*>(v + int64_t(k) * n + i));
    s[0] += a.x * g[clampi(i + o.off[k], n)];
    s[1] += a.y * g[clampi(i + 1 + o.off[k], n)];
    s[2] += a.z * g[clampi(i + 2 + o.off[k], n)];
    s[3] += a.w * g[clampi(i + 3 + o.off[k], n)];
  }
  const float4 bb = *reinterpret_cast<const float4*>(b + i);
  *reinterpret_cast<float4*>(r + i) =
      make_float4(bb.x - s[0], bb.y - s[1], bb.z - s[2], bb.w - s[3]);
}

template <int K>
__global__ void __launch_bounds__(256) k_dia_post4f(int n, DiagOffs o, const float* __restrict__ v,
                                                    const float* __restrict__ dinv,
                                                    const float* __restrict__ b,
                                                    const float* __restrict__ y,
                                                    float* __restrict__ x) {
  const int i = 4 * (xcd_contiguous_block() * blockDim.x + threadIdx.x);
  if (i >= n) return;
  float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const nt4f a = __builtin_nontemporal_load(reinterpret_cast<const nt4f*>(v + int64_t(k) * n + i));
    s[0] += a.x * y[clampi(i + o.off[k], n)];
    s[1] += a.y * y[clampi(i + 1 + o.off[k], n)];
    s[2] += a.z * y[clampi(i + 2 + o.off[k], n)];
    s[3] += a.w * y[clampi(i + 3 + o.off[k], n)];
  }
  const float4 yy = *reinterpret_cast<const float4*>(y + i);
  const float4 dd = *reinterpret_cast<const float4*>(dinv + i);
  const float4 bb = *reinterpret_cast<const float4*>(b + i);
  *reinterpret_cast<float4*>(x + i) =
      make_float4(yy.x + dd.x * (bb.x - s[0]), yy.y + dd.y * (bb.y - s[1]),
                  yy.z + dd.z * (bb.z - s[2]), yy.w + dd.w * (bb.w - s[3]));
}

// x = y + D^{-1} (b - A y)
template <class T, int K>
__global__ void __launch_bounds__(256) k_dia_post(int n, DiagOffs o, const T* __restrict__ v,
                                                  const T* __restrict__ dinv,
                                                  const T* __restrict__ b,
                                                  const T* __restrict__ y, T* __restrict__ x) {
  int i = xcd_contiguous_block() * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T sum = T(0);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int j = clampi(i + o.off[k], n);
    sum += v[int64_t(k) * n + i] * y[j];
  }
  x[i] = y[i] + dinv[i] * (b[i] - sum);
}

// The ELL prolongation with two rows per thread (n even): slots, values and
// row vectors read as pairs, each row's entries summed as in k_vc_prolong_ell;
// P is read once per cycle, so its slots are read non-temporally.
template <class T, int W>
__global__ void __launch_bounds__(256) k_vc_prolong_ell2(int n, const int* __restrict__ eci,
                                                         const T* __restrict__ ev,
                                                         const T* __restrict__ dinv,
                                                         const T* __restrict__ b,
                                                         const T* __restrict__ xc,
                                                         T* __restrict__ y) {
  using T2 = typename Vec2<T>::type;
  using I2 = int __attribute__((ext_vector_type(2)));
  const int i = 2 * (xcd_contiguous_block() * blockDim.x + threadIdx.x);
  if (i >= n) return;
  I2 c[W];
  nt2<T> a[W];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    c[k] = __builtin_nontemporal_load(reinterpret_cast<const I2*>(eci + int64_t(k) * n + i));
    a[k] = __builtin_nontemporal_load(reinterpret_cast<const nt2<T>*>(ev + int64_t(k) * n + i));
  }
  T s0 = T(0), s1 = T(0);
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if (c[k].x >= 0) s0 += a[k].x * xc[c[k].x];
    if (c[k].y >= 0) s1 += a[k].y * xc[c[k].y];
  }
  const T2 dd = *reinterpret_cast<const T2*>(dinv + i);
  const T2 bb = *reinterpret_cast<const T2*>(b + i);
  T2 out;
  out.x = dd.x * bb.x + s0;
  out.y = dd.y * bb.y + s1;
  *reinterpret_cast<T2*>(y + i) = out;
}

// ---------------------------------------------------------------- streamed CSR rows
// Smoother kernels of the large CSR levels (the Galerkin operators below
// level 0) whose rows take at most 8 lanes (64 entries on average), and the
// restriction into such levels.  A wavefront takes R = 64 / LPR consecutive
// rows, as the row kernels' grid assigns them, but reads their entries as
// one contiguous range: every load instruction covers 128 consecutive values
// and column indices (a pair per lane), where the row kernels' lane groups
// read R separate pieces of 8 LPR bytes (wider groups already read whole
// 128-byte lines and keep the row kernels).  The range is cut into windows
// of kStreamWin entries, and setup sorts each window's entries by column
// (Level::sw_ci): a load's gathers of g_j then touch a few cache lines of g
// instead of one or two per row segment.  The products a_ij g_j go back to
// their CSR positions in the wavefront's LDS window; each row's LPR lanes
// then sum their row's part of the window, in CSR order, and reduce across
// the group.  Work-groups are numbered XCD-contiguously, so the columns a
// stretch of rows gathers stay in one XCD's L2.  The pre-smoother reads the
// level's values and indices with ordinary loads, leaving what the
// memory-side cache keeps of them for the post-smoother, which reads them
// non-temporally as their last use in the cycle.
constexpr int kStreamWin = 512;
constexpr int kStreamLanes = 8;  // rows of up to this many lanes are streamed
constexpr int kGuessRows = 65536;  // CSR levels from this size form D^{-1} b first
// window-sorted entries: column in the low 23 bits, window position above
constexpr int kSwColBits = 23;
constexpr int kSwColMask = (1 << kSwColBits) - 1;
static_assert(kStreamWin <= (1 << (32 - kSwColBits)), "window positions fit above the column");

// LDS written by some lanes of a wavefront and then read by others: the LDS
// operations of one wavefront complete in order, so ordering the compiler's
// view at wavefront scope is enough
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Products of the window's sorted entries into win at their CSR positions.
// Lane l takes the entry pairs (e, e + 1), e = base + 2 (u * 64 + l) for
// u < U, base = ws rounded down to even, so values and packed indices are
// read as 16- and 8-byte pairs; pairs are clamped to the window's last one,
// so all loads are valid (the arrays carry one zero entry past the end) and
// issued before the first wait, and entries outside [ws, we) are dropped.
// NT: values and indices read non-temporally.
template <class T, int U, bool NT, class G>
__device__ inline void stream_window(int ws, int we, int lane, const int* __restrict__ sci,
                                     const T* __restrict__ v, G g, T* __restrict__ win) {
  using I2 = int __attribute__((ext_vector_type(2)));
  const int base = ws & ~1, last = (we - 1) & ~1;
  I2 c[U];
  nt2<T> a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = min(base + 2 * (u * kWave + lane), last);
    if constexpr (NT) {
      c[u] = __builtin_nontemporal_load(reinterpret_cast<const I2*>(sci + e));
      a[u] = __builtin_nontemporal_load(reinterpret_cast<const nt2<T>*>(v + e));
    } else {
      c[u] = *reinterpret_cast<const I2*>(sci + e);
      a[u] = *reinterpret_cast<const nt2<T>*>(v + e);
    }
  }
  T x0[U], x1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    x0[u] = g(c[u].x & kSwColMask);
    x1[u] = g(c[u].y & kSwColMask);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = base + 2 * (u * kWave + lane);
    if (e >= ws && e < we) win[unsigned(c[u].x) >> kSwColBits] = a[u].x * x0[u];
    if (e + 1 < we) win[unsigned(c[u].y) >> kSwColBits] = a[u].y * x1[u];
  }
}

// Row r0 + lane / LPR's dot with the gathered values g(col), valid in the
// group's first lane (0 for a row at or past n).  win: the wavefront's
// kStreamWin-entry LDS window.  A window issues the fewest pair loads per
// lane (1 to 5) that cover its entries.
template <class T, int LPR, bool NT, class G>
__device__ inline T stream_rows_dot(int n, int r0, int lane, const int* __restrict__ rp,
                                    const int* __restrict__ ci, const T* __restrict__ v, G g,
                                    T* __restrict__ win) {
  constexpr int R = kWave / LPR;
  static_assert(kStreamWin == 8 * kWave, "windows of up to five pair loads");
  const int s = rp[r0], t = rp[min(r0 + R, n)];
  const int row = r0 + lane / LPR, q = lane % LPR;
  const int lo = rp[min(row, n)], hi = rp[min(row + 1, n)];
  T sum = T(0);
  for (int ws = s; ws < t; ws += kStreamWin) {
    const int we = min(ws + kStreamWin, t);
    const int pairs = (we - (ws & ~1) + 1) / 2;  // at most kStreamWin / 2 + 1
    if (pairs > 4 * kWave)
      stream_window<T, 5, NT>(ws, we, lane, ci, v, g, win);
    else if (pairs > 3 * kWave)
      stream_window<T, 4, NT>(ws, we, lane, ci, v, g, win);
    else if (pairs > 2 * kWave)
      stream_window<T, 3, NT>(ws, we, lane, ci, v, g, win);
    else if (pairs > kWave)
      stream_window<T, 2, NT>(ws, we, lane, ci, v, g, win);
    else
      stream_window<T, 1, NT>(ws, we, lane, ci, v, g, win);
    wave_lds_sync();
    const int je = min(hi, we);
    for (int j = max(lo, ws) + q; j < je; j += LPR) sum += win[j - ws];
    wave_lds_sync();  // the window is rewritten next
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) sum += __shfl_down(sum, off, LPR);
  return sum;
}

// Setup of Level::sw_ci / sw_v / sw_v32 (and of R's copy): one wavefront per
// R = 64 / LPR rows (the smoothers' assignment, without the XCD
// renumbering); each window's keys column << 9 | position are sorted in
// registers by a bitonic network across the wavefront, then the packed
// entries and the values they point at are written.  Columns must be below
// 2^23.
template <int LPR>
__global__ void __launch_bounds__(256) k_window_sort(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const double* __restrict__ v,
                                                     int* __restrict__ sci,
                                                     double* __restrict__ sv,
                                                     float* __restrict__ sv32) {
  constexpr int PER = kStreamWin / kWave;
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // the zero entry past the end
    const int z = rp[n];
    sci[z] = 0;
    if (sv) sv[z] = 0.0;
    if (sv32) sv32[z] = 0.0f;
  }
  const int r0 = (blockIdx.x * (256 / kWave) + w) * (kWave / LPR);
  if (r0 >= n) return;  // the whole wavefront
  const int s = rp[r0], t = rp[min(r0 + kWave / LPR, n)];
  for (int ws = s; ws < t; ws += kStreamWin) {
    const int m = min(kStreamWin, t - ws);
    unsigned key[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = q * kWave + lane;
      key[q] = k < m ? (unsigned(ci[ws + k]) << (32 - kSwColBits)) | unsigned(k) : 0xffffffffu;
    }
    int p2 = 2;
    while (p2 < m) p2 <<= 1;
    // p2 <= kStreamWin = 64 PER: the network stays in registers and shuffles
    bitonic_regs<PER>(key, 0, lane, p2, static_cast<unsigned*>(nullptr));
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int k = q * kWave + lane;
      if (k < m) {
        const int p = int(key[q] & (kStreamWin - 1)), c = int(key[q] >> (32 - kSwColBits));
        sci[ws + k] = int(unsigned(c) | (unsigned(p) << kSwColBits));
        if (sv) sv[ws + k] = v[ws + p];
        if (sv32) sv32[ws + k] = float(v[ws + p]);
      }
    }
  }
}

// first row of this wavefront's R rows (wavefront-uniform)
template <int LPR>
__device__ inline int stream_first_row() {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  return (xcd_contiguous_block() * (256 / kWave) + w) * (kWave / LPR);
}

// r = b - A g with g = D^{-1} b formed beforehand; grid as k_vc_pre_g's
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_pre_gs(int n, const int* __restrict__ rp,
                                                   const int* __restrict__ ci,
                                                   const T* __restrict__ v,
                                                   const T* __restrict__ g,
                                                   const T* __restrict__ b, T* __restrict__ r) {
  __shared__ T win[256 / kWave][kStreamWin];
  const int r0 = stream_first_row<LPR>();
  if (r0 >= n) return;  // the whole wavefront
  const int lane = threadIdx.x % kWave;
  const T sum = stream_rows_dot<T, LPR, false>(
      n, r0, lane, rp, ci, v, [&](int j) { return g[j]; }, win[threadIdx.x / kWave]);
  const int row = r0 + lane / LPR;
  if (lane % LPR == 0 && row < n) r[row] = b[row] - sum;
}

// x = y + D^{-1} (b - A y); grid as k_vc_post's
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_posts(int n, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ v,
                                                  const T* __restrict__ dinv,
                                                  const T* __restrict__ b,
                                                  const T* __restrict__ y, T* __restrict__ x) {
  __shared__ T win[256 / kWave][kStreamWin];
  const int r0 = stream_first_row<LPR>();
  if (r0 >= n) return;
  const int lane = threadIdx.x % kWave;
  const T sum = stream_rows_dot<T, LPR, true>(
      n, r0, lane, rp, ci, v, [&](int j) { return y[j]; }, win[threadIdx.x / kWave]);
  const int row = r0 + lane / LPR;
  if (lane % LPR == 0 && row < n) x[row] = y[row] + dinv[row] * (b[row] - sum);
}

// b_c = R r and g_c = D_c^{-1} b_c from R's window-sorted copy (the rows of
// R are the coarse points); grid as k_vc_restrict_guess's.  R is read once
// per cycle: non-temporal.
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_vc_restrict_gs(int nc, const int* __restrict__ rrp,
                                                        const int* __restrict__ rci,
                                                        const T* __restrict__ rv,
                                                        const T* __restrict__ r,
                                                        const T* __restrict__ dinv_c,
                                                        T* __restrict__ bc, T* __restrict__ gc) {
  __shared__ T win[256 / kWave][kStreamWin];
  const int r0 = stream_first_row<LPR>();
  if (r0 >= nc) return;
  const int lane = threadIdx.x % kWave;
  const T sum = stream_rows_dot<T, LPR, true>(
      nc, r0, lane, rrp, rci, rv, [&](int j) { return r[j]; }, win[threadIdx.x / kWave]);
  const int row = r0 + lane / LPR;
  if (lane % LPR == 0 && row < nc) {
    bc[row] = sum;
    gc[row] = dinv_c[row] * sum;
  }
}

#define DISPATCH_DIAG(K, KK, ...)                               \
  switch (K) {                                                  \
    case 5: { constexpr int KK = 5; __VA_ARGS__ } break;        \
    case 7: { constexpr int KK = 7; __VA_ARGS__ } break;        \
    case 13: { constexpr int KK = 13; __VA_ARGS__ } break;      \
    case 25: { constexpr int KK = 25; __VA_ARGS__ } break;      \
    default: fail(TPF_ERR_STATE, "unsupported stencil width %d", K); \
  }

template <class T>
const T* vals_of(const Csr<double>& M, const Buf<float>& v32);
template <>
const double* vals_of<double>(const Csr<double>& M, const Buf<float>&) { return M.v.p; }
template <>
const float* vals_of<float>(const Csr<double>&, const Buf<float>& v32) { return v32.p; }

template <class T> T* work(Buf<double>& d, Buf<float>& f);
template <> double* work<double>(Buf<double>& d, Buf<float>&) { return d.p; }
template <> float* work<float>(Buf<double>&, Buf<float>& f) { return f.p; }
template <class T> const T* dinv_of(const Level& L);
template <class T> const T* ell_vals(const Level& L);
template <> const double* ell_vals<double>(const Level& L) { return L.pe_v.p; }
template <> const float* ell_vals<float>(const Level& L) { return L.pe_v32.p; }
template <class T> const T* sw_vals(const Level& L);
template <> const double* sw_vals<double>(const Level& L) { return L.sw_v.p; }
template <> const float* sw_vals<float>(const Level& L) { return L.sw_v32.p; }
template <class T> const T* rw_vals(const Level& L);
template <> const double* rw_vals<double>(const Level& L) { return L.rw_v.p; }
template <> const float* rw_vals<float>(const Level& L) { return L.rw_v32.p; }
constexpr int kEllMaxW = 4;  // widest ELL form of P
#define DISPATCH_ELL(w, W, ...)                         \
  switch (w) {                                          \
    case 1: { constexpr int W = 1; __VA_ARGS__ } break; \
    case 2: { constexpr int W = 2; __VA_ARGS__ } break; \
    case 3: { constexpr int W = 3; __VA_ARGS__ } break; \
    default: { constexpr int W = 4; __VA_ARGS__ } break; \
  }
template <> const double* dinv_of<double>(const Level& L) { return L.dinv.p; }
template <> const float* dinv_of<float>(const Level& L) { return L.dinv32.p; }

}  // namespace

// ---------------------------------------------------------------- setup
// A_c = R A P through the intermediate L.T: (R A) P when ra_first, else
// R (A P).  The intermediate is released afterwards (a numeric refresh
// recomputes it); its blocks stay cached for the stream, where the next
// level's product finds them.
static void galerkin(Level& L, bool ra_first, Csr<double>& Ac, hipStream_t s) {
  if (ra_first) {
    spgemm(ref(L.R), ref(L.A), L.T, s);
    spgemm(ref(L.T), ref(L.P), Ac, s);
  } else {
    spgemm(ref(L.A), ref(L.P), L.T, s);
    spgemm(ref(L.R), ref(L.T), Ac, s);
  }
  L.T = Csr<double>{};
}

void Hierarchy::build(Csr<double>&& A0, const AmgOpts& opts, hipStream_t st) {
  drop_graphs();
  o = opts;
  s = st;
  lv.clear();
  auto L0 = std::make_unique<Level>();
  L0->A = std::move(A0);
  lv.push_back(std::move(L0));
  // setup phase timers (recorded while kernel timing is on), per level
  const std::string ph_finish = "setup_finish[" + tag + "]";
  while (true) {
    Level& L = *lv.back();
    int n = L.A.nrows;
    if (n <= o.coarse_max || int(lv.size()) >= o.max_levels) break;
    const std::string sfx = "[" + tag + ",l" + std::to_string(lv.size() - 1) + "]";
    const std::string ph_strength = "setup_strength" + sfx, ph_coarsen = "setup_coarsen" + sfx,
                      ph_interp = "setup_interp" + sfx, ph_transpose = "setup_transpose" + sfx,
                      ph_galerkin = "setup_galerkin" + sfx;
    std::unique_ptr<TimedScope> phase(new TimedScope(ph_strength.c_str(), s));
    // strength of connection
    L.mask.alloc(L.A.nnz > 0 ? L.A.nnz : 1, s);
    Buf<int> cnt(n, s);
    const int lpr = lanes_per_row(n, L.A.nnz);
    const unsigned rblocks = grid_for(int64_t(n) * lpr, 256);
    DISPATCH_LPR(lpr, LL, {
      k_strength<LL><<<rblocks, 256, 0, s>>>(n, L.A.rp.p, L.A.ci.p, L.A.v.p, o.theta, L.mask.p,
                                             cnt.p);
    });
    TPF_CHECK_LAUNCH();
    L.S.nrows = L.S.ncols = n;
    L.S.rp.alloc(n + 1, s);
    L.S.nnz = scan_exclusive(cnt.p, L.S.rp.p, n, s);
    L.S.ci.alloc(L.S.nnz > 0 ? L.S.nnz : 1, s);
    DISPATCH_LPR(lpr, LL, {
      k_compact_pattern<LL><<<rblocks, 256, 0, s>>>(n, L.A.rp.p, L.A.ci.p, L.mask.p, L.S.rp.p,
                                                    L.S.ci.p);
    });
    TPF_CHECK_LAUNCH();
    Csr<double> ST;
    transpose(CsrRef<double>{n, n, L.S.nnz, L.S.rp.p, L.S.ci.p, nullptr}, ST, s);
    phase.reset();
    phase.reset(new TimedScope(ph_coarsen.c_str(), s));
    // PMIS
    Buf<double> w(n, s);
    L.cf.alloc(n, s);
    Buf<uint8_t> newc(n, s);
    Buf<int> und(1, s);
    k_pmis_init<<<grid_for(n, 256), 256, 0, s>>>(n, o.seed, ST.rp.p, w.p, L.cf.p);
    TPF_CHECK_LAUNCH();
    int rounds = 0;
    int* rounds_pinned = host_counts_slot();
    if (o.cljp) {
      // CLJP: one read-back per round
      const int64_t snnz = L.S.nnz > 0 ? L.S.nnz : 1;
      Buf<int> alive(snnz, s), st2s(snnz, s);
      fill_int(alive.p, 1, snnz, s);
      k_cljp_st2s<<<grid_for(n, 256), 256, 0, s>>>(n, L.S.rp.p, L.S.ci.p, ST.rp.p, ST.ci.p,
                                                   st2s.p);
      TPF_CHECK_LAUNCH();
      int* hflag = host_counts_slot();
      for (rounds = 1;; ++rounds) {
        TPF_REQUIRE(rounds <= n + 1, TPF_ERR_INVALID_ARG, "CLJP did not terminate");
        fill_int(und.p, 0, 1, s);
        const unsigned g = grid_for(n, 256);
        k_cljp_select<<<g, 256, 0, s>>>(n, L.S.rp.p, L.S.ci.p, ST.rp.p, ST.ci.p, st2s.p, alive.p,
                                        w.p, L.cf.p, newc.p);
        k_cljp_heuristics<<<g, 256, 0, s>>>(n, L.S.rp.p, L.S.ci.p, ST.rp.p, ST.ci.p, st2s.p,
                                            alive.p, w.p, newc.p);
        k_cljp_remove_in<<<g, 256, 0, s>>>(n, ST.rp.p, st2s.p, alive.p, newc.p);
        k_cljp_state<<<g, 256, 0, s>>>(n, newc.p, w.p, L.cf.p, und.p);
        TPF_CHECK_LAUNCH();
        TPF_HIP(hipMemcpyAsync(hflag, und.p, sizeof(int), hipMemcpyDeviceToHost, s));
        note_host_sync();
        TPF_HIP(hipStreamSynchronize(s));
        if (*hflag == 0) break;
      }
    } else if (n <= kPmisWgMax) {
      // every round in one launch; the count comes back with the next scan
      k_pmis_block<<<1, kPmisWg, 0, s>>>(n, L.S.rp.p, L.S.ci.p, ST.rp.p, ST.ci.p, w.p, L.cf.p,
                                         newc.p, und.p);
      TPF_CHECK_LAUNCH();
      TPF_HIP(hipMemcpyAsync(rounds_pinned, und.p, sizeof(int), hipMemcpyDeviceToHost, s));
    } else {
      // Rounds are queued in batches of kPmisBatch with one read-back of
      // their flags per batch (a round takes a few microseconds on the GPU,
      // less than the host's turn-around).  Once a round leaves no point
      // undecided, the rounds after it change nothing.
      constexpr int kPmisBatch = 4;
      Buf<int> flags(kPmisBatch, s);
      int* hflag = host_counts_slot();
      rounds = 0;
      for (int r0 = 0; rounds == 0; r0 += kPmisBatch) {
        TPF_REQUIRE(r0 <= n + 1, TPF_ERR_INVALID_ARG, "PMIS did not terminate");
        fill_int(flags.p, 0, kPmisBatch, s);
        for (int k = 0; k < kPmisBatch; ++k) {
          k_pmis_select<<<grid_for(n, 256), 256, 0, s>>>(n, L.S.rp.p, L.S.ci.p, ST.rp.p,
                                                         ST.ci.p, w.p, L.cf.p, newc.p);
          k_pmis_update<<<grid_for(n, 256), 256, 0, s>>>(n, L.S.rp.p, L.S.ci.p, newc.p, L.cf.p,
                                                         flags.p + k);
          TPF_CHECK_LAUNCH();
        }
        TPF_HIP(hipMemcpyAsync(hflag, flags.p, kPmisBatch * sizeof(int), hipMemcpyDeviceToHost, s));
        note_host_sync();
        TPF_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < kPmisBatch; ++k)
          if (hflag[k] == 0) {
            rounds = r0 + k + 1;
            break;
          }
      }
    }
    // coarse numbering
    Buf<int> isc(n, s), cidx(n + 1, s);
    k_is_c<<<grid_for(n, 256), 256, 0, s>>>(n, L.cf.p, isc.p);
    TPF_CHECK_LAUNCH();
    int64_t nc = scan_exclusive(isc.p, cidx.p, n, s);  // synchronises: the round count arrived
    if (!o.cljp && n <= kPmisWgMax) {
      rounds = *rounds_pinned;
      TPF_REQUIRE(rounds > 0, TPF_ERR_INVALID_ARG, "PMIS did not terminate");
    }
    L.pmis_rounds = rounds;
    if (nc == 0 || double(nc) > 0.9 * double(n)) break;
    phase.reset();
    phase.reset(new TimedScope(ph_interp.c_str(), s));
    // interpolation: direct, classical, or extended+i
    L.P.nrows = n;
    L.P.ncols = int(nc);
    L.P.rp.alloc(n + 1, s);
    if (o.ext_i) {
      constexpr int NC = kExtClasses;
      Buf<int> ub(n, s), fl(n, s), nk(n, s), counts(NC, s), lists(NC * int64_t(n), s);
      fill_int(counts.p, 0, NC, s);
      {
        Buf<int> sc(n, s);
        DISPATCH_LPR(lpr, LL, {
          k_strong_c_count<LL><<<rblocks, 256, 0, s>>>(n, L.A.rp.p, L.A.ci.p, L.mask.p, L.cf.p,
                                                        sc.p);
          k_exti_ub<LL><<<rblocks, 256, 0, s>>>(n, L.A.rp.p, L.A.ci.p, L.mask.p, L.cf.p, sc.p,
                                                ub.p, fl.p, nk.p);
        });
        TPF_CHECK_LAUNCH();
      }
      k_exti_classify<<<grid_for(n, 256 * kClassifyRows), 256, 0, s>>>(n, ub.p, fl.p, nk.p, L.cf.p, o.exti_first,
                                                       counts.p, lists.p);
      TPF_CHECK_LAUNCH();
      // single pass: rows staged at their candidate bound, then packed
      Buf<int64_t> toff(size_t(n) + 1, s);
      int* hc_pinned = host_counts_slot();
      TPF_HIP(hipMemcpyAsync(hc_pinned, counts.p, NC * sizeof(int), hipMemcpyDeviceToHost, s));
      int64_t staged = scan_exclusive_wide(ub.p, toff.p, n, s);  // synchronises
      int hc[NC];
      std::memcpy(hc, hc_pinned, sizeof(hc));
      Buf<int> tci(staged > 0 ? size_t(staged) : 1, s);
      Buf<double> tv(staged > 0 ? size_t(staged) : 1, s);
      Buf<int2> cur;
      if (hc[NC - 1] > 0) cur.alloc(L.A.nnz > 0 ? L.A.nnz : 1, s);
      auto list = [&](int c) { return lists.p + c * int64_t(n); };
      k_inject_c<<<grid_for(n, 256), 256, 0, s>>>(n, L.cf.p, cidx.p, toff.p, cnt.p, tci.p, tv.p);
      // the widest flattened class, the wide kernel and the per-thread rows:
      // few rows that each take long, on the side stream beside the others
      int nshort = 0, nlong = 0;
      for (int c = 0; c < NC; ++c) (c < kExtFlatN - 1 ? nshort : nlong) += hc[c];
      SideFork fork(s, nshort > 0 && nlong > 0);
      const hipStream_t ls = fork.side;
      auto flat = [&](auto kt, auto ct, auto ft, int c) {
        constexpr int K = decltype(kt)::value, C = decltype(ct)::value, F = decltype(ft)::value;
        static_assert(K <= kExtK && C <= kExtCapWide, "class table");
        if (hc[c] > 0)
          k_exti_flat<K, C, F><<<hc[c], 64, 0, c < kExtFlatN - 1 ? s : ls>>>(
              list(c), L.A.rp.p, L.A.ci.p, L.A.v.p, L.mask.p, L.cf.p, cidx.p, toff.p, cnt.p, tci.p,
              tv.p);
      };
      using I16 = std::integral_constant<int, 16>;
      using I64 = std::integral_constant<int, 64>;
      using I128 = std::integral_constant<int, 128>;
      using I256 = std::integral_constant<int, 256>;
      using I512 = std::integral_constant<int, 512>;
      using I1024 = std::integral_constant<int, 1024>;
      using I2048 = std::integral_constant<int, 2048>;
      // the classes of kExtFlatClasses (long-row ones first, on the side stream)
      if (hc[NC - 2] > 0)
        k_exti_wide<kExtCapWide><<<hc[NC - 2], 64, 0, ls>>>(list(NC - 2), L.A.rp.p, L.A.ci.p,
                                                            L.A.v.p, L.mask.p, L.cf.p, cidx.p,
                                                            toff.p, cnt.p, tci.p, tv.p);
      if (hc[NC - 1] > 0)
        k_exti_fill<<<grid_for(hc[NC - 1], 128), 128, 0, ls>>>(hc[NC - 1], list(NC - 1), L.A.rp.p,
                                                               L.A.ci.p, L.A.v.p, L.mask.p, L.cf.p,
                                                               cidx.p, cur.p, toff.p, cnt.p, tci.p,
                                                               tv.p);
      flat(I64{}, I1024{}, I2048{}, 5);
      flat(I16{}, I64{}, I128{}, 0);
      flat(I16{}, I64{}, I512{}, 1);
      flat(I16{}, I64{}, I1024{}, 2);
      flat(I16{}, I64{}, I2048{}, 3);
      flat(I64{}, I256{}, I512{}, 4);
      TPF_CHECK_LAUNCH();
      fork.join();
      if (o.truncates()) {
        // truncation packs the staged rows itself
        Buf<int> kept(n, s);
        k_truncate<int64_t><<<grid_for(n, 256), 256, 0, s>>>(
            n, toff.p, cnt.p, tci.p, tv.p, o.trunc_pmax, o.trunc_factor, kept.p, nullptr, nullptr,
            nullptr);
        TPF_CHECK_LAUNCH();
        L.P.nnz = scan_exclusive(kept.p, L.P.rp.p, n, s);
        L.P.ci.alloc(L.P.nnz > 0 ? L.P.nnz : 1, s);
        L.P.v.alloc(L.P.nnz > 0 ? L.P.nnz : 1, s);
        k_truncate<int64_t><<<grid_for(n, 256), 256, 0, s>>>(
            n, toff.p, cnt.p, tci.p, tv.p, o.trunc_pmax, o.trunc_factor, nullptr, L.P.rp.p,
            L.P.ci.p, L.P.v.p);
        TPF_CHECK_LAUNCH();
      } else {
        L.P.nnz = scan_exclusive(cnt.p, L.P.rp.p, n, s);
        L.P.ci.alloc(L.P.nnz > 0 ? L.P.nnz : 1, s);
        L.P.v.alloc(L.P.nnz > 0 ? L.P.nnz : 1, s);
        pack_rows(n, toff.p, L.P.rp.p, L.P.nnz, tci.p, tv.p, L.P.ci.p, L.P.v.p, s);
      }
    } else {
      DISPATCH_LPR(lpr, LL, {  // lanes per row of A, as for the strength kernels
        k_interp_count<LL><<<rblocks, 256, 0, s>>>(n, L.A.rp.p, L.A.ci.p, L.mask.p, L.cf.p,
                                                   cnt.p);
      });
      TPF_CHECK_LAUNCH();
      L.P.nnz = scan_exclusive(cnt.p, L.P.rp.p, n, s);
      L.P.ci.alloc(L.P.nnz, s);
      L.P.v.alloc(L.P.nnz, s);
      if (o.classical) {
        DISPATCH_LPR(lpr, LL, {
          k_classical_fill<LL><<<rblocks, 256, 0, s>>>(n, L.A.rp.p, L.A.ci.p, L.A.v.p, L.mask.p,
                                                       L.cf.p, cidx.p, L.P.rp.p, L.P.ci.p,
                                                       L.P.v.p);
        });
      } else {
        DISPATCH_LPR(lpr, LL, {
          k_interp_fill<LL><<<rblocks, 256, 0, s>>>(n, L.A.rp.p, L.A.ci.p, L.A.v.p, L.mask.p,
                                                    L.cf.p, cidx.p, L.P.rp.p, L.P.ci.p, L.P.v.p);
        });
      }
      TPF_CHECK_LAUNCH();
      if (o.truncates()) {
        Csr<double> Pt;
        Pt.nrows = n;
        Pt.ncols = int(nc);
        Pt.rp.alloc(n + 1, s);
        k_truncate<int><<<grid_for(n, 256), 256, 0, s>>>(n, L.P.rp.p, nullptr, L.P.ci.p, L.P.v.p,
                                                         o.trunc_pmax, o.trunc_factor, cnt.p,
                                                         nullptr, nullptr, nullptr);
        TPF_CHECK_LAUNCH();
        Pt.nnz = scan_exclusive(cnt.p, Pt.rp.p, n, s);
        Pt.ci.alloc(Pt.nnz > 0 ? Pt.nnz : 1, s);
        Pt.v.alloc(Pt.nnz > 0 ? Pt.nnz : 1, s);
        k_truncate<int><<<grid_for(n, 256), 256, 0, s>>>(n, L.P.rp.p, nullptr, L.P.ci.p, L.P.v.p,
                                                         o.trunc_pmax, o.trunc_factor, nullptr,
                                                         Pt.rp.p, Pt.ci.p, Pt.v.p);
        TPF_CHECK_LAUNCH();
        L.P = std::move(Pt);
      }
    }
    phase.reset();
    phase.reset(new TimedScope(ph_transpose.c_str(), s));
    transpose(ref(L.P), L.R, s);
    phase.reset();
    phase.reset(new TimedScope(ph_galerkin.c_str(), s));
    // Galerkin product A_c = R A P, as (R A) P on level 0 (R's rows of a
    // few fine points times the stencil rows, then P's short rows: about a
    // quarter fewer products than R (A P)), as R (A P) on the coarser levels
    // (whose dense rows would make R A the larger product)
    auto next = std::make_unique<Level>();
    galerkin(L, lv.size() == 1, next->A, s);
    lv.push_back(std::move(next));
  }
  TimedScope fin(ph_finish.c_str(), s);
  finish_levels(s);
}

// The Galerkin products are recomputed in full: the single-pass product
// yields the same pattern and is faster than a values-only pass over the
// kept one (k_spgemm_values searches B's rows per output entry).
void Hierarchy::refresh(hipStream_t st) {
  drop_graphs();
  s = st;
  for (size_t l = 0; l + 1 < lv.size(); ++l) {
    Level& L = *lv[l];
    galerkin(L, l == 0, lv[l + 1]->A, s);
  }
  finish_levels(s);
}

void Hierarchy::finish_levels(hipStream_t st) {
  drop_graphs();  // level buffers may move
  for (size_t l = 0; l < lv.size(); ++l) {
    Level& L = *lv[l];
    int n = L.A.nrows;
    std::string sfx = "[" + tag + ",l" + std::to_string(l) + "]";
    L.t_pre = "vcycle_pre_residual" + sfx;
    L.t_guess = "vcycle_jacobi_guess" + sfx;
    L.t_restrict = "vcycle_restrict" + sfx;
    L.t_prolong = "vcycle_prolong" + sfx;
    L.t_post = "vcycle_post_smooth" + sfx;
    L.t_coarse = "vcycle_coarse" + sfx;
    L.dinv.ensure(n, st);
    {
      const int lpr = lanes_per_row(n, L.A.nnz);
      DISPATCH_LPR(lpr, LL, {
        k_l1_dinv<LL><<<grid_for(int64_t(n) * lpr, 256), 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p,
                                                                       L.A.v.p, L.dinv.p);
      });
    }
    TPF_CHECK_LAUNCH();
    // FP64 cycle work vectors (the FP32 form cycles in FP32 only)
    const bool generic = !o.fused_cycle() && l + 1 < lv.size();
    if (!o.fp32) {
      L.r.ensure(n, st);
      L.y.ensure(n, st);
      if (&L != lv[0].get()) {
        L.b.ensure(n, st);
        L.x.ensure(n, st);
      }
      if (generic) {
        L.xa.ensure(n, st);
        L.xb.ensure(n, st);
        if (o.smoother == 1) L.dd.ensure(n, st);
      }
    }
    if (generic) {
      if (o.smoother == 1) chebyshev_setup(L, st);
      if (o.smoother == 2) gs_setup(L, st);
    }
    if (o.fp32) {
      L.Av32.ensure(L.A.nnz, st);
      cast<double, float>(L.Av32.p, L.A.v.p, L.A.nnz, st);
      L.dinv32.ensure(n, st);
      cast<double, float>(L.dinv32.p, L.dinv.p, n, st);
      if (L.P.rp.p) {
        L.Pv32.ensure(L.P.nnz, st);
        cast<double, float>(L.Pv32.p, L.P.v.p, L.P.nnz, st);
        L.Rv32.ensure(L.R.nnz, st);
        cast<double, float>(L.Rv32.p, L.R.v.p, L.R.nnz, st);
      }
      L.r32.ensure(n, st);
      L.y32.ensure(n, st);
      if (&L != lv[0].get()) {
        L.b32.ensure(n, st);
        L.x32.ensure(n, st);
      }
      if (generic) {
        L.xa32.ensure(n, st);
        L.xb32.ensure(n, st);
        if (o.smoother == 1) L.dd32.ensure(n, st);
      }
    }
    // ELL form of P for the fused cycle's prolongation: truncation to
    // trunc_pmax entries bounds every row of P
    const int W = o.trunc_pmax;
    if (o.fused_cycle() && L.P.rp.p && W >= 1 && W <= kEllMaxW) {
      L.pe_ci.ensure(size_t(W) * n, st);
      if (o.fp32) {
        L.pe_v.release();
        L.pe_v32.ensure(size_t(W) * n, st);
        k_csr_to_ell<float><<<grid_for(n, 256), 256, 0, st>>>(n, W, L.P.rp.p, L.P.ci.p, L.P.v.p,
                                                              L.pe_ci.p, L.pe_v32.p);
      } else {
        L.pe_v32.release();
        L.pe_v.ensure(size_t(W) * n, st);
        k_csr_to_ell<double><<<grid_for(n, 256), 256, 0, st>>>(n, W, L.P.rp.p, L.P.ci.p, L.P.v.p,
                                                               L.pe_ci.p, L.pe_v.p);
      }
      TPF_CHECK_LAUNCH();
      L.pe_w = W;
    } else {
      L.pe_w = 0;
      L.pe_ci.release();
      L.pe_v.release();
      L.pe_v32.release();
    }
  }
  // level-0 diagonal layout
  dia0.ok = false;
  int K = int(stencil.size());
  if (K == 5 || K == 7 || K == 13 || K == 25) {
    Level& L = *lv[0];
    int n = L.A.nrows;
    dia0.K = K;
    dia0.n = n;
    for (int k = 0; k < K; ++k) dia0.off[k] = stencil[k];
    DiagOffs off;
    for (int k = 0; k < kMaxDiag; ++k) off.off[k] = k < K ? stencil[k] : 0;
    dia0.v.ensure(size_t(K) * n, st);
    Buf<int> missed(1, st);
    fill_int(missed.p, 0, 1, st);
    if (K <= 8)  // lanes per row: about one entry each
      k_csr_to_dia<8><<<grid_for(n, kDiaRows), 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, L.A.v.p, K, off,
                                                             dia0.v.p, missed.p);
    else
      k_csr_to_dia<32><<<grid_for(n, kDiaRows), 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, L.A.v.p, K,
                                                              off, dia0.v.p, missed.p);
    TPF_CHECK_LAUNCH();
    dia0.ok = read_scalar(missed.p, st) == 0;
    if (dia0.ok && o.fp32) {
      dia0.v32.ensure(size_t(K) * n, st);
      cast<double, float>(dia0.v32.p, dia0.v.p, int64_t(K) * n, st);
    }
    if (!dia0.ok) {
      dia0.v.release();
      dia0.v32.release();
    } else if (o.fp32) {
      dia0.v.release();  // only the FP32 copy is cycled
    }
  }
  // window-sorted copies for the streamed smoothers
  for (size_t l = 0; l + 1 < lv.size(); ++l) {
    Level& L = *lv[l];
    const int n = L.A.nrows;
    const int lpr = lanes_per_row(n, L.A.nnz);
    if (streamed_level(int(l), n, lpr)) {
      L.sw_ci.ensure(L.A.nnz + 1, st);
      if (o.fp32) {
        L.sw_v.release();
        L.sw_v32.ensure(L.A.nnz + 1, st);
      } else {
        L.sw_v32.release();
        L.sw_v.ensure(L.A.nnz + 1, st);
      }
      const int64_t waves = (n + kWave / lpr - 1) / (kWave / lpr);
      DISPATCH_LPR(lpr, LL, {
        k_window_sort<LL><<<unsigned((waves + 3) / 4), 256, 0, st>>>(
            n, L.A.rp.p, L.A.ci.p, L.A.v.p, L.sw_ci.p, L.sw_v.p, L.sw_v32.p);
      });
      TPF_CHECK_LAUNCH();
      L.Av32.release();  // the FP32 cycle reads sw_v32 only
    } else {
      L.sw_ci.release();
      L.sw_v.release();
      L.sw_v32.release();
    }
    if (streamed_restriction(int(l))) {
      const int nc = L.R.nrows;
      const int rl = lanes_per_row(nc, L.R.nnz);
      L.rw_ci.ensure(L.R.nnz + 1, st);
      if (o.fp32) {
        L.rw_v.release();
        L.rw_v32.ensure(L.R.nnz + 1, st);
      } else {
        L.rw_v32.release();
        L.rw_v.ensure(L.R.nnz + 1, st);
      }
      const int64_t waves = (nc + kWave / rl - 1) / (kWave / rl);
      DISPATCH_LPR(rl, LL, {
        k_window_sort<LL><<<unsigned((waves + 3) / 4), 256, 0, st>>>(
            nc, L.R.rp.p, L.R.ci.p, L.R.v.p, L.rw_ci.p, L.rw_v.p, L.rw_v32.p);
      });
      TPF_CHECK_LAUNCH();
    } else {
      L.rw_ci.release();
      L.rw_v.release();
      L.rw_v32.release();
    }
  }
  coarse_setup(st);
}

// Restrictions into a coarse level that forms its guess there (fused
// cycles, coarse level of kGuessRows rows or more above the coarsest), with
// rows of at most kStreamLanes lanes and fine columns that fit the packed
// entries
bool Hierarchy::streamed_restriction(int l) const {
  if (!o.fused_cycle() || l + 2 >= int(lv.size())) return false;
  const Level& L = *lv[l];
  const int nc = L.R.nrows;
  return nc >= kGuessRows && lanes_per_row(nc, L.R.nnz) <= kStreamLanes &&
         L.A.nrows <= kSwColMask + 1;
}

// Levels whose smoothers stream their rows: fused V(1,1) cycles, CSR levels
// (not the diagonal level 0) of kGuessRows rows or more, below the coarsest,
// with rows of at most kStreamLanes lanes and columns that fit the packed
// entries
bool Hierarchy::streamed_level(int l, int n, int lpr) const {
  return o.fused_cycle() && l + 1 < int(lv.size()) && !(l == 0 && dia0.ok) && n >= kGuessRows &&
         lpr <= kStreamLanes && n <= kSwColMask + 1;
}

// Interval of the Chebyshev smoother on D^{-1} A: hi = 1.1 lambda^, lo = 0.3 hi,
// lambda^ from cheb_eig_iters power steps started at the PMIS hash vector
// (the estimate is ||w|| of the last step).  A zero estimate (D^{-1} A = 0)
// leaves the level with l1-Jacobi sweeps.
// ---------------------------------------------------------------- multicolour Gauss-Seidel
// Key of point i: the 24-bit PMIS hash weight above the index, so keys are
// distinct and ordered as (u_i, i).
__global__ void k_gs_keys(int n, uint64_t seed, int64_t* __restrict__ key) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t h = splitmix64(seed ^ uint64_t(i)) >> 40;
  key[i] = int64_t((h << 32) | uint64_t(i));
}

// One colouring round r: an uncoloured point takes colour r when its key
// beats that of every neighbour in the patterns of A and A^T that was
// uncoloured when the round began (a neighbour coloured in this round still
// counts, so the picked points are independent whatever the thread order).
// *flag is set when a point stays uncoloured.
__global__ void __launch_bounds__(256) k_gs_color_round(int n, const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const int* __restrict__ trp,
                                                        const int* __restrict__ tci,
                                                        const int64_t* __restrict__ key,
                                                        int* __restrict__ color, int r,
                                                        int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || color[i] >= 0) return;
  const int64_t ki = key[i];
  bool best = true;
  for (int e = rp[i]; e < rp[i + 1] && best; ++e) {
    const int j = ci[e];
    const int cj = color[j];
    if (j != i && (cj < 0 || cj == r) && key[j] > ki) best = false;
  }
  for (int e = trp[i]; e < trp[i + 1] && best; ++e) {
    const int j = tci[e];
    const int cj = color[j];
    if (j != i && (cj < 0 || cj == r) && key[j] > ki) best = false;
  }
  if (best)
    color[i] = r;
  else
    *flag = 1;
}

__global__ void k_gs_color_count(int n, const int* __restrict__ color, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[color[i]], 1);
}

__global__ void k_gs_color_place(int n, const int* __restrict__ color, int* __restrict__ pos,
                                 int* __restrict__ rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rows[atomicAdd(&pos[color[i]], 1)] = i;
}

// 1/a_ii, 0 where the diagonal is zero or absent
__global__ void k_plain_dinv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ v, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] == i) a += v[e];
  d[i] = a != 0.0 ? 1.0 / a : 0.0;
}

// One colour of a Gauss-Seidel sweep: x_i += (b_i - (A x)_i) / a_ii for the
// m points rows[0..m), LPR lanes per row.  No two points of a colour are
// neighbours, so each update reads only other colours' values.
template <class T, int LPR>
__global__ void __launch_bounds__(256) k_gs_color(int m, const int* __restrict__ rows,
                                                  const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ v,
                                                  const T* __restrict__ gd,
                                                  const T* __restrict__ b, T* __restrict__ x) {
  int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int t = int(gid / LPR), lane = int(gid % LPR);
  if (t >= m) return;
  const int i = rows[t];
  T sum = row_dot<T, LPR>(i, lane, rp, ci, v, [&](int j) { return x[j]; });
  if (lane == 0) x[i] += gd[i] * (b[i] - sum);
}

void Hierarchy::chebyshev_setup(Level& L, hipStream_t st) {
  const int n = L.A.nrows;
  Buf<double> v(n, st), w(n, st);
  k_hash_centered<<<grid_for(n, 256), 256, 0, st>>>(n, o.seed, v.p);
  TPF_CHECK_LAUNCH();
  const double nv = nrm2_host(v.p, n, st);
  double lam = 0.0;
  if (nv > 0.0) {
    k_div_scalar<<<grid_for(n, 256), 256, 0, st>>>(n, v.p, nv, v.p);
    TPF_CHECK_LAUNCH();
    const int lpr = lanes_per_row(n, L.A.nnz);
    for (int it = 0; it < o.cheb_eig_iters; ++it) {
      DISPATCH_LPR(lpr, LL, {
        k_dinv_spmv<LL><<<grid_for(int64_t(n) * LL, 256), 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p,
                                                                         L.A.v.p, L.dinv.p, v.p,
                                                                         w.p);
      });
      TPF_CHECK_LAUNCH();
      lam = nrm2_host(w.p, n, st);
      if (lam == 0.0) break;
      k_div_scalar<<<grid_for(n, 256), 256, 0, st>>>(n, w.p, lam, v.p);
      TPF_CHECK_LAUNCH();
    }
  }
  L.cheb_hi = 1.1 * lam;
  L.cheb_lo = 0.3 * L.cheb_hi;
}

// Colouring, colour lists and 1/a_ii of level L for the multicolour
// Gauss-Seidel smoother.  Rounds run in batches of eight per read-back;
// rounds after the last point is coloured change nothing.
void Hierarchy::gs_setup(Level& L, hipStream_t st) {
  const int n = L.A.nrows;
  L.gsd.ensure(n, st);
  k_plain_dinv<<<grid_for(n, 256), 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, L.A.v.p, L.gsd.p);
  TPF_CHECK_LAUNCH();
  if (int(L.gs_ptr.size()) == 0 || L.gs_rows.n != size_t(n)) {
    Csr<double> AT;
    transpose(CsrRef<double>{n, n, L.A.nnz, L.A.rp.p, L.A.ci.p, nullptr}, AT, st);
    Buf<int64_t> key(n, st);
    Buf<int> color(n, st);
    k_gs_keys<<<grid_for(n, 256), 256, 0, st>>>(n, o.seed, key.p);
    TPF_CHECK_LAUNCH();
    fill_int(color.p, -1, n, st);
    constexpr int kBatch = 8;
    int* hflag = host_counts_slot();
    int ncolors = 0;
    for (int r0 = 0; ncolors == 0; r0 += kBatch) {
      TPF_REQUIRE(r0 <= n, TPF_ERR_INVALID_ARG, "colouring did not terminate");
      Buf<int> flag(kBatch, st);
      fill_int(flag.p, 0, kBatch, st);
      for (int k = 0; k < kBatch; ++k) {  // flag[k]: a point is left after round r0 + k
        k_gs_color_round<<<grid_for(n, 256), 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, AT.rp.p,
                                                           AT.ci.p, key.p, color.p, r0 + k,
                                                           flag.p + k);
        TPF_CHECK_LAUNCH();
      }
      TPF_HIP(hipMemcpyAsync(hflag, flag.p, kBatch * sizeof(int), hipMemcpyDeviceToHost, st));
      note_host_sync();
      TPF_HIP(hipStreamSynchronize(st));
      for (int k = 0; k < kBatch; ++k)
        if (hflag[k] == 0) {
          ncolors = r0 + k + 1;
          break;
        }
    }
    Buf<int> cnt(ncolors, st), pos(ncolors + 1, st);
    fill_int(cnt.p, 0, ncolors, st);
    k_gs_color_count<<<grid_for(n, 256), 256, 0, st>>>(n, color.p, cnt.p);
    TPF_CHECK_LAUNCH();
    scan_exclusive(cnt.p, pos.p, ncolors, st);  // synchronises
    L.gs_ptr.assign(ncolors + 1, 0);
    TPF_HIP(hipMemcpyAsync(L.gs_ptr.data(), pos.p, (ncolors + 1) * sizeof(int),
                           hipMemcpyDeviceToHost, st));
    note_host_sync();
    TPF_HIP(hipStreamSynchronize(st));
    L.gs_ptr_dev.alloc(ncolors + 1, st);
    copy(L.gs_ptr_dev.p, pos.p, ncolors + 1, st);
    L.gs_rows.alloc(n, st);
    k_gs_color_place<<<grid_for(n, 256), 256, 0, st>>>(n, color.p, pos.p, L.gs_rows.p);
    TPF_CHECK_LAUNCH();
  }
  if (o.fp32) {
    L.gsd32.ensure(n, st);
    cast<double, float>(L.gsd32.p, L.gsd.p, n, st);
  }
}

// `steps` smoothing steps (each one l1-Jacobi sweep, or one Chebyshev
// polynomial of degree cheb_degree) on L from x0 (null: the zero iterate);
// the final iterate goes to `out`, the intermediate ones alternate between
// spare0 and spare1 (all distinct from x0 and out).
template <class T>
const T* Hierarchy::smooth(Level& L, const T* b, const T* x0, T* out, T* spare0, T* spare1,
                           int steps, bool post, hipStream_t st) {
  const int n = L.A.nrows;
  if (o.smoother == 2) {  // multicolour Gauss-Seidel, in place in `out`
    if (x0)
      copy(out, x0, n, st);
    else
      fill(out, T(0), n, st);
    const T* Av = vals_of<T>(L.A, L.Av32);
    const T* gd;
    if constexpr (std::is_same<T, float>::value)
      gd = L.gsd32.p;
    else
      gd = L.gsd.p;
    const int lpr = lanes_per_row(n, L.A.nnz);
    const int nc = int(L.gs_ptr.size()) - 1;
    for (int k = 0; k < steps; ++k)
      for (int q = 0; q < nc; ++q) {
        const int c = post ? nc - 1 - q : q;
        const int m = L.gs_ptr[c + 1] - L.gs_ptr[c];
        if (m == 0) continue;
        DISPATCH_LPR(lpr, LL, {
          k_gs_color<T, LL><<<grid_for(int64_t(m) * LL, 256), 256, 0, st>>>(
              m, L.gs_rows.p + L.gs_ptr[c], L.A.rp.p, L.A.ci.p, Av, gd, b, out);
        });
        TPF_CHECK_LAUNCH();
      }
    return out;
  }
  const bool cheb = o.smoother == 1 && L.cheb_hi > 0.0;
  const int per = cheb ? o.cheb_degree : 1;
  const int sweeps = steps * per;
  if (sweeps == 0) {
    if (x0)
      copy(out, x0, n, st);
    else
      fill(out, T(0), n, st);
    return out;
  }
  const T* Av = vals_of<T>(L.A, L.Av32);
  const T* dinv = dinv_of<T>(L);
  T* d = cheb ? work<T>(L.dd, L.dd32) : nullptr;
  const int lpr = lanes_per_row(n, L.A.nnz);
  const unsigned blocks = grid_for(int64_t(n) * lpr, 256);
  const double c = 0.5 * (L.cheb_hi + L.cheb_lo), h = 0.5 * (L.cheb_hi - L.cheb_lo);
  const double sigma = cheb ? c / h : 0.0;
  const T* cur = x0;
  double rho = 0.0;
  for (int k = 0; k < sweeps; ++k) {
    T* nxt = k == sweeps - 1 ? out : (k % 2 == 0 ? spare0 : spare1);
    double cd = 0.0, cr = 1.0;
    if (cheb) {
      if (k % per == 0) {  // a new polynomial: d_0 = r / c
        rho = 1.0 / sigma;
        cr = 1.0 / c;
      } else {
        const double rn = 1.0 / (2.0 * sigma - rho);
        cd = rn * rho;
        cr = 2.0 * rn / h;
        rho = rn;
      }
    }
    DISPATCH_LPR(lpr, LL, {
      k_smooth_sweep<T, LL><<<blocks, 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, Av, dinv, b, cur, d,
                                                    T(cd), T(cr), nxt);
    });
    TPF_CHECK_LAUNCH();
    cur = nxt;
  }
  return out;
}

void Hierarchy::coarse_setup(hipStream_t st) {
  Level& L = *lv.back();
  int n = L.A.nrows;
  coarse_dense = n <= o.dense_max;
  if (!coarse_dense) {
    Ainv.release();
    return;
  }
  Buf<int> flag(1, st);
  fill_int(flag.p, 0, 1, st);
  Ainv.ensure(size_t(n) * n, st);
  if (n <= kGjLds) {
    k_gauss_jordan_lds<<<1, 1024, 0, st>>>(n, L.A.rp.p, L.A.ci.p, L.A.v.p, Ainv.p, flag.p);
    TPF_CHECK_LAUNCH();
    int f = read_scalar(flag.p, st);
    TPF_REQUIRE(f == 0, TPF_ERR_SINGULAR, "coarsest AMG matrix (n = %d) is singular", n);
    return;
  }
  Buf<double> M(size_t(n) * 2 * n, st), fac(n, st);
  k_dense_augment<<<n, 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, L.A.v.p, M.p);
  TPF_CHECK_LAUNCH();
  k_gauss_jordan<<<1, 1024, 0, st>>>(n, M.p, fac.p, flag.p);
  TPF_CHECK_LAUNCH();
  int f = read_scalar(flag.p, st);
  TPF_REQUIRE(f == 0, TPF_ERR_SINGULAR, "coarsest AMG matrix (n = %d) is singular", n);
  k_dense_extract<<<grid_for(int64_t(n) * n, 256), 256, 0, st>>>(n, M.p, Ainv.p);
  TPF_CHECK_LAUNCH();
  note_host_sync();
  TPF_HIP(hipStreamSynchronize(st));
}

size_t Hierarchy::bytes() const {
  size_t b = Ainv.bytes() + dia0.bytes();
  for (auto& Lp : lv) {
    const Level& L = *Lp;
    b += L.A.bytes() + L.dinv.bytes() + L.mask.bytes() + L.S.bytes() + L.cf.bytes() + L.P.bytes() +
         L.R.bytes() + L.T.bytes() + L.Av32.bytes() + L.Pv32.bytes() + L.Rv32.bytes() +
         L.dinv32.bytes() + L.r.bytes() + L.y.bytes() + L.b.bytes() + L.x.bytes() + L.xa.bytes() +
         L.xb.bytes() + L.dd.bytes() + L.xa32.bytes() + L.xb32.bytes() + L.dd32.bytes() +
         L.r32.bytes() + L.y32.bytes() + L.b32.bytes() + L.x32.bytes() + L.pe_ci.bytes() +
         L.pe_v.bytes() + L.pe_v32.bytes() + L.sw_ci.bytes() + L.sw_v.bytes() + L.sw_v32.bytes() +
         L.rw_ci.bytes() + L.rw_v.bytes() + L.rw_v32.bytes();
  }
  return b;
}

// ---------------------------------------------------------------- V-cycle

template <class T>
void Hierarchy::vcycle_level(int l, const T* b, T* x, hipStream_t st, bool g_ready) {
  Level& L = *lv[l];
  int n = L.A.nrows;
  const T* Av = vals_of<T>(L.A, L.Av32);
  const T* dinv = dinv_of<T>(L);
  int lpr = lanes_per_row(n, L.A.nnz);
  unsigned blocks = grid_for(int64_t(n) * lpr, 256);
  bool last = l == int(lv.size()) - 1;
  if (last) {
    TimedScope ts(L.t_coarse.c_str(), st);
    if (coarse_dense) {
      k_dense_gemv<T><<<grid_for(int64_t(n) * kWave, 256), 256, 0, st>>>(n, Ainv.p, b, x);
    } else {
      DISPATCH_LPR(lpr, LL, {
        k_vc_two_sweeps<T, LL><<<blocks, 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, Av, dinv, b, x);
      });
    }
    TPF_CHECK_LAUNCH();
    return;
  }
  Level& C = *lv[l + 1];
  T* r = work<T>(L.r, L.r32);
  T* y = work<T>(L.y, L.y32);
  T* bc = work<T>(C.b, C.b32);
  T* xc = work<T>(C.x, C.x32);
  if (!o.fused_cycle()) {
    // V(nu1, nu2) with the generic sweeps (CSR operator on every level)
    T* xa = work<T>(L.xa, L.xa32);
    T* xb = work<T>(L.xb, L.xb32);
    const T* xpre = nullptr;
    {
      TimedScope ts(L.t_pre.c_str(), st);
      if (o.nu1 > 0) xpre = smooth<T>(L, b, nullptr, xa, xb, r, o.nu1, false, st);
      if (xpre) {
        DISPATCH_LPR(lpr, LL, {
          k_vc_pre_g<T, LL><<<blocks, 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, Av, xpre, b, r);
        });
        TPF_CHECK_LAUNCH();
      } else {
        copy(r, b, n, st);
      }
    }
    csr_spmv<T>(ref_with<T>(L.R, vals_of<T>(L.R, L.Rv32)), r, bc, st, L.t_restrict.c_str());
    vcycle_level<T>(l + 1, bc, xc, st);
    {
      const int plpr = lanes_per_row(n, L.P.nnz);
      TimedScope ts(L.t_prolong.c_str(), st);
      DISPATCH_LPR(plpr, LL, {
        k_vc_prolong_add<T, LL><<<grid_for(int64_t(n) * LL, 256), 256, 0, st>>>(
            n, L.P.rp.p, L.P.ci.p, vals_of<T>(L.P, L.Pv32), xpre, xc, y);
      });
      TPF_CHECK_LAUNCH();
    }
    {
      TimedScope ts(L.t_post.c_str(), st);
      smooth<T>(L, b, y, x, xa, xb, o.nu2, true, st);
    }
    return;
  }
  bool dia = l == 0 && dia0.ok;
  // the two-row diagonal kernels read pairs: n even and every vector aligned
  auto al2 = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % (2 * sizeof(T)) == 0; };
  const bool pairs = n % 2 == 0 && al2(b) && al2(x) && al2(r) && al2(y) && al2(dinv);
  // FP32: four rows per thread (16-byte loads) when n % 4 == 0 and every
  // vector and diagonal is 16-byte aligned
  auto al16 = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  DiagOffs doff;
  const T* dv = nullptr;
  if (dia) {
    for (int k = 0; k < kMaxDiag; ++k) doff.off[k] = dia0.off[k];
    if constexpr (std::is_same<T, float>::value)
      dv = dia0.v32.p;
    else
      dv = dia0.v.p;
  }
  const bool quads = std::is_same<T, float>::value && dia && n % 4 == 0 && al16(b) && al16(x) &&
                     al16(r) && al16(y) && al16(dinv) && al16(dv);
  // large levels form g = D^{-1} b once (in y, until the prolongation
  // overwrites it), so the residual gathers one vector
  const bool guess = dia || n >= kGuessRows;
  const T* swv = sw_vals<T>(L);
  const bool stream = L.sw_ci.p && swv;
  if (guess && !g_ready) {
    TimedScope ts(L.t_guess.c_str(), st);
    k_jacobi_guess<T><<<grid_for(n, 256), 256, 0, st>>>(n, dinv, b, y);
    TPF_CHECK_LAUNCH();
  }
  {
    TimedScope ts(L.t_pre.c_str(), st);
    if (dia) {
      if (quads) {
        DISPATCH_DIAG(dia0.K, KK, {
          k_dia_pre4f<KK><<<grid_for(n / 4, 256), 256, 0, st>>>(
              n, doff, reinterpret_cast<const float*>(dv), reinterpret_cast<const float*>(y),
              reinterpret_cast<const float*>(b), reinterpret_cast<float*>(r));
        });
      } else if (pairs) {
        DISPATCH_DIAG(dia0.K, KK, {
          k_dia_pre2<T, KK><<<grid_for(n / 2, 256), 256, 0, st>>>(n, doff, dv, y, b, r);
        });
      } else {
        DISPATCH_DIAG(dia0.K, KK, {
          k_dia_pre<T, KK><<<grid_for(n, 256), 256, 0, st>>>(n, doff, dv, y, b, r);
        });
      }
    } else if (stream) {
      DISPATCH_LPR(lpr, LL, {
        k_vc_pre_gs<T, LL><<<blocks, 256, 0, st>>>(n, L.A.rp.p, L.sw_ci.p, swv, y, b, r);
      });
    } else if (guess) {
      DISPATCH_LPR(lpr, LL, {
        k_vc_pre_g<T, LL><<<blocks, 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, Av, y, b, r);
      });
    } else {
      DISPATCH_LPR(lpr, LL, {
        k_vc_pre<T, LL><<<blocks, 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, Av, dinv, b, r);
      });
    }
    TPF_CHECK_LAUNCH();
  }
  // a large coarse level above the coarsest forms its guess in the restriction
  const bool c_guess = l + 2 < int(lv.size()) && C.A.nrows >= kGuessRows;
  if (c_guess) {
    TimedScope ts(L.t_restrict.c_str(), st);
    const int rlpr = lanes_per_row(C.A.nrows, L.R.nnz);
    const T* rwv = rw_vals<T>(L);
    if (L.rw_ci.p && rwv) {
      DISPATCH_LPR(rlpr, LL, {
        k_vc_restrict_gs<T, LL><<<grid_for(int64_t(C.A.nrows) * LL, 256), 256, 0, st>>>(
            C.A.nrows, L.R.rp.p, L.rw_ci.p, rwv, r, dinv_of<T>(C), bc, work<T>(C.y, C.y32));
      });
    } else {
      DISPATCH_LPR(rlpr, LL, {
        k_vc_restrict_guess<T, LL><<<grid_for(int64_t(C.A.nrows) * LL, 256), 256, 0, st>>>(
            C.A.nrows, L.R.rp.p, L.R.ci.p, vals_of<T>(L.R, L.Rv32), r, dinv_of<T>(C), bc,
            work<T>(C.y, C.y32));
      });
    }
    TPF_CHECK_LAUNCH();
  } else {
    csr_spmv<T>(ref_with<T>(L.R, vals_of<T>(L.R, L.Rv32)), r, bc, st, L.t_restrict.c_str());
  }
  vcycle_level<T>(l + 1, bc, xc, st, c_guess);
  {
    TimedScope ts(L.t_prolong.c_str(), st);
    const T* pev = ell_vals<T>(L);
    if (L.pe_w > 0 && pev && pairs && al2(pev)) {
      DISPATCH_ELL(L.pe_w, WW, {
        k_vc_prolong_ell2<T, WW><<<grid_for(n / 2, 256), 256, 0, st>>>(n, L.pe_ci.p, pev, dinv,
                                                                        b, xc, y);
      });
    } else if (L.pe_w > 0 && pev) {
      DISPATCH_ELL(L.pe_w, WW, {
        k_vc_prolong_ell<T, WW><<<grid_for(n, 256), 256, 0, st>>>(n, L.pe_ci.p, pev, dinv, b,
                                                                   xc, y);
      });
    } else {
      int plpr = lanes_per_row(n, L.P.nnz);
      DISPATCH_LPR(plpr, LL, {
        k_vc_prolong<T, LL><<<grid_for(int64_t(n) * LL, 256), 256, 0, st>>>(
            n, L.P.rp.p, L.P.ci.p, vals_of<T>(L.P, L.Pv32), dinv, b, xc, y);
      });
    }
    TPF_CHECK_LAUNCH();
  }
  {
    TimedScope ts(L.t_post.c_str(), st);
    if (dia) {
      if (quads) {
        DISPATCH_DIAG(dia0.K, KK, {
          k_dia_post4f<KK><<<grid_for(n / 4, 256), 256, 0, st>>>(
              n, doff, reinterpret_cast<const float*>(dv), reinterpret_cast<const float*>(dinv),
              reinterpret_cast<const float*>(b), reinterpret_cast<const float*>(y),
              reinterpret_cast<float*>(x));
        });
      } else if (pairs) {
        DISPATCH_DIAG(dia0.K, KK, {
          k_dia_post2<T, KK><<<grid_for(n / 2, 256), 256, 0, st>>>(n, doff, dv, dinv, b, y, x);
        });
      } else {
        DISPATCH_DIAG(dia0.K, KK, {
          k_dia_post<T, KK><<<grid_for(n, 256), 256, 0, st>>>(n, doff, dv, dinv, b, y, x);
        });
      }
    } else if (stream) {
      DISPATCH_LPR(lpr, LL, {
        k_vc_posts<T, LL><<<blocks, 256, 0, st>>>(n, L.A.rp.p, L.sw_ci.p, swv, dinv, b, y, x);
      });
    } else {
      DISPATCH_LPR(lpr, LL, {
        k_vc_post<T, LL><<<blocks, 256, 0, st>>>(n, L.A.rp.p, L.A.ci.p, Av, dinv, b, y, x);
      });
    }
    TPF_CHECK_LAUNCH();
  }
}

void Hierarchy::drop_graphs() {
  for (auto& g : vg) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = VGraph{};
  }
}

Hierarchy::~Hierarchy() {
  drop_graphs();
  if (cap_s) (void)hipStreamDestroy(cap_s);
}

// One V-cycle: its kernels (about five per level) are launched as one graph
// when graphs are enabled and kernel timing is off, eagerly otherwise.
template <class T>
void Hierarchy::vcycle(const T* b, T* x, hipStream_t st, bool g_ready) {
  TPF_REQUIRE(!lv.empty(), TPF_ERR_STATE, "AMG hierarchy not set up");
  if (std::is_same<T, float>::value) TPF_REQUIRE(o.fp32, TPF_ERR_STATE, "FP32 copies not built");
  TPF_REQUIRE(!g_ready || guess_buffer<T>(), TPF_ERR_STATE,
              "this hierarchy's cycle does not start from a formed guess");
  if (timing_enabled() || !graphs_enabled()) {
    vcycle_level<T>(0, b, x, st, g_ready);
    return;
  }
  VGraph& g = vg[(std::is_same<T, float>::value ? 1 : 0) + (g_ready ? 2 : 0)];
  if (!g.exec || g.b != b || g.x != x) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = VGraph{};
    if (!cap_s) TPF_HIP(hipStreamCreateWithFlags(&cap_s, hipStreamNonBlocking));
    TPF_HIP(hipStreamBeginCapture(cap_s, hipStreamCaptureModeThreadLocal));
    hipGraph_t gr = nullptr;
    try {
      vcycle_level<T>(0, b, x, cap_s, g_ready);
    } catch (...) {
      (void)hipStreamEndCapture(cap_s, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      throw;
    }
    TPF_HIP(hipStreamEndCapture(cap_s, &gr));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    TPF_HIP(e);
    g = VGraph{b, x, ex};
  }
  TPF_HIP(hipGraphLaunch(g.exec, st));
}

template const double* Hierarchy::smooth<double>(Level&, const double*, const double*, double*,
                                                  double*, double*, int, bool, hipStream_t);
template const float* Hierarchy::smooth<float>(Level&, const float*, const float*, float*, float*,
                                               float*, int, bool, hipStream_t);
template void Hierarchy::vcycle<double>(const double*, double*, hipStream_t, bool);
template void Hierarchy::vcycle<float>(const float*, float*, hipStream_t, bool);

// Level 0's guess buffer when the fused cycle starts from g = D^-1 b there
// (diagonal layout or a large CSR level above the coarsest), else null.
template <class T>
T* Hierarchy::guess_buffer() {
  if (lv.size() < 2 || !o.fused_cycle()) return nullptr;
  Level& L = *lv[0];
  if (!(dia0.ok || L.A.nrows >= kGuessRows)) return nullptr;
  return work<T>(L.y, L.y32);
}
template <class T>
const T* Hierarchy::level0_dinv() const {
  return dinv_of<T>(*lv[0]);
}
template double* Hierarchy::guess_buffer<double>();
template float* Hierarchy::guess_buffer<float>();
template const double* Hierarchy::level0_dinv<double>() const;
template const float* Hierarchy::level0_dinv<float>() const;

}  // namespace tpf
