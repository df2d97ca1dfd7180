// Block records -> handle state, and state + state merges.
//
// The partial results of disjoint row subsets are combined (sections
// "Validation and Infrastructure Testing" and "Data Representation and
// Sufficient Statistics").  Two representations are kept per entry:
//  - integer columns / pairs: exact 128-bit totals.  A block with shift K,
//    count n_b, S = sum (x - K), Q = sum (x - K)(x - K)^T contributes
//      s_i  += S_i + n_b K_i
//      C_ij += Q_ij + K_i S_j + S_i K_j + n_b K_i K_j
//    (all exact integers);
//  - every entry: (n, mean, centred co-moment M2), where a block gives
//    mean_i = K_i + S_i / n_b and M2_ij = Q_ij - S_i S_j / n_b, and two
//    partial results are combined with the pairwise update of Chan, Golub
//    and LeVeque: n = n_a + n_b, delta = mean_b - mean_a,
//    mean = mean_a + delta n_b / n, M2 = M2_a + M2_b + delta_i delta_j n_a n_b / n.
//    This never subtracts X^T X and n mu mu^T (section "Numerical
//    Considerations").
//
// Each entry (a column i, or a pair i <= j) is owned by one workgroup or
// thread that walks the partial results in a fixed order, so the result is
// deterministic.  The column means needed by a pair are recomputed by the
// pair's owner with the same operations as the column's owner, hence
// bitwise equal.
#include "common.hpp"

namespace st {
namespace {

constexpr int kThreads = 128;

struct Chan {
  double n, mi, mj, m2;
};

__device__ inline void chan_add(Chan& a, const Chan& b) {
  if (b.n == 0.0) return;
  if (a.n == 0.0) {
    a = b;
    return;
  }
  const double n = a.n + b.n;
  const double di = b.mi - a.mi, dj = b.mj - a.mj;
  const double fb = b.n / n;
  const double w = a.n * b.n / n;
  a.m2 = a.m2 + b.m2 + di * dj * w;
  a.mi = a.mi + di * fb;
  a.mj = a.mj + dj * fb;
  a.n = n;
}

// Entry e < p is column e; entry p + t is pair t of the packed triangle.
__device__ inline void entry_cols(int p, int64_t e, int* i, int* j, bool* is_col) {
  if (e < p) {
    *i = *j = (int)e;
    *is_col = true;
  } else {
    tri_inv(p, e - p, i, j);
    *is_col = false;
  }
}

__device__ inline double kval(uint64_t w, bool is_int) {
  return is_int ? (double)(int64_t)w : __longlong_as_double((long long)w);
}

__device__ inline Chan chan_of(const uint64_t* s, const Layout& L, int i, int j, int64_t t) {
  Chan c;
  c.n = (double)(int64_t)s[0];
  c.mi = __longlong_as_double((long long)s[L.off_mu + i]);
  c.mj = __longlong_as_double((long long)s[L.off_mu + j]);
  c.m2 = (t >= 0) ? __longlong_as_double((long long)s[L.off_M2 + t]) : 0.0;
  return c;
}

// State merge: next = cur followed by parts[0..nparts) in order.
__global__ __launch_bounds__(kThreads) void k_merge_l2(const uint64_t* __restrict__ cur,
                                                       const uint64_t* __restrict__ parts,
                                                       int64_t nparts, int p,
                                                       const uint8_t* __restrict__ intf,
                                                       uint64_t* __restrict__ next) {
  const Layout L = Layout::make(p);
  const int64_t E = p + L.T;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= E) return;
  int i, j;
  bool is_col;
  entry_cols(p, e, &i, &j, &is_col);
  const bool both = intf[i] && intf[j];
  const int64_t t = is_col ? -1 : e - p;
  Chan acc = chan_of(cur, L, i, j, t);
  int64_t ntot = (int64_t)cur[0];
  i128 exact = is_col ? load_i128(cur + L.off_s + 2 * i) : load_i128(cur + L.off_C + 2 * t);
  for (int64_t g = 0; g < nparts; ++g) {
    const uint64_t* s = parts + g * L.words;
    chan_add(acc, chan_of(s, L, i, j, t));
    ntot += (int64_t)s[0];
    if (is_col) exact += load_i128(s + L.off_s + 2 * i);
    else if (both) exact += load_i128(s + L.off_C + 2 * t);
  }
  if (e == 0) {
    next[0] = (uint64_t)ntot;
    next[1] = 0;
  }
  if (is_col) {
    store_i128(next + L.off_s + 2 * i, exact);
    next[L.off_mu + i] = (uint64_t)__double_as_longlong(acc.mi);
  } else {
    store_i128(next + L.off_C + 2 * t, exact);
    next[L.off_M2 + t] = (uint64_t)__double_as_longlong(acc.m2);
  }
}

// Records -> state in one pass: one workgroup per entry.  Thread t folds
// blocks t, t + 256, ... in order (the words of eight of them loaded before
// the first is folded), then the 256 partial results are combined
// by a fixed binary tree in LDS (Chan update + exact 128-bit sums) and the
// total is merged into the current state (cur -> next).  The tree shape is
// fixed, so the result is deterministic.
constexpr int kTreeThreads = 256;

__global__ __launch_bounds__(kTreeThreads) void k_merge_tree(const uint64_t* __restrict__ rec,
                                                             int64_t nblocks, int p,
                                                             const uint8_t* __restrict__ intf,
                                                             const uint64_t* __restrict__ cur,
                                                             uint64_t* __restrict__ next,
                                                             DevStatus* status) {
  __shared__ double s_n[kTreeThreads], s_mi[kTreeThreads], s_mj[kTreeThreads], s_m2[kTreeThreads];
  __shared__ uint64_t s_lo[kTreeThreads], s_hi[kTreeThreads];
  const Layout L = Layout::make(p);
  const int64_t e = blockIdx.x;
  int i, j;
  bool is_col;
  entry_cols(p, e, &i, &j, &is_col);
  const bool ii = intf[i], ij = intf[j];
  const int64_t W = rec_words(p);
  const int64_t t = is_col ? tri(p, i, i) : e - p;
  Chan acc = {0.0, 0.0, 0.0, 0.0};
  i128 exact = 0;
  uint32_t inexact = 0;
  // records b, b + 256, ... in order; the words of kU records are loaded
  // before the first of them is folded
  constexpr int kU = 8;
  for (int64_t b0 = threadIdx.x; b0 < nblocks; b0 += kTreeThreads * kU) {
    uint64_t wd[kU][7];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t b = b0 + (int64_t)u * kTreeThreads;
      const uint64_t* r = rec + (b < nblocks ? b : 0) * W;
      wd[u][0] = b < nblocks ? r[0] : 0;
      wd[u][1] = r[1];
      wd[u][2] = r[2 + i];
      wd[u][3] = r[2 + j];
      wd[u][4] = r[2 + p + i];
      wd[u][5] = r[2 + p + j];
      wd[u][6] = r[2 + 2 * p + t];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t nb = (int64_t)wd[u][0];
      if (nb == 0) continue;
      const double nbd = (double)nb;
      const uint64_t Kiw = wd[u][2], Kjw = wd[u][3];
      const double Si = __longlong_as_double((long long)wd[u][4]);
      const double Sj = __longlong_as_double((long long)wd[u][5]);
      const double Qij = __longlong_as_double((long long)wd[u][6]);
      Chan blk;
      blk.n = nbd;
      blk.mi = kval(Kiw, ii) + Si / nbd;
      blk.mj = kval(Kjw, ij) + Sj / nbd;
      blk.m2 = is_col ? 0.0 : Qij - Si * (Sj / nbd);
      chan_add(acc, blk);
      if (is_col && ii) {
        const int64_t K = (int64_t)Kiw;
        if (wd[u][1] != 0 || !(Qij < kExactQ) || K >= kMaxShift || K <= -kMaxShift) inexact = 1;
        exact += (i128)(int64_t)Si + (i128)nb * (i128)K;
      } else if (!is_col && ii && ij) {
        const i128 Ki = (i128)(int64_t)Kiw, Kj = (i128)(int64_t)Kjw;
        exact += (i128)(int64_t)Qij + Ki * (i128)(int64_t)Sj + (i128)(int64_t)Si * Kj + (i128)nb * Ki * Kj;
      }
    }
  }
  if (inexact) atomicOr(&status->bits, ST_INEXACT);
  const int tid = threadIdx.x;
  s_n[tid] = acc.n;
  s_mi[tid] = acc.mi;
  s_mj[tid] = acc.mj;
  s_m2[tid] = acc.m2;
  s_lo[tid] = (uint64_t)(u128)exact;
  s_hi[tid] = (uint64_t)((u128)exact >> 64);
  __syncthreads();
  for (int s = kTreeThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      Chan a = {s_n[tid], s_mi[tid], s_mj[tid], s_m2[tid]};
      const Chan b = {s_n[tid + s], s_mi[tid + s], s_mj[tid + s], s_m2[tid + s]};
      chan_add(a, b);
      s_n[tid] = a.n;
      s_mi[tid] = a.mi;
      s_mj[tid] = a.mj;
      s_m2[tid] = a.m2;
      const uint64_t w0[2] = {s_lo[tid], s_hi[tid]}, w1[2] = {s_lo[tid + s], s_hi[tid + s]};
      const i128 sum = load_i128(w0) + load_i128(w1);
      s_lo[tid] = (uint64_t)(u128)sum;
      s_hi[tid] = (uint64_t)((u128)sum >> 64);
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t tt = is_col ? -1 : t;
    Chan tot = chan_of(cur, L, i, j, tt);
    const Chan add = {s_n[0], s_mi[0], s_mj[0], s_m2[0]};
    chan_add(tot, add);
    const uint64_t w[2] = {s_lo[0], s_hi[0]};
    const i128 add_exact = load_i128(w);
    if (is_col) {
      store_i128(next + L.off_s + 2 * i, load_i128(cur + L.off_s + 2 * i) + add_exact);
      next[L.off_mu + i] = (uint64_t)__double_as_longlong(tot.mi);
      if (e == 0) {
        next[0] = (uint64_t)((int64_t)cur[0] + (int64_t)s_n[0]);
        next[1] = 0;
      }
    } else {
      const i128 base = load_i128(cur + L.off_C + 2 * t);
      store_i128(next + L.off_C + 2 * t, (ii && ij) ? base + add_exact : base);
      next[L.off_M2 + t] = (uint64_t)__double_as_longlong(tot.m2);
    }
  }
}

// Deferred errors of a merged source (exactness guard, text parse) carry
// over to the destination: bits are OR-ed, the smaller parse offset is kept.
__global__ void k_status_or(DevStatus* dst, const DevStatus* src) {
  if (threadIdx.x == 0) {
    const DevStatus s = *src;
    dst->bits |= s.bits;
    if (s.parse_off < dst->parse_off) dst->parse_off = s.parse_off;
  }
}

}  // namespace

void launch_status_or(DevStatus* dst, const DevStatus* src, hipStream_t s) {
  hipLaunchKernelGGL(k_status_or, dim3(1), dim3(64), 0, s, dst, src);
}

void launch_merge_records(const uint64_t* rec, int64_t nblocks, int p, const uint8_t* intf,
                          const uint64_t* cur, uint64_t* next, DevStatus* status, hipStream_t s) {
  const Layout L = Layout::make(p);
  const int64_t E = p + L.T;
  hipLaunchKernelGGL(k_merge_tree, dim3((unsigned)E), dim3(kTreeThreads), 0, s, rec, nblocks, p,
                     intf, cur, next, status);
}

void launch_merge_states(const uint64_t* a, const uint64_t* b, uint64_t* out, int p,
                         const uint8_t* intf, hipStream_t s) {
  const Layout L = Layout::make(p);
  const int64_t E = p + L.T;
  dim3 grid((unsigned)((E + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(k_merge_l2, grid, dim3(kThreads), 0, s, a, b, (int64_t)1, p, intf, out);
}

}  // namespace st
