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
// One thread owns one entry (a column i, or a pair i <= j) and walks the
// partial results in a fixed order, so the result is deterministic.  The
// column means needed by a pair are recomputed by the pair's own thread with
// the same operations as the column's thread, hence bitwise equal.
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

// Level 1: records [g*G, min((g+1)*G, nblocks)) -> one partial state per g.
__global__ __launch_bounds__(kThreads) void k_merge_l1(const uint64_t* __restrict__ rec,
                                                       int64_t nblocks, int64_t G, int p,
                                                       const uint8_t* __restrict__ intf,
                                                       uint64_t* __restrict__ part,
                                                       DevStatus* status) {
  const Layout L = Layout::make(p);
  const int64_t E = p + L.T;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t g = blockIdx.y;
  if (e >= E) return;
  int i, j;
  bool is_col;
  entry_cols(p, e, &i, &j, &is_col);
  const bool ii = intf[i], ij = intf[j];
  const int64_t W = rec_words(p);
  const int64_t b0 = g * G, b1 = min(b0 + G, nblocks);
  Chan acc = {0.0, 0.0, 0.0, 0.0};
  i128 exact = 0;
  int64_t ntot = 0;
  uint32_t inexact = 0;
  const int64_t t = is_col ? tri(p, i, i) : e - p;
  for (int64_t b = b0; b < b1; ++b) {
    const uint64_t* r = rec + b * W;
    const int64_t nb = (int64_t)r[0];
    if (nb == 0) continue;
    const double nbd = (double)nb;
    const uint64_t Kiw = r[2 + i], Kjw = r[2 + j];
    const double Si = __longlong_as_double((long long)r[2 + p + i]);
    const double Sj = __longlong_as_double((long long)r[2 + p + j]);
    const double Qij = __longlong_as_double((long long)r[2 + 2 * p + t]);
    Chan blk;
    blk.n = nbd;
    blk.mi = kval(Kiw, ii) + Si / nbd;
    blk.mj = kval(Kjw, ij) + Sj / nbd;
    blk.m2 = is_col ? 0.0 : Qij - Si * (Sj / nbd);
    chan_add(acc, blk);
    ntot += nb;
    if (is_col && ii) {
      const int64_t K = (int64_t)Kiw;
      const double Qii = __longlong_as_double((long long)r[2 + 2 * p + tri(p, i, i)]);
      if (r[1] != 0 || !(Qii < kExactQ) || K >= kMaxShift || K <= -kMaxShift) inexact = 1;
      exact += (i128)(int64_t)Si + (i128)nb * (i128)K;
    } else if (!is_col && ii && ij) {
      const i128 Ki = (i128)(int64_t)Kiw, Kj = (i128)(int64_t)Kjw;
      exact += (i128)(int64_t)Qij + Ki * (i128)(int64_t)Sj + (i128)(int64_t)Si * Kj + (i128)nb * Ki * Kj;
    }
  }
  uint64_t* o = part + g * L.words;
  if (e == 0) {
    o[0] = (uint64_t)ntot;
    o[1] = 0;
  }
  if (is_col) {
    store_i128(o + L.off_s + 2 * i, exact);
    o[L.off_mu + i] = (uint64_t)__double_as_longlong(acc.mi);
    // (the diagonal co-moment M2_ii is written by the pair thread (i, i))
  } else {
    store_i128(o + L.off_C + 2 * t, exact);
    o[L.off_M2 + t] = (uint64_t)__double_as_longlong(acc.m2);
  }
  if (inexact) atomicOr(&status->bits, ST_INEXACT);
}

__device__ inline Chan chan_of(const uint64_t* s, const Layout& L, int i, int j, int64_t t) {
  Chan c;
  c.n = (double)(int64_t)s[0];
  c.mi = __longlong_as_double((long long)s[L.off_mu + i]);
  c.mj = __longlong_as_double((long long)s[L.off_mu + j]);
  c.m2 = (t >= 0) ? __longlong_as_double((long long)s[L.off_M2 + t]) : 0.0;
  return c;
}

// Level 2: next = cur followed by parts[0..nparts) in order.
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

}  // namespace

void launch_merge_records(const uint64_t* rec, int64_t nblocks, int p, uint32_t /*intmask_lo*/,
                          const uint8_t* intf, uint64_t* l1, int64_t l1_groups,
                          const uint64_t* cur, uint64_t* next, DevStatus* status, hipStream_t s) {
  const Layout L = Layout::make(p);
  const int64_t E = p + L.T;
  const int64_t G = (nblocks + l1_groups - 1) / l1_groups;
  const int64_t groups = (nblocks + G - 1) / G;
  dim3 grid1((unsigned)((E + kThreads - 1) / kThreads), (unsigned)groups);
  hipLaunchKernelGGL(k_merge_l1, grid1, dim3(kThreads), 0, s, rec, nblocks, G, p, intf, l1,
                     status);
  dim3 grid2((unsigned)((E + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(k_merge_l2, grid2, dim3(kThreads), 0, s, cur, l1, groups, p, intf, next);
}

void launch_merge_states(const uint64_t* a, const uint64_t* b, uint64_t* out, int p,
                         const uint8_t* intf, hipStream_t s) {
  const Layout L = Layout::make(p);
  const int64_t E = p + L.T;
  dim3 grid((unsigned)((E + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(k_merge_l2, grid, dim3(kThreads), 0, s, a, b, (int64_t)1, p, intf, out);
}

}  // namespace st
