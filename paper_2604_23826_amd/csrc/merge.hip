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
// Each entry (a column i, or a pair i <= j) is folded in a fixed order: by
// one workgroup or thread over all partial results, or, for launches with
// many block records, over fixed slices of them whose totals are then folded
// in a fixed order (the slices depend only on the record count and p), so
// the result is deterministic.  The column means needed by a pair are recomputed by the
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

// Records -> state.  One workgroup per entry (and, in the split form, per
// slice of the records): thread t folds records lo + t, lo + t + 256, ...
// below hi in order (the words of eight of them loaded before the first is
// folded), then the 256 partial results are combined by a fixed binary tree
// in LDS (Chan update + exact 128-bit sums).  The tree shape and the slices
// are fixed, so the result is deterministic.
constexpr int kTreeThreads = 256;

struct Tree {
  double n[kTreeThreads], mi[kTreeThreads], mj[kTreeThreads], m2[kTreeThreads];
  uint64_t lo[kTreeThreads], hi[kTreeThreads];
};

struct Entry {
  int i, j;
  bool is_col, ii, ij;
  int64_t t;  // packed-triangle index of (i, j); of (i, i) for a column
};

__device__ inline Entry entry_of(int p, int64_t e, const uint8_t* intf) {
  Entry E;
  entry_cols(p, e, &E.i, &E.j, &E.is_col);
  E.ii = intf[E.i];
  E.ij = intf[E.j];
  E.t = E.is_col ? tri(p, E.i, E.i) : e - p;
  return E;
}

// The fixed binary tree over the 256 slots of S (Chan update + exact sums);
// called after the slots are written and a barrier; slot 0 holds the total
// after it returns.
__device__ void tree_reduce(Tree& S) {
  const int tid = threadIdx.x;
  for (int s = kTreeThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      Chan a = {S.n[tid], S.mi[tid], S.mj[tid], S.m2[tid]};
      const Chan b = {S.n[tid + s], S.mi[tid + s], S.mj[tid + s], S.m2[tid + s]};
      chan_add(a, b);
      S.n[tid] = a.n;
      S.mi[tid] = a.mi;
      S.mj[tid] = a.mj;
      S.m2[tid] = a.m2;
      const uint64_t w0[2] = {S.lo[tid], S.hi[tid]}, w1[2] = {S.lo[tid + s], S.hi[tid + s]};
      const i128 sum = load_i128(w0) + load_i128(w1);
      S.lo[tid] = (uint64_t)(u128)sum;
      S.hi[tid] = (uint64_t)((u128)sum >> 64);
    }
    __syncthreads();
  }
}

// One block record's words (n_b, flags, K_i, K_j, S_i, S_j, Q_ij) folded
// into an entry's running total.
__device__ inline void fold_one(const uint64_t* wd, const Entry& E, Chan& acc, i128& exact,
                                uint32_t& inexact) {
  const int64_t nb = (int64_t)wd[0];
  if (nb == 0) return;
  const double nbd = (double)nb;
  const uint64_t Kiw = wd[2], Kjw = wd[3];
  const double Si = __longlong_as_double((long long)wd[4]);
  const double Sj = __longlong_as_double((long long)wd[5]);
  const double Qij = __longlong_as_double((long long)wd[6]);
  Chan blk;
  blk.n = nbd;
  blk.mi = kval(Kiw, E.ii) + Si / nbd;
  blk.mj = kval(Kjw, E.ij) + Sj / nbd;
  blk.m2 = E.is_col ? 0.0 : Qij - Si * (Sj / nbd);
  chan_add(acc, blk);
  if (E.is_col && E.ii) {
    const int64_t K = (int64_t)Kiw;
    if (wd[1] != 0 || !(Qij < kExactQ) || K >= kMaxShift || K <= -kMaxShift) inexact = 1;
    exact += (i128)(int64_t)Si + (i128)nb * (i128)K;
  } else if (!E.is_col && E.ii && E.ij) {
    const i128 Ki = (i128)(int64_t)Kiw, Kj = (i128)(int64_t)Kjw;
    exact += (i128)(int64_t)Qij + Ki * (i128)(int64_t)Sj + (i128)(int64_t)Si * Kj + (i128)nb * Ki * Kj;
  }
}

__device__ inline void load_rec_words(const uint64_t* r, int p, const Entry& E, uint64_t* wd) {
  wd[1] = r[1];
  wd[2] = r[2 + E.i];
  wd[3] = r[2 + E.j];
  wd[4] = r[2 + p + E.i];
  wd[5] = r[2 + p + E.j];
  wd[6] = r[2 + 2 * p + E.t];
}

// Leaves the entry's total over records [lo, hi) in slot 0 of S (all
// threads of the workgroup take part; S is valid after the last barrier).
__device__ void fold_records(const uint64_t* __restrict__ rec, int64_t lo, int64_t hi, int p,
                             const Entry& E, DevStatus* status, Tree& S) {
  const int64_t W = rec_words(p);
  Chan acc = {0.0, 0.0, 0.0, 0.0};
  i128 exact = 0;
  uint32_t inexact = 0;
  constexpr int kU = 8;
  for (int64_t b0 = lo + threadIdx.x; b0 < hi; b0 += kTreeThreads * kU) {
    uint64_t wd[kU][7];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t b = b0 + (int64_t)u * kTreeThreads;
      const uint64_t* r = rec + (b < hi ? b : lo) * W;
      wd[u][0] = b < hi ? r[0] : 0;
      load_rec_words(r, p, E, wd[u]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) fold_one(wd[u], E, acc, exact, inexact);
  }
  if (inexact) atomicOr(&status->bits, ST_INEXACT);
  const int tid = threadIdx.x;
  S.n[tid] = acc.n;
  S.mi[tid] = acc.mi;
  S.mj[tid] = acc.mj;
  S.m2[tid] = acc.m2;
  S.lo[tid] = (uint64_t)(u128)exact;
  S.hi[tid] = (uint64_t)((u128)exact >> 64);
  __syncthreads();
  tree_reduce(S);
}

// next = cur followed by the records' total (add, add_exact) for entry e.
__device__ void finish_entry(int p, int64_t e, const Entry& E, const Chan& add, i128 add_exact,
                             const uint64_t* __restrict__ cur, uint64_t* __restrict__ next) {
  const Layout L = Layout::make(p);
  Chan tot = chan_of(cur, L, E.i, E.j, E.is_col ? -1 : E.t);
  chan_add(tot, add);
  if (E.is_col) {
    store_i128(next + L.off_s + 2 * E.i, load_i128(cur + L.off_s + 2 * E.i) + add_exact);
    next[L.off_mu + E.i] = (uint64_t)__double_as_longlong(tot.mi);
    if (e == 0) {
      next[0] = (uint64_t)((int64_t)cur[0] + (int64_t)add.n);
      next[1] = 0;
    }
  } else {
    const i128 base = load_i128(cur + L.off_C + 2 * E.t);
    store_i128(next + L.off_C + 2 * E.t, (E.ii && E.ij) ? base + add_exact : base);
    next[L.off_M2 + E.t] = (uint64_t)__double_as_longlong(tot.m2);
  }
}

// One pass over all records per entry (few records, or many entries).
__global__ __launch_bounds__(kTreeThreads) void k_merge_tree(const uint64_t* __restrict__ rec,
                                                             int64_t nblocks, int p,
                                                             const uint8_t* __restrict__ intf,
                                                             const uint64_t* __restrict__ cur,
                                                             uint64_t* __restrict__ next,
                                                             DevStatus* status) {
  __shared__ Tree S;
  const int64_t e = blockIdx.x;
  const Entry E = entry_of(p, e, intf);
  fold_records(rec, 0, nblocks, p, E, status, S);
  if (threadIdx.x == 0) {
    const Chan add = {S.n[0], S.mi[0], S.mj[0], S.m2[0]};
    const uint64_t w[2] = {S.lo[0], S.hi[0]};
    finish_entry(p, e, E, add, load_i128(w), cur, next);
  }
}

// Split form, first stage: workgroup (e, g) folds slice g of the records
// (slices of `per` consecutive records) and writes its total to
// part[(e * nslices + g) * 6 ...] as n, mean_i, mean_j, M2 and the two
// words of the exact sum.
__global__ __launch_bounds__(kTreeThreads) void k_merge_slices(const uint64_t* __restrict__ rec,
                                                               int64_t nblocks, int64_t per, int p,
                                                               const uint8_t* __restrict__ intf,
                                                               uint64_t* __restrict__ part,
                                                               DevStatus* status) {
  __shared__ Tree S;
  const int64_t e = blockIdx.x;
  const int64_t g = blockIdx.y;
  const Entry E = entry_of(p, e, intf);
  const int64_t lo = g * per;
  const int64_t hi = lo + per < nblocks ? lo + per : nblocks;
  fold_records(rec, lo, hi, p, E, status, S);
  if (threadIdx.x == 0) {
    uint64_t* o = part + (e * (int64_t)gridDim.y + g) * 6;
    o[0] = (uint64_t)__double_as_longlong(S.n[0]);
    o[1] = (uint64_t)__double_as_longlong(S.mi[0]);
    o[2] = (uint64_t)__double_as_longlong(S.mj[0]);
    o[3] = (uint64_t)__double_as_longlong(S.m2[0]);
    o[4] = S.lo[0];
    o[5] = S.hi[0];
  }
}

// Split form for many entries, first stage: thread (e, g) folds slice g of
// the records for entry e alone (adjacent threads read adjacent words of a
// record) and writes its total as k_merge_slices does.
__global__ __launch_bounds__(256) void k_merge_slices_thr(const uint64_t* __restrict__ rec,
                                                          int64_t nblocks, int64_t per, int p,
                                                          const uint8_t* __restrict__ intf,
                                                          uint64_t* __restrict__ part,
                                                          DevStatus* status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = blockIdx.y;
  const int64_t W = rec_words(p);
  if (e >= p + Layout::make(p).T) return;
  const Entry E = entry_of(p, e, intf);
  const int64_t lo = g * per;
  const int64_t hi = lo + per < nblocks ? lo + per : nblocks;
  Chan acc = {0.0, 0.0, 0.0, 0.0};
  i128 exact = 0;
  uint32_t inexact = 0;
  constexpr int kU = 4;
  for (int64_t b0 = lo; b0 < hi; b0 += kU) {
    uint64_t wd[kU][7];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t b = b0 + u;
      const uint64_t* r = rec + (b < hi ? b : lo) * W;
      wd[u][0] = b < hi ? r[0] : 0;
      load_rec_words(r, p, E, wd[u]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) fold_one(wd[u], E, acc, exact, inexact);
  }
  if (inexact) atomicOr(&status->bits, ST_INEXACT);
  uint64_t* o = part + (e * (int64_t)gridDim.y + g) * 6;
  o[0] = (uint64_t)__double_as_longlong(acc.n);
  o[1] = (uint64_t)__double_as_longlong(acc.mi);
  o[2] = (uint64_t)__double_as_longlong(acc.mj);
  o[3] = (uint64_t)__double_as_longlong(acc.m2);
  o[4] = (uint64_t)(u128)exact;
  o[5] = (uint64_t)((u128)exact >> 64);
}

// Split form for few entries (at most 256), first stage: workgroup g folds
// slice g.  Each of its four waves takes every fourth record of the slice and
// each lane the entries lane, lane + 64, ... (adjacent lanes read adjacent
// words of a record, so a record is read once per wave); the four waves'
// totals are then combined per entry in wave order and written out as
// k_merge_slices does.
constexpr int kLanesMaxE = 256;

// KK = ceil(entries / 64) entries per lane; the words of kU records per
// wave are loaded before the first of them is folded.
template <int KK>
__global__ __launch_bounds__(256) void k_merge_slices_lanes(const uint64_t* __restrict__ rec,
                                                            int64_t nblocks, int64_t per, int p,
                                                            const uint8_t* __restrict__ intf,
                                                            uint64_t* __restrict__ part,
                                                            DevStatus* status) {
  __shared__ double s_n[4][kLanesMaxE], s_mi[4][kLanesMaxE], s_mj[4][kLanesMaxE], s_m2[4][kLanesMaxE];
  __shared__ uint64_t s_lo[4][kLanesMaxE], s_hi[4][kLanesMaxE];
  const int E = p + (int)Layout::make(p).T;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  const int64_t W = rec_words(p);
  const int64_t lo = g * per;
  const int64_t hi = lo + per < nblocks ? lo + per : nblocks;
  constexpr int kK = KK;
  constexpr int kU = KK <= 2 ? 4 : 2;
  Entry en[kK];
  Chan acc[kK];
  i128 ex[kK];
  bool has[kK];
  uint32_t inexact = 0;
#pragma unroll
  for (int k = 0; k < kK; ++k) {
    const int e = lane + 64 * k;
    has[k] = e < E;
    en[k] = entry_of(p, has[k] ? e : 0, intf);
    acc[k] = Chan{0.0, 0.0, 0.0, 0.0};
    ex[k] = 0;
  }
  // wave w folds records lo + w, lo + w + 4, ... in order
  for (int64_t b0 = lo + w; b0 < hi; b0 += 4 * kU) {
    uint64_t wd[kU][kK][7];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t b = b0 + 4 * u;
      const uint64_t* r = rec + (b < hi ? b : lo) * W;
#pragma unroll
      for (int k = 0; k < kK; ++k) {
        wd[u][k][0] = (b < hi && has[k]) ? r[0] : 0;
        load_rec_words(r, p, en[k], wd[u][k]);
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int k = 0; k < kK; ++k) fold_one(wd[u][k], en[k], acc[k], ex[k], inexact);
  }
  if (inexact) atomicOr(&status->bits, ST_INEXACT);
#pragma unroll
  for (int k = 0; k < kK; ++k) {
    const int e = lane + 64 * k;
    if (e < E) {
      s_n[w][e] = acc[k].n;
      s_mi[w][e] = acc[k].mi;
      s_mj[w][e] = acc[k].mj;
      s_m2[w][e] = acc[k].m2;
      s_lo[w][e] = (uint64_t)(u128)ex[k];
      s_hi[w][e] = (uint64_t)((u128)ex[k] >> 64);
    }
  }
  __syncthreads();
  const int e = threadIdx.x;
  if (e < E) {
    Chan a = {s_n[0][e], s_mi[0][e], s_mj[0][e], s_m2[0][e]};
    i128 x = (i128)(((u128)s_hi[0][e] << 64) | (u128)s_lo[0][e]);
    for (int v = 1; v < 4; ++v) {
      const Chan b = {s_n[v][e], s_mi[v][e], s_mj[v][e], s_m2[v][e]};
      chan_add(a, b);
      x += (i128)(((u128)s_hi[v][e] << 64) | (u128)s_lo[v][e]);
    }
    uint64_t* o = part + ((int64_t)e * (int64_t)gridDim.x + g) * 6;
    o[0] = (uint64_t)__double_as_longlong(a.n);
    o[1] = (uint64_t)__double_as_longlong(a.mi);
    o[2] = (uint64_t)__double_as_longlong(a.mj);
    o[3] = (uint64_t)__double_as_longlong(a.m2);
    o[4] = (uint64_t)(u128)x;
    o[5] = (uint64_t)((u128)x >> 64);
  }
}

// Second stage for many slices: one workgroup per entry; thread t folds the
// slice totals t, t + 256, ... in order, then the fixed LDS tree, then the
// total is merged into the state (cur -> next).
__global__ __launch_bounds__(kTreeThreads) void k_merge_slices_tree(const uint64_t* __restrict__ part,
                                                                    int64_t nslices, int p,
                                                                    const uint8_t* __restrict__ intf,
                                                                    const uint64_t* __restrict__ cur,
                                                                    uint64_t* __restrict__ next) {
  __shared__ Tree S;
  const int64_t e = blockIdx.x;
  const Entry E = entry_of(p, e, intf);
  Chan acc = {0.0, 0.0, 0.0, 0.0};
  i128 exact = 0;
  for (int64_t g = threadIdx.x; g < nslices; g += kTreeThreads) {
    const uint64_t* o = part + (e * nslices + g) * 6;
    const Chan c = {__longlong_as_double((long long)o[0]), __longlong_as_double((long long)o[1]),
                    __longlong_as_double((long long)o[2]), __longlong_as_double((long long)o[3])};
    chan_add(acc, c);
    exact += load_i128(o + 4);
  }
  const int tid = threadIdx.x;
  S.n[tid] = acc.n;
  S.mi[tid] = acc.mi;
  S.mj[tid] = acc.mj;
  S.m2[tid] = acc.m2;
  S.lo[tid] = (uint64_t)(u128)exact;
  S.hi[tid] = (uint64_t)((u128)exact >> 64);
  __syncthreads();
  tree_reduce(S);
  if (tid == 0) {
    const Chan add = {S.n[0], S.mi[0], S.mj[0], S.m2[0]};
    const uint64_t w[2] = {S.lo[0], S.hi[0]};
    finish_entry(p, e, E, add, load_i128(w), cur, next);
  }
}

// Split form, second stage: entry e's slice totals combined in slice order
// (Chan update + exact sum), then merged into the state (cur -> next).
__global__ void k_merge_slices_fold(const uint64_t* __restrict__ part, int nslices, int p,
                                    const uint8_t* __restrict__ intf,
                                    const uint64_t* __restrict__ cur, uint64_t* __restrict__ next) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Layout L = Layout::make(p);
  if (e >= p + L.T) return;
  const Entry E = entry_of(p, e, intf);
  Chan acc = {0.0, 0.0, 0.0, 0.0};
  i128 exact = 0;
  for (int g = 0; g < nslices; ++g) {
    const uint64_t* o = part + (e * nslices + g) * 6;
    const Chan c = {__longlong_as_double((long long)o[0]), __longlong_as_double((long long)o[1]),
                    __longlong_as_double((long long)o[2]), __longlong_as_double((long long)o[3])};
    chan_add(acc, c);
    exact += load_i128(o + 4);
  }
  finish_entry(p, e, E, acc, exact, cur, next);
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

// Slices of the split merge (1: the one-pass form).  Up to 256 entries and
// from 8192 records, a workgroup folds each slice of 64 records for all
// entries (lanes hold entries), and the slice totals are folded by a tree.
// Otherwise, up to 1023 entries a
// workgroup folds each (entry, slice): enough of them to cover the GPU about
// three times, each slice at least 2048 records (eight per thread).  From
// 1024 entries a thread folds each (entry, slice): 64 slices of at least 16
// records.  At most 64 slices, so an entry's total passes through at most
// ceil(slice / 256) + 8 + 64 (workgroup form) or slice + 64 (thread form)
// successive Chan updates.
struct MergePlan {
  int64_t g;
  bool per_thread;
  bool lanes;
};

static MergePlan merge_plan(int64_t nblocks, int64_t E) {
  MergePlan m;
  m.lanes = false;
  if (E <= kLanesMaxE && nblocks >= 8192) {
    m.per_thread = false;
    m.lanes = true;
    m.g = (nblocks + 63) / 64;
    return m;
  }
  m.per_thread = E >= 1024;
  int64_t g, by_len;
  if (m.per_thread) {
    g = 64;
    by_len = nblocks / 16;
  } else {
    g = (768 + E - 1) / E;
    by_len = nblocks / 2048;
  }
  if (g > by_len) g = by_len;
  if (g > 64) g = 64;
  m.g = g < 1 ? 1 : g;
  return m;
}

void launch_status_or(DevStatus* dst, const DevStatus* src, hipStream_t s) {
  hipLaunchKernelGGL(k_status_or, dim3(1), dim3(64), 0, s, dst, src);
}

int64_t merge_slice_words(int64_t nblocks, int p) {
  const int64_t E = p + Layout::make(p).T;
  const int64_t g = merge_plan(nblocks, E).g;
  return g > 1 ? E * g * 6 : 0;
}

void launch_merge_records(const uint64_t* rec, int64_t nblocks, int p, const uint8_t* intf,
                          const uint64_t* cur, uint64_t* next, DevStatus* status, hipStream_t s,
                          uint64_t* part) {
  const Layout L = Layout::make(p);
  const int64_t E = p + L.T;
  const MergePlan m = merge_plan(nblocks, E);
  const int64_t g = m.g;
  if (part == nullptr || g <= 1) {
    hipLaunchKernelGGL(k_merge_tree, dim3((unsigned)E), dim3(kTreeThreads), 0, s, rec, nblocks, p,
                       intf, cur, next, status);
    return;
  }
  const int64_t per = (nblocks + g - 1) / g;
  if (m.lanes) {
    const dim3 grid((unsigned)g), block(256);
    switch ((E + 63) / 64) {
      case 1: hipLaunchKernelGGL(k_merge_slices_lanes<1>, grid, block, 0, s, rec, nblocks, per, p, intf, part, status); break;
      case 2: hipLaunchKernelGGL(k_merge_slices_lanes<2>, grid, block, 0, s, rec, nblocks, per, p, intf, part, status); break;
      case 3: hipLaunchKernelGGL(k_merge_slices_lanes<3>, grid, block, 0, s, rec, nblocks, per, p, intf, part, status); break;
      default: hipLaunchKernelGGL(k_merge_slices_lanes<4>, grid, block, 0, s, rec, nblocks, per, p, intf, part, status); break;
    }
    hipLaunchKernelGGL(k_merge_slices_tree, dim3((unsigned)E), dim3(kTreeThreads), 0, s, part, g, p, intf,
                       cur, next);
    return;
  }
  if (m.per_thread)
    hipLaunchKernelGGL(k_merge_slices_thr, dim3((unsigned)((E + 255) / 256), (unsigned)g), dim3(256), 0,
                       s, rec, nblocks, per, p, intf, part, status);
  else
    hipLaunchKernelGGL(k_merge_slices, dim3((unsigned)E, (unsigned)g), dim3(kTreeThreads), 0, s, rec,
                       nblocks, per, p, intf, part, status);
  hipLaunchKernelGGL(k_merge_slices_fold, dim3((unsigned)((E + 63) / 64)), dim3(64), 0, s, part,
                     (int)g, p, intf, cur, next);
}

void launch_merge_states(const uint64_t* a, const uint64_t* b, uint64_t* out, int p,
                         const uint8_t* intf, hipStream_t s) {
  const Layout L = Layout::make(p);
  const int64_t E = p + L.T;
  dim3 grid((unsigned)((E + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(k_merge_l2, grid, dim3(kThreads), 0, s, a, b, (int64_t)1, p, intf, out);
}

}  // namespace st
