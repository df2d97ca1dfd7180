// Statistics with missing values (NaN), pairwise-complete: for every pair of
// columns (i, j) the rows where both are present, their count n_ij, the two
// columns' means over those rows and the centred co-moments -- the
// missing-value extension the paper names as future work (section
// "Limitations and Future Work").  Covariance and correlation of a pair use
// only its complete rows (pairwise deletion).
//
// Per block of rows, with K_i the first present value of column i in the
// block (shift) and, per row, d_i = x_i - K_i and v_i = 1 where x_i is present
// (d_i = v_i = 0 where it is NaN), four matrix products over the block's rows
// hold everything:
//     N = V^T V          n_ij
//     S = D^T V          S[i][j] = sum over rows with j present of d_i
//     Q = (D o D)^T V    Q[i][j] = sum over rows with j present of d_i^2
//     C = D^T D          sum of d_i d_j (zero wherever either is missing)
// On the FP64 matrix cores (v_mfma_f64_16x16x4f64, p <= 16) a lane holds
// d, d^2 and v of column (lane % 16) in row (lane / 16) of a 4-row step,
// which is its element of both operands: four products per 4 rows.
#include <cstring>
#include <vector>

#include "common.hpp"
#include "runtime.hpp"

namespace st {
namespace pw {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kMaxP = 16;
constexpr int kScan = 256;  // rows searched for a block's shift

// Block record: n (rows), K[16], then the four 16 x 16 tiles N, S, Q, C.
constexpr int kRecWords = 1 + kMaxP + 4 * 256;

struct Args {
  const char* colbase[kMaxP];
  int64_t colstride[kMaxP];
  int32_t dtype[kMaxP];  // STATS_F32 / STATS_F64
  int p;
  int64_t nrows, R;
  double* rec;
};

__device__ inline double load_value(const Args& a, int c, int64_t r) {
  const char* ptr = a.colbase[c] + r * a.colstride[c];
  return a.dtype[c] == STATS_F32 ? (double)__builtin_nontemporal_load((const float*)ptr)
                                 : __builtin_nontemporal_load((const double*)ptr);
}

__global__ __launch_bounds__(kThreads) void k_pairwise(Args a) {
  __shared__ double sK[kMaxP];
  __shared__ double red[4][4][4][64];  // [wave][tile][register][lane]
  const int64_t r0 = (int64_t)blockIdx.x * a.R, r1 = min(r0 + a.R, a.nrows);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const bool cv = col < a.p;
  // shift: the first present value of each column among the block's first rows
  if (threadIdx.x < kMaxP) {
    double K = 0.0;
    if ((int)threadIdx.x < a.p) {
      const int64_t lim = min(r1, r0 + kScan);
      for (int64_t r = r0; r < lim; ++r) {
        const double x = load_value(a, threadIdx.x, r);
        if (x == x) {
          K = x;
          break;
        }
      }
    }
    sK[threadIdx.x] = K;
  }
  __syncthreads();
  const double K = cv ? sK[col] : 0.0;
  d4 tN = {}, tS = {}, tQ = {}, tC = {};
  // wave w takes rows r0 + 4 (w + 4 s) + kq: 16 rows per step of the workgroup
  constexpr int U = 4;  // steps in flight per wave
  for (int64_t base = r0 + 4 * wave; base < r1; base += 16 * U) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = base + 16 * u + kq;
      x[u] = (cv && r < r1) ? load_value(a, col, r) : __builtin_nan("");
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = x[u] == x[u];
      const double d = ok ? x[u] - K : 0.0;
      const double v = ok ? 1.0 : 0.0;
      const double d2 = d * d;
      tN = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, tN, 0, 0, 0);
      tS = __builtin_amdgcn_mfma_f64_16x16x4f64(d, v, tS, 0, 0, 0);
      tQ = __builtin_amdgcn_mfma_f64_16x16x4f64(d2, v, tQ, 0, 0, 0);
      tC = __builtin_amdgcn_mfma_f64_16x16x4f64(d, d, tC, 0, 0, 0);
    }
  }
  // the four waves' tiles, added in a fixed order
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    red[wave][0][k][lane] = tN[k];
    red[wave][1][k][lane] = tS[k];
    red[wave][2][k][lane] = tQ[k];
    red[wave][3][k][lane] = tC[k];
  }
  __syncthreads();
  double* out = a.rec + (int64_t)blockIdx.x * kRecWords;
  // register k of lane l holds D[4 k + l / 16][l % 16]
  for (int e = threadIdx.x; e < 4 * 4 * 64; e += kThreads) {
    const int t = e >> 8, k = (e >> 6) & 3, l = e & 63;
    const double v = red[0][t][k][l] + red[1][t][k][l] + red[2][t][k][l] + red[3][t][k][l];
    const int i = 4 * k + (l >> 4), j = l & 15;
    out[1 + kMaxP + 256 * t + 16 * i + j] = v;
  }
  if (threadIdx.x < kMaxP) out[1 + threadIdx.x] = sK[threadIdx.x];
  if (threadIdx.x == 0) out[0] = (double)(r1 - r0);
}

// ---- merge: block records -> per-pair state, states -> state ----------------
//
// State of pair t = (i, j), i <= j (packed upper triangle): n, mean_i, mean_j,
// M2_ii, M2_jj, C_ij over the rows where both columns are present.  Blocks
// are combined by the pairwise update of Chan, Golub and LeVeque (the same
// update as the complete-data path), along a fixed tree, so results repeat
// bit for bit.

struct Pair {
  double n, mi, mj, m2i, m2j, c;
};

__device__ inline Pair combine(const Pair& a, const Pair& b) {
  if (b.n == 0.0) return a;
  if (a.n == 0.0) return b;
  Pair r;
  r.n = a.n + b.n;
  const double di = b.mi - a.mi, dj = b.mj - a.mj, f = a.n * b.n / r.n;
  r.mi = a.mi + di * (b.n / r.n);
  r.mj = a.mj + dj * (b.n / r.n);
  r.m2i = a.m2i + b.m2i + di * di * f;
  r.m2j = a.m2j + b.m2j + dj * dj * f;
  r.c = a.c + b.c + di * dj * f;
  return r;
}

// Pair (i, j) of block record rec (shifted sums -> centred form).
__device__ inline Pair from_record(const double* rec, int i, int j) {
  const double* K = rec + 1;
  const double* N = rec + 1 + kMaxP;
  const double* S = N + 256;
  const double* Q = S + 256;
  const double* C = Q + 256;
  Pair r;
  r.n = N[16 * i + j];
  if (r.n == 0.0) return Pair{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double si = S[16 * i + j], sj = S[16 * j + i];
  r.mi = K[i] + si / r.n;
  r.mj = K[j] + sj / r.n;
  r.m2i = Q[16 * i + j] - si * (si / r.n);
  r.m2j = Q[16 * j + i] - sj * (sj / r.n);
  r.c = C[16 * i + j] - si * (sj / r.n);
  return r;
}

__device__ inline void pair_of(int p, int t, int& i, int& j) {
  i = 0;
  int rem = t;
  while (rem >= p - i) {
    rem -= p - i;
    ++i;
  }
  j = i + rem;
}

constexpr int kMergeThreads = 256;

// One workgroup per pair: thread k combines a contiguous range of blocks,
// then a fixed binary tree over the threads; the result is combined with the
// incoming state (cur) into next.
__global__ __launch_bounds__(kMergeThreads) void k_pw_merge(const double* rec, int64_t nblocks, int p,
                                                           const double* cur, double* next) {
  __shared__ Pair part[kMergeThreads];
  const int t = blockIdx.x;
  int i, j;
  pair_of(p, t, i, j);
  const int64_t a0 = nblocks * threadIdx.x / kMergeThreads, a1 = nblocks * (threadIdx.x + 1) / kMergeThreads;
  Pair acc{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t b = a0; b < a1; ++b) acc = combine(acc, from_record(rec + b * kRecWords, i, j));
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kMergeThreads / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] = combine(part[threadIdx.x], part[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double* c = cur + 6 * t;
    const Pair old{c[0], c[1], c[2], c[3], c[4], c[5]};
    const Pair r = combine(old, part[0]);
    double* o = next + 6 * t;
    o[0] = r.n;
    o[1] = r.mi;
    o[2] = r.mj;
    o[3] = r.m2i;
    o[4] = r.m2j;
    o[5] = r.c;
  }
}

__global__ void k_pw_merge_states(const double* a, const double* b, double* out, int T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double* x = a + 6 * t;
  const double* y = b + 6 * t;
  const Pair r = combine(Pair{x[0], x[1], x[2], x[3], x[4], x[5]}, Pair{y[0], y[1], y[2], y[3], y[4], y[5]});
  double* o = out + 6 * t;
  o[0] = r.n;
  o[1] = r.mi;
  o[2] = r.mj;
  o[3] = r.m2i;
  o[4] = r.m2j;
  o[5] = r.c;
}

// n, mean (each column over its own present rows), cov and corr (p x p):
// out = [n (p*p) | mean (p) | cov (p*p) | corr (p*p)].
__global__ void k_pw_finalize(const double* st, int p, int ddof, double* out) {
  const int T = p * (p + 1) / 2;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  int i, j;
  pair_of(p, t, i, j);
  const double* s = st + 6 * t;
  const double n = s[0];
  const double nan = __builtin_nan("");
  double* on = out;
  double* om = out + p * p;
  double* ocov = om + p;
  double* ocorr = ocov + p * p;
  on[i * p + j] = on[j * p + i] = n;
  const double cov = n > (double)ddof ? s[5] / (n - (double)ddof) : nan;
  ocov[i * p + j] = ocov[j * p + i] = cov;
  double corr = nan;
  if (s[3] > 0.0 && s[4] > 0.0) corr = i == j ? 1.0 : s[5] / sqrt(s[3] * s[4]);
  ocorr[i * p + j] = ocorr[j * p + i] = corr;
  if (i == j) om[i] = n > 0.0 ? s[1] : nan;
}

}  // namespace pw

// ---- host ----------------------------------------------------------------------

int pairwise_state_words(int p) { return 6 * p * (p + 1) / 2; }

int accumulate_pairwise(stats_ctx* h, const void* const* planes, int64_t nrows) {
  const int p = h->p;
  pw::Args a;
  memset(&a, 0, sizeof a);
  a.p = p;
  for (int c = 0; c < p; ++c) {
    const stats_column& col = h->cols[c];
    a.colbase[c] = (const char*)planes[col.plane] + col.byte_offset;
    a.colstride[c] = h->row_stride[col.plane];
    a.dtype[c] = col.dtype;
  }
  const int64_t R = block_rows_for(h, nrows);
  const int64_t max_rows = std::max<int64_t>(R, std::min<int64_t>(16384 * R, ((int64_t)1 << 28) / R * R));
  const int T = p * (p + 1) / 2;
  int64_t done = 0;
  while (done < nrows) {
    const int64_t rows = std::min(nrows - done, max_rows);
    const int64_t nblocks = (rows + R - 1) / R;
    int rc = ensure_dev(h, (void**)&h->rec, &h->rec_cap, (size_t)(nblocks * pw::kRecWords * 8));
    if (rc) return rc;
    pw::Args b = a;
    for (int c = 0; c < p; ++c) b.colbase[c] = a.colbase[c] + done * a.colstride[c];
    b.nrows = rows;
    b.R = R;
    b.rec = (double*)h->rec;
    {
      Timer t;
      t.begin(h, STATS_K_ACCUM);
      hipLaunchKernelGGL(pw::k_pairwise, dim3((unsigned)nblocks), dim3(pw::kThreads), 0, h->stream, b);
      t.end();
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "pairwise kernel launch");
    {
      Timer t;
      t.begin(h, STATS_K_MERGE);
      hipLaunchKernelGGL(pw::k_pw_merge, dim3((unsigned)T), dim3(pw::kMergeThreads), 0, h->stream,
                         (const double*)h->rec, nblocks, p, (const double*)h->state[h->cur],
                         (double*)h->state[h->cur ^ 1]);
      t.end();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "pairwise merge launch");
    h->cur ^= 1;
    done += rows;
  }
  return STATS_OK;
}

void launch_pairwise_merge_states(const uint64_t* a, const uint64_t* b, uint64_t* out, int p, hipStream_t s) {
  const int T = p * (p + 1) / 2;
  hipLaunchKernelGGL(pw::k_pw_merge_states, dim3((T + 255) / 256), dim3(256), 0, s, (const double*)a,
                     (const double*)b, (double*)out, T);
}

}  // namespace st

using namespace st;

extern "C" int stats_finalize_pairwise(stats_ctx* h, int32_t ddof, int64_t* n_out, double* mean_out,
                                       double* cov_out, double* corr_out) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (!(h->flags & STATS_CFG_PAIRWISE)) return fail(STATS_E_STATE, "not a pairwise (missing-value) handle");
  if (ddof < 0) return fail(STATS_E_ARG, "ddof < 0");
  const int p = h->p;
  DeviceGuard g(h->device);
  if (!g.ok) return fail(STATS_E_HIP, "hipSetDevice failed");
  const size_t words = (size_t)3 * p * p + p;
  int rc = ensure_dev(h, (void**)&h->fin_out, &h->fin_out_cap, words * 8);
  if (rc) return rc;
  const int T = p * (p + 1) / 2;
  {
    Timer t;
    t.begin(h, STATS_K_FINALIZE);
    hipLaunchKernelGGL(pw::k_pw_finalize, dim3((T + 255) / 256), dim3(256), 0, h->stream,
                       (const double*)h->state[h->cur], p, ddof, h->fin_out);
    t.end();
  }
  std::vector<double> host(words);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(host.data(), h->fin_out, words * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "pairwise finalize");
  collect_timings(h);
  const double* hn = host.data();
  const double* hm = hn + (size_t)p * p;
  const double* hc = hm + p;
  const double* hr = hc + (size_t)p * p;
  for (int k = 0; k < p * p; ++k) {
    if (n_out) n_out[k] = (int64_t)hn[k];
    if (cov_out) cov_out[k] = hc[k];
    if (corr_out) corr_out[k] = hr[k];
  }
  if (mean_out)
    for (int c = 0; c < p; ++c) mean_out[c] = hm[c];
  return STATS_OK;
}
