// Means, covariance, correlation and PCA from the statistics alone.
//
// Section "Data Representation and Sufficient Statistics": once (N, s, X^T X)
// are known, means, covariance and correlation follow without the rows.
// Section "Numerical Considerations": the identifier column is excluded
// (column selection) and the covariance is never formed as X^T X - N mu mu^T
// in floating point: integer pairs use the exact numerator
// N C_ij - s_i s_j (256-bit) divided once with correct rounding, other pairs
// the merged centred co-moment M2 / (N - ddof).
// Section "Principal Component Analysis Results": eigenpairs of the (small,
// dense) correlation or covariance matrix; here a cyclic Jacobi method in
// FP64 with the round-robin (Brent-Luk) ordering, so that in every round
// q/2 disjoint rotations are computed and applied in parallel.  Output as in
// Table 3: eigenvalues descending, variance %, cumulative %, loadings (one
// row per component).
//
// One workgroup does the whole job.  The working matrices live in LDS when
// they fit (q <= kLdsQ, every PCA of the narrow path), else in a global
// scratch buffer that stays in L2; there each thread loads the 2 x 2 blocks
// of several rotations before it writes any (the blocks of one round are
// disjoint), so the L2 latency is paid once per batch.
#include "common.hpp"

namespace st {
namespace {

constexpr int kThreads = 1024;
constexpr int kLdsQ = 60;  // A and V in LDS up to this size (2 q^2 doubles <= 57.6 KiB)
constexpr int kNB = 4;     // 2 x 2 blocks per thread and batch
constexpr int kNV = 4;     // V row pairs per thread and batch
constexpr int kMaxSweeps = 60;
constexpr int kJThreads = 256;  // workgroup of the multi-kernel rounds

struct Args {
  const uint64_t* state;
  int p;
  const int32_t* sel;
  int q;
  const uint8_t* intf;
  int ddof;
  int pca_on;
  int want_vectors;
  double* out;
  double* scratch;
  int lds_mat;  // A and V in dynamic LDS after the rotation tables
  int phase;     // kAll, or kPre / kPost around the multi-kernel Jacobi
  unsigned* jc;  // kPre / kPost: [0] rotations of a sweep, [1] no decomposition (non-finite
                 // input, or n <= ddof),
                 // [2] pairs that would still rotate after the sweep
};

enum { kAll = 0, kPre = 1, kPost = 2 };

// Round-robin schedule on m (even) players: player at position pos in round
// r (0 <= pos < m, 0 <= r < m - 1).
__device__ inline int rr_player(int pos, int r, int m) {
  if (pos == 0) return 0;
  const int x = pos - 1 + r;  // < 2 (m - 1)
  return (x >= m - 1 ? x - (m - 1) : x) + 1;
}

// The two players of pair k in round r, smaller first.
__device__ inline void rr_pair(int k, int r, int m, int& a, int& b) {
  const int x = rr_player(k, r, m), y = rr_player(m - 1 - k, r, m);
  a = min(x, y);
  b = max(x, y);
}

// Rotation tables of one round: cosine, sine, tangent, the annihilated
// element and the pair (a, b) of every pair k.
struct RotTab {
  double* c;
  double* s;
  double* t;
  double* apq;
  int2* pair;
  __device__ static RotTab at(double* base, int npairs) {
    return RotTab{base, base + npairs, base + 2 * npairs, base + 3 * npairs, (int2*)(base + 4 * npairs)};
  }
};

// Whether the element apq of the pair with diagonal entries app, aqq is
// rotated away: not when it is already negligible against them.
__device__ inline bool rotates(double apq, double app, double aqq) {
  const double tol = 2.220446049250313e-16;
  return apq != 0.0 && fabs(apq) > tol * sqrt(fabs(app * aqq));
}

// Jacobi rotation annihilating A[a][b] (a < b < q), or none (c = 1, s = 0)
// when the element is already negligible.  Returns whether it rotates.
__device__ inline bool jacobi_rotation(const double* A, int q, int a, int b, double& c, double& s, double& t,
                                       double& apq) {
  c = 1.0;
  s = t = 0.0;
  apq = A[(int64_t)a * q + b];
  const double app = A[(int64_t)a * q + a], aqq = A[(int64_t)b * q + b];
  if (rotates(apq, app, aqq)) {
    const double theta = (aqq - app) / (2.0 * apq);
    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    c = 1.0 / sqrt(t * t + 1.0);
    s = t * c;
    return true;
  }
  apq = 0.0;
  return false;
}

// A <- J^T A J on the 2x2 blocks idx = u * npairs + v of one round (pair u
// rows, pair v columns), idx = start, start + stride, ...  The blocks of a
// round are disjoint, so a batch is loaded before it is written; (u, v)
// advance by stride without division.
__device__ inline void jacobi_blocks(double* A, int q, int npairs, const RotTab& R, int start, int stride) {
  const int nblk = npairs * npairs;
  const int du = stride / npairs, dv = stride % npairs;
  int cu = start / npairs, cv = start % npairs;
  for (int base = start; base < nblk; base += stride * kNB) {
    double x[kNB][4];
    int ia[kNB], ib[kNB], ic[kNB], id[kNB], iu[kNB], iv[kNB];
#pragma unroll
    for (int e = 0; e < kNB; ++e) {
      iu[e] = cu;
      iv[e] = cv;
      cv += dv;
      cu += du;
      if (cv >= npairs) {
        cv -= npairs;
        ++cu;
      }
      x[e][0] = x[e][1] = x[e][2] = x[e][3] = 0.0;
      ia[e] = ib[e] = ic[e] = id[e] = 0;
      if (base + e * stride >= nblk) continue;
      const int2 pu = R.pair[iu[e]], pv = R.pair[iv[e]];
      ia[e] = pu.x;
      ib[e] = pu.y;
      ic[e] = pv.x;
      id[e] = pv.y;
      const bool bq = ib[e] < q, dq = id[e] < q;
      x[e][0] = A[(int64_t)ia[e] * q + ic[e]];
      if (dq) x[e][1] = A[(int64_t)ia[e] * q + id[e]];
      if (bq) x[e][2] = A[(int64_t)ib[e] * q + ic[e]];
      if (bq && dq) x[e][3] = A[(int64_t)ib[e] * q + id[e]];
    }
#pragma unroll
    for (int e = 0; e < kNB; ++e) {
      if (base + e * stride >= nblk) continue;
      const int u = iu[e], v = iv[e];
      const double cu_ = R.c[u], su = R.s[u], cv_ = R.c[v], sv = R.s[v];
      if (su == 0.0 && sv == 0.0) continue;
      const int a = ia[e], b = ib[e], c2 = ic[e], d2 = id[e];
      const bool bq = b < q, dq = d2 < q;
      const double x00 = x[e][0], x01 = x[e][1], x10 = x[e][2], x11 = x[e][3];
      // rows: (row a, row b) <- (c row a - s row b, s row a + c row b)
      const double y00 = cu_ * x00 - su * x10, y10 = su * x00 + cu_ * x10;
      const double y01 = cu_ * x01 - su * x11, y11 = su * x01 + cu_ * x11;
      // columns: (col c2, col d2) <- (c col c2 - s col d2, s col c2 + c col d2)
      double z00 = cv_ * y00 - sv * y01, z01 = sv * y00 + cv_ * y01;
      double z10 = cv_ * y10 - sv * y11, z11 = sv * y10 + cv_ * y11;
      if (u == v && su != 0.0) {  // the rotated 2x2 block itself: exact update
        const double t = R.t[u], apq = R.apq[u];
        z00 = x00 - t * apq;
        z11 = x11 + t * apq;
        z01 = 0.0;
        z10 = 0.0;
      }
      A[(int64_t)a * q + c2] = z00;
      if (dq) A[(int64_t)a * q + d2] = z01;
      if (bq) A[(int64_t)b * q + c2] = z10;
      if (bq && dq) A[(int64_t)b * q + d2] = z11;
    }
  }
}

// V <- V J on the entries idx = row * npairs + u, batched the same way.
__device__ inline void jacobi_vectors(double* V, int q, int npairs, const RotTab& R, int start, int stride) {
  const int nv = q * npairs;
  const int du = stride / npairs, dv = stride % npairs;
  int vr = start / npairs, vu = start % npairs;
  for (int base = start; base < nv; base += stride * kNV) {
    double va[kNV], vb[kNV];
    int jr[kNV], ju[kNV];
#pragma unroll
    for (int e = 0; e < kNV; ++e) {
      jr[e] = vr;
      ju[e] = vu;
      vu += dv;
      vr += du;
      if (vu >= npairs) {
        vu -= npairs;
        ++vr;
      }
      va[e] = vb[e] = 0.0;
      if (base + e * stride >= nv) continue;
      const int2 pu = R.pair[ju[e]];
      if (pu.y >= q) continue;  // the dummy player of odd q
      va[e] = V[(int64_t)jr[e] * q + pu.x];
      vb[e] = V[(int64_t)jr[e] * q + pu.y];
    }
#pragma unroll
    for (int e = 0; e < kNV; ++e) {
      if (base + e * stride >= nv) continue;
      const int u = ju[e];
      const double s = R.s[u];
      if (s == 0.0) continue;  // also the dummy player's pair
      const int2 pu = R.pair[u];
      const double c = R.c[u];
      V[(int64_t)jr[e] * q + pu.x] = c * va[e] - s * vb[e];
      V[(int64_t)jr[e] * q + pu.y] = s * va[e] + c * vb[e];
    }
  }
}

// End of a sweep (after its last barrier): true when no pair would rotate,
// i.e. the next sweep would change nothing, so stopping now gives the same
// result one sweep earlier.  *cnt is workgroup-shared scratch (reset here).
__device__ inline bool converged(const double* A, int q, int tid, int nth, int* cnt) {
  if (tid == 0) *cnt = 0;
  __syncthreads();
  int any = 0;
  for (int idx = tid; idx < q * q; idx += nth) {
    const int i = idx / q, j = idx % q;
    if (i < j && rotates(A[idx], A[i * q + i], A[j * q + j])) any = 1;
  }
  if (any) atomicOr(cnt, 1);
  __syncthreads();
  return *cnt == 0;
}

__global__ __launch_bounds__(kThreads) void k_finalize(Args f) {
  const Layout L = Layout::make(f.p);
  const uint64_t* st = f.state;
  const int64_t n = (int64_t)st[0];
  const int q = f.q;
  const int tid = threadIdx.x;
  const int nth = blockDim.x;  // 64 .. kThreads, chosen by the launcher from q
  double* mean = f.out;
  double* cov = mean + q;
  double* corr = cov + (int64_t)q * q;
  double* ev = corr + (int64_t)q * q;
  double* evec = ev + q;
  double* varp = evec + (int64_t)q * q;
  double* cump = varp + q;

  __shared__ int s_flag;
  __shared__ int s_rot;
  __shared__ int s_conv;  // converged(): its own word, so that no wave reads s_rot after a reset
  const int m = q + (q & 1);  // players (a dummy when q is odd)
  const int npairs = m / 2;
  // c[npairs], s[npairs], t[npairs], apq[npairs], the round's pairs, A, V
  extern __shared__ double s_dyn[];
  const RotTab R = RotTab::at(s_dyn, npairs);
  double* A = f.scratch;
  if (f.lds_mat) A = s_dyn + 5 * npairs;
  double* V = A + (int64_t)q * q;

  if (f.phase == kPost) {
    if (f.jc[1]) return;  // no decomposition: see the pre phase
  } else if (n <= f.ddof) {
    // covariance undefined (the host reports it); nothing is computed, and
    // the exact divisions by n and n - ddof are never reached
    if (f.phase == kPre && tid == 0) {
      f.jc[0] = 0;
      f.jc[1] = 1;
    }
    return;
  } else {
  // ---- means and covariance ----
  const double dn = (double)(n - f.ddof);
  for (int a = tid; a < q; a += nth) {
    const int i = f.sel[a];
    mean[a] = f.intf[i] ? exact_mean(st, L, i, n)
                        : __longlong_as_double((long long)st[L.off_mu + i]);
  }
  // q <= 1024: every index below fits 32 bits (64-bit division is a long
  // software sequence on the GPU)
  const int qq = q * q;
  for (int idx = tid; idx < qq; idx += nth) {
    const int a = idx / q, b = idx % q;
    if (a > b) continue;
    const int i = f.sel[a], j = f.sel[b];  // sel ascending, so i <= j
    double v;
    if (f.intf[i] && f.intf[j]) v = exact_cov(st, L, i, j, n, f.ddof);
    else v = __longlong_as_double((long long)st[L.off_M2 + tri(L.p, i, j)]) / dn;
    cov[(int64_t)a * q + b] = v;
    cov[(int64_t)b * q + a] = v;
  }
  __syncthreads();
  // ---- correlation ----
  for (int idx = tid; idx < qq; idx += nth) {
    const int a = idx / q, b = idx % q;
    const double caa = cov[(int64_t)a * q + a], cbb = cov[(int64_t)b * q + b];
    double v;
    if (caa == 0.0 || cbb == 0.0) v = __builtin_nan("");
    else if (a == b) v = 1.0;
    else v = cov[idx] / sqrt(caa * cbb);
    corr[idx] = v;
  }
  if (tid == 0) s_flag = 0;
  __syncthreads();
  // ---- PCA input ----
  const double* M = f.pca_on ? cov : corr;
  int bad = 0;
  for (int idx = tid; idx < qq; idx += nth) {
    const double v = M[idx];
    if (!isfinite(v)) bad = 1;
    A[idx] = v;
    V[idx] = (idx / q == idx % q) ? 1.0 : 0.0;
  }
  if (bad) atomicOr(&s_flag, 1);
  __syncthreads();
  if (f.phase == kPre && tid == 0) {
    f.jc[0] = 0;
    f.jc[1] = s_flag ? 1u : 0u;
  }
  if (s_flag) {
    for (int idx = tid; idx < qq; idx += nth) evec[idx] = __builtin_nan("");
    for (int a = tid; a < q; a += nth) {
      ev[a] = varp[a] = cump[a] = __builtin_nan("");
    }
    return;
  }
  if (f.phase == kPre) return;

  // ---- cyclic Jacobi, round-robin ordering: q/2 disjoint rotations per round ----
  if (nth == 64 && q <= 16) {
    // One wave, at most one 2x2 block and two V row pairs per lane.  Each
    // round issues all of its loads (block, V pairs, rotation inputs) right
    // after the barrier, with the pair indices computed, not looked up; the
    // rotation tables are read once, after the second barrier.  The same
    // arithmetic as jacobi_blocks / jacobi_vectors.
    const int nblk = npairs * npairs, nv = q * npairs;
    const bool hasb = tid < nblk;
    const int bu = tid / npairs, bv = tid % npairs;
    int vrow[2], vu[2];
    bool hasv[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int idx = tid + 64 * j;
      hasv[j] = idx < nv;
      vrow[j] = idx / npairs;
      vu[j] = idx % npairs;
    }
    for (int sweep = 0; sweep < kMaxSweeps && q > 1; ++sweep) {
      if (tid == 0) s_rot = 0;
      __syncthreads();
      for (int r = 0; r < m - 1; ++r) {
        int a = 0, b = 0, c2 = 0, d2 = 0;
        double x00 = 0.0, x01 = 0.0, x10 = 0.0, x11 = 0.0;
        if (hasb) {
          rr_pair(bu, r, m, a, b);
          rr_pair(bv, r, m, c2, d2);
          x00 = A[a * q + c2];
          if (d2 < q) x01 = A[a * q + d2];
          if (b < q) x10 = A[b * q + c2];
          if (b < q && d2 < q) x11 = A[b * q + d2];
        }
        int pa[2], pb[2];
        double va[2] = {0.0, 0.0}, vb[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          rr_pair(vu[j], r, m, pa[j], pb[j]);
          if (hasv[j] && pb[j] < q) {
            va[j] = V[vrow[j] * q + pa[j]];
            vb[j] = V[vrow[j] * q + pb[j]];
          }
        }
        if (tid < npairs) {
          int ra, rb;
          rr_pair(tid, r, m, ra, rb);
          double c = 1.0, s = 0.0, t = 0.0, apq = 0.0;
          if (rb < q && jacobi_rotation(A, q, ra, rb, c, s, t, apq)) atomicAdd(&s_rot, 1);
          R.c[tid] = c;
          R.s[tid] = s;
          R.t[tid] = t;
          R.apq[tid] = apq;
        }
        __syncthreads();
        if (hasb) {
          const double cu_ = R.c[bu], su = R.s[bu], cv_ = R.c[bv], sv = R.s[bv];
          if (su != 0.0 || sv != 0.0) {
            const double y00 = cu_ * x00 - su * x10, y10 = su * x00 + cu_ * x10;
            const double y01 = cu_ * x01 - su * x11, y11 = su * x01 + cu_ * x11;
            double z00 = cv_ * y00 - sv * y01, z01 = sv * y00 + cv_ * y01;
            double z10 = cv_ * y10 - sv * y11, z11 = sv * y10 + cv_ * y11;
            if (bu == bv && su != 0.0) {  // the rotated 2x2 block itself: exact update
              const double t = R.t[bu], apq = R.apq[bu];
              z00 = x00 - t * apq;
              z11 = x11 + t * apq;
              z01 = 0.0;
              z10 = 0.0;
            }
            A[a * q + c2] = z00;
            if (d2 < q) A[a * q + d2] = z01;
            if (b < q) A[b * q + c2] = z10;
            if (b < q && d2 < q) A[b * q + d2] = z11;
          }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (!hasv[j] || pb[j] >= q) continue;
          const double s = R.s[vu[j]];
          if (s == 0.0) continue;
          const double c = R.c[vu[j]];
          V[vrow[j] * q + pa[j]] = c * va[j] - s * vb[j];
          V[vrow[j] * q + pb[j]] = s * va[j] + c * vb[j];
        }
        __syncthreads();
      }
      if (s_rot == 0 || converged(A, q, tid, nth, &s_conv)) break;
      __syncthreads();
    }
  } else {
  for (int sweep = 0; sweep < kMaxSweeps && q > 1; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      for (int k = tid; k < npairs; k += nth) {
        int a, b;
        rr_pair(k, r, m, a, b);
        double c = 1.0, s = 0.0, t = 0.0, apq = 0.0;
        if (b < q && jacobi_rotation(A, q, a, b, c, s, t, apq)) atomicAdd(&s_rot, 1);
        R.c[k] = c;
        R.s[k] = s;
        R.t[k] = t;
        R.apq[k] = apq;
        R.pair[k] = make_int2(a, b);
      }
      __syncthreads();
      jacobi_blocks(A, q, npairs, R, tid, nth);
      jacobi_vectors(V, q, npairs, R, tid, nth);
      __syncthreads();
    }
    if (s_rot == 0 || converged(A, q, tid, nth, &s_conv)) break;
    __syncthreads();
  }
  }
  }  // phase kAll / kPre

  // ---- sort descending (ties: lower index first), sign rule, percentages ----
  for (int k = tid; k < q; k += nth) {
    const double lk = A[(int64_t)k * q + k];
    int rank = 0;
    for (int j = 0; j < q; ++j) {
      const double lj = A[(int64_t)j * q + j];
      rank += (lj > lk) || (lj == lk && j < k);
    }
    ev[rank] = lk;
    // eigenvector k = column k of V; sign: largest |entry| positive (lowest index on ties)
    int arg = 0;
    double best = -1.0;
    for (int j = 0; j < q; ++j) {
      const double a = fabs(V[(int64_t)j * q + k]);
      if (a > best) {
        best = a;
        arg = j;
      }
    }
    const double sg = V[(int64_t)arg * q + k] < 0.0 ? -1.0 : 1.0;
    if (f.want_vectors)
      for (int j = 0; j < q; ++j) evec[(int64_t)rank * q + j] = sg * V[(int64_t)j * q + k];
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int k = 0; k < q; ++k) tot += ev[k];
    double run = 0.0;
    for (int k = 0; k < q; ++k) {
      varp[k] = 100.0 * ev[k] / tot;
      run += varp[k];
      cump[k] = run;
    }
  }
}

// Multi-kernel Jacobi for q > kLdsQ (A and V in global memory): one round is
// k_jrot (one workgroup: the round's rotation tables, and the count of
// rotations) followed by k_japply (the 2x2 blocks of A and the rows of V,
// spread over many workgroups).  Same arithmetic as the one-workgroup loop.
__global__ __launch_bounds__(kThreads) void k_jrot(const double* __restrict__ A, int q, int m, int r,
                                                   double* tab, unsigned* jc) {
  const int npairs = m / 2;
  const RotTab R = RotTab::at(tab, npairs);
  unsigned cnt = 0;
  for (int k = threadIdx.x; k < npairs; k += blockDim.x) {
    int a, b;
    rr_pair(k, r, m, a, b);
    double c = 1.0, s = 0.0, t = 0.0, apq = 0.0;
    if (!jc[1] && b < q && jacobi_rotation(A, q, a, b, c, s, t, apq)) ++cnt;
    R.c[k] = c;
    R.s[k] = s;
    R.t[k] = t;
    R.apq[k] = apq;
    R.pair[k] = make_int2(a, b);
  }
  if (cnt) atomicAdd(&jc[0], cnt);
}

// End of a sweep: count (into jc[2]) the pairs that would still rotate; none
// means the next sweep would change nothing.
__global__ __launch_bounds__(kJThreads) void k_jcheck(const double* __restrict__ A, int q, unsigned* jc) {
  const int64_t n = (int64_t)q * q;
  unsigned any = 0;
  for (int64_t idx = (int64_t)blockIdx.x * kJThreads + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * kJThreads) {
    const int i = (int)(idx / q), j = (int)(idx % q);
    if (i < j && rotates(A[idx], A[(int64_t)i * q + i], A[(int64_t)j * q + j])) any = 1;
  }
  if (any) atomicOr(&jc[2], 1u);
}

__global__ __launch_bounds__(kJThreads) void k_japply(double* A, double* V, int q, int m, const double* tab) {
  const int npairs = m / 2;
  extern __shared__ double s_tab[];  // the round's tables, copied once
  for (int i = threadIdx.x; i < 5 * npairs; i += kJThreads) s_tab[i] = tab[i];
  __syncthreads();
  const RotTab R = RotTab::at(s_tab, npairs);
  const int start = blockIdx.x * kJThreads + threadIdx.x, stride = gridDim.x * kJThreads;
  jacobi_blocks(A, q, npairs, R, start, stride);
  jacobi_vectors(V, q, npairs, R, start, stride);
}

__global__ void k_raw(const uint64_t* st, int p, const uint8_t* intf, double* out) {
  // out: s_f64[p], C_f64[p*p]
  const Layout L = Layout::make(p);
  const int64_t n = (int64_t)st[0];
  const double dn = (double)n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < p + (int64_t)p * p;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx < p) {
      const int i = (int)idx;
      double v;
      if (intf[i]) {
        bool neg;
        const u128 m = abs128(load_i128(st + L.off_s + 2 * i), &neg);
        v = u256_div_to_double(neg, u256_from_u128(m), u256_from_u128(1));
      } else {
        v = dn * __longlong_as_double((long long)st[L.off_mu + i]);
      }
      out[i] = v;
    } else {
      const int64_t e = idx - p;
      int i = (int)(e / p), j = (int)(e % p);
      if (i > j) {
        const int x = i;
        i = j;
        j = x;
      }
      double v;
      if (intf[i] && intf[j]) {
        bool neg;
        const u128 m = abs128(load_i128(st + L.off_C + 2 * tri(p, i, j)), &neg);
        v = u256_div_to_double(neg, u256_from_u128(m), u256_from_u128(1));
      } else {
        const double mi = __longlong_as_double((long long)st[L.off_mu + i]);
        const double mj = __longlong_as_double((long long)st[L.off_mu + j]);
        v = __longlong_as_double((long long)st[L.off_M2 + tri(p, i, j)]) + dn * mi * mj;
      }
      out[idx] = v;
    }
  }
}

}  // namespace

hipError_t launch_finalize(const FinalizeLaunch& F, hipStream_t s) {
  Args a;
  a.state = F.state;
  a.p = F.p;
  a.sel = F.sel_dev;
  a.q = F.q;
  a.intf = F.intflags_dev;
  a.ddof = F.ddof;
  a.pca_on = F.pca_on;
  a.want_vectors = F.want_vectors;
  a.out = F.out;
  a.scratch = F.scratch;
  a.jc = F.jc;
  const int npairs = (F.q + (F.q & 1)) / 2;
  size_t shm = (size_t)npairs * 5 * sizeof(double);
  a.lds_mat = F.q <= kLdsQ;
  if (a.lds_mat) {
    // one workgroup does everything; one wave for the small matrices of the
    // narrow path (its barriers cost nothing)
    shm += 2 * sizeof(double) * (size_t)F.q * F.q;
    a.phase = kAll;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(F.q <= 16 ? 64 : 256), shm, s, a);
    return hipGetLastError();
  }
  // wide matrices: the Jacobi rounds as separate kernels over the whole GPU,
  // sweeps until one makes no rotation
  a.phase = kPre;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), shm, s, a);
  hipError_t e = hipGetLastError();
  double* A = F.scratch;
  double* V = A + (int64_t)F.q * F.q;
  const int m = 2 * npairs;
  int dev = 0, ncu = 256;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t work = (int64_t)npairs * npairs + (int64_t)F.q * npairs;
  const int nwg = (int)std::max<int64_t>(1, std::min<int64_t>((work + kJThreads * kNB - 1) / (kJThreads * kNB), 4 * ncu));
  const size_t tab_shm = (size_t)npairs * 5 * sizeof(double);
  for (int sweep = 0; sweep < kMaxSweeps && F.q > 1 && e == hipSuccess; ++sweep) {
    e = hipMemsetAsync(F.jc, 0, sizeof(unsigned), s);
    for (int r = 0; r < m - 1 && e == hipSuccess; ++r) {
      hipLaunchKernelGGL(k_jrot, dim3(1), dim3(kThreads), 0, s, A, F.q, m, r, F.jtab, F.jc);
      hipLaunchKernelGGL(k_japply, dim3(nwg), dim3(kJThreads), tab_shm, s, A, V, F.q, m, F.jtab);
      e = hipGetLastError();
    }
    // stop when this sweep rotated nothing, or when nothing would rotate in
    // the next one (same result, one sweep earlier)
    if (e == hipSuccess) e = hipMemsetAsync(F.jc + 2, 0, sizeof(unsigned), s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_jcheck, dim3(nwg), dim3(kJThreads), 0, s, A, F.q, F.jc);
      e = hipGetLastError();
    }
    unsigned w[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(w, F.jc, sizeof w, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess || w[0] == 0 || w[2] == 0) break;
  }
  if (e != hipSuccess) return e;
  a.phase = kPost;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), shm, s, a);
  return hipGetLastError();
}

void launch_raw(const uint64_t* state, int p, const uint8_t* intf, double* out, hipStream_t s) {
  const int64_t work = p + (int64_t)p * p;
  const unsigned blocks = (unsigned)std::min<int64_t>((work + 255) / 256, 1024);
  hipLaunchKernelGGL(k_raw, dim3(blocks), dim3(256), 0, s, state, p, intf, out);
}

}  // namespace st
