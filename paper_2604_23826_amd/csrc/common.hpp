// Internal definitions shared by the kernels and the runtime of libstats.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/stats.h"

namespace st {

// Packed index of (i, j), i <= j, in the row-major upper triangle of a p x p
// matrix; T = p (p + 1) / 2 entries.
__host__ __device__ inline int64_t tri(int p, int i, int j) {
  return (int64_t)i * p - (int64_t)i * (i - 1) / 2 + (j - i);
}
__host__ __device__ inline int64_t tri_count(int p) { return (int64_t)p * (p + 1) / 2; }

// Inverse of tri(): the (i, j) of packed index t.
__host__ __device__ inline void tri_inv(int p, int64_t t, int* i, int* j) {
  int a = 0;
  int64_t rowlen = p;
  while (t >= rowlen) {
    t -= rowlen;
    --rowlen;
    ++a;
  }
  *i = a;
  *j = a + (int)t;
}

// ---- statistics state of one handle (or one group), in 64-bit words --------
//   [0]            n
//   [1]            reserved
//   s_int   p x2   exact column sums (int128 as lo, hi) of integer columns
//   C_int   T x2   exact cross products of integer pairs
//   mu      p      running mean of every column (FP64)
//   M2      T      centred co-moment of every pair (FP64)
struct Layout {
  int p;
  int64_t T;
  int64_t off_s, off_C, off_mu, off_M2, words;
  __host__ __device__ static Layout make(int p) {
    Layout L;
    L.p = p;
    L.T = tri_count(p);
    L.off_s = 2;
    L.off_C = L.off_s + 2 * (int64_t)p;
    L.off_mu = L.off_C + 2 * L.T;
    L.off_M2 = L.off_mu + p;
    L.words = L.off_M2 + L.T;
    return L;
  }
};

// Block record written by the reduction kernels, in 64-bit words:
//   [0] n_b   [1] flags (bit c: integer column c held a non-integer value)
//   K[p]      shift = the block's first row (int64 for integer columns,
//             FP64 bits otherwise)
//   S[p]      sum of (x - K)            (FP64; exact integers for int columns)
//   Q[T]      sum of (x - K)(x - K)^T   (FP64; exact integers for int pairs)
__host__ __device__ inline int64_t rec_words(int p) { return 2 + 2 * (int64_t)p + tri_count(p); }

// Exactness limits for integer columns: per block, every partial sum of
// (x - K)^2 stays below 2^53 so FP64 accumulation is exact (Cauchy-Schwarz
// bounds the cross terms by the same number); the shift itself must satisfy
// |K| < 2^40 so the 128-bit totals cannot overflow for N < 2^46 rows.
constexpr double kExactQ = 9007199254740992.0;  // 2^53
constexpr int64_t kMaxShift = (int64_t)1 << 40;

// Status word bits (device, one per handle).
enum : uint32_t { ST_INEXACT = 1u, ST_PARSE = 2u };

struct DevStatus {
  uint32_t bits;
  uint32_t pad;
  unsigned long long parse_off;  // smallest offending byte offset (atomicMin)
};

// Column description handed to kernels.
struct ColInfo {
  int p;
  uint32_t intmask_lo;  // bits for columns 0..31 (small-p kernels use these)
  uint32_t chkmask_lo;  // F32/F64 columns flagged INTEGER (values checked)
};

// ---- 128 / 256-bit integer helpers ------------------------------------------
typedef __int128 i128;
typedef unsigned __int128 u128;

__host__ __device__ inline i128 load_i128(const uint64_t* w) {
  return (i128)(((u128)w[1] << 64) | (u128)w[0]);
}
__host__ __device__ inline void store_i128(uint64_t* w, i128 v) {
  w[0] = (uint64_t)(u128)v;
  w[1] = (uint64_t)((u128)v >> 64);
}

struct U256 {
  uint64_t w[4];  // little-endian limbs
};

__host__ __device__ inline U256 u256_from_u128(u128 v) {
  U256 r;
  r.w[0] = (uint64_t)v;
  r.w[1] = (uint64_t)(v >> 64);
  r.w[2] = 0;
  r.w[3] = 0;
  return r;
}

__host__ __device__ inline U256 u256_mul128(u128 a, u128 b) {
  // schoolbook on 64-bit limbs
  uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64), b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
  u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
  U256 r;
  r.w[0] = (uint64_t)p00;
  u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
  r.w[1] = (uint64_t)mid;
  u128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
  r.w[2] = (uint64_t)hi;
  r.w[3] = (uint64_t)((hi >> 64) + (p11 >> 64));
  return r;
}

__host__ __device__ inline int u256_cmp(const U256& a, const U256& b) {
  for (int k = 3; k >= 0; --k) {
    if (a.w[k] != b.w[k]) return a.w[k] < b.w[k] ? -1 : 1;
  }
  return 0;
}

__host__ __device__ inline U256 u256_sub(const U256& a, const U256& b) {
  U256 r;
  uint64_t borrow = 0;
  for (int k = 0; k < 4; ++k) {
    uint64_t x = a.w[k], y = b.w[k];
    uint64_t d = x - y - borrow;
    borrow = (x < y) || (x - y < borrow) ? 1 : 0;
    r.w[k] = d;
  }
  return r;
}

__host__ __device__ inline bool u256_is_zero(const U256& a) {
  return (a.w[0] | a.w[1] | a.w[2] | a.w[3]) == 0;
}

__host__ __device__ inline int u256_bitlen(const U256& a) {
  for (int k = 3; k >= 0; --k)
    if (a.w[k]) return 64 * k + 64 - __builtin_clzll(a.w[k]);
  return 0;
}

// a * m for m < 2^64 (the product must fit in 256 bits).
__host__ __device__ inline U256 u256_mul64(const U256& a, uint64_t m) {
  U256 r;
  u128 carry = 0;
  for (int k = 0; k < 4; ++k) {
    const u128 t = (u128)a.w[k] * m + carry;
    r.w[k] = (uint64_t)t;
    carry = t >> 64;
  }
  return r;
}

__host__ __device__ inline U256 u256_shl(const U256& a, int s) {
  U256 r = {{0, 0, 0, 0}};
  if (s >= 256) return r;
  const int q = s >> 6, b = s & 63;
  for (int k = 3; k >= 0; --k) {
    int src = k - q;
    if (src < 0) continue;
    uint64_t v = a.w[src] << b;
    if (b && src - 1 >= 0) v |= a.w[src - 1] >> (64 - b);
    r.w[k] = v;
  }
  return r;
}

__host__ __device__ inline U256 u256_shr1(const U256& a) {
  U256 r;
  for (int k = 0; k < 4; ++k) r.w[k] = (a.w[k] >> 1) | (k < 3 ? a.w[k + 1] << 63 : 0);
  return r;
}

// Correctly rounded (to nearest, ties to even) value of (neg ? -1 : 1) * a / b
// for b > 0 and a < 2^190.  Exact long division of the top 65 quotient bits
// plus a sticky remainder bit (the general case of u256_div_to_double).
__host__ __device__ inline double u256_div_long(bool neg, U256 a, U256 b) {
  if (u256_is_zero(a)) return 0.0;
  const int la = u256_bitlen(a), lb = u256_bitlen(b);
  int k = 64 - (la - lb);  // quotient of (a * 2^k) / b has 64 or 65 bits
  U256 N = a, D = b;
  if (k >= 0) N = u256_shl(a, k);
  else D = u256_shl(b, -k);
  // shift-subtract division, quotient < 2^66
  const int s = u256_bitlen(N) - u256_bitlen(D);
  U256 Ds = u256_shl(D, s < 0 ? 0 : s);
  uint64_t qhi = 0;  // bits 64.. of the quotient
  uint64_t q = 0;
  for (int i = (s < 0 ? -1 : s); i >= 0; --i) {
    if (u256_cmp(N, Ds) >= 0) {
      N = u256_sub(N, Ds);
      if (i >= 64) qhi |= (uint64_t)1 << (i - 64);
      else q |= (uint64_t)1 << i;
    }
    Ds = u256_shr1(Ds);
  }
  bool sticky = !u256_is_zero(N);
  int e = -k;
  while (qhi) {  // bring the quotient below 2^64
    sticky = sticky || (q & 1);
    q = (q >> 1) | (qhi << 63);
    qhi >>= 1;
    ++e;
  }
  while (q < ((uint64_t)1 << 63)) {  // (cannot happen with the chosen k, kept for safety)
    q <<= 1;
    --e;
  }
  const uint64_t low = q & 0x7FF;
  uint64_t m = q >> 11;
  e += 11;
  const uint64_t half = 0x400;
  if (low > half || (low == half && (sticky || (m & 1)))) ++m;
  if (m == ((uint64_t)1 << 53)) {
    m >>= 1;
    ++e;
  }
  double r = ldexp((double)m, e);
  return neg ? -r : r;
}

// a * 2^(1 - e) compared with t * b (t odd): the sign of a / b - (t / 2) 2^e.
__host__ __device__ inline int u256_cmp_half(const U256& a, const U256& b, int e, uint64_t t) {
  U256 x = a, y = u256_mul64(b, t);
  if (1 - e >= 0) x = u256_shl(a, 1 - e);
  else y = u256_shl(y, e - 1);
  return u256_cmp(x, y);
}

// Top 64 bits of a (bit length la > 0) times 2^(la - 64), as a double.
__host__ __device__ inline double u256_approx(const U256& a, int la) {
  if (la <= 64) return (double)a.w[0];
  const int sh = la - 64, q = sh >> 6, r = sh & 63;
  uint64_t v = a.w[q] >> r;
  if (r && q + 1 < 4) v |= a.w[q + 1] << (64 - r);
  return ldexp((double)v, sh);
}

// Correctly rounded (to nearest, ties to even) value of (neg ? -1 : 1) * a / b
// for b > 0, a < 2^190, b < 2^190.  A double quotient of the leading bits is
// within a few units in the last place; its mantissa m is then moved to the
// right neighbour by exact comparisons of a / b with the midpoints
// (m +- 1/2) 2^e, and a tie goes to the even mantissa.  Quotients outside the
// normal range, or an estimate that does not settle, take the long division.
__host__ __device__ inline double u256_div_to_double(bool neg, U256 a, U256 b) {
  if (u256_is_zero(a)) return 0.0;
  const int la = u256_bitlen(a), lb = u256_bitlen(b);
  if (la > 190 || lb > 190) return u256_div_long(neg, a, b);
  const double q0 = u256_approx(a, la) / u256_approx(b, lb);
  int E;
  const double f = frexp(q0, &E);  // q0 = f 2^E, f in [1/2, 1)
  if (!(E > -1000 && E < 1000)) return u256_div_long(neg, a, b);
  int64_t m = (int64_t)ldexp(f, 53);  // [2^52, 2^53)
  int e = E - 53;
  const int64_t lo = (int64_t)1 << 52, hi = (int64_t)1 << 53;
  for (int it = 0; it < 8; ++it) {
    const int up = u256_cmp_half(a, b, e, (uint64_t)(2 * m + 1));
    if (up > 0) {  // a/b above the upper midpoint
      ++m;
      if (m == hi) {
        m = lo;
        ++e;
      }
      continue;
    }
    if (up == 0) {  // exactly halfway to m + 1
      if (m & 1) ++m;
      if (m == hi) {
        m = lo;
        ++e;
      }
      const double r = ldexp((double)m, e);
      return neg ? -r : r;
    }
    // below the upper midpoint; the lower midpoint of m = 2^52 sits at a
    // quarter unit (the binade below has half the spacing)
    const int dn = m == lo ? u256_cmp_half(a, b, e - 1, (uint64_t)(4 * m - 1))
                           : u256_cmp_half(a, b, e, (uint64_t)(2 * m - 1));
    if (dn < 0) {
      if (m == lo) {
        m = hi - 1;
        --e;
      } else {
        --m;
      }
      continue;
    }
    if (dn == 0) {  // exactly halfway to the lower neighbour
      if (m & 1) {
        if (m == lo) {
          m = hi - 1;
          --e;
        } else {
          --m;
        }
      }
      const double r = ldexp((double)m, e);
      return neg ? -r : r;
    }
    const double r = ldexp((double)m, e);
    return neg ? -r : r;
  }
  return u256_div_long(neg, a, b);
}

// (neg, |v|) of a signed 128-bit value.
__host__ __device__ inline u128 abs128(i128 v, bool* neg) {
  *neg = v < 0;
  return *neg ? (u128)0 - (u128)v : (u128)v;
}

// Signed 256-bit a*b - c*d for 128-bit operands, as (neg, magnitude).
__host__ __device__ inline U256 i256_mul_sub(i128 a, i128 b, i128 c, i128 d, bool* neg) {
  bool na, nb, nc, nd;
  U256 x = u256_mul128(abs128(a, &na), abs128(b, &nb));
  U256 y = u256_mul128(abs128(c, &nc), abs128(d, &nd));
  const bool sx = (na != nb) && !u256_is_zero(x);
  const bool sy = (nc != nd) && !u256_is_zero(y);
  // value = (sx ? -x : x) - (sy ? -y : y)
  if (sx != sy) {  // X and -Y share a sign: magnitudes add
    U256 r;
    uint64_t carry = 0;
    for (int k = 0; k < 4; ++k) {
      uint64_t t = x.w[k] + y.w[k];
      uint64_t c1 = t < x.w[k];
      uint64_t t2 = t + carry;
      uint64_t c2 = t2 < t;
      r.w[k] = t2;
      carry = c1 | c2;
    }
    *neg = sx;
    return r;
  }
  // same signs: the difference of the magnitudes, sign flipped when y > x
  if (u256_cmp(x, y) >= 0) {
    *neg = sx;
    return u256_sub(x, y);
  }
  *neg = !sx;
  return u256_sub(y, x);
}

// Covariance of integer columns i <= j from the exact totals: the 256-bit
// numerator n C_ij - s_i s_j over n (n - ddof), correctly rounded.
__device__ inline double exact_cov(const uint64_t* st, const Layout& L, int i, int j, int64_t n,
                                   int ddof) {
  const i128 si = load_i128(st + L.off_s + 2 * i);
  const i128 sj = load_i128(st + L.off_s + 2 * j);
  const i128 cij = load_i128(st + L.off_C + 2 * tri(L.p, i, j));
  bool neg;
  U256 num = i256_mul_sub((i128)n, cij, si, sj, &neg);  // n C_ij - s_i s_j
  const U256 den = u256_mul128((u128)n, (u128)(n - ddof));
  return u256_div_to_double(neg, num, den);
}

// Mean of an integer column, s_i / n correctly rounded.
__device__ inline double exact_mean(const uint64_t* st, const Layout& L, int i, int64_t n) {
  bool neg;
  const u128 m = abs128(load_i128(st + L.off_s + 2 * i), &neg);
  return u256_div_to_double(neg, u256_from_u128(m), u256_from_u128((u128)n));
}

// ---- kernel launchers (defined in the .hip files) ----------------------------

struct AccumLaunch {
  const char* colbase[16];  // address of column c in row 0
  int64_t colstride[16];    // bytes between rows of column c
  int32_t dtype[16];
  int p;
  uint32_t intmask, chkmask;
  int kind;  // 0 generic, 1 AoS FP64 (contiguous), 2 dense planes
  int64_t nrows;
  int64_t block_rows;
  uint64_t* rec;  // nblocks records
};

// Small-p (p <= 16) fused shift + colsum + upper-triangle X^T X + in-block
// reduction.  Returns the number of blocks written.
int64_t launch_accum_small_p(const AccumLaunch& a, hipStream_t s);

// Merge nblocks records into the state: cur -> next (double-buffered).
// With part (merge_slice_words(nblocks, p) words of device memory, when that
// is not 0) many records are folded in slices by several workgroups per
// entry, then the slice totals in order; without it, in one pass per entry.
void launch_merge_records(const uint64_t* rec, int64_t nblocks, int p, const uint8_t* intflags_dev,
                          const uint64_t* cur, uint64_t* next, DevStatus* status, hipStream_t s,
                          uint64_t* part = nullptr);
int64_t merge_slice_words(int64_t nblocks, int p);

// dst status |= src status (stream-ordered; see k_status_or).
void launch_status_or(DevStatus* dst, const DevStatus* src, hipStream_t s);

// Merge two states: out = merge(a, b).
void launch_merge_states(const uint64_t* a, const uint64_t* b, uint64_t* out, int p,
                         const uint8_t* intflags_dev, hipStream_t s);

struct FinalizeLaunch {
  const uint64_t* state;
  int p;
  const int32_t* sel_dev;  // q selected column indices
  int q;
  const uint8_t* intflags_dev;
  int ddof;
  int pca_on;
  int want_vectors;
  double* out;      // mean q, cov q*q, corr q*q, eigval q, eigvec q*q, var q, cum q
  double* scratch;  // 2 q*q (Jacobi A and V)
  double* jtab;     // q > 60: 5 * ceil(q / 2) (rotation tables of a round)
  unsigned* jc;     // q > 60: 3 words (rotations, non-finite flag, pairs still to rotate)
};
// Enqueues the finalize kernels on s.  Matrices above 60 x 60 run one kernel
// pair per Jacobi round and wait on s after every sweep.
hipError_t launch_finalize(const FinalizeLaunch& f, hipStream_t s);

// Raw statistics as FP64: s_f64[p], C_f64[p*p] (full) from a state.
void launch_raw(const uint64_t* state, int p, const uint8_t* intflags_dev, double* out,
                hipStream_t s);

}  // namespace st
