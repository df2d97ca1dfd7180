// Fused single-pass reduction for narrow tables (p <= 16): shared device code.
//
// One workgroup reduces one block of R consecutive rows (section "Data
// Representation and Sufficient Statistics": column sums and X^T X in one
// streaming pass; each worker reduces a disjoint subset of rows).  Every
// value is shifted by the block's first row K before it is accumulated, so the
// block statistics are S = sum (x - K) and Q = sum (x - K)(x - K)^T (upper
// triangle).  For integer columns these are exact integers in FP64 as long as
// sum (x - K)^2 < 2^53 (checked when the records are merged); the merge turns
// them into exact 128-bit totals (section "Numerical Considerations").
//
// Per lane: RPI rows per step, loaded raw with every load of the step issued
// before the first use, then shifted and accumulated row by row into
// p + p(p+1)/2 FP64 registers.  Per wave: DPP butterflies leave the wave sum in
// lane 63.  Per workgroup: the four wave sums are added through LDS in a fixed
// order, so results are bitwise reproducible.
//
// Layout classes (compile-time, so the load phase has no branches):
//   Aos:     all columns FP64, contiguous in a 16-byte aligned row;
//   Planes:  one dense plane per column, the first NI slots int32 and the
//            rest FP64 (columns are permuted into this order on the host);
//   Generic: anything else; two 32-bit loads per element, converted by type.
#pragma once
#include "common.hpp"

namespace st {
namespace acc {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

struct Args {
  const char* colbase[16];  // slot order
  int64_t colstride[16];
  int32_t dtype[16];
  uint32_t chkmask;         // slots: FP column flagged INTEGER (values checked)
  uint32_t intmask;         // slots: integer column
  int64_t nrows;
  int64_t R;
  uint64_t* rec;
  int16_t dst[16 + 136];    // record position (relative to S) of slot entry e
  int8_t kdst[16];          // record column of slot c
};

template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi2, lo2);
}

// Sum over the 64 lanes of a wave; the total is valid in lane 63.
__device__ inline double wave_sum_to_lane63(double v) {
  v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x124, 0xF>(v);  // row_ror:4
  v += dpp_f64<0x128, 0xF>(v);  // row_ror:8   -> every lane holds its row (16 lanes) sum
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3 -> lane 63 holds the total
  return v;
}

__device__ inline uint64_t uniform64(uint64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Shift of slot c: the value in row r0 (uniform; kept in SGPRs).  For int64
// columns the exact integer goes to Ki.
__device__ inline void load_shift(const Args& a, int c, int64_t r0, double& K, int64_t& Ki) {
  const char* p0 = a.colbase[c] + r0 * a.colstride[c];
  uint64_t kb;
  switch (a.dtype[c]) {
    case STATS_I32: kb = (uint64_t)__double_as_longlong((double)*(const int32_t*)p0); break;
    case STATS_I64: kb = (uint64_t)*(const int64_t*)p0; break;
    case STATS_F32: kb = (uint64_t)__double_as_longlong((double)*(const float*)p0); break;
    default: kb = (uint64_t)__double_as_longlong(*(const double*)p0); break;
  }
  kb = uniform64(kb);
  if (a.dtype[c] == STATS_I64) {
    Ki = (int64_t)kb;
    K = (double)(int64_t)kb;
  } else {
    Ki = 0;
    K = __longlong_as_double((long long)kb);
  }
}

template <int P>
struct Acc {
  static constexpr int T = P * (P + 1) / 2;
  double S[P];
  double Q[T];
  __device__ inline void zero() {
#pragma unroll
    for (int c = 0; c < P; ++c) S[c] = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t) Q[t] = 0.0;
  }
  __device__ inline void add(const double (&d)[P]) {
    int t = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      S[i] += d[i];
#pragma unroll
      for (int j = i; j < P; ++j) {
        Q[t] = __builtin_fma(d[i], d[j], Q[t]);
        ++t;
      }
    }
  }
};

__device__ inline uint32_t not_integer(double v) { return v != __builtin_rint(v) ? 1u : 0u; }

// Generic element: low and high 32-bit words (the high load re-reads the low
// word for 4-byte types so every slot issues the same two loads).
__device__ inline double convert(int dt, uint32_t lo, uint32_t hi, double K, int64_t Ki) {
  switch (dt) {
    case STATS_I32: return (double)(int32_t)lo - K;
    case STATS_F32: return (double)__uint_as_float(lo) - K;
    case STATS_I64: return (double)((int64_t)(((uint64_t)hi << 32) | lo) - Ki);
    default: return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo)) - K;
  }
}

// Block epilogue: wave + workgroup reduction, record write.
template <int P>
__device__ inline void finish_block(const Args& a, Acc<P>& A, const double (&K)[P],
                                    const int64_t (&Ki)[P], uint32_t bad, int64_t r0, int64_t r1) {
  constexpr int T = P * (P + 1) / 2;
  constexpr int E = P + T;
  __shared__ double red[kWaves][E];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const double v = wave_sum_to_lane63(A.S[c]);
    if (lane == 63) red[wave][c] = v;
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const double v = wave_sum_to_lane63(A.Q[t]);
    if (lane == 63) red[wave][P + t] = v;
  }
  const int anybad = __syncthreads_or((int)bad);
  uint64_t* out = a.rec + (int64_t)blockIdx.x * (2 + 2 * P + T);
  for (int e = threadIdx.x; e < E; e += kThreads) {
    double v = red[0][e];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) v += red[w][e];
    out[2 + P + a.dst[e]] = (uint64_t)__double_as_longlong(v);
  }
  if (threadIdx.x < P) {
    const int c = threadIdx.x;
    uint64_t kw;
    if ((a.intmask >> c) & 1u) {
      if (a.dtype[c] == STATS_I64) {
        kw = (uint64_t)Ki[c];
      } else {
        const double kc = K[c];
        kw = (fabs(kc) < 4.0e18) ? (uint64_t)(int64_t)kc : (uint64_t)0x7FFFFFFFFFFFFFFFll;
      }
    } else {
      kw = (uint64_t)__double_as_longlong(K[c]);
    }
    out[2 + a.kdst[c]] = kw;
  }
  if (threadIdx.x == 0) {
    out[0] = (uint64_t)(r1 - r0);
    out[1] = anybad ? 1u : 0u;
  }
}

// Generic tail / fallback for one row.
template <int P>
__device__ inline void generic_row(const Args& a, int64_t r, const double (&K)[P],
                                   const int64_t (&Ki)[P], double (&d)[P], uint32_t& bad) {
  uint32_t lo[P], hi[P];
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const char* p = a.colbase[c] + r * a.colstride[c];
    const int hoff = (a.dtype[c] == STATS_I64 || a.dtype[c] == STATS_F64) ? 4 : 0;
    lo[c] = __builtin_nontemporal_load((const uint32_t*)p);
    hi[c] = __builtin_nontemporal_load((const uint32_t*)(p + hoff));
  }
#pragma unroll
  for (int c = 0; c < P; ++c) {
    d[c] = convert(a.dtype[c], lo[c], hi[c], K[c], Ki[c]);
    if ((a.chkmask >> c) & 1u) {
      const double x = d[c] + K[c];
      bad |= not_integer(x);
    }
  }
}

// ---- kernels ------------------------------------------------------------------

template <int P>
__device__ inline void prologue(const Args& a, int64_t& r0, int64_t& r1, double (&K)[P],
                                int64_t (&Ki)[P]) {
  r0 = (int64_t)blockIdx.x * a.R;
  r1 = min(r0 + a.R, a.nrows);
#pragma unroll
  for (int c = 0; c < P; ++c) load_shift(a, c, r0, K[c], Ki[c]);
}

// Uniform FP64 shift of a column whose values are read as T (int32 / FP64).
template <typename T>
__device__ inline double shift_of(const char* p) {
  const double v = (double)*(const T*)p;
  return __longlong_as_double((long long)uniform64((uint64_t)__double_as_longlong(v)));
}

}  // namespace acc
}  // namespace st
