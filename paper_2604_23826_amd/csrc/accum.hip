// Fused single-pass reduction for narrow tables (p <= 16).
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
// Per lane: the p shifted values of RPI rows per step, p + p(p+1)/2 FP64
// register accumulators.  Per wave: DPP butterflies leave the wave sum in
// lane 63.  Per workgroup: the four wave sums are added through LDS in a
// fixed order, so results are bitwise reproducible.
#include "common.hpp"

namespace st {
namespace {

constexpr int kThreads = 256;

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef long long v2l __attribute__((ext_vector_type(2)));
constexpr int kWaves = kThreads / 64;

// ---- DPP wave reduction (FP64 as two 32-bit halves) --------------------------
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

struct Args {
  const char* colbase[16];
  int64_t colstride[16];
  int32_t dtype[16];
  uint32_t intmask, chkmask;
  int64_t nrows;
  int64_t R;
  uint64_t* rec;
};

// Value of column c in row r as FP64 (exact for I32 / F32 / F64).
__device__ inline double load_scalar(const Args& a, int c, int64_t r) {
  const char* p = a.colbase[c] + r * a.colstride[c];
  switch (a.dtype[c]) {
    case STATS_I32: return (double)__builtin_nontemporal_load((const int32_t*)p);
    case STATS_I64: return (double)__builtin_nontemporal_load((const int64_t*)p);
    case STATS_F32: return (double)__builtin_nontemporal_load((const float*)p);
    default: return __builtin_nontemporal_load((const double*)p);
  }
}

__device__ inline int64_t load_i64(const Args& a, int c, int64_t r) {
  return *(const int64_t*)(a.colbase[c] + r * a.colstride[c]);
}

// KIND 0: any layout, one element load per value.
// KIND 1: all columns FP64, contiguous in a row, row starts 16-byte aligned.
// KIND 2: every column its own dense plane (stride = element size), planes
//         16-byte aligned; RPI consecutive rows per lane are one vector load.
template <int P, int KIND, int RPI>
__device__ inline void load_rows(const Args& a, int64_t r, int nv, const double* K,
                                 const int64_t* Ki, double (&d)[RPI][P], uint32_t& bad) {
  if (KIND == 2 && nv == RPI) {
#pragma unroll
    for (int c = 0; c < P; ++c) {
      const int dt = a.dtype[c];
      const char* base = a.colbase[c];
      if (dt == STATS_I32) {
        if constexpr (RPI == 2) {
          v2i v = __builtin_nontemporal_load((const v2i*)(base + r * 4));
          d[0][c] = (double)v.x - K[c];
          d[1][c] = (double)v.y - K[c];
        } else {
          v4i v = __builtin_nontemporal_load((const v4i*)(base + r * 4));
          d[0][c] = (double)v.x - K[c];
          d[1][c] = (double)v.y - K[c];
          d[2][c] = (double)v.z - K[c];
          d[3][c] = (double)v.w - K[c];
        }
      } else if (dt == STATS_F64) {
#pragma unroll
        for (int k = 0; k < RPI; k += 2) {
          v2d v = __builtin_nontemporal_load((const v2d*)(base + (r + k) * 8));
          d[k][c] = v.x - K[c];
          d[k + 1][c] = v.y - K[c];
          if (a.chkmask & (1u << c)) {
            bad |= (v.x != __builtin_rint(v.x)) | (v.y != __builtin_rint(v.y));
          }
        }
      } else if (dt == STATS_F32) {
#pragma unroll
        for (int k = 0; k < RPI; k += 2) {
          v2f v = __builtin_nontemporal_load((const v2f*)(base + (r + k) * 4));
          d[k][c] = (double)v.x - K[c];
          d[k + 1][c] = (double)v.y - K[c];
          if (a.chkmask & (1u << c)) {
            bad |= (v.x != __builtin_rintf(v.x)) | (v.y != __builtin_rintf(v.y));
          }
        }
      } else {  // I64: subtract in integers, then convert
#pragma unroll
        for (int k = 0; k < RPI; k += 2) {
          v2l v = __builtin_nontemporal_load((const v2l*)(base + (r + k) * 8));
          d[k][c] = (double)(v.x - Ki[c]);
          d[k + 1][c] = (double)(v.y - Ki[c]);
        }
      }
    }
    return;
  }
  if (KIND == 1 && nv == RPI) {
#pragma unroll
    for (int k = 0; k < RPI; ++k) {
      const double* row = (const double*)(a.colbase[0] + (r + k) * a.colstride[0]);
#pragma unroll
      for (int c = 0; c + 1 < P; c += 2) {
        v2d v = __builtin_nontemporal_load((const v2d*)(row + c));
        d[k][c] = v.x - K[c];
        d[k][c + 1] = v.y - K[c + 1];
        if (a.chkmask & (3u << c)) {
          bad |= ((a.chkmask >> c) & 1u) & (v.x != __builtin_rint(v.x));
          bad |= ((a.chkmask >> (c + 1)) & 1u) & (v.y != __builtin_rint(v.y));
        }
      }
      if (P & 1) {
        const double v = __builtin_nontemporal_load(row + (P - 1));
        d[k][P - 1] = v - K[P - 1];
        if ((a.chkmask >> (P - 1)) & 1u) bad |= (v != __builtin_rint(v));
      }
    }
    return;
  }
  // generic path, and the ragged tail of the vector paths
#pragma unroll
  for (int k = 0; k < RPI; ++k) {
    if (k < nv) {
#pragma unroll
      for (int c = 0; c < P; ++c) {
        if (a.dtype[c] == STATS_I64) {
          d[k][c] = (double)(load_i64(a, c, r + k) - Ki[c]);
        } else {
          const double v = load_scalar(a, c, r + k);
          d[k][c] = v - K[c];
          if ((a.chkmask >> c) & 1u) bad |= (v != __builtin_rint(v));
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < P; ++c) d[k][c] = 0.0;
    }
  }
}

template <int P, int KIND, int RPI>
__global__ __launch_bounds__(kThreads, 2) void k_accum_small_p(Args a) {
  constexpr int T = P * (P + 1) / 2;
  constexpr int E = P + T;
  __shared__ double red[kWaves][E];

  const int64_t r0 = (int64_t)blockIdx.x * a.R;
  const int64_t r1 = min(r0 + a.R, a.nrows);

  // Shift: the block's first row (same address for every lane, kept in SGPRs).
  double K[P];
  int64_t Ki[P];
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const char* p0 = a.colbase[c] + r0 * a.colstride[c];
    int64_t kb;
    switch (a.dtype[c]) {
      case STATS_I32: kb = __double_as_longlong((double)*(const int32_t*)p0); break;
      case STATS_I64: kb = *(const int64_t*)p0; break;
      case STATS_F32: kb = __double_as_longlong((double)*(const float*)p0); break;
      default: kb = __double_as_longlong(*(const double*)p0); break;
    }
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)kb);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)kb >> 32));
    const int64_t kw = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    if (a.dtype[c] == STATS_I64) {
      Ki[c] = kw;
      K[c] = (double)kw;
    } else {
      K[c] = __longlong_as_double(kw);
      Ki[c] = 0;
    }
  }

  double S[P];
  double Q[T];
#pragma unroll
  for (int c = 0; c < P; ++c) S[c] = 0.0;
#pragma unroll
  for (int t = 0; t < T; ++t) Q[t] = 0.0;
  uint32_t bad = 0;

  for (int64_t r = r0 + (int64_t)threadIdx.x * RPI; r < r1; r += (int64_t)kThreads * RPI) {
    const int nv = (int)min((int64_t)RPI, r1 - r);
    double d[RPI][P];
    load_rows<P, KIND, RPI>(a, r, nv, K, Ki, d, bad);
#pragma unroll
    for (int k = 0; k < RPI; ++k) {
      int t = 0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        S[i] += d[k][i];
#pragma unroll
        for (int j = i; j < P; ++j) {
          Q[t] = __builtin_fma(d[k][i], d[k][j], Q[t]);
          ++t;
        }
      }
    }
  }

  // ---- in-block reduction: wave (DPP) then workgroup (LDS, fixed order) ----
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    const double v = wave_sum_to_lane63(S[c]);
    if (lane == 63) red[wave][c] = v;
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const double v = wave_sum_to_lane63(Q[t]);
    if (lane == 63) red[wave][P + t] = v;
  }
  const int anybad = __syncthreads_or((int)bad);

  uint64_t* out = a.rec + (int64_t)blockIdx.x * (2 + 2 * P + T);
  for (int e = threadIdx.x; e < E; e += kThreads) {
    double v = red[0][e];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) v += red[w][e];
    out[2 + P + e] = (uint64_t)__double_as_longlong(v);
  }
  if (threadIdx.x < P) {
    const int c = threadIdx.x;
    uint64_t kw;
    if ((a.intmask >> c) & 1u) {
      if (a.dtype[c] == STATS_I64) {
        kw = (uint64_t)Ki[c];
      } else {
        // integer-valued FP64 shift; out-of-range shifts are caught when merged
        const double kc = K[c];
        kw = (fabs(kc) < 4.0e18) ? (uint64_t)(int64_t)kc : (uint64_t)0x7FFFFFFFFFFFFFFFll;
      }
    } else {
      kw = (uint64_t)__double_as_longlong(K[c]);
    }
    out[2 + c] = kw;
  }
  if (threadIdx.x == 0) {
    out[0] = (uint64_t)(r1 - r0);
    out[1] = anybad ? 1u : 0u;
  }
}

template <int P>
void launch_p(const Args& a, int kind, int64_t nblocks, hipStream_t s) {
  const dim3 grid((unsigned)nblocks), block(kThreads);
  if (kind == 1) hipLaunchKernelGGL((k_accum_small_p<P, 1, 1>), grid, block, 0, s, a);
  else if (kind == 2) hipLaunchKernelGGL((k_accum_small_p<P, 2, 2>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_accum_small_p<P, 0, 1>), grid, block, 0, s, a);
}

}  // namespace

int64_t launch_accum_small_p(const AccumLaunch& L, hipStream_t s) {
  Args a;
  for (int c = 0; c < 16; ++c) {
    a.colbase[c] = c < L.p ? L.colbase[c] : nullptr;
    a.colstride[c] = c < L.p ? L.colstride[c] : 0;
    a.dtype[c] = c < L.p ? L.dtype[c] : STATS_F64;
  }
  a.intmask = L.intmask;
  a.chkmask = L.chkmask;
  a.nrows = L.nrows;
  a.R = L.block_rows;
  a.rec = L.rec;
  const int64_t nblocks = (L.nrows + L.block_rows - 1) / L.block_rows;
  if (nblocks <= 0) return 0;
  switch (L.p) {
#define ST_CASE(PP) \
  case PP: launch_p<PP>(a, L.kind, nblocks, s); break;
    ST_CASE(1) ST_CASE(2) ST_CASE(3) ST_CASE(4) ST_CASE(5) ST_CASE(6) ST_CASE(7) ST_CASE(8)
    ST_CASE(9) ST_CASE(10) ST_CASE(11) ST_CASE(12) ST_CASE(13) ST_CASE(14) ST_CASE(15) ST_CASE(16)
#undef ST_CASE
    default: return -1;
  }
  return nblocks;
}

}  // namespace st
