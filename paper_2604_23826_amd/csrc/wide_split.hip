// Wide tables, split-precision mode: X_b^T X_b on BF16 matrix cores.
//
// Per block of rows and per column slot, the shifted values d = x - K are put
// on a common fixed-point grid, v = d / 2^e with |d| < 2^e (e from the block's
// largest |d| in that column), and cut into three signed 9-bit digits, each
// exactly representable in BF16:
//     v = s1 2^-8 + s2 2^-17 + s3 2^-26 (+ a remainder below 2^-27),
//     s_k = round-to-nearest digit, |s_k| <= 256.
// A product of two values is then 2^(e_a + e_b - 16) sum_l 2^(-9 l) L_l with
// L_l = sum over i + j = l of s_i s_j' (levels l = 0..4, nine BF16 products).
// Each product of digits is exact in FP32 and at most 2^16, so a level sum of
// up to 3 products per row over a 64-row window stays below 2^24 and the FP32
// matrix-core accumulation is exact; every window is flushed to FP64.  The
// only approximation is the dropped remainder (2^-27 of the column's block
// range); values with at most 27 significant bits on that grid (FP32 data
// shifted within its binade, or integers below 2^26) are multiplied exactly.
// The per-block shift and the window size implement the per-block mean
// shifting and hi/lo splitting that win the accuracy back (section "Numerical
// Considerations").
#include "common.hpp"
#include "wide.hpp"

namespace st {
namespace wide {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));

constexpr int KS = 64;         // rows per window (= staging step)
constexpr int RUN = KS + 8;    // bf16 per slot run in LDS (padded)

__device__ inline double load_value(const SlotInfo& si, int64_t r, int64_t Ki, double K,
                                    uint32_t& bad) {
  const char* p = si.base + r * si.stride;
  switch (si.kind) {
    case STATS_I32: return (double)*(const int32_t*)p - K;
    case STATS_F32: {
      const double x = (double)*(const float*)p;
      if (si.chk) bad |= (x != __builtin_rint(x));
      return x - K;
    }
    case STATS_I64: return (double)(*(const int64_t*)p - Ki);
    case STATS_F64: {
      const double x = *(const double*)p;
      if (si.chk) bad |= (x != __builtin_rint(x));
      return x - K;
    }
    default: return 0.0;
  }
}

__device__ inline unsigned short bf16_bits(double s) {
  // s is an integer with |s| <= 256: exact in FP32 and in BF16 (upper half)
  return (unsigned short)(__float_as_uint((float)s) >> 16);
}

template <int ST>
__global__ __launch_bounds__(kThreads) void k_wide_split(Args a) {
  constexpr int NSUB = ST / 32;  // 32 x 32 sub-tiles per side
  __shared__ unsigned short sSl[3][2 * ST][RUN];
  __shared__ double sK[2 * ST];
  __shared__ int64_t sKi[2 * ST];
  __shared__ double sRed[kThreads];
  __shared__ int sE[2 * ST];

  const int64_t id = blockIdx.x;
  const int64_t xcd = id % 8, y = id / 8;
  const int t = (int)(y % a.ntiles);
  const int64_t b = (y / a.ntiles) * 8 + xcd;
  if (b >= a.nblocks) return;
  const int A = a.tiles[t].x, B = a.tiles[t].y;
  const bool diag = A == B;
  const int nsl = diag ? ST : 2 * ST;
  const int64_t r0 = b * a.R, r1 = min(r0 + a.R, a.nrows);
  const int p = a.p;

  for (int s = threadIdx.x; s < nsl; s += kThreads) {
    const int gs = (s < ST ? A * ST + s : B * ST + (s - ST));
    double K = 0.0;
    int64_t Ki = 0;
    if (gs < p) {
      const SlotInfo si = a.slots[gs];
      const char* p0 = si.base + r0 * si.stride;
      switch (si.kind) {
        case STATS_I32: K = (double)*(const int32_t*)p0; break;
        case STATS_F32: K = (double)*(const float*)p0; break;
        case STATS_I64: Ki = *(const int64_t*)p0; K = (double)Ki; break;
        default: K = *(const double*)p0; break;
      }
    }
    sK[s] = K;
    sKi[s] = Ki;
  }
  __syncthreads();

  const int my_s = threadIdx.x % nsl;
  const int row_step = kThreads / nsl;
  const int my_r = threadIdx.x / nsl;
  const int gs = (my_s < ST ? A * ST + my_s : B * ST + (my_s - ST));
  SlotInfo si;
  si.kind = -1;
  si.chk = 0;
  si.isint = 0;
  si.base = nullptr;
  si.stride = 0;
  if (gs < p) si = a.slots[gs];
  const double myK = sK[my_s];
  const int64_t myKi = sKi[my_s];
  uint32_t bad = 0;

  // ---- pass 1: the block's largest |d| per slot -> grid exponent ----
  double mx = 0.0;
  if (gs < p)
    for (int64_t r = r0 + my_r; r < r1; r += row_step) mx = fmax(mx, fabs(load_value(si, r, myKi, myK, bad)));
  sRed[threadIdx.x] = mx;
  __syncthreads();
  if (threadIdx.x < nsl) {
    double m = 0.0;
    for (int g = 0; g < row_step; ++g) m = fmax(m, sRed[g * nsl + threadIdx.x]);
    int e = 0;
    if (m > 0.0) (void)frexp(m, &e);  // m < 2^e
    sE[threadIdx.x] = e;
  }
  __syncthreads();
  const int myE = sE[my_s];

  // ---- pass 2: digits in LDS, nine BF16 products per 16 rows ----
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave -> one 32 x 32 sub-tile (mi, nj); diagonal super-tiles skip mi > nj
  const int mi = (NSUB == 2) ? (wave >> 1) : 0;
  const int nj = (NSUB == 2) ? (wave & 1) : 0;
  const bool active = (NSUB == 2 || wave == 0) && !(diag && nj < mi);
  const int boff = diag ? 0 : ST;
  f16v L[5];
#pragma unroll
  for (int l = 0; l < 5; ++l) L[l] = (f16v){};
  double Q[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) Q[k] = 0.0;
  double mysum = 0.0;

  for (int64_t k0 = r0; k0 < r1; k0 += KS) {
    for (int rr = my_r; rr < KS; rr += row_step) {
      const int64_t r = k0 + rr;
      double s1 = 0.0, s2 = 0.0, s3 = 0.0;
      if (r < r1 && gs < p) {
        const double v = ldexp(load_value(si, r, myKi, myK, bad), 8 - myE);  // |v| < 2^8
        s1 = __builtin_rint(v);
        const double t2 = (v - s1) * 512.0;
        s2 = __builtin_rint(t2);
        s3 = __builtin_rint((t2 - s2) * 512.0);
        mysum += ldexp(s1 + ldexp(s2, -9) + ldexp(s3, -18), myE - 8);
      }
      sSl[0][my_s][rr] = bf16_bits(s1);
      sSl[1][my_s][rr] = bf16_bits(s2);
      sSl[2][my_s][rr] = bf16_bits(s3);
    }
    __syncthreads();
    if (active) {
      const int ra = 32 * mi + (lane & 31), rb = boff + 32 * nj + (lane & 31);
#pragma unroll
      for (int k16 = 0; k16 < KS / 16; ++k16) {
        const int kr = 16 * k16 + 8 * (lane >> 5);
        bf8 fa[3], fb[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          fa[q] = __builtin_bit_cast(bf8, *(const s8v*)&sSl[q][ra][kr]);
          fb[q] = __builtin_bit_cast(bf8, *(const s8v*)&sSl[q][rb][kr]);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            L[i + j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], L[i + j], 0, 0, 0);
      }
      // window flush: exact FP32 level sums into FP64
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        Q[k] += (double)L[0][k] + 0x1p-9 * (double)L[1][k] + 0x1p-18 * (double)L[2][k] +
                0x1p-27 * (double)L[3][k] + 0x1p-36 * (double)L[4][k];
      }
#pragma unroll
      for (int l = 0; l < 5; ++l) L[l] = (f16v){};
    }
    __syncthreads();
  }

  uint64_t* out = a.rec + b * rec_words(p);
  if (active) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = (k / 4) * 8 + (lane >> 5) * 4 + (k % 4), j = lane & 31;
      const int sa = 32 * mi + i, sb = boff + 32 * nj + j;
      const int ga = A * ST + 32 * mi + i, gb = B * ST + 32 * nj + j;
      if (ga <= gb && gb < p) {
        const double v = ldexp(Q[k], sE[sa] + sE[sb] - 16);
        out[2 + 2 * p + tri(p, ga, gb)] = (uint64_t)__double_as_longlong(v);
      }
    }
  }
  if (bad) atomicOr(&a.status->bits, ST_INEXACT);
  if (diag) {
    sRed[threadIdx.x] = 0.0;
    __syncthreads();
    for (int g = 0; g < row_step; ++g) {
      if (my_r == g) sRed[my_s] += mysum;
      __syncthreads();
    }
    for (int s = threadIdx.x; s < ST; s += kThreads) {
      const int c = A * ST + s;
      if (c < p) {
        out[2 + p + c] = (uint64_t)__double_as_longlong(sRed[s]);
        uint64_t kw;
        const SlotInfo& sc = a.slots[c];
        if (sc.isint) {
          if (sc.kind == STATS_I64) kw = (uint64_t)sKi[s];
          else kw = (fabs(sK[s]) < 4.0e18) ? (uint64_t)(int64_t)sK[s] : (uint64_t)0x7FFFFFFFFFFFFFFFll;
        } else {
          kw = (uint64_t)__double_as_longlong(sK[s]);
        }
        out[2 + c] = kw;
      }
    }
    if (A == 0 && threadIdx.x == 0) {
      out[0] = (uint64_t)(r1 - r0);
      out[1] = 0;
    }
  }
}

}  // namespace wide

void launch_wide_split(const wide::Args& a, int st, hipStream_t s) {
  const int64_t nb8 = (a.nblocks + 7) / 8 * 8;
  const dim3 grid((unsigned)(nb8 * a.ntiles)), block(wide::kThreads);
  if (st == 32) hipLaunchKernelGGL(wide::k_wide_split<32>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(wide::k_wide_split<64>, grid, block, 0, s, a);
}

}  // namespace st
