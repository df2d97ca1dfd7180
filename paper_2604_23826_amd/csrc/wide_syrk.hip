// Wide FP32 tables on BF16 matrix cores: X_b^T X_b from exact digit products.
//
// Scope: the vector columns are F FP32 values at consecutive 4-byte offsets
// of one row-major plane (16-byte aligned rows), plus up to two extra
// columns of any type (an identifier, say).  Other layouts use the general
// kernels of wide.hip / wide_split.hip.
//
// Method (section "Numerical Considerations": per-block mean shifting and
// hi/lo splitting of the operands to recover the accuracy of low-precision
// matrix units).  Every value is shifted by the block's first row K.  For a
// window of 64 rows and one column, E is chosen with |x - K| <= 2^E over the
// window, and v = (x - K) 2^(8-E) (|v| <= 256) is cut into three signed
// digits, each an integer of magnitude <= 256 and hence exact in BF16:
//     v = s1 + s2 2^-9 + s3 2^-18 + r,   |r| <= 2^-19.
// For columns a, b the window's cross product is then
//     2^(E_a + E_b - 16) sum_l 2^(-9 l) L_l,   L_l = sum_{i+j=l} sum_rows s_i s'_j,
// nine BF16 products in five levels.  Each product is exact in FP32 and at most
// 2^16; a level holds at most three products per row, so over 64 rows every
// partial sum stays below 2^24 and the FP32 accumulation on the matrix cores
// is exact.  Each window's levels are scaled and added into FP64.  The only
// rounding is the dropped remainder r (2^-27 of the window's range): data
// whose shifted values have at most 27 significant bits on that grid (FP32
// values shifted within a few binades, integers below 2^26) give exact
// window products.
//
// Work split: vector columns form groups of 128.  A workgroup owns one block
// of rows and one pair of groups (A, B), A <= B, and computes that 128 x 128
// part of Q with 32 x 32 x 16 BF16 MFMAs; the diagonal pair (A, A) also sums
// its columns (S), writes their shifts, and forms their products with the
// extra columns in FP64 on the vector units.  Staged columns sit in LDS in a
// permuted order that keeps both the digit writes and the operand reads free
// of bank conflicts.  Workgroup ids put all pairs of
// one block on the same XCD (ids congruent modulo 8), so the block's rows are
// fetched from HBM once and re-read from that XCD's L2.
//
// Per window: each wave-instruction loads 16 bytes per lane, i.e. one row's
// 256 columns of the pair (off-diagonal) or two rows' 128 (diagonal), fully
// coalesced; the next window's loads are issued as soon as the current one is
// converted, so they overlap the matrix-core phase.
#include "common.hpp"
#include "wide.hpp"

namespace st {
namespace syrk {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef float fl4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int G = wide::kSyrkGroup;  // vector columns per group
constexpr int WR = 64;               // rows per window
constexpr int DS = WR + 8;           // LDS bf16 per staged column (rows contiguous, padded)
constexpr int MAXT = 4;              // 32 x 32 tiles per wave

// Upper 32 x 32 tiles (i, j) of a diagonal pair, dealt to waves round-robin.
__device__ inline void diag_tile(int k, int& i, int& j) {
  switch (k) {
    case 0: i = 0; j = 0; break;
    case 1: i = 0; j = 1; break;
    case 2: i = 0; j = 2; break;
    case 3: i = 0; j = 3; break;
    case 4: i = 1; j = 1; break;
    case 5: i = 1; j = 2; break;
    case 6: i = 1; j = 3; break;
    case 7: i = 2; j = 2; break;
    case 8: i = 2; j = 3; break;
    default: i = 3; j = 3; break;
  }
}

// LDS position of staged column s: a rotation within each group of four, so
// that both access patterns are free of bank conflicts with the odd 16-byte
// column pitch: the conversion (lane q writes column 4q + i) and the operand
// reads (lane q reads column 32t + q).
__device__ inline int lpos(int s) { return (s & ~3) | ((s + (s >> 4)) & 3); }

// Tile u of wave w (off-diagonal: the wave's tiles share one tile column).
template <bool DIAG>
__device__ inline void wave_tile(int u, int w, int& i, int& j) {
  if (DIAG) {
    diag_tile(4 * u + w, i, j);
  } else {
    i = u;
    j = w;
  }
}

struct Smem {
  unsigned short dig[3][2 * G][DS];  // digits, [digit][LDS column position][row]
  float mx[8][2 * G];                // per row group: window max / min of x
  float mn[8][2 * G];
  double pw[2 * G];                  // 2^(E - 8) of the window
  double sc[2 * G];                  // 2^(8 - E)
  double K[2 * G];                   // shifts of the staged columns
  double red[8][G];                  // row-group partials (diagonal pair)
};

// Extra column value in row r as FP64, shifted (int64 through Ki).
__device__ inline double extra_value(const wide::SyrkExtra& e, int64_t r, double K, int64_t Ki,
                                     uint32_t& bad) {
  const char* p = e.base + r * e.stride;
  switch (e.kind) {
    case STATS_I32: return (double)*(const int32_t*)p - K;
    case STATS_I64: return (double)(*(const int64_t*)p - Ki);
    case STATS_F32: {
      const double x = (double)*(const float*)p;
      if (e.chk) bad |= (x != __builtin_rint(x));
      return x - K;
    }
    default: {
      const double x = *(const double*)p;
      if (e.chk) bad |= (x != __builtin_rint(x));
      return x - K;
    }
  }
}

__device__ inline void extra_shift(const wide::SyrkExtra& e, int64_t r0, double& K, int64_t& Ki) {
  const char* p = e.base + r0 * e.stride;
  Ki = 0;
  switch (e.kind) {
    case STATS_I32: K = (double)*(const int32_t*)p; break;
    case STATS_I64: Ki = *(const int64_t*)p; K = (double)Ki; break;
    case STATS_F32: K = (double)*(const float*)p; break;
    default: K = *(const double*)p; break;
  }
}

__device__ inline uint64_t shift_word(bool isint, int kind, double K, int64_t Ki) {
  if (!isint) return (uint64_t)__double_as_longlong(K);
  if (kind == STATS_I64) return (uint64_t)Ki;
  return (fabs(K) < 4.0e18) ? (uint64_t)(int64_t)K : (uint64_t)0x7FFFFFFFFFFFFFFFll;
}

// Two BF16 digits (integers |s| <= 256, exact) packed low = row 2m, high = row 2m+1.
__device__ inline uint32_t pack_bf16(double lo, double hi) {
  return __builtin_amdgcn_perm(__float_as_uint((float)hi), __float_as_uint((float)lo), 0x07060302u);
}

// One block of rows and one pair of column groups (A, B).
template <bool DIAG>
__device__ void pair_block(const wide::SyrkArgs& a, Smem& sm, int64_t b, int A, int B) {
  constexpr int NR = DIAG ? 8 : 16;  // rows per lane per window
  const int64_t r0 = b * a.R, r1 = min(r0 + a.R, a.nrows);
  const int lane = threadIdx.x & 63, h = lane >> 5, q = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = DIAG ? A : (h ? B : A);
  const int sl0 = (DIAG ? 0 : h * G) + 4 * q;
  const int c0 = grp * G + 4 * q;
  const bool colv = c0 < a.F;
  const int rb = DIAG ? 16 * wave + 8 * h : 16 * wave;
  const int rg = DIAG ? 2 * wave + h : wave;
  constexpr int NRG = DIAG ? 8 : 4;
  constexpr int NSL = DIAG ? G : 2 * G;
  const int ne = a.ne;
  const int boff = DIAG ? 0 : G;
  const int nt = DIAG ? (wave < 2 ? 3 : 2) : 4;
  const char* xrow0 = a.xbase + 4 * (int64_t)c0;
  fl4 Kf = (fl4){0.f, 0.f, 0.f, 0.f};
  if (colv) Kf = *(const fl4*)(xrow0 + r0 * a.xstride);
  double Kd[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) Kd[i] = (double)Kf[i];
  if (rg == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) sm.K[sl0 + i] = Kd[i];
  }
  double eK[wide::kSyrkMaxExtra];
  int64_t eKi[wide::kSyrkMaxExtra];
#pragma unroll
  for (int e = 0; e < wide::kSyrkMaxExtra; ++e) {
    eK[e] = 0.0;
    eKi[e] = 0;
    if (DIAG && e < ne) extra_shift(a.ex[e], r0, eK[e], eKi[e]);
  }
  double Q[MAXT][16];
#pragma unroll
  for (int u = 0; u < MAXT; ++u)
#pragma unroll
    for (int k = 0; k < 16; ++k) Q[u][k] = 0.0;
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  double strip[wide::kSyrkMaxExtra][4];
#pragma unroll
  for (int e = 0; e < wide::kSyrkMaxExtra; ++e)
#pragma unroll
    for (int i = 0; i < 4; ++i) strip[e][i] = 0.0;
  const bool self = DIAG && A == 0 && q == 0;
  double eS[wide::kSyrkMaxExtra] = {};
  double eQ[wide::kSyrkMaxExtra * (wide::kSyrkMaxExtra + 1) / 2] = {};
  uint32_t bad = 0;
  fl4 raw[NR];
  auto load_window = [&](int64_t w0) {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int64_t r = w0 + rb + j;
      raw[j] = Kf;
      if (colv && r < r1) raw[j] = __builtin_nontemporal_load((const fl4*)(xrow0 + r * a.xstride));
    }
  };
  load_window(r0);
  __syncthreads();  // shifts in LDS
  for (int64_t w0 = r0; w0 < r1; w0 += WR) {
    // ---- window range per column -> grid exponent E ----
    fl4 mx = raw[0], mn = raw[0];
#pragma unroll
    for (int j = 1; j < NR; ++j) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        mx[i] = fmaxf(mx[i], raw[j][i]);
        mn[i] = fminf(mn[i], raw[j][i]);
      }
    }
    *(fl4*)&sm.mx[rg][sl0] = mx;
    *(fl4*)&sm.mn[rg][sl0] = mn;
    __syncthreads();  // also: the previous window's digit reads are over
    for (int s = threadIdx.x; s < NSL; s += kThreads) {
      float M = sm.mx[0][s], m = sm.mn[0][s];
#pragma unroll
      for (int g = 1; g < NRG; ++g) {
        M = fmaxf(M, sm.mx[g][s]);
        m = fminf(m, sm.mn[g][s]);
      }
      const double k = sm.K[s];
      const double dm = fmax((double)M - k, k - (double)m);
      int E = 0;
      if (dm > 0.0) (void)frexp(dm, &E);  // dm < 2^E
      sm.pw[s] = ldexp(1.0, E - 8);
      sm.sc[s] = ldexp(1.0, 8 - E);
    }
    __syncthreads();
    // ---- digits (and, on the diagonal pair, column sums and extra strips) ----
    double sc[4], pw[4], nKs[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      sc[i] = sm.sc[sl0 + i];
      pw[i] = sm.pw[sl0 + i];
      nKs[i] = -Kd[i] * sc[i];
    }
    double de[wide::kSyrkMaxExtra][NR];
    if (DIAG) {
#pragma unroll
      for (int e = 0; e < wide::kSyrkMaxExtra; ++e)
#pragma unroll
        for (int j = 0; j < NR; ++j) {
          de[e][j] = 0.0;
          const int64_t r = w0 + rb + j;
          if (e < ne && r < r1) de[e][j] = extra_value(a.ex[e], r, eK[e], eKi[e], bad);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uint32_t pk[3][NR / 2];
      double ws = 0.0;
      double wstrip[wide::kSyrkMaxExtra] = {};
#pragma unroll
      for (int j = 0; j < NR; j += 2) {
        double s1[2], s2[2], s3[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const double v = __builtin_fma((double)raw[j + m][i], sc[i], nKs[i]);  // (x - K) sc, exact
          ws += v;
          if (DIAG) {
#pragma unroll
            for (int e = 0; e < wide::kSyrkMaxExtra; ++e)
              if (e < ne) wstrip[e] = __builtin_fma(v, de[e][j + m], wstrip[e]);
          }
          s1[m] = __builtin_rint(v);
          const double t1 = __builtin_fma(s1[m], -512.0, v * 512.0);  // (v - s1) 2^9, exact
          s2[m] = __builtin_rint(t1);
          s3[m] = __builtin_rint((t1 - s2[m]) * 512.0);
        }
        pk[0][j / 2] = pack_bf16(s1[0], s1[1]);
        pk[1][j / 2] = pack_bf16(s2[0], s2[1]);
        pk[2][j / 2] = pack_bf16(s3[0], s3[1]);
      }
      S[i] = __builtin_fma(ws, pw[i], S[i]);
      if (DIAG) {
#pragma unroll
        for (int e = 0; e < wide::kSyrkMaxExtra; ++e)
          if (e < ne) strip[e][i] = __builtin_fma(wstrip[e], pw[i], strip[e][i]);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < NR / 8; ++c)
          *(u4*)&sm.dig[d][lpos(sl0 + i)][rb + 8 * c] =
              (u4){pk[d][4 * c], pk[d][4 * c + 1], pk[d][4 * c + 2], pk[d][4 * c + 3]};
    }
    if (self) {
      int t = 0;
#pragma unroll
      for (int e = 0; e < wide::kSyrkMaxExtra; ++e) {
        if (e < ne) {
#pragma unroll
          for (int j = 0; j < NR; ++j) eS[e] += de[e][j];
        }
#pragma unroll
        for (int f = e; f < wide::kSyrkMaxExtra; ++f, ++t)
          if (f < ne) {
#pragma unroll
            for (int j = 0; j < NR; ++j) eQ[t] = __builtin_fma(de[e][j], de[f][j], eQ[t]);
          }
      }
    }
    if (w0 + WR < r1) load_window(w0 + WR);  // in flight during the matrix-core phase
    __syncthreads();                        // digits complete
    // ---- matrix cores: one tile at a time, five FP32 levels ----
#pragma unroll
    for (int u = 0; u < MAXT; ++u) {
      if (u >= nt) break;
      int ti, tj;
      wave_tile<DIAG>(u, wave, ti, tj);
      if (A * G + 32 * ti >= a.F || B * G + 32 * tj >= a.F) continue;
      f16v L[5];
#pragma unroll
      for (int l = 0; l < 5; ++l) L[l] = (f16v){};
      const int sa = 32 * ti + q, sb = boff + 32 * tj + q;
#pragma unroll
      for (int k16 = 0; k16 < WR / 16; ++k16) {
        const int kr = 16 * k16 + 8 * h;
        bf8 fa[3], fb[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          fa[d] = __builtin_bit_cast(bf8, *(const u4*)&sm.dig[d][lpos(sa)][kr]);
          fb[d] = __builtin_bit_cast(bf8, *(const u4*)&sm.dig[d][lpos(sb)][kr]);
        }
        // level order interleaved so that dependent products are apart
        L[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], fb[0], L[0], 0, 0, 0);
        L[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], fb[1], L[1], 0, 0, 0);
        L[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], fb[2], L[2], 0, 0, 0);
        L[3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1], fb[2], L[3], 0, 0, 0);
        L[4] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[2], fb[2], L[4], 0, 0, 0);
        L[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1], fb[0], L[1], 0, 0, 0);
        L[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1], fb[1], L[2], 0, 0, 0);
        L[3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[2], fb[1], L[3], 0, 0, 0);
        L[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[2], fb[0], L[2], 0, 0, 0);
      }
      // window flush: exact FP32 level sums, scaled into FP64
      const double pj = sm.pw[sb];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int i = (k >> 2) * 8 + h * 4 + (k & 3);
        const double pij = sm.pw[32 * ti + i] * pj;
        double t = (double)L[4][k];
        t = __builtin_fma(t, 0x1p-9, (double)L[3][k]);
        t = __builtin_fma(t, 0x1p-9, (double)L[2][k]);
        t = __builtin_fma(t, 0x1p-9, (double)L[1][k]);
        t = __builtin_fma(t, 0x1p-9, (double)L[0][k]);
        Q[u][k] = __builtin_fma(t, pij, Q[u][k]);
      }
    }
  }
  // ---- record ----
  const int p = a.p;
  uint64_t* out = a.rec + b * rec_words(p);
#pragma unroll
  for (int u = 0; u < MAXT; ++u) {
    if (u >= nt) break;
    int ti, tj;
    wave_tile<DIAG>(u, wave, ti, tj);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = (k >> 2) * 8 + h * 4 + (k & 3);
      const int ca = A * G + 32 * ti + i, cb = B * G + 32 * tj + q;
      if (ca < a.F && cb < a.F && ca <= cb) {
        const int ua = a.col_of[ca], ub = a.col_of[cb];
        out[2 + 2 * p + tri(p, min(ua, ub), max(ua, ub))] = (uint64_t)__double_as_longlong(Q[u][k]);
      }
    }
  }
  if (bad) atomicOr(&a.status->bits, ST_INEXACT);
  if (!DIAG) return;
  // column sums and extra strips: fixed-order sums over the 8 row groups
  auto reduce_write = [&](const double (&v)[4], int extra) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) sm.red[rg][sl0 + i] = v[i];
    __syncthreads();
    if (threadIdx.x < G) {
      const int s = threadIdx.x, c = A * G + s;
      double t = sm.red[0][s];
#pragma unroll
      for (int g = 1; g < 8; ++g) t += sm.red[g][s];
      if (c < a.F) {
        const int uc = a.col_of[c];
        if (extra < 0) {
          out[2 + p + uc] = (uint64_t)__double_as_longlong(t);
          out[2 + uc] = (uint64_t)__double_as_longlong(sm.K[s]);
        } else {
          const int ue = a.col_of[a.F + extra];
          out[2 + 2 * p + tri(p, min(uc, ue), max(uc, ue))] = (uint64_t)__double_as_longlong(t);
        }
      }
    }
  };
  reduce_write(S, -1);
  for (int e = 0; e < ne; ++e) reduce_write(strip[e], e);
  if (A == 0) {
    // extras' sums and products: row-group partials held by lanes q == 0
    __syncthreads();
    if (q == 0) {
      int t = 0;
#pragma unroll
      for (int e = 0; e < wide::kSyrkMaxExtra; ++e) {
        sm.red[rg][e] = eS[e];
#pragma unroll
        for (int f = e; f < wide::kSyrkMaxExtra; ++f, ++t) sm.red[rg][wide::kSyrkMaxExtra + t] = eQ[t];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int e = 0; e < ne; ++e) {
        double s = sm.red[0][e];
        for (int g = 1; g < 8; ++g) s += sm.red[g][e];
        const int ue = a.col_of[a.F + e];
        out[2 + p + ue] = (uint64_t)__double_as_longlong(s);
        out[2 + ue] = shift_word(a.ex[e].isint, a.ex[e].kind, eK[e], eKi[e]);
      }
      for (int e = 0; e < wide::kSyrkMaxExtra; ++e)
        for (int f = e; f < wide::kSyrkMaxExtra; ++f, ++t)
          if (f < ne) {
            double s = sm.red[0][wide::kSyrkMaxExtra + t];
            for (int g = 1; g < 8; ++g) s += sm.red[g][wide::kSyrkMaxExtra + t];
            const int ue = a.col_of[a.F + e], uf = a.col_of[a.F + f];
            out[2 + 2 * p + tri(p, min(ue, uf), max(ue, uf))] = (uint64_t)__double_as_longlong(s);
          }
      out[0] = (uint64_t)(r1 - r0);
      out[1] = 0;
    }
  }
}

__global__ __launch_bounds__(kThreads, 1) void k_syrk_split(wide::SyrkArgs a) {
  __shared__ __attribute__((aligned(16))) Smem sm;
  const int64_t id = blockIdx.x;
  const int64_t xcd = id & 7, y = id >> 3;
  const int t = (int)(y % a.npairs);
  const int64_t b = (y / a.npairs) * 8 + xcd;
  if (b >= a.nblocks) return;
  const int A = a.pairs[t].x, B = a.pairs[t].y;
  if (A == B) pair_block<true>(a, sm, b, A, B);
  else pair_block<false>(a, sm, b, A, B);
}

}  // namespace syrk

void launch_syrk_split(const wide::SyrkArgs& a, hipStream_t s) {
  const int64_t nb8 = (a.nblocks + 7) / 8 * 8;
  hipLaunchKernelGGL(syrk::k_syrk_split, dim3((unsigned)(nb8 * a.npairs)), dim3(syrk::kThreads), 0, s, a);
}

}  // namespace st
