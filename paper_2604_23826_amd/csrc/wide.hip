// Wide tables (p > 16): block statistics with a dense SYRK on the matrix cores.
//
// For p columns the per-row work is p(p+1)/2 products, a real dense
// contraction X_b^T X_b over the rows of a block (section "Data
// Representation and Sufficient Statistics": X^T X accumulated in one
// streaming pass).  The block record is the same as the narrow path's (shift
// K = the block's first row, S = sum (x - K), Q = sum (x - K)(x - K)^T) and is
// merged by the same kernels.
//
// Tiling: slots 0..p-1 are the columns, padded to a multiple of ST (32 or 64).
// A workgroup owns one block of rows and one super-tile (A, B), A <= B, of the
// upper triangle of Q.  Each step it loads KR rows of the 2 ST slots it needs,
// shifts them and stages them in LDS; each wave multiplies 16 x 16 sub-tiles.
//   FP64 mode: the shifted values in FP64, v_mfma_f64_16x16x4_f64.  Exact for
//     integer columns under the same 2^53 guard as the narrow path.
//   Split mode (BF16): see wide_split.hip.
// The workgroup that owns a diagonal super-tile (A, A) also sums its slots'
// shifted values (S) and writes their shifts.
// Blocks are mapped to workgroup ids so that all super-tiles of one block run
// on the same XCD (ids congruent modulo 8), sharing its L2.
#include "common.hpp"
#include "wide.hpp"

namespace st {
namespace wide {

typedef double d4 __attribute__((ext_vector_type(4)));

// Value of slot s in row r, shifted; ones/pad slots excluded by the caller.
__device__ inline double load_shifted(const SlotInfo& si, int64_t r, double K, int64_t Ki,
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

// One block of rows [r0, r1) and super-tile (A, B): shifts, staged FP64
// values, MFMA sub-tiles, and this super-tile's part of the record at out.
template <int ST>
__device__ void wide_f64_block(const Args& a, uint64_t* out, int64_t r0, int64_t r1, int A, int B) {
  constexpr int NSUB = ST / 16;       // sub-tiles per super-group side
  constexpr int MAXW = (NSUB * NSUB + 3) / 4;  // sub-tiles per wave
  __shared__ double sD[KR][2 * ST + 1];
  __shared__ double sK[2 * ST];
  __shared__ int64_t sKi[2 * ST];
  __shared__ double sS[2 * ST];

  const bool diag = A == B;
  const int nsl = diag ? ST : 2 * ST;  // staged slots

  // shifts of the staged slots
  for (int s = threadIdx.x; s < nsl; s += kThreads) {
    const int gs = (s < ST ? A * ST + s : B * ST + (s - ST));
    double K = 0.0;
    int64_t Ki = 0;
    if (gs < a.p) {
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
    sS[s] = 0.0;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // sub-tiles of this wave: index u = mi * NSUB + nj over the super-tile,
  // round-robin over the ones in the upper triangle (diagonal tiles)
  int my_mi[MAXW], my_nj[MAXW];
  int nmine = 0;
  {
    int k = 0;
    for (int mi = 0; mi < NSUB; ++mi)
      for (int nj = 0; nj < NSUB; ++nj) {
        if (diag && nj < mi) continue;
        if (k % 4 == wave && nmine < MAXW) {
          my_mi[nmine] = mi;
          my_nj[nmine] = nj;
          ++nmine;
        }
        ++k;
      }
  }
  d4 acc[MAXW];
#pragma unroll
  for (int u = 0; u < MAXW; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};
  // slot this thread stages and its S accumulator
  const int my_s = threadIdx.x % nsl;
  const int row_step = kThreads / nsl;  // rows staged per pass
  const int my_r = threadIdx.x / nsl;
  const int gs = (my_s < ST ? A * ST + my_s : B * ST + (my_s - ST));
  SlotInfo si;
  si.kind = -1;
  si.chk = 0;
  si.base = nullptr;
  si.stride = 0;
  if (gs < a.p) si = a.slots[gs];
  const double myK = sK[my_s];
  const int64_t myKi = sKi[my_s];
  double mysum = 0.0;
  uint32_t bad = 0;
  const int boff = diag ? 0 : ST;

  for (int64_t k0 = r0; k0 < r1; k0 += KR) {
    // stage KR rows x nsl slots
    for (int rr = my_r; rr < KR; rr += row_step) {
      const int64_t r = k0 + rr;
      double d = 0.0;
      if (r < r1 && gs < a.p) d = load_shifted(si, r, myK, myKi, bad);
      sD[rr][my_s] = d;
      mysum += d;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KR / 4; ++k4) {
      const int row = 4 * k4 + (lane >> 4);
      const int col = lane & 15;
#pragma unroll
      for (int u = 0; u < MAXW; ++u) {
        if (u < nmine) {
          const double av = sD[row][16 * my_mi[u] + col];
          const double bv = sD[row][boff + 16 * my_nj[u] + col];
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // ---- write this super-tile's part of the block record ----
  const int p = a.p;
#pragma unroll
  for (int u = 0; u < MAXW; ++u) {
    if (u >= nmine) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // v_mfma_f64_16x16x4: register r of lane l holds D[4 r + l / 16][l % 16]
      const int i = 4 * r + (lane >> 4), j = lane & 15;
      const int ga = A * ST + 16 * my_mi[u] + i;
      const int gb = B * ST + 16 * my_nj[u] + j;
      if (ga <= gb && gb < p) out[2 + 2 * p + tri(p, ga, gb)] = (uint64_t)__double_as_longlong(acc[u][r]);
    }
  }
  if (bad) atomicOr(&a.status->bits, ST_INEXACT);
  if (diag) {
    // column sums of the staged slots (fixed-order reduction over row groups)
    for (int q = threadIdx.x; q < 2 * ST; q += kThreads) sS[q] = 0.0;
    __syncthreads();
    for (int g = 0; g < row_step; ++g) {
      if (my_r == g) sS[my_s] += mysum;
      __syncthreads();
    }
    for (int s = threadIdx.x; s < ST; s += kThreads) {
      const int c = A * ST + s;
      if (c < p) {
        out[2 + p + c] = (uint64_t)__double_as_longlong(sS[s]);
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

template <int ST>
__global__ __launch_bounds__(kThreads) void k_wide_f64(Args a) {
  // block / super-tile from the XCD-aware id
  const int64_t id = blockIdx.x;
  const int64_t xcd = id % 8, y = id / 8;
  const int t = (int)(y % a.ntiles);
  const int64_t b = (y / a.ntiles) * 8 + xcd;
  if (b >= a.nblocks) return;
  const int64_t r0 = b * a.R, r1 = min(r0 + a.R, a.nrows);
  wide_f64_block<ST>(a, a.rec + b * rec_words(a.p), r0, r1, a.tiles[t].x, a.tiles[t].y);
}

// Persistent variant for batched groups: workgroups take (row tile,
// super-tile) items from an atomic queue until it is empty; record slots are
// indexed by row tile, so results do not depend on which workgroup ran what.
template <int ST>
__global__ __launch_bounds__(kThreads) void k_seg_f64(Args a, SegArgs g) {
  __shared__ int64_t s_item;
  const int64_t nitems = *g.nrowtiles * a.ntiles;
  for (;;) {
    __syncthreads();  // previous item's LDS use is over
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(g.counter, 1ull);
    __syncthreads();
    const int64_t item = s_item;
    if (item >= nitems) break;
    const int64_t rt = item / a.ntiles;
    const int t = (int)(item % a.ntiles);
    const SegTile tile = g.rowtiles[rt];
    wide_f64_block<ST>(a, a.rec + rt * rec_words(a.p), tile.r0, tile.r1, a.tiles[t].x, a.tiles[t].y);
  }
}

__global__ void k_zero_counter(unsigned long long* c) { *c = 0ull; }

// Blocks of the int8 split kernel whose values left their grids (or were not
// finite): the same (block, super-tile) grid as k_wide_f64, flagged blocks only.
template <int ST>
__global__ __launch_bounds__(kThreads) void k_wide_fixup(Args a, const int* ovf) {
  const int64_t id = blockIdx.x;
  const int64_t xcd = id % 8, y = id / 8;
  const int t = (int)(y % a.ntiles);
  const int64_t b = (y / a.ntiles) * 8 + xcd;
  if (b >= a.nblocks || !ovf[b]) return;
  const int64_t r0 = b * a.R, r1 = min(r0 + a.R, a.nrows);
  wide_f64_block<ST>(a, a.rec + b * rec_words(a.p), r0, r1, a.tiles[t].x, a.tiles[t].y);
}

}  // namespace wide

void launch_wide(const wide::Args& a, int st, int mode, hipStream_t s) {
  const int64_t nb8 = (a.nblocks + 7) / 8 * 8;
  const dim3 grid((unsigned)(nb8 * a.ntiles)), block(wide::kThreads);
  if (mode == wide::MODE_SPLIT) {
    launch_wide_split(a, st, s);
    return;
  }
  if (st == 32) hipLaunchKernelGGL(wide::k_wide_f64<32>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(wide::k_wide_f64<64>, grid, block, 0, s, a);
}

void launch_wide_fixup(const wide::Args& a, int st, const int* ovf, hipStream_t s) {
  const int64_t nb8 = (a.nblocks + 7) / 8 * 8;
  const dim3 grid((unsigned)(nb8 * a.ntiles)), block(wide::kThreads);
  if (st == 32) hipLaunchKernelGGL(wide::k_wide_fixup<32>, grid, block, 0, s, a, ovf);
  else hipLaunchKernelGGL(wide::k_wide_fixup<64>, grid, block, 0, s, a, ovf);
}

void launch_seg(const wide::Args& a, const wide::SegArgs& g, int st, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(wide::k_zero_counter, dim3(1), dim3(1), 0, s, g.counter);
  if (st == 32) hipLaunchKernelGGL(wide::k_seg_f64<32>, dim3(nwg), dim3(wide::kThreads), 0, s, a, g);
  else hipLaunchKernelGGL(wide::k_seg_f64<64>, dim3(nwg), dim3(wide::kThreads), 0, s, a, g);
}

}  // namespace st
