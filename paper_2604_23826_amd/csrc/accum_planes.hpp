// Narrow-table kernel for dense column planes (one plane per column).
#pragma once
#include "accum_common.hpp"

namespace st {
namespace acc {

// Dense planes: slots [0, NI) int32, [NI, P) FP64.  Four rows per lane per
// step: one 16-byte load per int32 slot, two per FP64 slot.  A launch covers
// at most 2^28 rows, so plane offsets fit in 32 bits.
template <int P, int NI>
__global__ __launch_bounds__(kThreads, (P <= 12 ? 2 : 1)) void k_planes(Args a) {
  const int64_t r0 = (int64_t)blockIdx.x * a.R;
  const int64_t r1 = min(r0 + a.R, a.nrows);
  double K[P];
  int64_t Ki[P];
#pragma unroll
  for (int c = 0; c < P; ++c) {
    K[c] = c < NI ? shift_of<int32_t>(a.colbase[c] + r0 * 4) : shift_of<double>(a.colbase[c] + r0 * 8);
    Ki[c] = 0;
  }
  Acc<P> A;
  A.zero();
  uint32_t bad = 0;
  const bool chk = a.chkmask != 0;
  constexpr int RPI = 4;
  constexpr int NF = P - NI;
  int64_t r = r0 + (int64_t)threadIdx.x * RPI;
  for (; r + RPI <= r1; r += (int64_t)kThreads * RPI) {
    const uint32_t o4 = (uint32_t)r * 4u, o8 = (uint32_t)r * 8u;
    v4i ri[NI > 0 ? NI : 1];
    v2d rf[NF > 0 ? NF : 1][2];
#pragma unroll
    for (int c = 0; c < NI; ++c) ri[c] = __builtin_nontemporal_load((const v4i*)(a.colbase[c] + o4));
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const v2d* p = (const v2d*)(a.colbase[NI + f] + o8);
      rf[f][0] = __builtin_nontemporal_load(p);
      rf[f][1] = __builtin_nontemporal_load(p + 1);
    }
    __builtin_amdgcn_sched_barrier(0);  // every load of the step is in flight before any use
#pragma unroll
    for (int k = 0; k < RPI; ++k) {
      double d[P];
#pragma unroll
      for (int c = 0; c < NI; ++c) d[c] = (double)ri[c][k] - K[c];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double x = (k & 1) ? rf[f][k >> 1].y : rf[f][k >> 1].x;
        d[NI + f] = x - K[NI + f];
        if (chk && ((a.chkmask >> (NI + f)) & 1u)) bad |= not_integer(x);
      }
      A.add(d);
    }
  }
  for (; r < r1; ++r) {
    double d[P];
    generic_row<P>(a, r, K, Ki, d, bad);
    A.add(d);
  }
  finish_block<P>(a, A, K, Ki, bad, r0, r1);
}

}  // namespace acc
}  // namespace st
