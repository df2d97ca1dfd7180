// Narrow-table kernel for row-major FP64 records.
#pragma once
#include "accum_common.hpp"

namespace st {
namespace acc {

// Row-major FP64 rows through LDS by direct DMA: 16-byte global loads that
// write LDS without passing through registers.  A stage is 256 consecutive
// rows (256 * RS contiguous bytes); each wave fetches a quarter of it as
// 1 KiB pieces -- the 64 rows its own lanes reduce.  NS stages rotate in LDS
// with NS - 1 of them in flight while one is reduced, one row per lane per
// stage, so the HBM queue stays full without staging registers.  Completion
// is tracked per wave by the vector-memory counter (loads retire in order);
// no workgroup barrier is needed.
template <int P>
struct AosDma {
  static constexpr int RS = (8 * P + 15) / 16 * 16;  // row stride (checked on the host)
  static constexpr int SB = kThreads * RS;            // stage bytes
  static constexpr int LPW = RS / 16;                 // 1 KiB pieces per wave per stage
  static constexpr int BUDGET = (P <= 12 ? 72 : 136) * 1024;
  static constexpr int NS0 = BUDGET / SB;
  static constexpr int NS = NS0 > 8 ? 8 : NS0;        // stages in LDS
  static_assert(NS >= 3, "at least two stages in flight");
  static_assert((NS - 2) * LPW < 64, "vector-memory counter range");
};

// Cache-policy operand of the DMA loads: non-temporal.  Every byte is read
// once, so the loads should not displace other lines; measured on 10^9
// 80-byte rows this raises the kernel from 6.1 to 6.9 TB/s.
constexpr int kNonTemporal = 2;

// s_waitcnt immediate that waits until at most N vector-memory loads of this
// wave are outstanding (expcnt and lgkmcnt left at their maxima).
template <int N>
struct VmWait {
  static constexpr int imm = (N & 15) | (7 << 4) | (15 << 8) | (((N >> 4) & 3) << 14);
};

// N 16-byte LDS reads at byte address a, a + 16, ..., completed before
// return.  Written as one asm block: the compiler would otherwise make every
// LDS read wait for all outstanding DMA loads, including those for stages
// that are still in flight by design.
template <int N>
__device__ inline void lds_row(uint32_t a, v4u (&v)[8]);
template <>
__device__ inline void lds_row<1>(uint32_t a, v4u (&v)[8]) {
  asm volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=&v"(v[0]) : "v"(a));
}
template <>
__device__ inline void lds_row<2>(uint32_t a, v4u (&v)[8]) {
  asm volatile("ds_read_b128 %0, %2\n\tds_read_b128 %1, %2 offset:16\n\ts_waitcnt lgkmcnt(0)"
               : "=&v"(v[0]), "=&v"(v[1]) : "v"(a));
}
template <>
__device__ inline void lds_row<3>(uint32_t a, v4u (&v)[8]) {
  asm volatile("ds_read_b128 %0, %3\n\tds_read_b128 %1, %3 offset:16\n\t"
               "ds_read_b128 %2, %3 offset:32\n\ts_waitcnt lgkmcnt(0)"
               : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]) : "v"(a));
}
template <>
__device__ inline void lds_row<4>(uint32_t a, v4u (&v)[8]) {
  asm volatile("ds_read_b128 %0, %4\n\tds_read_b128 %1, %4 offset:16\n\t"
               "ds_read_b128 %2, %4 offset:32\n\tds_read_b128 %3, %4 offset:48\n\ts_waitcnt lgkmcnt(0)"
               : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]) : "v"(a));
}
template <>
__device__ inline void lds_row<5>(uint32_t a, v4u (&v)[8]) {
  asm volatile("ds_read_b128 %0, %5\n\tds_read_b128 %1, %5 offset:16\n\t"
               "ds_read_b128 %2, %5 offset:32\n\tds_read_b128 %3, %5 offset:48\n\t"
               "ds_read_b128 %4, %5 offset:64\n\ts_waitcnt lgkmcnt(0)"
               : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]) : "v"(a));
}
template <>
__device__ inline void lds_row<6>(uint32_t a, v4u (&v)[8]) {
  asm volatile("ds_read_b128 %0, %6\n\tds_read_b128 %1, %6 offset:16\n\t"
               "ds_read_b128 %2, %6 offset:32\n\tds_read_b128 %3, %6 offset:48\n\t"
               "ds_read_b128 %4, %6 offset:64\n\tds_read_b128 %5, %6 offset:80\n\ts_waitcnt lgkmcnt(0)"
               : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5])
               : "v"(a));
}
template <>
__device__ inline void lds_row<7>(uint32_t a, v4u (&v)[8]) {
  asm volatile("ds_read_b128 %0, %7\n\tds_read_b128 %1, %7 offset:16\n\t"
               "ds_read_b128 %2, %7 offset:32\n\tds_read_b128 %3, %7 offset:48\n\t"
               "ds_read_b128 %4, %7 offset:64\n\tds_read_b128 %5, %7 offset:80\n\t"
               "ds_read_b128 %6, %7 offset:96\n\ts_waitcnt lgkmcnt(0)"
               : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]),
                 "=&v"(v[6])
               : "v"(a));
}
template <>
__device__ inline void lds_row<8>(uint32_t a, v4u (&v)[8]) {
  asm volatile("ds_read_b128 %0, %8\n\tds_read_b128 %1, %8 offset:16\n\t"
               "ds_read_b128 %2, %8 offset:32\n\tds_read_b128 %3, %8 offset:48\n\t"
               "ds_read_b128 %4, %8 offset:64\n\tds_read_b128 %5, %8 offset:80\n\t"
               "ds_read_b128 %6, %8 offset:96\n\tds_read_b128 %7, %8 offset:112\n\ts_waitcnt lgkmcnt(0)"
               : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]),
                 "=&v"(v[6]), "=&v"(v[7])
               : "v"(a));
}

template <int P>
__global__ __launch_bounds__(kThreads, (P <= 12 ? 2 : 1)) void k_aos_dma(Args a) {
  typedef AosDma<P> G;
  constexpr int RS = G::RS, SB = G::SB, LPW = G::LPW, NS = G::NS;
  __shared__ __attribute__((aligned(16))) unsigned char s_st[NS * SB];
  const int64_t r0 = (int64_t)blockIdx.x * a.R;
  const int64_t r1 = min(r0 + a.R, a.nrows);
  const char* base = a.colbase[0];
  double K[P];
  int64_t Ki[P];
#pragma unroll
  for (int c = 0; c < P; ++c) {
    K[c] = shift_of<double>(base + r0 * RS + 8 * c);
    Ki[c] = 0;
  }
  Acc<P> A;
  A.zero();
  uint32_t bad = 0;
  const bool chk = a.chkmask != 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nst = (r1 - r0) / kThreads;  // whole stages
  const char* src0 = base + r0 * RS + wave * (SB / kWaves) + lane * 16;
  const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)s_st;
  auto issue = [&](int64_t t) {
    const char* src = src0 + t * SB;
    __attribute__((address_space(3))) unsigned char* dst =
        (__attribute__((address_space(3))) unsigned char*)s_st + (int)(t % NS) * SB + wave * (SB / kWaves);
#pragma unroll
    for (int j = 0; j < LPW; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(src + j * 1024),
                                       (__attribute__((address_space(3))) void*)(dst + j * 1024), 16, 0, kNonTemporal);
  };
#pragma unroll
  for (int t = 0; t < NS - 1; ++t)
    if (t < nst) issue(t);
  for (int64_t t = 0; t < nst; ++t) {
    // stage t is this wave's oldest outstanding group of loads
    if (t + NS - 2 < nst) __builtin_amdgcn_s_waitcnt(VmWait<(NS - 2) * LPW>::imm);
    else __builtin_amdgcn_s_waitcnt(VmWait<0>::imm);
    // Wave w fetches rows [64w, 64w + 64) of every stage -- exactly the rows
    // its lanes reduce -- so its own completion wait is the only
    // synchronisation: the slot of stage t-1, refilled next, was read by
    // this wave in the previous iteration.
    if (t + NS - 1 < nst) issue(t + NS - 1);
    v4u raw[8];
    lds_row<LPW>(lds0 + (uint32_t)(t % NS) * SB + threadIdx.x * RS, raw);
    double d[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      const v4u& q = raw[c >> 1];
      const uint64_t w = (c & 1) ? (((uint64_t)q.w << 32) | q.z) : (((uint64_t)q.y << 32) | q.x);
      d[c] = __longlong_as_double((long long)w) - K[c];
    }
    if (chk) {
#pragma unroll
      for (int c = 0; c < P; ++c)
        if ((a.chkmask >> c) & 1u) bad |= not_integer(d[c] + K[c]);
    }
    A.add(d);
  }
  // rows after the last whole stage
  for (int64_t r = r0 + nst * kThreads + threadIdx.x; r < r1; r += kThreads) {
    double d[P];
    generic_row<P>(a, r, K, Ki, d, bad);
    A.add(d);
  }
  finish_block<P>(a, A, K, Ki, bad, r0, r1);
}

}  // namespace acc
}  // namespace st
