// FP64 row-major records on the FP64 matrix cores: all p columns FP64 at byte
// offsets 8c of RS-byte rows, RS = 256 (p <= 32: the batched workload's
// layout) or RS = 128 (p <= 16).  Items come from a tile table (groups) or
// are uniform blocks of rows (one table).
//
// Same contract as the persistent segmented kernel of wide.hip (items = row
// tiles of groups from an atomic queue, one block record per row tile, merged
// per group afterwards), with the data path of the row-major narrow kernel:
// 64-row stages (16 KiB) move from HBM to LDS by direct DMA
// (global_load_lds_dwordx4), three stages rotate with two in flight.  Each
// wave fetches and consumes its own quarter of every stage (16 rows), so the
// only wait is on its own vector-memory counter: no barrier in the loop.
//
// Products on the FP64 matrix cores: for v_mfma_f64_16x16x4f64 a lane holds
// the shifted value of column (lane % 16) (or 16 + lane % 16) in row
// (lane / 16) of a 4-row step, which is at the same time its element of the
// A operand (column i, row k) and of the B operand (row k, column j).  Three
// products per step give the upper 32 x 32 triangle in 16 x 16 tiles
// (0,0), (0,1), (1,1); each wave takes a quarter of the stage's rows, and the
// four waves' tiles are added in a fixed order at the end of the item.  For
// integer-valued columns every partial sum is an integer below 2^53 under the
// per-block guard checked by the merge, so the matrix-core sums are exact.
#include "common.hpp"
#include "wide.hpp"

namespace st {
namespace aos64 {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kSR = 64;       // rows per stage
constexpr int kNS = 3;        // stages in LDS

// Cache-policy operand of the DMA loads: non-temporal (each row is read once).
constexpr int kNonTemporal = 2;

// s_waitcnt immediate: at most N vector-memory loads of this wave outstanding.
template <int N>
struct VmWait {
  static constexpr int imm = (N & 15) | (7 << 4) | (15 << 8) | (((N >> 4) & 3) << 14);
};

// The four 4-row steps of a wave's 16 rows: values of columns c and c + 16 of
// rows a/256 + 4s (256-byte rows), or of column c of rows a/128 + 4s (128-byte
// rows), read in one asm block (with its own completion wait) so that the
// compiler does not make them wait for the DMA stages in flight.
__device__ inline void lds_steps128(uint32_t a, double (&x0)[4]) {
  asm volatile(
      "ds_read_b64 %0, %4\n\t"
      "ds_read_b64 %1, %4 offset:512\n\t"
      "ds_read_b64 %2, %4 offset:1024\n\t"
      "ds_read_b64 %3, %4 offset:1536\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x0[0]), "=&v"(x0[1]), "=&v"(x0[2]), "=&v"(x0[3])
      : "v"(a));
}

__device__ inline void lds_steps(uint32_t a, double (&x0)[4], double (&x1)[4]) {
  asm volatile(
      "ds_read_b64 %0, %8\n\t"
      "ds_read_b64 %4, %8 offset:128\n\t"
      "ds_read_b64 %1, %8 offset:1024\n\t"
      "ds_read_b64 %5, %8 offset:1152\n\t"
      "ds_read_b64 %2, %8 offset:2048\n\t"
      "ds_read_b64 %6, %8 offset:2176\n\t"
      "ds_read_b64 %3, %8 offset:3072\n\t"
      "ds_read_b64 %7, %8 offset:3200\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x0[0]), "=&v"(x0[1]), "=&v"(x0[2]), "=&v"(x0[3]), "=&v"(x1[0]), "=&v"(x1[1]),
        "=&v"(x1[2]), "=&v"(x1[3])
      : "v"(a));
}

__device__ inline uint32_t not_integer(double v) { return v != __builtin_rint(v) ? 1u : 0u; }

template <int RS>
struct Smem {
  union {
    unsigned char st[kNS][kSR * RS];  // stage ring
    struct {
      double acc[4][3][4][64];     // per wave: tiles x registers x lanes
      double s[4][64][2];          // per wave and lane: sums of columns c, c + 16
    } red;
  } u;
  double K[32];
  uint32_t chk, isint;
  int64_t item;
};

template <int RS>
__global__ __launch_bounds__(kThreads) void k_seg_aos64(wide::Args a, wide::SegArgs g) {
  constexpr int kRS = RS;
  constexpr int kSB = kSR * RS;          // stage bytes
  constexpr int kLPW = kSB / 1024 / 4;   // 1 KiB DMA pieces per wave per stage
  constexpr bool kTwo = RS == 256;       // a second half of 16 columns
  constexpr int kTiles = kTwo ? 3 : 1;   // upper 16 x 16 tiles
  __shared__ __attribute__((aligned(16))) Smem<RS> sm;
  const int p = a.p;
  const int tid = threadIdx.x, lane = tid & 63, q16 = lane & 15, kq = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const char* base = a.slots[0].base;  // column c at base + 8c (checked on the host)
  if (tid == 0) {
    uint32_t chk = 0, isint = 0;
    for (int c = 0; c < p; ++c) {
      if (a.slots[c].chk) chk |= 1u << c;
      if (a.slots[c].isint) isint |= 1u << c;
    }
    sm.chk = chk;
    sm.isint = isint;
  }
  const int c0 = q16, c1 = 16 + q16;
  const int64_t nitems = g.tile_rows ? (g.total_rows + g.tile_rows - 1) / g.tile_rows : *g.nrowtiles;
  const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)&sm.u.st[0][0];
  for (;;) {
    __syncthreads();  // previous item's LDS use is over
    if (tid == 0) sm.item = (int64_t)atomicAdd(g.counter, 1ull);
    __syncthreads();
    const int64_t item = sm.item;
    if (item >= nitems) break;
    int64_t r0, r1;
    if (g.tile_rows) {
      r0 = item * g.tile_rows;
      r1 = min(r0 + g.tile_rows, g.total_rows);
    } else {
      const wide::SegTile tile = g.rowtiles[item];
      r0 = tile.r0;
      r1 = tile.r1;
    }
    if (tid < p) sm.K[tid] = *(const double*)(base + r0 * kRS + 8 * tid);
    __syncthreads();
    const bool v0ok = c0 < p, v1ok = kTwo && c1 < p;
    const double K0 = v0ok ? sm.K[c0] : 0.0, K1 = v1ok ? sm.K[c1] : 0.0;
    const uint32_t chk0 = (sm.chk >> c0) & 1u, chk1 = v1ok ? (sm.chk >> c1) & 1u : 0u;
    d4 acc00 = (d4){0.0, 0.0, 0.0, 0.0}, acc01 = acc00, acc11 = acc00;
    double S0 = 0.0, S1 = 0.0;
    uint32_t bad = 0;
    auto step = [&](double x0, double x1) {
      const double v0 = v0ok ? x0 - K0 : 0.0, v1 = v1ok ? x1 - K1 : 0.0;
      if (chk0) bad |= not_integer(x0);
      if (chk1) bad |= not_integer(x1);
      S0 += v0;
      acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(v0, v0, acc00, 0, 0, 0);
      if constexpr (kTwo) {
        S1 += v1;
        acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(v0, v1, acc01, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(v1, v1, acc11, 0, 0, 0);
      }
    };

    const int64_t nst = (r1 - r0) / kSR;  // whole stages
    const char* src0 = base + r0 * kRS + wave * (kSB / 4) + lane * 16;
    auto issue = [&](int64_t t) {
      const char* src = src0 + t * kSB;
      __attribute__((address_space(3))) unsigned char* dst =
          (__attribute__((address_space(3))) unsigned char*)&sm.u.st[(int)(t % kNS)][0] + wave * (kSB / 4);
#pragma unroll
      for (int j = 0; j < kLPW; ++j)
        __builtin_amdgcn_global_load_lds((const void*)(src + j * 1024),
                                         (__attribute__((address_space(3))) void*)(dst + j * 1024), 16, 0, kNonTemporal);
    };
#pragma unroll
    for (int t = 0; t < kNS - 1; ++t)
      if (t < nst) issue(t);
    for (int64_t t = 0; t < nst; ++t) {
      // stage t is this wave's oldest outstanding group of loads; the slot of
      // stage t-1, refilled next, was read by this wave in the last iteration
      if (t + kNS - 2 < nst) __builtin_amdgcn_s_waitcnt(VmWait<(kNS - 2) * kLPW>::imm);
      else __builtin_amdgcn_s_waitcnt(VmWait<0>::imm);
      if (t + kNS - 1 < nst) issue(t + kNS - 1);
      double x0[4], x1[4] = {0.0, 0.0, 0.0, 0.0};
      const uint32_t la = lds0 + (uint32_t)(t % kNS) * kSB + (uint32_t)(16 * wave + kq) * kRS + 8 * c0;
      if constexpr (kTwo) lds_steps(la, x0, x1);
      else lds_steps128(la, x0);
#pragma unroll
      for (int s = 0; s < 4; ++s) step(x0[s], x1[s]);
    }
    // rows after the last whole stage: direct loads, 16 rows per wave per pass
    for (int64_t rb = r0 + nst * kSR; rb < r1; rb += kSR) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t r = rb + 16 * wave + 4 * s + kq;
        double x0 = K0, x1 = K1;
        if (r < r1) {
          if (v0ok) x0 = *(const double*)(base + r * kRS + 8 * c0);
          if (v1ok) x1 = *(const double*)(base + r * kRS + 8 * c1);
        }
        step(x0, x1);
      }
    }
    if (bad) atomicOr(&a.status->bits, ST_INEXACT);

    // ---- fixed-order sum over the waves; record ----
    __syncthreads();  // stage ring no longer read
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      sm.u.red.acc[wave][0][r][lane] = acc00[r];
      sm.u.red.acc[wave][1][r][lane] = acc01[r];
      sm.u.red.acc[wave][2][r][lane] = acc11[r];
    }
    sm.u.red.s[wave][lane][0] = S0;
    sm.u.red.s[wave][lane][1] = S1;
    __syncthreads();
    uint64_t* out = a.rec + item * rec_words(p);
    // tiles x 4 registers x 64 lanes, in fixed order
    for (int e = tid; e < kTiles * 4 * 64; e += kThreads) {
      const int tile_ = e >> 8, r = (e >> 6) & 3, l = e & 63;
      double v = sm.u.red.acc[0][tile_][r][l];
#pragma unroll
      for (int w = 1; w < 4; ++w) v += sm.u.red.acc[w][tile_][r][l];
      // register r of lane l holds D[4r + l/16][l%16]
      const int i = 4 * r + (l >> 4), j = l & 15;
      const int ci = tile_ == 2 ? 16 + i : i, cj = tile_ == 0 ? j : 16 + j;
      if (ci <= cj && cj < p) out[2 + 2 * p + tri(p, ci, cj)] = (uint64_t)__double_as_longlong(v);
    }
    if (tid < p) {
      const int c = tid, h = c >> 4, l0 = c & 15;
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int k = 0; k < 4; ++k) t += sm.u.red.s[w][l0 + 16 * k][h];
      out[2 + p + c] = (uint64_t)__double_as_longlong(t);
      const double Kc = sm.K[c];
      uint64_t kw;
      if ((sm.isint >> c) & 1u) kw = (fabs(Kc) < 4.0e18) ? (uint64_t)(int64_t)Kc : (uint64_t)0x7FFFFFFFFFFFFFFFll;
      else kw = (uint64_t)__double_as_longlong(Kc);
      out[2 + c] = kw;
    }
    if (tid == 0) {
      out[0] = (uint64_t)(r1 - r0);
      out[1] = 0;
    }
  }
}

__global__ void k_zero_queue(unsigned long long* c) { *c = 0ull; }

}  // namespace aos64

void launch_seg_aos64(const wide::Args& a, const wide::SegArgs& g, int nwg, hipStream_t s, int row_bytes) {
  hipLaunchKernelGGL(aos64::k_zero_queue, dim3(1), dim3(1), 0, s, g.counter);
  if (row_bytes == 128)
    hipLaunchKernelGGL(aos64::k_seg_aos64<128>, dim3(nwg), dim3(aos64::kThreads), 0, s, a, g);
  else
    hipLaunchKernelGGL(aos64::k_seg_aos64<256>, dim3(nwg), dim3(aos64::kThreads), 0, s, a, g);
}

}  // namespace st
