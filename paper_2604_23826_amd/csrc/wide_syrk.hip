// Wide FP32 tables on the int8 matrix cores: X_b^T X_b from exact digit
// products.
//
// Scope: the vector columns are F FP32 values at consecutive 4-byte offsets
// of one row-major plane (16-byte aligned rows, F a multiple of 4), plus up
// to two extra columns of any type (an identifier, say).  Other layouts use
// the general kernels of wide.hip / wide_split.hip.
//
// Method (section "Numerical Considerations": per-block mean shifting and
// splitting of the operands to recover the accuracy of low-precision matrix
// units).  Every value is shifted by the block's first row K and put on a
// binary grid of its column: v = rint((x - K) 2^s), an integer.  s is chosen
// per block and column from 1024 rows spread over the block (its first and
// last included) so that they need at most 21 bits, leaving a factor of two
// to four of headroom below the limit |v| < 2^22.  v is cut into three signed byte
// digits, exact in int8:
//     v = d0 2^16 + d1 2^8 + d2,    d1, d2 in [-128, 127], |d0| <= 64.
// The rounding and the digits take three vector operations per value:
// y + 1.5 * 2^23 leaves rint(y) in the low mantissa bits, and one integer
// add turns the bit pattern into v + 0x8080, whose bytes are d2 + 128,
// d1 + 128 and d0; the bias of the two low bytes is removed on the packed
// dwords (one XOR per four values).
// For columns a, b the block's cross product is
//     sum_rows v_a v_b = sum_l 2^(32 - 8 l) L_l,   L_l = sum_{i+j=l} sum_rows d_i d'_j,
// nine digit products in five levels on v_mfma_i32_32x32x32_i8, whose int32
// accumulation is exact (|L_l| < 3 * 2^14 per row, 2^31 over 32768 rows);
// the levels are combined and scaled by 2^(-s_a - s_b) in FP64 once per
// block.  The only rounding before FP64 is the grid: FP32 values within a
// few binades of the shift (and integers below 2^21) lie on it, so their
// products are exact.
//
// Two passes per launch.  k_syrk_i8 forms the digits and the products above
// and writes each block's grid exponents; k_syrk_sums then forms the rest of
// the record (column sums, products with the extra columns, shifts, row
// count) and checks every value: a block with a value beyond its column's
// limit, a value off its grid (x 2^s not an integer: one v_fract per value),
// or a non-finite value is flagged (ovf[b]), and the FP64 matrix-core routine
// of wide.hip computes that block's whole record again (launch_wide_fixup),
// so every block is either exact on its grid or FP64.  Each workgroup of the
// first pass also finds the lowest set bit of its first 128 sampled rows:
// when one lies below the grid spacing the block cannot be exact (zero-mean
// data with full significands, say), and the workgroup flags it and stops
// before the main loop.
//
// Work split: vector columns form groups of 128.  A workgroup owns one block
// of rows and one half of a pair of groups (A, B), A <= B: two tile rows of
// A for an off-diagonal pair (8 tiles), tile rows {0, 3} or {1, 2} of a
// diagonal one (5 upper tiles; its other three waves only load and convert).
// Eight waves, two per SIMD, with at most one 32 x 32 tile each (its five
// int32 levels in 80 accumulation registers), so that each wave's waits are
// covered by the other wave of its SIMD.  The sums stay out of this pass: in
// the workgroups of the diagonal pairs they would double the vector work on
// the pass's critical path.  Workgroup ids put all pairs of one block on the
// same XCD (ids congruent modulo 8), so that a block's rows can come from
// that XCD's L2 for the pairs after the first (the two halves of a pair, which
// run at the same speed, do share them; pairs of different kinds drift apart).
//
// Data path per 32-row sub-step: each wave loads its own four rows (a lane
// four consecutive columns of each, two on a diagonal half) from global
// memory straight into
// registers, two alternating register sets, one sub-step ahead, and converts
// exactly those rows.  The digits go to a double-buffered LDS array,
// [digit][4-row group][column] as dwords of four rows; one barrier per
// sub-step separates the conversion of sub-step t + 1 from the products of
// sub-step t.  The K index of a product is the row, so a lane's operand
// dwords j = 0..3 are its column's row groups 4h + j.  The conversion of
// sub-step t + 1 and the products of sub-step t are independent; the
// schedule interleaves them (one product, then a share of the conversion),
// so the vector work issues while the matrix cores run.
#include <type_traits>

#include "common.hpp"
#include "wide.hpp"

namespace st {
namespace syrk {

typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i16 __attribute__((ext_vector_type(16)));
typedef float fl4 __attribute__((ext_vector_type(4)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 512;
constexpr int NW = kThreads / 64;    // waves
constexpr int RW = 32 / NW;          // rows per wave per sub-step
constexpr int MT = 1;                // tiles per wave
constexpr int G = wide::kSyrkGroup;  // vector columns per group
constexpr int SR = 32;               // rows per sub-step (K of one product)
constexpr int PITCH_MAX = 2 * G + 8;
constexpr int NSAMP = 1024;          // rows sampled per block for the grids
constexpr int SB = 16;               // sampled rows per wave in flight
constexpr float kVlim = 4194303.0f;  // |v| < 2^22: the rounding constant below holds v exactly
constexpr float kRound = 12582912.0f; // 1.5 * 2^23: y + kRound is rint(y) in the low mantissa bits
constexpr int kBias = 0x8080 - 0x4B400000;  // bits(y + kRound) + kBias = v + 0x8080
constexpr int NE = wide::kSyrkMaxExtra;
static_assert(NE <= 2, "the sums pass brings two dwords of at most two extras per row");

// s_waitcnt immediate: at most N vector-memory loads of this wave outstanding.
template <int N>
struct VmWait {
  static constexpr int imm = (N & 15) | (7 << 4) | (15 << 8) | (((N >> 4) & 3) << 14);
};

// Shapes of the two workgroup kinds.
template <bool DIAG>
struct Shape {
  static constexpr int NC = DIAG ? G : 2 * G;  // staged columns
  static constexpr int CPL = NC / 64;           // columns converted per lane
  static constexpr int PITCH = NC + 8;          // dwords per 4-row group (4 PITCH = 32 mod 64 banks)
};

// Tiles (ti, tj) of a wave, at most MT; off-diagonal pairs: tile row w.
struct WaveTiles {
  int n;
  int ti[MT], tj[MT];
};

template <bool DIAG>
__device__ inline WaveTiles wave_tiles(int w, int half) {
  WaveTiles r;
  if (!DIAG) {
    // tile row 2 half + w / 4 of A, tile column w % 4 of B
    r.n = 1;
    r.ti[0] = 2 * half + (w >> 2);
    r.tj[0] = w & 3;
    return r;
  }
  // a diagonal half: the upper tiles of tile rows {0, 3} (half 0) or {1, 2}
  // (half 1) of the 4 x 4 tiles, one per wave; waves without a tile only
  // stage and convert rows
  switch (half * 8 + w) {
    case 0: r.n = 1; r.ti[0] = 0; r.tj[0] = 0; break;
    case 1: r.n = 1; r.ti[0] = 0; r.tj[0] = 1; break;
    case 2: r.n = 1; r.ti[0] = 0; r.tj[0] = 2; break;
    case 3: r.n = 1; r.ti[0] = 0; r.tj[0] = 3; break;
    case 4: r.n = 1; r.ti[0] = 3; r.tj[0] = 3; break;
    case 8: r.n = 1; r.ti[0] = 1; r.tj[0] = 1; break;
    case 9: r.n = 1; r.ti[0] = 1; r.tj[0] = 2; break;
    case 10: r.n = 1; r.ti[0] = 1; r.tj[0] = 3; break;
    case 11: r.n = 1; r.ti[0] = 2; r.tj[0] = 2; break;
    case 12: r.n = 1; r.ti[0] = 2; r.tj[0] = 3; break;
    default: r.n = 0; r.ti[0] = 0; r.tj[0] = 0; break;
  }
  return r;
}

// Barrier after this wave's LDS writes, without waiting for the DMA loads in
// flight (a __syncthreads() fence would wait for them too).
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ inline bool wide_kind(int kind) { return kind == STATS_I64 || kind == STATS_F64; }

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

// Grid exponent s of a column whose sampled shifted values reach m
// (m < 2^e): s = 21 - e.  With m = 0 the grid is the spacing of FP32 values
// in K's binade, or 1 for K = 0.  Clamped so that 2^s is a normal FP32
// number.
__device__ inline int grid_exp(double m, float K) {
  int e = 0;
  int s;
  if (m > 0.0) {
    (void)frexp(m, &e);
    s = 21 - e;
  } else if (K != 0.0f) {
    (void)frexp((double)K, &e);
    s = 23 - e;
  } else {
    s = 0;
  }
  return max(-126, min(127, s));
}

// One workgroup's view of its block: DIAG for a half of a diagonal pair (one
// group of columns), else a half of an off-diagonal pair (two groups).
template <bool DIAG>
struct Ctx {
  static constexpr int NC = Shape<DIAG>::NC;
  static constexpr int CPL = Shape<DIAG>::CPL;
  static constexpr int PITCH = Shape<DIAG>::PITCH;
  const wide::SyrkArgs& a;
  int* dig;             // LDS digits [2][3][8][PITCH]
  const float* s_sc;    // 2^s per staged column (0: not converted)
  const float* s_nks;   // -K 2^s
  float sc[CPL], nks[CPL];  // the lane's columns' 2^s and -K 2^s, in registers for the block
  int64_t r0, r1;
  int A, B, lane, wave, h, q;
  int cl0;              // first staged column converted by this lane

  __device__ Ctx(const wide::SyrkArgs& a_) : a(a_) {}

  // global vector column of staged column c
  __device__ __attribute__((always_inline)) int gcol(int c) const { return DIAG ? A * G + c : (c < G ? A * G + c : B * G + (c - G)); }

  // Raw values of one sub-step for this lane: RW rows x CPL columns.
  struct Raw {
    float x[RW][CPL];
  };

  // Loads of this wave's rows of sub-step t, straight into registers: CPL
  // consecutive columns of each row per lane (rows past the block end read
  // its last row, columns past F read column 0; both are ignored).
  __device__ __attribute__((always_inline)) void load(int64_t t, Raw& r) const {
    const int64_t rb = r0 + t * SR + RW * wave;
    const int dc = gcol(cl0);
    const int64_t col = dc < a.F ? dc : 0;
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      int64_t row = rb + j;
      row = row < r1 ? row : r1 - 1;
      load_row(a.xbase + row * a.xstride + 4 * col, r.x[j]);
    }
  }

  // The same for a sub-step that lies inside the block: rp is this lane's
  // address in the wave's first row of the sub-step (advanced by the caller).
  __device__ __attribute__((always_inline)) void load_inside(const char* rp, Raw& r) const {
#pragma unroll
    for (int j = 0; j < RW; ++j) load_row(rp + j * a.xstride, r.x[j]);
  }

  __device__ __attribute__((always_inline)) static void load_row(const char* p, float (&x)[CPL]) {
    if constexpr (CPL == 4) {
      const fl4 v = *(const fl4*)p;
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = v[i];
    } else {
      const fl2 v = *(const fl2*)p;
#pragma unroll
      for (int i = 0; i < 2; ++i) x[i] = v[i];
    }
  }

  // Digits of sub-step t into digit buffer t & 1 (rows past the block end
  // give zeros).
  __device__ __attribute__((always_inline)) void load_grids() {
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      sc[i] = s_sc[cl0 + i];
      nks[i] = s_nks[cl0 + i];
    }
  }

  template <bool TAIL>
  __device__ __attribute__((always_inline)) void digitize(int64_t t, Raw& r) const {
    const int64_t rb = r0 + t * SR + RW * wave;
#pragma unroll
    for (int g = 0; g < RW / 4; ++g) {
      uint32_t dw[3][CPL];
#pragma unroll
      for (int i = 0; i < CPL; ++i) {
        int w[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          float y = __builtin_fmaf(r.x[4 * g + jj][i], sc[i], nks[i]);
          if (TAIL) y = (rb + 4 * g + jj < r1) ? y : 0.0f;
          const float fr = y + kRound;
          w[jj] = __float_as_int(fr) + kBias;  // v + 0x8080: bytes d2 + 128, d1 + 128, d0
        }
        // byte transpose: digit k of the four rows into one dword
        const uint32_t p01 = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);
        const uint32_t p23 = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);
        const uint32_t q01 = __builtin_amdgcn_perm(w[1], w[0], 0x0C0C0602u);
        const uint32_t q23 = __builtin_amdgcn_perm(w[3], w[2], 0x0C0C0602u);
        dw[2][i] = __builtin_amdgcn_perm(p23, p01, 0x05040100u) ^ 0x80808080u;  // d2 (lowest)
        dw[1][i] = __builtin_amdgcn_perm(p23, p01, 0x07060302u) ^ 0x80808080u;  // d1
        dw[0][i] = __builtin_amdgcn_perm(q23, q01, 0x05040100u);                // d0 (highest)
      }
      int* out = dig + ((int)(t & 1) * 3 * 8 + (RW / 4) * wave + g) * PITCH + cl0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if constexpr (CPL == 4) *(u4*)(out + d * 8 * PITCH) = (u4){dw[d][0], dw[d][1], dw[d][2], dw[d][3]};
        else *(u2*)(out + d * 8 * PITCH) = (u2){dw[d][0], dw[d][1]};
      }
    }
  }
};

// One operand: digit d of staged column c in rows 16h..16h+15 of buffer buf.
template <bool DIAG>
__device__ inline i4 operand(const int* base, int d, int c) {
  constexpr int PITCH = Shape<DIAG>::PITCH;
  i4 r;
#pragma unroll
  for (int j = 0; j < 4; ++j) r[j] = base[(d * 8 + j) * PITCH + c];
  return r;
}

// Operands of one sub-step's digits (buffer buf) for the wave's tile: the
// three digits of its column block of A and of its column block of B.
struct Ops {
  i4 fa[3], fb[3];
};

template <bool DIAG>
__device__ inline void load_ops(const int* dig, int buf, const WaveTiles& wt, int h, int q, Ops& o) {
  constexpr int PITCH = Shape<DIAG>::PITCH;
  const int* base = dig + (buf * 3 * 8 + 4 * h) * PITCH + q;
  constexpr int boff = DIAG ? 0 : G;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    o.fa[d] = operand<DIAG>(base, d, 32 * wt.ti[0]);
    o.fb[d] = operand<DIAG>(base, d, boff + 32 * wt.tj[0]);
  }
}

// The nine digit products of one sub-step into the tile's levels: digit d of
// the B operand meets the three digits of A in levels d..d+2 (tiles past the
// last vector column multiply zero digits and are not written).
__device__ inline void mma_ops(const Ops& o, i16 (&L)[MT][5]) {
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int k = 0; k < 3; ++k) L[0][d + k] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.fa[k], o.fb[d], L[0][d + k], 0, 0, 0);
}

struct Lds {
  int* dig;
  double* red;      // [NW][256], shares memory with dig
  int* s_exp;
  float* s_K;
  float* s_sc;
  float* s_nks;
  int* s_flag;      // sampled values off their grid: the block goes to FP64
};

// One block of rows and one pair of column groups (A, B).
template <bool DIAG>
__device__ __attribute__((always_inline)) void pair_block(const wide::SyrkArgs& a, const Lds& m, int64_t b, int A,
                                                         int B, int half) {
  constexpr int NC = Shape<DIAG>::NC;
  constexpr int CPL = Shape<DIAG>::CPL;
  Ctx<DIAG> c(a);
  c.dig = m.dig;
  c.s_sc = m.s_sc;
  c.s_nks = m.s_nks;
  c.r0 = b * a.R;
  c.r1 = min(c.r0 + a.R, a.nrows);
  c.A = A;
  c.B = B;
  c.lane = threadIdx.x & 63;
  c.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  c.h = c.lane >> 5;
  c.q = c.lane & 31;
  c.cl0 = CPL * c.lane;
  const bool colv = c.gcol(c.cl0) < a.F;
  const int64_t nrow = c.r1 - c.r0;
  const int64_t nsub = (nrow + SR - 1) / SR;
  const int tid = threadIdx.x;
  uint64_t* out = a.rec + b * rec_words(a.p);

  // rows of sub-steps 0 and 1 in flight during the sampling
  typename Ctx<DIAG>::Raw rs[2];
  c.load(0, rs[0]);
  if (nsub > 1) c.load(1, rs[1]);
  // ---- shifts; grids from NSAMP rows spread over the block ----
  for (int k = tid; k < NC; k += kThreads) {
    const int g = c.gcol(k);
    m.s_K[k] = *(const float*)(a.xbase + c.r0 * a.xstride + 4 * (int64_t)(g < a.F ? g : 0));
    m.s_exp[k] = 0x7FFFFFFF;  // lowest set bit of the sampled values, below
  }
  if (tid == 0) m.s_flag[0] = 0;
  lds_barrier();
  {
    double K[CPL], mx[CPL];
    int lb[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      K[i] = (double)m.s_K[c.cl0 + i];
      mx[i] = 0.0;
      lb[i] = 0x7FFFFFFF;
    }
    const char* col0 = a.xbase + 4 * (int64_t)(colv ? c.gcol(c.cl0) : 0);
    const int ns = nrow < NSAMP ? (int)nrow : NSAMP;
    // SB rows per wave in flight: sample k is row r0 + k (nrow - 1) / (ns - 1)
    for (int k0 = c.wave; k0 < ns; k0 += NW * SB) {
      float x[SB][CPL];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int k = min(k0 + NW * u, ns - 1);
        // 32-bit: nrow <= 2^16 rows per block and k < NSAMP
        const int64_t r = c.r0 + (ns > 1 ? (int)((unsigned)k * (unsigned)(nrow - 1) / (unsigned)(ns - 1)) : 0);
        if constexpr (CPL == 4) {
          const fl4 v = *(const fl4*)(col0 + r * a.xstride);
#pragma unroll
          for (int i = 0; i < 4; ++i) x[u][i] = v[i];
        } else {
          const fl2 v = *(const fl2*)(col0 + r * a.xstride);
#pragma unroll
          for (int i = 0; i < 2; ++i) x[u][i] = v[i];
        }
      }
#pragma unroll
      for (int u = 0; u < SB; ++u)
#pragma unroll
        for (int i = 0; i < CPL; ++i) mx[i] = fmax(mx[i], fabs((double)x[u][i] - K[i]));
      if (k0 == c.wave) {
        // the first NW x SB samples: exponent of each value's lowest set
        // bit (x = sig 2^(E - 150) for a normal FP32 value)
#pragma unroll
        for (int u = 0; u < SB; ++u)
#pragma unroll
          for (int i = 0; i < CPL; ++i) {
            const uint32_t bits = __float_as_uint(x[u][i]) & 0x7FFFFFFFu;
            const uint32_t E = bits >> 23;
            const uint32_t sig = E ? (bits & 0x7FFFFFu) | 0x800000u : bits;
            const int l = (E ? (int)E : 1) - 150 + __builtin_ctz(sig | 0x80000000u);
            lb[i] = sig ? min(lb[i], l) : lb[i];
          }
      }
    }
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      m.red[c.wave * NC + c.cl0 + i] = mx[i];
      atomicMin(&m.s_exp[c.cl0 + i], lb[i]);
    }
  }
  lds_barrier();
  for (int k = tid; k < NC; k += kThreads) {
    double mx = m.red[k];
#pragma unroll
    for (int w = 1; w < NW; ++w) mx = fmax(mx, m.red[w * NC + k]);
    const float K = m.s_K[k];
    const bool valid = c.gcol(k) < a.F && __builtin_isfinite(mx) && __builtin_isfinite(K);
    const int s = grid_exp(mx, K);
    // a sampled value below the grid's spacing 2^-s: this block's values do
    // not sit on a common grid (e.g. zero-mean data with full significands)
    if (valid && m.s_exp[k] < -s) m.s_flag[0] = 1;
    m.s_exp[k] = s;
    m.s_sc[k] = valid ? ldexpf(1.0f, s) : 0.0f;
    m.s_nks[k] = valid ? -K * ldexpf(1.0f, s) : 0.0f;
    // the grids of the block, for the sums pass (one writer per column)
    if (DIAG && half == 0 && c.gcol(k) < a.F) a.sexp[b * a.F + c.gcol(k)] = s;
  }
  lds_barrier();
  if (m.s_flag[0]) {
    // the whole block is recomputed in FP64
    if (tid == 0) a.ovf[b] = 1;
    return;
  }

  c.load_grids();
  const WaveTiles wt = wave_tiles<DIAG>(c.wave, half);
  // whether the wave has a tile that holds vector columns (a short last
  // group leaves some tiles out); 0: no products
  int nt = 0;
#pragma unroll
  for (int u = 0; u < MT; ++u)
    if (u < wt.n && A * G + 32 * wt.ti[u] < a.F && B * G + 32 * wt.tj[u] < a.F) nt = u + 1;
  nt = __builtin_amdgcn_readfirstlane(nt);
  i16 L[MT][5];
#pragma unroll
  for (int u = 0; u < MT; ++u)
#pragma unroll
    for (int l = 0; l < 5; ++l) L[u][l] = (i16){};

  if (SR > nrow) c.template digitize<true>(0, rs[0]);
  else c.template digitize<false>(0, rs[0]);
  lds_barrier();
  // Sub-step t: loads of t + 2 into the registers of t (converted one
  // sub-step ago), operands of t, products of t and digits of t + 1 (loaded
  // one sub-step ago), interleaved so that the conversion's vector
  // instructions issue while the matrix cores work.  Register sets
  // alternate, so the main loop takes two sub-steps per trip; the last
  // sub-steps run one at a time.  Waves without a tile run the same loop
  // without the products (same barriers).
  const int64_t step_bytes = (int64_t)SR * a.xstride;
  const char* rp0;  // this lane's address in the wave's first row of sub-step 2
  {
    const int dc = c.gcol(c.cl0);
    const int64_t col = dc < a.F ? dc : 0;
    rp0 = a.xbase + (c.r0 + 2 * SR + RW * c.wave) * a.xstride + 4 * col;
  }
  using T_ = std::true_type;
  using F_ = std::false_type;
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  auto run = [&](auto prod_c) __attribute__((always_inline)) {
    constexpr bool PROD = decltype(prod_c)::value;
    const char* rp = rp0;
    // PAR = t & 1; LOAD: 0 none, 1 inside the block (rp), 2 clamped
    auto step = [&](int64_t t, auto par_c, auto load_c, auto more_c, auto tail_c) __attribute__((always_inline)) {
      constexpr int PAR = decltype(par_c)::value;
      constexpr int LOAD = decltype(load_c)::value;
      constexpr bool MORE = decltype(more_c)::value;
      constexpr bool TAIL = decltype(tail_c)::value;
      if constexpr (LOAD == 1) c.load_inside(rp, rs[PAR]);
      if constexpr (LOAD == 2) c.load(t + 2, rs[PAR]);
      Ops o;
      if constexpr (PROD) load_ops<DIAG>(m.dig, PAR, wt, c.h, c.q, o);
      if constexpr (PROD) mma_ops(o, L);
      if constexpr (MORE) c.template digitize<TAIL>(t + 1, rs[PAR ^ 1]);
      if constexpr (PROD && MORE) {
        // one product, then a share of the conversion, nine times
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, DIAG ? 4 : 8, 0);
        }
      }
      lds_barrier();
    };
    int64_t t = 0;
    // pairs of sub-steps whose loads (t + 2, t + 3) lie wholly inside the block
    for (; t + 3 < nsub && c.r0 + (t + 4) * SR <= c.r1; t += 2) {
      step(t, I0{}, I1{}, T_{}, F_{});
      rp += step_bytes;
      step(t + 1, I1{}, I1{}, T_{}, F_{});
      rp += step_bytes;
    }
    // the rest one by one: loads clamped to the block, rows past its end
    // give zero digits
    for (; t + 2 < nsub; ++t) {
      if (t & 1) step(t, I1{}, std::integral_constant<int, 2>{}, T_{}, T_{});
      else step(t, I0{}, std::integral_constant<int, 2>{}, T_{}, T_{});
    }
    if (t + 1 < nsub) {
      if (t & 1) step(t, I1{}, I0{}, T_{}, T_{});
      else step(t, I0{}, I0{}, T_{}, T_{});
      ++t;
    }
    if (t & 1) step(t, I1{}, I0{}, F_{}, F_{});
    else step(t, I0{}, I0{}, F_{}, F_{});
  };
  if (nt) run(T_{});
  else run(F_{});

  // ---- tiles: levels combined, scaled by the grids, into the record ----
  const int p = a.p;
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    if (u >= nt) break;
    const int sbl = (DIAG ? 0 : G) + 32 * wt.tj[u] + c.q;
    const int cb = B * G + 32 * wt.tj[u] + c.q;
    const int ub = a.col_of[cb < a.F ? cb : 0];
    const int sb = m.s_exp[sbl];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int sal = 32 * wt.ti[u] + (k >> 2) * 8 + c.h * 4 + (k & 3);
      const int ca = A * G + sal;
      if (ca < a.F && cb < a.F && (ca <= cb || wt.ti[u] != wt.tj[u])) {
        double P = (double)L[u][4][k];
        P = __builtin_fma(P, 0x1p-8, (double)L[u][3][k]);
        P = __builtin_fma(P, 0x1p-8, (double)L[u][2][k]);
        P = __builtin_fma(P, 0x1p-8, (double)L[u][1][k]);
        P = __builtin_fma(P, 0x1p-8, (double)L[u][0][k]);
        const int ua = a.col_of[ca];
        out[2 + 2 * p + tri(p, min(ua, ub), max(ua, ub))] =
            (uint64_t)__double_as_longlong(ldexp(P, 32 - m.s_exp[sal] - sb));
      }
    }
  }
}

// ---- column sums, products with the extra columns, checks of the grids ----
//
// The rest of a block's record needs no matrix cores.  On the block's grids
// every shifted value d = x - K has at most 22 significant bits, every
// shifted integer extra at most the bits of the block's identifier range, and
// the products and their sums over 32768 rows stay far below 2^53: formed in
// FP64 from the FP32 values they are exact, so they equal the sums of the grid
// integers scaled by 2^-s whatever the order.  d itself is formed in FP32,
// exact on the grid.  The same pass checks every value against its grid: x 2^s
// an integer (one v_fract), |d| 2^s <= 2^22 - 1, finite; a value that fails
// flags the block for the FP64 routine (which also takes blocks already
// flagged by the matrix-core kernel; they are skipped here).
//
// One workgroup per block and 256 vector columns.  Wave w takes rows
// r0 + w + 4 k; its rows move from HBM to its own LDS ring by direct DMA
// (one 1 KiB global_load_lds_dwordx4 per row, lane l bringing columns
// 4 l .. 4 l + 3 of the chunk; lanes 0..15 bring the extras' words), four
// rows a stage, three stages, two in flight, so the only wait is on the
// wave's own vector-memory counter.  The waves' sums are added in a fixed
// order at the end.  The first chunk also forms the extras' own sums and
// products.
constexpr int kSumThreads = 256;
constexpr int kSumRPW = 4;                    // rows per wave and stage
constexpr int kSumNS = 3;                     // stages per wave
constexpr int kSumSB = kSumRPW * 1024 + 64;   // stage bytes: rows + extras' words

template <int NS>  // the number of extra columns (a.ne)
__global__ __launch_bounds__(kSumThreads, 3) void k_syrk_sums(wide::SyrkArgs a) {
  constexpr int NQ = NE * (NE + 1) / 2;
  constexpr int NW4 = kSumThreads / 64;
  constexpr int RED = 4 * 64 * (1 + NE) + NE + NQ;  // doubles per wave in the final sums
  __shared__ __attribute__((aligned(16))) unsigned char s_ring[NW4 * kSumNS * kSumSB];
  static_assert(sizeof(s_ring) >= NW4 * RED * sizeof(double), "the final sums reuse the ring");
  const int F = a.F, p = a.p;
  const int nch = (F + 255) / 256;
  const int64_t b = blockIdx.x / nch;
  const int cb = 256 * (int)(blockIdx.x % nch);  // first column of the chunk
  if (a.ovf[b]) return;                          // recomputed in FP64
  const int64_t r0 = b * a.R, r1 = min(r0 + a.R, a.nrows);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ne = cb == 0 ? a.ne : 0;  // the extras' own sums: first chunk
  constexpr int ns = NS;               // strips with the extras: every chunk
  const int c0 = cb + 4 * lane;
  const bool cv = c0 < F;  // F is a multiple of 4
  float K[4], lim[4], sc[4];
  {
    const fl4 k4 = cv ? *(const fl4*)(a.xbase + r0 * a.xstride + 4 * (int64_t)c0) : (fl4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int sx = cv ? a.sexp[b * F + c0 + i] : 0;
      K[i] = k4[i];
      sc[i] = ldexpf(1.0f, sx);
      lim[i] = ldexpf(kVlim, -sx);  // exact: kVlim has 22 significant bits
    }
  }
  double eK[NE];
  int64_t eKi[NE];
  bool e64[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    eK[e] = 0.0;
    eKi[e] = 0;
    e64[e] = e < ns && wide_kind(a.ex[e].kind);
    if (e < ns) extra_shift(a.ex[e], r0, eK[e], eKi[e]);
  }
  double S[4] = {0.0, 0.0, 0.0, 0.0}, ST[NE][4], es[NE], eq[NQ];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    es[e] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) ST[e][i] = 0.0;
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) eq[q] = 0.0;
  float fo = 0.0f;
  bool over = false;
  uint32_t bad = 0;

  // rows of this wave: r0 + wave + 4 k, k < nk; stage t holds k = 4 t .. 4 t + 3
  const int64_t nk = (r1 - r0 - wave + 3) / 4;
  const int64_t nst = (nk + kSumRPW - 1) / kSumRPW;
  unsigned char* ring = s_ring + wave * kSumNS * kSumSB;
  const int64_t colb = cv ? c0 : cb;  // a valid column for idle lanes
  const bool exl = lane < 16 && (lane >> 3) < ns && (((lane >> 2) & 1) == 0 || e64[lane >> 3]);
  auto issue = [&](int64_t t) {
    unsigned char* st = ring + (int)(t % kSumNS) * kSumSB;
#pragma unroll
    for (int j = 0; j < kSumRPW; ++j) {
      int64_t r = r0 + wave + 4 * (kSumRPW * t + j);
      r = r < r1 ? r : r1 - 1;
      __builtin_amdgcn_global_load_lds((const void*)(a.xbase + r * a.xstride + 4 * colb),
                                       (__attribute__((address_space(3))) void*)(st + j * 1024), 16, 0, 0);
    }
    if (ns > 0) {
      // lane 8e + 4w + j: dword w of extra e in row j of the stage
      if (exl) {
        const int e = lane >> 3, wd = (lane >> 2) & 1, j = lane & 3;
        int64_t r = r0 + wave + 4 * (kSumRPW * t + j);
        r = r < r1 ? r : r1 - 1;
        __builtin_amdgcn_global_load_lds((const void*)(a.ex[e].base + r * a.ex[e].stride + 4 * wd),
                                         (__attribute__((address_space(3))) void*)(st + kSumRPW * 1024), 4, 0, 0);
      }
    }
  };
#pragma unroll
  for (int t = 0; t < kSumNS - 1; ++t)
    if (t < nst) issue(t);
  for (int64_t t = 0; t < nst; ++t) {
    // stage t is this wave's oldest outstanding group of loads
    if (t + kSumNS - 2 < nst) {
      if (ns > 0) __builtin_amdgcn_s_waitcnt(VmWait<(kSumNS - 2) * (kSumRPW + 1)>::imm);
      else __builtin_amdgcn_s_waitcnt(VmWait<(kSumNS - 2) * kSumRPW>::imm);
    } else {
      __builtin_amdgcn_s_waitcnt(VmWait<0>::imm);
    }
    // the slot refilled next was read by this wave in the last iteration
    if (t + kSumNS - 1 < nst) issue(t + kSumNS - 1);
    const unsigned char* st = ring + (int)(t % kSumNS) * kSumSB;
#pragma unroll
    for (int j = 0; j < kSumRPW; ++j) {
      if (kSumRPW * t + j >= nk) break;
      const fl4 v = *(const __attribute__((address_space(3))) fl4*)(st + j * 1024 + 16 * lane);
      double de[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        de[e] = 0.0;
        if (e < ns) {
          const __attribute__((address_space(3))) uint32_t* w =
              (const __attribute__((address_space(3))) uint32_t*)(st + kSumRPW * 1024);
          const uint32_t lo = w[8 * e + j], hi = w[8 * e + 4 + j];
          const wide::SyrkExtra& x = a.ex[e];
          switch (x.kind) {
            case STATS_I32: de[e] = (double)(int32_t)lo - eK[e]; break;
            case STATS_I64: de[e] = (double)((int64_t)(((uint64_t)hi << 32) | lo) - eKi[e]); break;
            case STATS_F32: {
              const double y = (double)__uint_as_float(lo);
              if (x.chk) bad |= (y != __builtin_rint(y));
              de[e] = y - eK[e];
              break;
            }
            default: {
              const double y = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
              if (x.chk) bad |= (y != __builtin_rint(y));
              de[e] = y - eK[e];
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float x = v[i];
        const float d32 = x - K[i];  // exact on the grid
        const double d = (double)d32;
        S[i] += d;
#pragma unroll
        for (int e = 0; e < NS; ++e) ST[e][i] = __builtin_fma(d, de[e], ST[e][i]);
        fo = fmaxf(fo, __builtin_amdgcn_fractf(x * sc[i]));
        over |= !(fabsf(d32) <= lim[i]);
      }
      int q = 0;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        if (e < NS) es[e] += de[e];
#pragma unroll
        for (int g = e; g < NE; ++g, ++q)
          if (g < NS) eq[q] = __builtin_fma(de[e], de[g], eq[q]);
      }
    }
  }
  over |= !(fo == 0.0f);
  if (!cv) over = false;
  if (over) a.ovf[b] = 1;
  if (bad) atomicOr(&a.status->bits, ST_INEXACT);
  __syncthreads();  // every wave is done with its ring
  double* s_red = (double*)s_ring;
  double* red = s_red + wave * RED;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    red[4 * lane + i] = S[i];
#pragma unroll
    for (int e = 0; e < NE; ++e) red[256 * (1 + e) + 4 * lane + i] = ST[e][i];
  }
  if (lane == 0) {
#pragma unroll
    for (int e = 0; e < NE; ++e) red[256 * (1 + NE) + e] = es[e];
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[256 * (1 + NE) + NE + q] = eq[q];
  }
  __syncthreads();
  uint64_t* out = a.rec + b * rec_words(p);
  for (int k = threadIdx.x; k < 256 && cb + k < F; k += kSumThreads) {
    const int uc = a.col_of[cb + k];
    double sum = s_red[k];
#pragma unroll
    for (int w = 1; w < NW4; ++w) sum += s_red[w * RED + k];
    out[2 + p + uc] = (uint64_t)__double_as_longlong(sum);
    out[2 + uc] = (uint64_t)__double_as_longlong((double)*(const float*)(a.xbase + r0 * a.xstride + 4 * (int64_t)(cb + k)));
    for (int e = 0; e < ns; ++e) {
      double st = s_red[256 * (1 + e) + k];
#pragma unroll
      for (int w = 1; w < NW4; ++w) st += s_red[w * RED + 256 * (1 + e) + k];
      const int ue = a.col_of[F + e];
      out[2 + 2 * p + tri(p, min(uc, ue), max(uc, ue))] = (uint64_t)__double_as_longlong(st);
    }
  }
  if (threadIdx.x == 0 && cb == 0) {
    int q = 0;
    for (int e = 0; e < NE; ++e) {
      if (e < ne) {
        double se = s_red[256 * (1 + NE) + e];
        for (int w = 1; w < NW4; ++w) se += s_red[w * RED + 256 * (1 + NE) + e];
        const int ue = a.col_of[F + e];
        out[2 + p + ue] = (uint64_t)__double_as_longlong(se);
        out[2 + ue] = shift_word(a.ex[e].isint, a.ex[e].kind, eK[e], eKi[e]);
      }
      for (int g = e; g < NE; ++g, ++q)
        if (g < ne) {
          double sq = s_red[256 * (1 + NE) + NE + q];
          for (int w = 1; w < NW4; ++w) sq += s_red[w * RED + 256 * (1 + NE) + NE + q];
          const int ue = a.col_of[F + e], uf = a.col_of[F + g];
          out[2 + 2 * p + tri(p, min(ue, uf), max(ue, uf))] = (uint64_t)__double_as_longlong(sq);
        }
    }
    out[0] = (uint64_t)(r1 - r0);
    out[1] = 0;
  }
}

__global__ __launch_bounds__(kThreads, 1) void k_syrk_i8(wide::SyrkArgs a) {
  __shared__ __attribute__((aligned(16))) union {
    int dig[2 * 3 * 8 * PITCH_MAX];
    double red[NW * 2 * G];
  } s_u;
  __shared__ int s_exp[2 * G];
  __shared__ float s_K[2 * G], s_sc[2 * G], s_nks[2 * G];
  __shared__ int s_flag;
  const int64_t id = blockIdx.x;
  const int64_t xcd = id & 7, y = id >> 3;
  const int t = (int)(y % a.npairs);
  const int64_t b = (y / a.npairs) * 8 + xcd;
  if (b >= a.nblocks) return;
  const int A = a.pairs[t].x & 15, B = a.pairs[t].y, half = a.pairs[t].x >> 4;
  Lds m;
  m.dig = s_u.dig;
  m.red = s_u.red;
  m.s_exp = s_exp;
  m.s_K = s_K;
  m.s_sc = s_sc;
  m.s_nks = s_nks;
  m.s_flag = &s_flag;
  if (A != B) pair_block<false>(a, m, b, A, B, half);
  else pair_block<true>(a, m, b, A, B, half);
}

__global__ void k_zero_flags(int* f, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = 0;
}

}  // namespace syrk

void launch_syrk_split(const wide::SyrkArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(syrk::k_zero_flags, dim3((unsigned)((a.nblocks + 255) / 256)), dim3(256), 0, s, a.ovf,
                     a.nblocks);
  const int64_t nb8 = (a.nblocks + 7) / 8 * 8;
  hipLaunchKernelGGL(syrk::k_syrk_i8, dim3((unsigned)(nb8 * a.npairs)), dim3(syrk::kThreads), 0, s, a);
  const int64_t nch = (a.F + 255) / 256;
  const dim3 gs((unsigned)(a.nblocks * nch));
  switch (a.ne) {
    case 0: hipLaunchKernelGGL(syrk::k_syrk_sums<0>, gs, dim3(syrk::kSumThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL(syrk::k_syrk_sums<1>, gs, dim3(syrk::kSumThreads), 0, s, a); break;
    default: hipLaunchKernelGGL(syrk::k_syrk_sums<2>, gs, dim3(syrk::kSumThreads), 0, s, a); break;
  }
}

}  // namespace st
