/* Host (CPU) side of the seeded synthetic-data generator.
 *
 * Produces rows shaped like the paper's Table 1 dataset (section "Background
 * and Motivation", Table 1): an identifier A, three uniform integers B, C, D,
 * and deterministic functions E..K of them.  Plus the extended 32-column rows
 * (Table 1 columns and 22 i.i.d. U{0..100} integers) and CSV text lines.
 *
 * Everything here is input generation.  It is shared by the CPU oracle, the
 * tests and the benchmark; it computes none of the statistics. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "philox.h"

/* ---- Table 1 lookup tables, built once with the host libm ------------------
 * Index conventions: E[b][c] with B = b + 3, C = c + 1; F[b][d] with D = d + 1.
 * Reading of the formulas (Table 1): int() truncates toward zero, round() is
 * C round (half away from zero), log is natural, trig in radians. */
typedef struct {
  double E[6][10], F[6][100], G[10], H[100], cot[10], I[10], J[100];
  int32_t K[10][100];
  int built;
} dg_tables;

static dg_tables T;

static int build_tables(void) {
  int bad = 0;
  for (int b = 0; b < 6; ++b) {
    const int B = b + 3;
    for (int c = 0; c < 10; ++c) {
      const int C = c + 1;
      T.E[b][c] = (double)(int)(log((double)C) / log((double)B) * 100.0);
    }
    for (int d = 0; d < 100; ++d) {
      const int D = d + 1;
      T.F[b][d] = round((log((double)D) / log((double)B)) * 10000.0);
    }
  }
  for (int c = 0; c < 10; ++c) {
    const int C = c + 1;
    T.G[c] = (double)(int)(fabs(cos((double)C)) * 100.0);
    T.cot[c] = 1.0 / tan((double)C);
    T.I[c] = round(fabs(T.cot[c]) * 1000.0);
    for (int d = 0; d < 100; ++d) T.K[c][d] = (d + 1) / C;
  }
  for (int d = 0; d < 100; ++d) {
    const int D = d + 1;
    T.H[d] = (double)(int)(fabs(sin((double)D)) * 100.0);
    T.J[d] = fabs(tan((double)D));
  }
  /* The 15 (B, C) pairs where log(C)/log(B)*100 is mathematically an integer:
   * C = 1 gives 0, C = B gives 100, (3,9) gives 200, (4,2) gives 50, (4,8)
   * gives 150.  A one-ulp libm error would flip the truncation there. */
  for (int b = 0; b < 6; ++b) {
    if (T.E[b][0] != 0.0) ++bad;
    if (T.E[b][b + 2] != 100.0) ++bad; /* C = B */
  }
  if (T.E[0][8] != 200.0) ++bad; /* B = 3, C = 9 */
  if (T.E[1][1] != 50.0) ++bad;  /* B = 4, C = 2 */
  if (T.E[1][7] != 150.0) ++bad; /* B = 4, C = 8 */
  T.built = 1;
  return bad;
}

static void ensure_tables(void) {
  if (!T.built) build_tables();
}

/* Returns the number of the 15 exact-integer E cases the host libm got wrong
 * (0 expected) and copies the tables out (any pointer may be NULL). */
int dg_table1_tables(double* E60, double* F600, double* G10, double* H100, double* cot10,
                     double* I10, double* J100, int32_t* K1000) {
  int bad = build_tables();
  if (E60) memcpy(E60, T.E, sizeof T.E);
  if (F600) memcpy(F600, T.F, sizeof T.F);
  if (G10) memcpy(G10, T.G, sizeof T.G);
  if (H100) memcpy(H100, T.H, sizeof T.H);
  if (cot10) memcpy(cot10, T.cot, sizeof T.cot);
  if (I10) memcpy(I10, T.I, sizeof T.I);
  if (J100) memcpy(J100, T.J, sizeof T.J);
  if (K1000) memcpy(K1000, T.K, sizeof T.K);
  return bad;
}

/* Philox block for tests against published known-answer vectors. */
void dg_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  dg_u32x4 u = dg_philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
  memcpy(out, u.v, sizeof u.v);
}

/* One Table-1 row.  Column order: A B C D E F G H cotC I J K. */
static void table1_row(uint64_t seed, uint64_t grow, int64_t a, double* v) {
  int32_t B, C, D;
  dg_table1_draws(seed, grow, &B, &C, &D);
  const int b = B - 3, c = C - 1, d = D - 1;
  v[0] = (double)a;
  v[1] = B; v[2] = C; v[3] = D;
  v[4] = T.E[b][c]; v[5] = T.F[b][d]; v[6] = T.G[c]; v[7] = T.H[d];
  v[8] = T.cot[c]; v[9] = T.I[c]; v[10] = T.J[d]; v[11] = (double)T.K[c][d];
}

/* Row-major FP64 rows of `ncols` (10 or 12) Table-1 columns.  Global row
 * index row0 + r seeds the draws; the identifier is a0 + r. */
void dg_table1_aos(uint64_t seed, int64_t row0, int64_t a0, int64_t n, int32_t ncols, double* out) {
  ensure_tables();
  double v[12];
  for (int64_t r = 0; r < n; ++r) {
    table1_row(seed, (uint64_t)(row0 + r), a0 + r, v);
    memcpy(out + r * ncols, v, sizeof(double) * (size_t)ncols);
  }
}

/* Planar layout, one plane per column, columns A B C D E F G H cotC I:
 * int32 planes for the nine integer columns, an FP64 plane for cotC. */
void dg_table1_planar(uint64_t seed, int64_t row0, int64_t a0, int64_t n, void* const* planes) {
  ensure_tables();
  double v[12];
  for (int64_t r = 0; r < n; ++r) {
    table1_row(seed, (uint64_t)(row0 + r), a0 + r, v);
    for (int k = 0; k < 10; ++k) {
      if (k == 8) ((double*)planes[k])[r] = v[k];
      else ((int32_t*)planes[k])[r] = (int32_t)v[k];
    }
  }
}

/* 32-column FP64 rows: the 10 Table-1 columns then 22 i.i.d. U{0..100}. */
void dg_groups_aos(uint64_t seed, int64_t row0, int64_t a0, int64_t n, double* out) {
  ensure_tables();
  double v[12];
  for (int64_t r = 0; r < n; ++r) {
    const uint64_t g = (uint64_t)(row0 + r);
    table1_row(seed, g, a0 + r, v);
    double* o = out + r * 32;
    memcpy(o, v, sizeof(double) * 10);
    for (int blk = 0; blk < 6; ++blk) {
      dg_u32x4 u = dg_extra_block(seed, g, blk);
      for (int w = 0; w < 4; ++w) {
        const int k = blk * 4 + w;
        if (k < 22) o[10 + k] = (double)dg_uniform_int(u.v[w], 0, 101);
      }
    }
  }
}

/* Log-uniform group sizes floor(exp(U(ln lo, ln hi))), U from 53-bit draws. */
void dg_group_sizes(uint64_t seed, int32_t ngroups, double lo, double hi, int64_t* sizes) {
  const double a = log(lo), b = log(hi);
  for (int32_t g = 0; g < ngroups; ++g) {
    dg_u32x4 u = dg_philox4x32_10((uint32_t)g, 0u, DG_STREAM_GROUPS, 0u, (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    const uint64_t m = ((uint64_t)u.v[0] << 21) ^ (uint64_t)(u.v[1] >> 11);
    const double x = (double)(m & ((1ull << 53) - 1)) * 0x1p-53;
    sizes[g] = (int64_t)floor(exp(a + (b - a) * x));
  }
}

/* ---- CSV text -------------------------------------------------------------
 * One line per row: "A,B,C,D,E,F,G,H,cotC,I\n", integers in decimal and
 * cotC printed with "%.17g" (17 significant digits round-trip a double). */
static int put_int(char* o, int64_t x) {
  char tmp[24];
  int n = 0, neg = x < 0;
  uint64_t u = neg ? (uint64_t)(-(x + 1)) + 1u : (uint64_t)x;
  do { tmp[n++] = (char)('0' + u % 10u); u /= 10u; } while (u);
  int k = 0;
  if (neg) o[k++] = '-';
  while (n) o[k++] = tmp[--n];
  return k;
}

static char cot_txt[10][32];
static int cot_len[10];
static int cot_built;

static void ensure_cot_txt(void) {
  ensure_tables();
  if (cot_built) return;
  for (int c = 0; c < 10; ++c) cot_len[c] = snprintf(cot_txt[c], sizeof cot_txt[c], "%.17g", T.cot[c]);
  cot_built = 1;
}

static int csv_line(uint64_t seed, uint64_t grow, int64_t a, char* o) {
  double v[12];
  table1_row(seed, grow, a, v);
  int k = 0;
  for (int j = 0; j < 10; ++j) {
    if (j) o[k++] = ',';
    if (j == 8) {
      const int c = (int)v[2] - 1;
      memcpy(o + k, cot_txt[c], (size_t)cot_len[c]);
      k += cot_len[c];
    } else {
      k += put_int(o + k, (int64_t)v[j]);
    }
  }
  o[k++] = '\n';
  return k;
}

/* Number of bytes dg_table1_csv would write for these rows. */
int64_t dg_table1_csv_size(uint64_t seed, int64_t row0, int64_t a0, int64_t n) {
  ensure_cot_txt();
  char line[256];
  int64_t tot = 0;
  for (int64_t r = 0; r < n; ++r) tot += csv_line(seed, (uint64_t)(row0 + r), a0 + r, line);
  return tot;
}

/* Writes the rows as CSV into out (capacity cap); returns the bytes written,
 * or -1 if cap is too small (nothing past cap is touched). */
int64_t dg_table1_csv(uint64_t seed, int64_t row0, int64_t a0, int64_t n, char* out, int64_t cap) {
  ensure_cot_txt();
  char line[256];
  int64_t off = 0;
  for (int64_t r = 0; r < n; ++r) {
    const int k = csv_line(seed, (uint64_t)(row0 + r), a0 + r, line);
    if (off + k > cap) return -1;
    memcpy(out + off, line, (size_t)k);
    off += k;
  }
  return off;
}

/* Fuzz words for text-parser tests: n raw 64-bit Philox words. */
void dg_fuzz_words(uint64_t seed, int64_t n, uint64_t* out) {
  for (int64_t i = 0; i < n; i += 2) {
    dg_u32x4 u = dg_philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), DG_STREAM_FUZZ, 0u,
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
    out[i] = ((uint64_t)u.v[1] << 32) | u.v[0];
    if (i + 1 < n) out[i + 1] = ((uint64_t)u.v[3] << 32) | u.v[2];
  }
}
