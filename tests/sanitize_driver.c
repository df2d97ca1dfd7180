/* Host driver for the sanitizer test: exercises the C oracle and the host
 * data generator under AddressSanitizer and UndefinedBehaviorSanitizer on
 * small inputs (ragged lengths, every column type, CSV round trip,
 * missing-value passes).  Exit status 0 when every call returns what it
 * should; the sanitizers abort on any error they catch. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  const void* base;
  int64_t stride;
  int32_t dtype;
  int32_t is_int;
} oc_col;

int oracle_pass1(const oc_col*, int32_t, int64_t, int64_t, uint64_t*, double*, uint64_t*, double*);
int oracle_pass_int(const oc_col*, int32_t, int64_t, int64_t, uint64_t*, uint64_t*);
void oracle_pass2(const oc_col*, int32_t, int64_t, int64_t, const double*, double*);
void oracle_pw_pass1(const oc_col*, int32_t, int64_t, int64_t, int64_t*, double*, double*);
void oracle_pw_pass2(const oc_col*, int32_t, int64_t, int64_t, const double*, const double*, double*, double*,
                     double*);
int64_t oracle_parse_csv(const char*, int64_t, int32_t, const int32_t*, double*, int64_t);
void dg_table1_aos(uint64_t, int64_t, int64_t, int64_t, int32_t, double*);
void dg_table1_planar(uint64_t, int64_t, int64_t, int64_t, void* const*);
void dg_groups_aos(uint64_t, int64_t, int64_t, int64_t, double*);
void dg_group_sizes(uint64_t, int32_t, double, double, int64_t*);
int64_t dg_table1_csv_size(uint64_t, int64_t, int64_t, int64_t);
int64_t dg_table1_csv(uint64_t, int64_t, int64_t, int64_t, char*, int64_t);

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main(void) {
  enum { P = 10, T = P * (P + 1) / 2 };
  const int64_t sizes[] = {1, 2, 7, 1000, 4097};
  for (int k = 0; k < 5; ++k) {
    const int64_t n = sizes[k];
    double* x = malloc(sizeof(double) * P * n);
    dg_table1_aos(3, 0, 1, n, P, x);
    oc_col cols[P];
    for (int c = 0; c < P; ++c) {
      cols[c].base = x + c;
      cols[c].stride = 8 * P;
      cols[c].dtype = 4;
      cols[c].is_int = c != 8;
    }
    uint64_t s_int[2 * P], C_int[2 * T];
    double s_fp[2 * P], C_fp[2 * T], M2[2 * T], mu[P];
    CHECK(oracle_pass1(cols, P, 0, n, s_int, s_fp, C_int, C_fp) == 0);
    CHECK(s_int[0] == (uint64_t)(n * (n + 1) / 2));
    for (int c = 0; c < P; ++c) mu[c] = (s_fp[2 * c] + s_fp[2 * c + 1]) / (double)n;
    oracle_pass2(cols, P, 0, n, mu, M2);
    int32_t isint[P];
    for (int c = 0; c < P; ++c) isint[c] = c != 8;
    oc_col icols[9];
    int m = 0;
    for (int c = 0; c < P; ++c)
      if (c != 8) icols[m++] = cols[c];
    uint64_t si2[18], ci2[90];
    CHECK(oracle_pass_int(icols, 9, 0, n, si2, ci2) == 0);
    /* planes of every storage type */
    void* planes[10];
    for (int c = 0; c < 10; ++c) planes[c] = malloc(8 * (size_t)n);
    dg_table1_planar(5, 0, 1, n, planes);
    for (int c = 0; c < 10; ++c) free(planes[c]);
    /* CSV round trip */
    const int64_t sz = dg_table1_csv_size(3, 0, 1, n);
    char* txt = malloc((size_t)sz);
    CHECK(dg_table1_csv(3, 0, 1, n, txt, sz) == sz);
    CHECK(dg_table1_csv(3, 0, 1, n, txt, sz - 1) == -1);
    double* y = malloc(sizeof(double) * P * n);
    CHECK(oracle_parse_csv(txt, sz, P, isint, y, n) == n);
    CHECK(memcmp(x, y, sizeof(double) * P * n) == 0);
    /* missing values */
    for (int64_t r = 0; r < n; r += 3) x[r * P + (r % P)] = NAN;
    int64_t cnt[T];
    double a[2 * T], b[2 * T], ma[T], mb[T], cij[2 * T], cii[2 * T], cjj[2 * T];
    memset(cnt, 0, sizeof cnt);
    oracle_pw_pass1(cols, P, 0, n, cnt, a, b);
    for (int t = 0; t < T; ++t) {
      ma[t] = cnt[t] ? (a[2 * t] + a[2 * t + 1]) / (double)cnt[t] : 0.0;
      mb[t] = cnt[t] ? (b[2 * t] + b[2 * t + 1]) / (double)cnt[t] : 0.0;
    }
    oracle_pw_pass2(cols, P, 0, n, ma, mb, cij, cii, cjj);
    free(x);
    free(y);
    free(txt);
  }
  double g[32 * 100];
  dg_groups_aos(4, 0, 1, 100, g);
  int64_t gs[64];
  dg_group_sizes(4, 64, 1e3, 1e7, gs);
  for (int k = 0; k < 64; ++k) CHECK(gs[k] >= 1000 && gs[k] <= 10000000);
  printf("sanitized oracle and generator: ok\n");
  return 0;
}
