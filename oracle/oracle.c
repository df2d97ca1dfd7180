/* CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, two-pass reference for the single-pass sufficient statistics
 * of the paper (section "Data Representation and Sufficient Statistics"):
 * the row count n, the column sums s = X^T 1 and the cross products
 * C = X^T X, plus the centred co-moments M2 = sum (x - mu)(x - mu)^T that the
 * covariance needs (section "Numerical Considerations": forming X^T X and
 * n mu mu^T separately and subtracting cancels catastrophically, so the
 * oracle never does that for floating-point columns).
 *
 *  - Integer-valued columns: sums and cross products are exact integers,
 *    accumulated in __int128.
 *  - Any pair involving a floating-point column: pass 1 gives the mean, pass
 *    2 accumulates the centred products with error-free transformations
 *    (TwoSum, FMA-based TwoProduct) into a compensated sum, i.e. the
 *    "accurate dot product" of Ogita, Rump and Oishi (SIAM J. Sci. Comput.
 *    2005), whose result is as accurate as if computed in twice the working
 *    precision.  Each partial result is returned as an unevaluated (hi, lo)
 *    pair so the Python side can combine row ranges exactly.
 *  - CSV fields are parsed with strtod / strtoll (correctly rounded / exact).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this code.  It shares nothing with the GPU library. */
#include <errno.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

enum { OC_I32 = 1, OC_I64 = 2, OC_F32 = 3, OC_F64 = 4 };

/* One input column: element r lives at base + r * stride (bytes). */
typedef struct {
  const void* base;
  int64_t stride;
  int32_t dtype;
  int32_t is_int; /* 1: integer-valued column, summed exactly */
} oc_col;

static double get_f64(const oc_col* c, int64_t r) {
  const char* p = (const char*)c->base + r * c->stride;
  switch (c->dtype) {
    case OC_I32: return (double)*(const int32_t*)p;
    case OC_I64: return (double)*(const int64_t*)p;
    case OC_F32: return (double)*(const float*)p;
    default: return *(const double*)p;
  }
}

/* Integer value of an integer-valued column; *bad is set when an F32/F64
 * element is not an integer or is too large for the exact path. */
static i128 get_int(const oc_col* c, int64_t r, int32_t* bad) {
  const char* p = (const char*)c->base + r * c->stride;
  double v;
  switch (c->dtype) {
    case OC_I32: return (i128) * (const int32_t*)p;
    case OC_I64: return (i128) * (const int64_t*)p;
    case OC_F32: v = (double)*(const float*)p; break;
    default: v = *(const double*)p; break;
  }
  if (!(v == floor(v)) || fabs(v) >= 0x1p62) {
    *bad = 1;
    return 0;
  }
  return (i128)(int64_t)v;
}

/* Error-free transformations. */
static void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}

static void two_prod(double a, double b, double* p, double* e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

/* Compensated accumulator: value = hi + lo (lo gathers every rounding error). */
typedef struct { double hi, lo; } comp;

static void comp_add(comp* c, double v) {
  double s, e;
  two_sum(c->hi, v, &s, &e);
  c->hi = s;
  c->lo += e;
}

/* Adds the exact product (ah + al) * (bh + bl), up to the al*bl term which
 * is below the working precision squared. */
static void comp_add_prod(comp* c, double ah, double al, double bh, double bl) {
  double p, e;
  two_prod(ah, bh, &p, &e);
  comp_add(c, p);
  c->lo += e + (ah * bl + al * bh) + al * bl;
}

/* Packed index of (i, j), i <= j, in the row-major upper triangle. */
static int64_t tri(int p, int i, int j) { return (int64_t)i * p - (int64_t)i * (i - 1) / 2 + (j - i); }

/* Pass 1 over rows [r0, r1).
 *   s_int[i]      exact sum of integer column i (two int64 halves: lo, hi)
 *   s_fp[2i..]    compensated (hi, lo) sum of column i (every column)
 *   C_int[t]      exact sum of x_i x_j for integer pairs (t = packed i <= j)
 *   C_fp[2t..]    compensated (hi, lo) sum of x_i x_j (every pair)
 * Returns 0, or 1 if an integer column holds a non-integer value. */
int oracle_pass1(const oc_col* cols, int32_t p, int64_t r0, int64_t r1, uint64_t* s_int,
                 double* s_fp, uint64_t* C_int, double* C_fp) {
  const int64_t T = (int64_t)p * (p + 1) / 2;
  i128* si = (i128*)calloc((size_t)p, sizeof(i128));
  i128* ci = (i128*)calloc((size_t)T, sizeof(i128));
  comp* sf = (comp*)calloc((size_t)p, sizeof(comp));
  comp* cf = (comp*)calloc((size_t)T, sizeof(comp));
  i128* xi = (i128*)calloc((size_t)p, sizeof(i128));
  double* xf = (double*)calloc((size_t)p, sizeof(double));
  int32_t bad = 0;
  for (int64_t r = r0; r < r1; ++r) {
    for (int i = 0; i < p; ++i) {
      xf[i] = get_f64(&cols[i], r);
      if (cols[i].is_int) xi[i] = get_int(&cols[i], r, &bad);
    }
    for (int i = 0; i < p; ++i) {
      comp_add(&sf[i], xf[i]);
      if (cols[i].is_int) si[i] += xi[i];
      for (int j = i; j < p; ++j) {
        const int64_t t = tri(p, i, j);
        comp_add_prod(&cf[t], xf[i], 0.0, xf[j], 0.0);
        if (cols[i].is_int && cols[j].is_int) ci[t] += xi[i] * xi[j];
      }
    }
  }
  for (int i = 0; i < p; ++i) {
    s_int[2 * i] = (uint64_t)si[i];
    s_int[2 * i + 1] = (uint64_t)(si[i] >> 64);
    s_fp[2 * i] = sf[i].hi;
    s_fp[2 * i + 1] = sf[i].lo;
  }
  for (int64_t t = 0; t < T; ++t) {
    C_int[2 * t] = (uint64_t)ci[t];
    C_int[2 * t + 1] = (uint64_t)(ci[t] >> 64);
    C_fp[2 * t] = cf[t].hi;
    C_fp[2 * t + 1] = cf[t].lo;
  }
  free(si); free(ci); free(sf); free(cf); free(xi); free(xf);
  return bad;
}

/* Exact pass over rows [r0, r1) for integer-valued columns only: the sums
 * and cross products of the definition (section "Data Representation and
 * Sufficient Statistics"), in __int128, nothing else.  Same output layout as
 * the integer part of oracle_pass1 (two int64 halves per entry, packed upper
 * triangle).  Returns 0, or 1 if a column holds a non-integer value. */
int oracle_pass_int(const oc_col* cols, int32_t p, int64_t r0, int64_t r1, uint64_t* s_int,
                    uint64_t* C_int) {
  const int64_t T = (int64_t)p * (p + 1) / 2;
  i128* si = (i128*)calloc((size_t)p, sizeof(i128));
  i128* ci = (i128*)calloc((size_t)T, sizeof(i128));
  i128* xi = (i128*)calloc((size_t)p, sizeof(i128));
  int32_t bad = 0;
  for (int64_t r = r0; r < r1; ++r) {
    for (int i = 0; i < p; ++i) xi[i] = get_int(&cols[i], r, &bad);
    for (int i = 0; i < p; ++i) {
      si[i] += xi[i];
      for (int j = i; j < p; ++j) ci[tri(p, i, j)] += xi[i] * xi[j];
    }
  }
  for (int i = 0; i < p; ++i) {
    s_int[2 * i] = (uint64_t)si[i];
    s_int[2 * i + 1] = (uint64_t)(si[i] >> 64);
  }
  for (int64_t t = 0; t < T; ++t) {
    C_int[2 * t] = (uint64_t)ci[t];
    C_int[2 * t + 1] = (uint64_t)(ci[t] >> 64);
  }
  free(si); free(ci); free(xi);
  return bad;
}

/* Pass 2 over rows [r0, r1): compensated (hi, lo) of the centred products
 * sum (x_i - mu_i)(x_j - mu_j) for every pair, where each difference is
 * itself kept exactly as a TwoSum pair. */
void oracle_pass2(const oc_col* cols, int32_t p, int64_t r0, int64_t r1, const double* mu,
                  double* M2) {
  const int64_t T = (int64_t)p * (p + 1) / 2;
  comp* acc = (comp*)calloc((size_t)T, sizeof(comp));
  double* dh = (double*)calloc((size_t)p, sizeof(double));
  double* dl = (double*)calloc((size_t)p, sizeof(double));
  for (int64_t r = r0; r < r1; ++r) {
    for (int i = 0; i < p; ++i) two_sum(get_f64(&cols[i], r), -mu[i], &dh[i], &dl[i]);
    for (int i = 0; i < p; ++i)
      for (int j = i; j < p; ++j) comp_add_prod(&acc[tri(p, i, j)], dh[i], dl[i], dh[j], dl[j]);
  }
  for (int64_t t = 0; t < T; ++t) {
    M2[2 * t] = acc[t].hi;
    M2[2 * t + 1] = acc[t].lo;
  }
  free(acc); free(dh); free(dl);
}

/* Missing values (NaN) and pairwise deletion: pass 1 over rows [r0, r1) gives,
 * for every pair t = (i <= j), the number of rows where both columns are
 * present and the compensated (hi, lo) sums of x_i and of x_j over those
 * rows. */
void oracle_pw_pass1(const oc_col* cols, int32_t p, int64_t r0, int64_t r1, int64_t* n, double* si,
                     double* sj) {
  const int64_t T = (int64_t)p * (p + 1) / 2;
  comp* a = (comp*)calloc((size_t)T, sizeof(comp));
  comp* b = (comp*)calloc((size_t)T, sizeof(comp));
  double* x = (double*)calloc((size_t)p, sizeof(double));
  for (int64_t r = r0; r < r1; ++r) {
    for (int i = 0; i < p; ++i) x[i] = get_f64(&cols[i], r);
    for (int i = 0; i < p; ++i) {
      if (isnan(x[i])) continue;
      for (int j = i; j < p; ++j) {
        if (isnan(x[j])) continue;
        const int64_t t = tri(p, i, j);
        n[t] += 1;
        comp_add(&a[t], x[i]);
        comp_add(&b[t], x[j]);
      }
    }
  }
  for (int64_t t = 0; t < T; ++t) {
    si[2 * t] = a[t].hi;
    si[2 * t + 1] = a[t].lo;
    sj[2 * t] = b[t].hi;
    sj[2 * t + 1] = b[t].lo;
  }
  free(a); free(b); free(x);
}

/* Pass 2: over the rows where both columns of pair t are present, the
 * compensated sums of (x_i - ma_t)(x_j - mb_t), (x_i - ma_t)^2 and
 * (x_j - mb_t)^2 (each difference kept exactly as a TwoSum pair). */
void oracle_pw_pass2(const oc_col* cols, int32_t p, int64_t r0, int64_t r1, const double* ma,
                     const double* mb, double* cij, double* cii, double* cjj) {
  const int64_t T = (int64_t)p * (p + 1) / 2;
  comp* c = (comp*)calloc((size_t)T, sizeof(comp));
  comp* u = (comp*)calloc((size_t)T, sizeof(comp));
  comp* w = (comp*)calloc((size_t)T, sizeof(comp));
  double* x = (double*)calloc((size_t)p, sizeof(double));
  for (int64_t r = r0; r < r1; ++r) {
    for (int i = 0; i < p; ++i) x[i] = get_f64(&cols[i], r);
    for (int i = 0; i < p; ++i) {
      if (isnan(x[i])) continue;
      for (int j = i; j < p; ++j) {
        if (isnan(x[j])) continue;
        const int64_t t = tri(p, i, j);
        double ah, al, bh, bl;
        two_sum(x[i], -ma[t], &ah, &al);
        two_sum(x[j], -mb[t], &bh, &bl);
        comp_add_prod(&c[t], ah, al, bh, bl);
        comp_add_prod(&u[t], ah, al, ah, al);
        comp_add_prod(&w[t], bh, bl, bh, bl);
      }
    }
  }
  for (int64_t t = 0; t < T; ++t) {
    cij[2 * t] = c[t].hi;
    cij[2 * t + 1] = c[t].lo;
    cii[2 * t] = u[t].hi;
    cii[2 * t + 1] = u[t].lo;
    cjj[2 * t] = w[t].hi;
    cjj[2 * t + 1] = w[t].lo;
  }
  free(c); free(u); free(w); free(x);
}

/* CSV parse: complete lines of p comma-separated fields.  Field j is read
 * with strtoll when is_int[j] (stored as double, exact below 2^53) and with
 * strtod otherwise.  Writes up to max_rows rows (row-major, p doubles each);
 * returns the number of rows, or -(1 + byte offset) of the first bad field. */
int64_t oracle_parse_csv(const char* buf, int64_t nbytes, int32_t p, const int32_t* is_int,
                         double* out, int64_t max_rows) {
  int64_t off = 0, rows = 0;
  char field[512];
  while (off < nbytes && rows < max_rows) {
    for (int j = 0; j < p; ++j) {
      const char term = (j == p - 1) ? '\n' : ',';
      int64_t e = off;
      while (e < nbytes && buf[e] != term && buf[e] != ',' && buf[e] != '\n') ++e;
      const int64_t len = e - off;
      const int at_end = (e >= nbytes);
      if (len <= 0 || len >= (int64_t)sizeof field || (!at_end && buf[e] != term) ||
          (at_end && j != p - 1))
        return -(1 + off);
      memcpy(field, buf + off, (size_t)len);
      field[len] = 0;
      char* endp = NULL;
      errno = 0;
      if (is_int[j]) {
        long long v = strtoll(field, &endp, 10);
        if (*endp || errno) return -(1 + off);
        out[rows * p + j] = (double)v;
      } else {
        double v = strtod(field, &endp);
        if (*endp) return -(1 + off);
        out[rows * p + j] = v;
      }
      off = e + 1;
    }
    ++rows;
  }
  return rows;
}
