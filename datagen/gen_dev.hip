// Device (gfx950) side of the seeded synthetic-data generator.
//
// Writes the same bytes as the host generator (same Philox counters, same
// lookup tables, which the host builds with its libm and uploads here), so
// workloads far larger than host memory can be produced directly in HBM.
// Input generation only: nothing here computes a statistic.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "philox.h"

namespace {

struct Tables {
  double E[6][10], F[6][100], G[10], H[100], cot[10], I[10], J[100];
  int32_t K[10][100];
};

__constant__ Tables g_tab;

__device__ inline void table1_row(uint64_t seed, uint64_t grow, int64_t a, double* v) {
  int32_t B, C, D;
  dg_table1_draws(seed, grow, &B, &C, &D);
  const int b = B - 3, c = C - 1, d = D - 1;
  v[0] = (double)a;
  v[1] = B; v[2] = C; v[3] = D;
  v[4] = g_tab.E[b][c]; v[5] = g_tab.F[b][d]; v[6] = g_tab.G[c]; v[7] = g_tab.H[d];
  v[8] = g_tab.cot[c]; v[9] = g_tab.I[c]; v[10] = g_tab.J[d]; v[11] = (double)g_tab.K[c][d];
}

__global__ void k_table1_aos(uint64_t seed, int64_t row0, int64_t a0, int64_t n, int ncols,
                             double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    double v[12];
    table1_row(seed, (uint64_t)(row0 + r), a0 + r, v);
    double* o = out + r * ncols;
#pragma unroll
    for (int k = 0; k < 12; ++k)
      if (k < ncols) o[k] = v[k];
  }
}

struct Planes10 { void* p[10]; };

__global__ void k_table1_planar(uint64_t seed, int64_t row0, int64_t a0, int64_t n, Planes10 pl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    double v[12];
    table1_row(seed, (uint64_t)(row0 + r), a0 + r, v);
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      if (k == 8) ((double*)pl.p[k])[r] = v[k];
      else ((int32_t*)pl.p[k])[r] = (int32_t)v[k];
    }
  }
}

// Rows r in [0, n) of a wave; group g owns [off[g], off[g+1]) and its
// identifier starts at a0[g].  Randomness is keyed by the global row row0 + r.
__global__ void k_groups_aos(uint64_t seed, int64_t row0, const int64_t* __restrict__ off,
                             const int64_t* __restrict__ a0, int ngroups, int64_t n,
                             double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    int lo = 0, hi = ngroups - 1;  // last g with off[g] <= r
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= r) lo = mid; else hi = mid - 1;
    }
    const uint64_t g = (uint64_t)(row0 + r);
    double v[12];
    table1_row(seed, g, a0[lo] + (r - off[lo]), v);
    double* o = out + r * 32;
#pragma unroll
    for (int k = 0; k < 10; ++k) o[k] = v[k];
#pragma unroll
    for (int blk = 0; blk < 6; ++blk) {
      dg_u32x4 u = dg_extra_block(seed, g, blk);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int k = blk * 4 + w;
        if (k < 22) o[10 + k] = (double)dg_uniform_int(u.v[w], 0, 101);
      }
    }
  }
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return g < 1 ? 1 : (int)g;
}

}  // namespace

extern "C" {

int dgd_set_tables(const double* E60, const double* F600, const double* G10, const double* H100,
                   const double* cot10, const double* I10, const double* J100,
                   const int32_t* K1000) {
  Tables t;
  memcpy(t.E, E60, sizeof t.E);
  memcpy(t.F, F600, sizeof t.F);
  memcpy(t.G, G10, sizeof t.G);
  memcpy(t.H, H100, sizeof t.H);
  memcpy(t.cot, cot10, sizeof t.cot);
  memcpy(t.I, I10, sizeof t.I);
  memcpy(t.J, J100, sizeof t.J);
  memcpy(t.K, K1000, sizeof t.K);
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tab), &t, sizeof t) == hipSuccess ? 0 : -1;
}

int dgd_table1_aos(uint64_t seed, int64_t row0, int64_t a0, int64_t n, int32_t ncols, double* out,
                   void* stream) {
  if (n <= 0) return 0;
  if (ncols < 1 || ncols > 12 || !out) return -1;
  k_table1_aos<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(seed, row0, a0, n, ncols, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dgd_table1_planar(uint64_t seed, int64_t row0, int64_t a0, int64_t n, void* const* planes,
                      void* stream) {
  if (n <= 0) return 0;
  Planes10 pl;
  for (int k = 0; k < 10; ++k) {
    if (!planes[k]) return -1;
    pl.p[k] = planes[k];
  }
  k_table1_planar<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(seed, row0, a0, n, pl);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dgd_groups_aos(uint64_t seed, int64_t row0, const int64_t* off_dev, const int64_t* a0_dev,
                   int32_t ngroups, int64_t n, double* out, void* stream) {
  if (n <= 0) return 0;
  if (ngroups < 1 || !off_dev || !a0_dev || !out) return -1;
  k_groups_aos<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(seed, row0, off_dev, a0_dev, ngroups,
                                                             n, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
