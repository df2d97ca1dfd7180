/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from the
 * published round definition: two 32x32->64 multiplies per round with the
 * constants 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 /
 * 0xBB67AE85 between rounds, 10 rounds.
 *
 * Seeded input generation only: this header belongs to the data generator
 * and is shared by its host (C) and device (HIP) builds so both produce the
 * same bytes.  It contains none of the statistics being computed. */
#ifndef DATAGEN_PHILOX_H
#define DATAGEN_PHILOX_H
#include <stdint.h>

#if defined(__HIPCC__)
#define DG_HD __host__ __device__ inline
#else
#define DG_HD static inline
#endif

typedef struct { uint32_t v[4]; } dg_u32x4;

DG_HD dg_u32x4 dg_philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  dg_u32x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

/* Map a uniform 32-bit word onto {lo, ..., lo+m-1} by multiply-shift
 * (no rejection; the relative bias is at most m / 2^32). */
DG_HD int32_t dg_uniform_int(uint32_t u, int32_t lo, uint32_t m) {
  return lo + (int32_t)(((uint64_t)u * (uint64_t)m) >> 32);
}

/* Stream identifiers (third counter word) so workloads never share draws. */
enum { DG_STREAM_TABLE1 = 0x7AB1E001u, DG_STREAM_EXTRA = 0x7AB1E002u,
       DG_STREAM_GROUPS = 0x7AB1E003u, DG_STREAM_FUZZ = 0x7AB1E004u };

/* Table-1 draws for global row r: B ~ U{3..8}, C ~ U{1..10}, D ~ U{1..100},
 * drawn in that order from one Philox block keyed by the seed. */
DG_HD void dg_table1_draws(uint64_t seed, uint64_t row, int32_t* B, int32_t* C, int32_t* D) {
  dg_u32x4 u = dg_philox4x32_10((uint32_t)row, (uint32_t)(row >> 32), DG_STREAM_TABLE1, 0u,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  *B = dg_uniform_int(u.v[0], 3, 6);
  *C = dg_uniform_int(u.v[1], 1, 10);
  *D = dg_uniform_int(u.v[2], 1, 100);
}

/* Extra i.i.d. U{0..100} integers for row r: block b of 4 words comes from
 * counter (r, EXTRA, b); extra column k uses word k%4 of block k/4. */
DG_HD dg_u32x4 dg_extra_block(uint64_t seed, uint64_t row, int b) {
  return dg_philox4x32_10((uint32_t)row, (uint32_t)(row >> 32), DG_STREAM_EXTRA, (uint32_t)b,
                          (uint32_t)seed, (uint32_t)(seed >> 32));
}

#endif
