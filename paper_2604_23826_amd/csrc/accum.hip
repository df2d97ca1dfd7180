// Host dispatch of the narrow-table reduction (p <= 16): picks the layout
// class, permutes columns into the kernel's slot order and tells the kernel
// where each slot's results go in the block record.
#include <cstring>

#include "accum_impl.hpp"

namespace st {

int64_t launch_accum_small_p(const AccumLaunch& L, hipStream_t s) {
  const int p = L.p;
  if (p < 1 || p > 16) return -1;
  const int64_t nblocks = (L.nrows + L.block_rows - 1) / L.block_rows;
  if (nblocks <= 0) return 0;
  // slot order: for dense int32/FP64 planes, int32 columns first
  int perm[16];
  int ni = -1;
  int kind = L.kind == 1 ? ACC_AOS : (L.kind == 2 ? ACC_PLANES : ACC_GENERIC);
  if (kind == ACC_PLANES) {
    bool ok = true;
    for (int c = 0; c < p; ++c) ok = ok && (L.dtype[c] == STATS_I32 || L.dtype[c] == STATS_F64);
    if (ok) {
      int k = 0;
      for (int c = 0; c < p; ++c)
        if (L.dtype[c] == STATS_I32) perm[k++] = c;
      ni = k;
      for (int c = 0; c < p; ++c)
        if (L.dtype[c] == STATS_F64) perm[k++] = c;
    } else {
      kind = ACC_GENERIC;
    }
  }
  if (kind != ACC_PLANES)
    for (int c = 0; c < p; ++c) perm[c] = c;
  acc::Args a;
  memset(&a, 0, sizeof a);
  for (int sl = 0; sl < 16; ++sl) {
    const int c = sl < p ? perm[sl] : 0;
    a.colbase[sl] = sl < p ? L.colbase[c] : nullptr;
    a.colstride[sl] = sl < p ? L.colstride[c] : 0;
    a.dtype[sl] = sl < p ? L.dtype[c] : STATS_F64;
    if (sl < p && ((L.intmask >> c) & 1u)) a.intmask |= 1u << sl;
    if (sl < p && ((L.chkmask >> c) & 1u)) a.chkmask |= 1u << sl;
    a.kdst[sl] = (int8_t)(sl < p ? c : 0);
  }
  for (int e = 0; e < p; ++e) a.dst[e] = (int16_t)perm[e];
  int e = p;
  for (int x = 0; x < p; ++x)
    for (int y = x; y < p; ++y) {
      const int i = perm[x] < perm[y] ? perm[x] : perm[y];
      const int j = perm[x] < perm[y] ? perm[y] : perm[x];
      a.dst[e++] = (int16_t)(p + tri(p, i, j));
    }
  a.nrows = L.nrows;
  a.R = L.block_rows;
  a.rec = L.rec;
  switch (p) {
#define ST_CASE(PP) \
  case PP: launch_accum_p<PP>(a, kind, ni, nblocks, s); break;
    ST_CASE(1) ST_CASE(2) ST_CASE(3) ST_CASE(4) ST_CASE(5) ST_CASE(6) ST_CASE(7) ST_CASE(8)
    ST_CASE(9) ST_CASE(10) ST_CASE(11) ST_CASE(12) ST_CASE(13) ST_CASE(14) ST_CASE(15) ST_CASE(16)
#undef ST_CASE
  }
  return nblocks;
}

}  // namespace st
