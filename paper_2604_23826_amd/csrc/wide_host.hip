// Host side of the wide-table path: slot table, super-tile list, launch
// splitting and the choice between FP64 and split-precision matrix-core modes.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "runtime.hpp"
#include "wide.hpp"

namespace st {

// Split precision is used when asked for; by default (PREC_AUTO) only where
// the int8 kernel takes the layout (syrk_layout below), whose blocks are
// either on their sampled grid or recomputed in FP64.  The general split
// kernel keeps 2^-27 of each block's range per element, which one outlier
// widens for its whole block, so PREC_AUTO sends the other layouts to FP64.
static int wide_mode(const stats_ctx* h) {
  return h->precision == STATS_PREC_FP64 ? wide::MODE_FP64 : wide::MODE_SPLIT;
}

// Layout test for the int8 matrix-core kernel (wide_syrk.hip): F FP32
// columns (not flagged INTEGER) at byte offsets 0, 4, ..., 4 (F - 1) of one
// plane with 16-byte aligned rows, F a multiple of 4, and at most
// kSyrkMaxExtra other columns.  col_of receives the user column of each slot.
static bool syrk_layout(const stats_ctx* h, const void* const* planes, int* F_out, int* plane_out,
                        std::vector<int32_t>* col_of) {
  const int p = h->p;
  int best = -1, best_n = 0;
  for (int pl = 0; pl < h->n_planes; ++pl) {
    int n = 0;
    for (const auto& c : h->cols)
      if (c.plane == pl && c.dtype == STATS_F32 && !(c.flags & STATS_COL_INTEGER)) ++n;
    if (n > best_n) {
      best_n = n;
      best = pl;
    }
  }
  if (best < 0) return false;
  const int64_t stride = h->row_stride[best];
  if (stride % 16 != 0 || ((uintptr_t)planes[best] & 15u) != 0) return false;
  std::vector<int32_t> at(stride / 4, -1);
  for (int c = 0; c < p; ++c) {
    const stats_column& col = h->cols[c];
    if (col.plane == best && col.dtype == STATS_F32 && !(col.flags & STATS_COL_INTEGER) &&
        col.byte_offset % 4 == 0) {
      if (at[col.byte_offset / 4] >= 0) return false;
      at[col.byte_offset / 4] = c;
    }
  }
  int F = 0;
  while (F < (int)at.size() && at[F] >= 0) ++F;
  F &= ~3;
  if (F < 4 || p - F > wide::kSyrkMaxExtra) return false;
  col_of->assign(at.begin(), at.begin() + F);
  std::vector<uint8_t> used(p, 0);
  for (int j = 0; j < F; ++j) used[at[j]] = 1;
  for (int c = 0; c < p; ++c)
    if (!used[c]) col_of->push_back(c);
  if ((int)col_of->size() != p) return false;
  *F_out = F;
  *plane_out = best;
  return true;
}

static int64_t wide_block_rows(const stats_ctx* h, int64_t nrows) {
  int64_t R = h->block_rows;
  if (!R) {
    R = (nrows + 1023) / 1024;
    R = (R + 1023) / 1024 * 1024;
    R = std::max<int64_t>(1024, std::min<int64_t>(R, 32768));
  }
  return R;
}

static int accumulate_syrk(stats_ctx* h, const void* const* planes, int64_t nrows, int F, int xplane,
                           const std::vector<int32_t>& col_of) {
  const int p = h->p;
  const int ne = p - F;
  const int ng = (F + wide::kSyrkGroup - 1) / wide::kSyrkGroup;
  // the int32 digit sums are exact up to 32768 rows per block
  const int64_t R = std::min<int64_t>(wide_block_rows(h, nrows), 32768);
  const int64_t W = rec_words(p);
  // records of one launch stay below ~1 GB
  const int64_t max_blocks = std::max<int64_t>(1, ((int64_t)1 << 30) / (W * 8));
  // FP64 super-tiles of the blocks that are computed again (launch_wide_fixup)
  const int ST = p <= 32 ? 32 : 64;
  const int fng = (p + ST - 1) / ST;
  std::vector<int2> tiles;
  for (int A = 0; A < fng; ++A)
    for (int B = A; B < fng; ++B) tiles.push_back(make_int2(A, B));
  auto up = [](size_t n) { return (n + 255) / 256 * 256; };
  const size_t col_bytes = up(sizeof(int32_t) * (size_t)p);
  const size_t tile_bytes = up(sizeof(int2) * tiles.size());
  const size_t slot_bytes = up(sizeof(wide::SlotInfo) * (size_t)p);
  const int64_t nb_max = std::min<int64_t>(max_blocks, (nrows + R - 1) / R);
  const size_t ovf_bytes = up(sizeof(int) * (size_t)nb_max);
  const size_t sexp_bytes = up(sizeof(int) * (size_t)nb_max * (size_t)F);  // grid exponents
  int rc = ensure_dev(h, &h->aux3_dev, &h->aux3_cap, col_bytes + tile_bytes + slot_bytes + ovf_bytes + sexp_bytes);
  if (rc) return rc;
  char* aux = (char*)h->aux3_dev;
  int32_t* col_dev = (int32_t*)aux;
  int2* tiles_dev = (int2*)(aux + col_bytes);
  wide::SlotInfo* slots_dev = (wide::SlotInfo*)(aux + col_bytes + tile_bytes);
  int* ovf_dev = (int*)(aux + col_bytes + tile_bytes + slot_bytes);
  int* sexp_dev = (int*)(aux + col_bytes + tile_bytes + slot_bytes + ovf_bytes);
  hipError_t e = hipMemcpyAsync(col_dev, col_of.data(), sizeof(int32_t) * (size_t)p,
                                hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(tiles_dev, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "uploading column map");
  wide::SyrkArgs a;
  memset(&a, 0, sizeof a);
  a.F = F;
  a.ne = ne;
  a.p = p;
  a.col_of = col_dev;
  a.npairs = 0;
  for (int A = 0; A < ng; ++A)
    for (int B = A; B < ng; ++B) {
      a.pairs[a.npairs++] = make_int2(A, B);
      a.pairs[a.npairs++] = make_int2(A + 16, B);
    }
  a.xstride = h->row_stride[xplane];
  a.R = R;
  a.status = h->status_dev;
  a.ovf = ovf_dev;
  a.sexp = sexp_dev;
  std::vector<wide::SlotInfo> slots(p);
  int64_t done = 0;
  while (done < nrows) {
    const int64_t rows = std::min(nrows - done, max_blocks * R);
    const int64_t nblocks = (rows + R - 1) / R;
    a.xbase = (const char*)planes[xplane] + done * a.xstride;
    for (int x = 0; x < ne; ++x) {
      const stats_column& col = h->cols[col_of[F + x]];
      wide::SyrkExtra& ex = a.ex[x];
      ex.stride = h->row_stride[col.plane];
      ex.base = (const char*)planes[col.plane] + col.byte_offset + done * ex.stride;
      ex.kind = col.dtype;
      ex.chk = (col.dtype == STATS_F32 || col.dtype == STATS_F64) && (col.flags & STATS_COL_INTEGER);
      ex.isint = h->intf[col_of[F + x]];
    }
    for (int c = 0; c < p; ++c) {
      const stats_column& col = h->cols[c];
      wide::SlotInfo& sl = slots[c];
      sl.stride = h->row_stride[col.plane];
      sl.base = (const char*)planes[col.plane] + col.byte_offset + done * sl.stride;
      sl.kind = col.dtype;
      sl.chk = (col.dtype == STATS_F32 || col.dtype == STATS_F64) && (col.flags & STATS_COL_INTEGER);
      sl.isint = h->intf[c];
      sl.pad[0] = sl.pad[1] = 0;
    }
    // the previous launch has read the table before this copy is ordered after it
    e = hipMemcpyAsync(slots_dev, slots.data(), sizeof(wide::SlotInfo) * (size_t)p, hipMemcpyHostToDevice,
                       h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "uploading slot table");
    rc = ensure_dev(h, (void**)&h->rec, &h->rec_cap, (size_t)((nblocks * W + merge_slice_words(nblocks, p)) * 8));
    if (rc) return rc;
    a.rec = h->rec;
    a.nblocks = nblocks;
    a.nrows = rows;
    wide::Args f;
    f.slots = slots_dev;
    f.p = p;
    f.tiles = tiles_dev;
    f.ntiles = (int)tiles.size();
    f.nblocks = nblocks;
    f.nrows = rows;
    f.R = R;
    f.rec = h->rec;
    f.status = h->status_dev;
    {
      Timer t;
      t.begin(h, STATS_K_SYRK);
      launch_syrk_split(a, h->stream);
      t.end();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "matrix-core kernel launch");
    launch_wide_fixup(f, ST, ovf_dev, h->stream);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "FP64 block launch");
    {
      Timer t;
      t.begin(h, STATS_K_MERGE);
      launch_merge_records(h->rec, nblocks, p, h->intf_dev, h->state[h->cur], h->state[h->cur ^ 1],
                           h->status_dev, h->stream, h->rec + nblocks * W);
      t.end();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "merge kernel launch");
    h->cur ^= 1;
    done += rows;
  }
  return STATS_OK;
}

int accumulate_device_wide(stats_ctx* h, const void* const* planes, int64_t nrows) {
  const int p = h->p;
  if (wide_mode(h) == wide::MODE_SPLIT) {
    int F = 0, xplane = 0;
    std::vector<int32_t> col_of;
    if (syrk_layout(h, planes, &F, &xplane, &col_of))
      return accumulate_syrk(h, planes, nrows, F, xplane, col_of);
  }
  const int ST = p <= 32 ? 32 : 64;
  const int ng = (p + ST - 1) / ST;
  const int mode = h->precision == STATS_PREC_SPLIT ? wide::MODE_SPLIT : wide::MODE_FP64;
  std::vector<int2> tiles;
  for (int A = 0; A < ng; ++A)
    for (int B = A; B < ng; ++B) tiles.push_back(make_int2(A, B));
  const int64_t R = wide_block_rows(h, nrows);
  const int64_t W = rec_words(p);
  // records of one launch stay below ~256 MB
  const int64_t max_blocks = std::max<int64_t>(1, ((int64_t)256 << 20) / (W * 8));
  const size_t slot_bytes = sizeof(wide::SlotInfo) * (size_t)p;
  const size_t tile_bytes = sizeof(int2) * tiles.size();
  int rc = ensure_dev(h, &h->aux3_dev, &h->aux3_cap, tile_bytes + slot_bytes + 256);
  if (rc) return rc;
  int2* tiles_dev = (int2*)h->aux3_dev;
  wide::SlotInfo* slots_dev = (wide::SlotInfo*)((char*)h->aux3_dev + (tile_bytes + 255) / 256 * 256);
  hipError_t e = hipMemcpyAsync(tiles_dev, tiles.data(), tile_bytes, hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "uploading tile list");
  std::vector<wide::SlotInfo> slots(p);
  int64_t done = 0;
  while (done < nrows) {
    const int64_t rows = std::min(nrows - done, max_blocks * R);
    const int64_t nblocks = (rows + R - 1) / R;
    for (int c = 0; c < p; ++c) {
      const stats_column& col = h->cols[c];
      wide::SlotInfo& s = slots[c];
      s.stride = h->row_stride[col.plane];
      s.base = (const char*)planes[col.plane] + col.byte_offset + done * s.stride;
      s.kind = col.dtype;
      s.chk = (col.dtype == STATS_F32 || col.dtype == STATS_F64) && (col.flags & STATS_COL_INTEGER);
      s.isint = h->intf[c];
      s.pad[0] = s.pad[1] = 0;
    }
    // the previous launch has read the table before this copy is ordered after it
    e = hipMemcpyAsync(slots_dev, slots.data(), slot_bytes, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "uploading slot table");
    rc = ensure_dev(h, (void**)&h->rec, &h->rec_cap, (size_t)((nblocks * W + merge_slice_words(nblocks, p)) * 8));
    if (rc) return rc;
    wide::Args a;
    a.slots = slots_dev;
    a.p = p;
    a.tiles = tiles_dev;
    a.ntiles = (int)tiles.size();
    a.nblocks = nblocks;
    a.nrows = rows;
    a.R = R;
    a.rec = h->rec;
    a.status = h->status_dev;
    {
      Timer t;
      t.begin(h, STATS_K_SYRK);
      launch_wide(a, ST, mode, h->stream);
      t.end();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "wide kernel launch");
    {
      Timer t;
      t.begin(h, STATS_K_MERGE);
      launch_merge_records(h->rec, nblocks, p, h->intf_dev, h->state[h->cur], h->state[h->cur ^ 1],
                           h->status_dev, h->stream, h->rec + nblocks * W);
      t.end();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "merge kernel launch");
    h->cur ^= 1;
    done += rows;
  }
  return STATS_OK;
}

}  // namespace st
