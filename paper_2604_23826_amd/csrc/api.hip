// C ABI of libstats.so: handles, argument checks, streams, staging and the
// order of kernel launches.  Every arithmetic step runs in the kernels of
// accum.hip / merge.hip / finalize.hip (and the wide, segmented and text
// kernels); this file only moves bytes and sequences work.
#include <algorithm>
#include <cerrno>
#include <thread>

#include <fcntl.h>
#include <unistd.h>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "runtime.hpp"
#include "wide.hpp"

using namespace st;

namespace st {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(stats_ctx* h, hipError_t e, const char* what) {
  if (h) h->poisoned = true;
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return STATS_E_HIP;
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  ok = hipSetDevice(dev) == hipSuccess;
}
DeviceGuard::~DeviceGuard() {
  if (prev >= 0) (void)hipSetDevice(prev);
}

int elem_size(int dtype) {
  switch (dtype) {
    case STATS_I32: return 4;
    case STATS_F32: return 4;
    case STATS_I64: return 8;
    case STATS_F64: return 8;
    default: return 0;
  }
}

bool is_int_col(const stats_column& c) {
  return c.dtype == STATS_I32 || c.dtype == STATS_I64 || (c.flags & STATS_COL_INTEGER);
}

// Device allocation that reports STATS_E_NOMEM; grows *cap_bytes if needed.
int ensure_dev(stats_ctx* h, void** ptr, size_t* cap, size_t need) {
  if (*cap >= need && *ptr) return STATS_OK;
  if (*ptr) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    (void)hipFree(*ptr);
    *ptr = nullptr;
    *cap = 0;
  }
  if (std::getenv("STATS_FAIL_ALLOC")) return fail(STATS_E_NOMEM, "allocation refused (STATS_FAIL_ALLOC)");
  hipError_t e = hipMalloc(ptr, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(STATS_E_NOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed");
  }
  *cap = need;
  return STATS_OK;
}

void Timer::begin(stats_ctx* h, int which, hipStream_t s) {
  if (!(h->flags & STATS_CFG_TIMING)) return;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  s_ = s ? s : h->stream;
  (void)hipEventRecord(a, s_);
  h_ = h;
  which_ = which;
  a_ = a;
  b_ = b;
}

void Timer::end() {
  if (!h_) return;
  (void)hipEventRecord(b_, s_);
  h_->pending[which_].push_back({a_, b_});
  h_ = nullptr;
}

void collect_timings(stats_ctx* h) {
  for (int k = 0; k < STATS_K_COUNT; ++k) {
    for (auto& pr : h->pending[k]) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        h->kt_ms[k] += ms;
        h->kt_n[k] += 1;
      }
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    h->pending[k].clear();
  }
}

// Zero status bits; the smallest-parse-error offset starts at the maximum.
hipError_t clear_status(stats_ctx* h) {
  static const DevStatus init = {0u, 0u, ~0ull};
  return hipMemcpyAsync(h->status_dev, &init, sizeof init, hipMemcpyHostToDevice, h->stream);
}

// The error recorded in a status word read back from the device, if any.
static int status_error(const DevStatus& s) {
  if (s.bits & ST_PARSE) {
    char buf[128];
    snprintf(buf, sizeof buf, "malformed text field at byte offset %llu",
             (unsigned long long)s.parse_off);
    return fail(STATS_E_PARSE, buf);
  }
  if (s.bits & ST_INEXACT)
    return fail(STATS_E_INEXACT,
                "an integer column left the exact range (non-integer value, |x - shift|^2 sum "
                ">= 2^53 in a block, or |value| >= 2^40)");
  return STATS_OK;
}

int check_status(stats_ctx* h) {
  DevStatus s;
  hipError_t e = hipMemcpy(&s, h->status_dev, sizeof s, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "hipMemcpy(status)");
  return status_error(s);
}

int sync_handle(stats_ctx* h) {
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
  if (h->copy_stream) {
    e = hipStreamSynchronize(h->copy_stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize(copy)");
  }
  collect_timings(h);
  return check_status(h);
}

}  // namespace st

// ---------------------------------------------------------------------------
// open / close

static int validate_cfg(const stats_config* cfg) {
  if (!cfg) return fail(STATS_E_ARG, "cfg is NULL");
  if (cfg->p < 1 || cfg->p > STATS_MAX_P) return fail(STATS_E_ARG, "p must be in 1..1024");
  if (!cfg->cols) return fail(STATS_E_ARG, "cols is NULL");
  if (cfg->n_planes < 1 || cfg->n_planes > STATS_MAX_PLANES)
    return fail(STATS_E_ARG, "n_planes must be in 1..32");
  for (int k = 0; k < cfg->n_planes; ++k)
    if (cfg->row_stride[k] <= 0) return fail(STATS_E_ARG, "row_stride must be positive");
  for (int c = 0; c < cfg->p; ++c) {
    const stats_column& col = cfg->cols[c];
    const int es = elem_size(col.dtype);
    if (!es) return fail(STATS_E_ARG, "column " + std::to_string(c) + ": unknown dtype");
    if (col.plane < 0 || col.plane >= cfg->n_planes)
      return fail(STATS_E_ARG, "column " + std::to_string(c) + ": plane out of range");
    if (col.byte_offset < 0 || col.byte_offset + es > cfg->row_stride[col.plane])
      return fail(STATS_E_ARG, "column " + std::to_string(c) + ": element outside the row stride");
    if (col.byte_offset % es != 0)
      return fail(STATS_E_ARG, "column " + std::to_string(c) + ": misaligned byte_offset");
    if (col.flags & ~(uint32_t)(STATS_COL_INTEGER | STATS_COL_IDENTIFIER))
      return fail(STATS_E_ARG, "column " + std::to_string(c) + ": unknown flags");
  }
  if (cfg->precision < STATS_PREC_FP64 || cfg->precision > STATS_PREC_AUTO)
    return fail(STATS_E_ARG, "unknown precision");
  if (cfg->block_rows < 0 || (cfg->block_rows % 1024) != 0)
    return fail(STATS_E_ARG, "block_rows must be 0 or a positive multiple of 1024");
  if (cfg->block_rows > ((int64_t)1 << 24)) return fail(STATS_E_ARG, "block_rows too large");
  if (cfg->staging_rows < 0) return fail(STATS_E_ARG, "staging_rows must be >= 0");
  if (cfg->flags & ~(uint32_t)(STATS_CFG_TIMING | STATS_CFG_PAIRWISE)) return fail(STATS_E_ARG, "unknown flags");
  if (cfg->flags & STATS_CFG_PAIRWISE) {
    if (cfg->p > 16) return fail(STATS_E_ARG, "pairwise (missing-value) statistics support p <= 16");
    for (int c = 0; c < cfg->p; ++c)
      if (cfg->cols[c].dtype != STATS_F32 && cfg->cols[c].dtype != STATS_F64)
        return fail(STATS_E_ARG, "pairwise statistics need FP32 or FP64 columns (NaN = missing)");
  }
  return STATS_OK;
}

namespace st {

// Words of one handle state: the complete-data layout, or the per-pair
// statistics of a pairwise (missing-value) handle.
int64_t state_words(const stats_ctx* h) {
  if (h->flags & STATS_CFG_PAIRWISE) return pairwise_state_words(h->p);
  return Layout::make(h->p).words;
}

int open_handle(const stats_config* cfg, int ngroups, stats_ctx** out) {
  if (!out) return fail(STATS_E_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate_cfg(cfg);
  if (rc) return rc;
  if (ngroups > 0 && (cfg->flags & STATS_CFG_PAIRWISE))
    return fail(STATS_E_ARG, "pairwise statistics are not available for groups handles");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(STATS_E_HIP, "no HIP device available");
  if (cfg->device < 0 || cfg->device >= ndev) return fail(STATS_E_ARG, "device out of range");
  DeviceGuard g(cfg->device);
  if (!g.ok) return fail(STATS_E_HIP, "hipSetDevice failed");
  stats_ctx* h = new (std::nothrow) stats_ctx();
  if (!h) return fail(STATS_E_NOMEM, "host allocation failed");
  h->device = cfg->device;
  h->p = cfg->p;
  h->cols.assign(cfg->cols, cfg->cols + cfg->p);
  h->n_planes = cfg->n_planes;
  for (int k = 0; k < STATS_MAX_PLANES; ++k) h->row_stride[k] = k < cfg->n_planes ? cfg->row_stride[k] : 0;
  h->precision = cfg->precision;
  h->staging_rows = cfg->staging_rows ? cfg->staging_rows : ((int64_t)1 << 28);
  h->block_rows = cfg->block_rows;
  h->flags = cfg->flags;
  h->ngroups = ngroups;
  h->intf.resize(h->p);
  for (int c = 0; c < h->p; ++c) h->intf[c] = is_int_col(h->cols[c]) ? 1 : 0;
  if (cfg->stream) {
    h->stream = (hipStream_t)cfg->stream;
    h->own_stream = false;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete h;
      return hip_fail(nullptr, e, "hipStreamCreate");
    }
    h->own_stream = true;
  }
  const int64_t words = state_words(h);
  const int64_t nstates = ngroups > 0 ? ngroups : 1;
  size_t cap;
  for (int k = 0; k < 2; ++k) {
    cap = 0;
    rc = ensure_dev(h, (void**)&h->state[k], &cap, (size_t)(words * 8 * nstates));
    if (rc) {
      stats_close(h);
      return rc;
    }
  }
  cap = 0;
  rc = ensure_dev(h, (void**)&h->intf_dev, &cap, (size_t)h->p);
  if (!rc) {
    cap = 0;
    rc = ensure_dev(h, (void**)&h->status_dev, &cap, sizeof(DevStatus));
  }
  if (rc) {
    stats_close(h);
    return rc;
  }
  hipError_t e = hipMemcpyAsync(h->intf_dev, h->intf.data(), (size_t)h->p, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->state[0], 0, (size_t)(words * 8 * nstates), h->stream);
  if (e == hipSuccess) e = clear_status(h);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    int r = hip_fail(h, e, "initialising handle state");
    stats_close(h);
    return r;
  }
  h->cur = 0;
  *out = h;
  return STATS_OK;
}

}  // namespace st

extern "C" int stats_open(const stats_config* cfg, stats_ctx** out) {
  return open_handle(cfg, 0, out);
}

extern "C" int stats_open_groups(const stats_config* cfg, int32_t ngroups, stats_ctx** out) {
  if (ngroups < 1 || ngroups > (1 << 24)) {
    if (out) *out = nullptr;
    return fail(STATS_E_ARG, "ngroups must be in 1..2^24");
  }
  return open_handle(cfg, ngroups, out);
}

extern "C" void stats_close(stats_ctx* h) {
  if (!h) return;
  DeviceGuard g(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->copy_stream) (void)hipStreamSynchronize(h->copy_stream);
  collect_timings(h);
  void* bufs[] = {h->state[0], h->state[1], h->intf_dev, h->status_dev, h->rec,
                  h->fin_out, h->fin_scratch, h->sel_dev, h->raw_out, h->stage_dev[0],
                  h->stage_dev[1], h->aux_dev, h->aux2_dev, h->aux3_dev, h->seg_part,
                  h->conv_dev};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (int k = 0; k < 2; ++k) {
    if (h->stage_host[k]) (void)hipHostFree(h->stage_host[k]);
    if (h->ev_copy[k]) (void)hipEventDestroy(h->ev_copy[k]);
    if (h->ev_free[k]) (void)hipEventDestroy(h->ev_free[k]);
  }
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->copy_stream) (void)hipStreamDestroy(h->copy_stream);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

extern "C" const char* stats_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// accumulate

namespace st {

// Chooses the kernel layout class for the given plane pointers.
static int layout_kind(const stats_ctx* h, const void* const* planes) {
  const int p = h->p;
  // AoS FP64: one plane, all columns FP64 at consecutive offsets, 16-byte rows.
  bool aos = true;
  for (int c = 0; c < p && aos; ++c) {
    const stats_column& col = h->cols[c];
    aos = col.dtype == STATS_F64 && col.plane == h->cols[0].plane &&
          col.byte_offset == h->cols[0].byte_offset + 8 * c;
  }
  if (aos) {
    const int pl = h->cols[0].plane;
    const uintptr_t base = (uintptr_t)planes[pl] + (uintptr_t)h->cols[0].byte_offset;
    // the staged-tile kernel expects the row stride 8p rounded up to 16 bytes
    if (base % 16 == 0 && h->row_stride[pl] == (8 * p + 15) / 16 * 16) return 1;
  }
  // Dense planes: each column alone in its plane with stride = element size.
  bool dense = true;
  std::vector<int> seen(h->n_planes, 0);
  for (int c = 0; c < p && dense; ++c) {
    const stats_column& col = h->cols[c];
    dense = col.byte_offset == 0 && h->row_stride[col.plane] == elem_size(col.dtype) &&
            !seen[col.plane] && ((uintptr_t)planes[col.plane] % 16 == 0);
    if (dense) seen[col.plane] = 1;
  }
  return dense ? 2 : 0;
}

static int64_t auto_block_rows(int64_t nrows) {
  // target ~2048 blocks per launch, between 4096 rows and 2^17 rows per block;
  // below 4096 rows per block the per-block reduction and pipeline start
  // dominate (10^6 FP64 rows of 80 bytes: 22 us with 4096-row blocks, 31 us
  // with 1024)
  int64_t R = (nrows + 2047) / 2048;
  R = ((R + 1023) / 1024) * 1024;
  return std::max<int64_t>(4096, std::min<int64_t>(R, (int64_t)1 << 17));
}

// FP64 row-major records of RS bytes with every column at byte offset 8c,
// 16-byte aligned: the FP64 matrix-core kernel k_seg_aos64<RS> (one 16x16x4
// product per 4 rows and 16 columns).  Used for RS = 128 with 11 <= p <= 16,
// where per-lane accumulators (136 products) would leave one wave per SIMD,
// and for RS = 256 with 17 <= p <= 32 in FP64 mode.
static bool aos_rows_layout(const stats_ctx* h, const void* const* planes, int RS) {
  const int pl = h->cols[0].plane;
  if (h->row_stride[pl] != RS || ((uintptr_t)planes[pl] & 15u) != 0) return false;
  for (int c = 0; c < h->p; ++c) {
    const stats_column& col = h->cols[c];
    if (col.plane != pl || col.dtype != STATS_F64 || col.byte_offset != 8 * c) return false;
  }
  return true;
}

static int accumulate_aos_rows(stats_ctx* h, const void* const* planes, int64_t nrows, int64_t R, int RS) {
  const int p = h->p;
  const int pl = h->cols[0].plane;
  // slot table and queue word in aux3 (shared with the wide path,
  // accumulate_device_wide; one of them runs per launch, stream-ordered)
  const size_t slot_bytes = (sizeof(wide::SlotInfo) * (size_t)p + 255) / 256 * 256;
  int rc = ensure_dev(h, &h->aux3_dev, &h->aux3_cap, slot_bytes + 256);
  if (rc) return rc;
  wide::SlotInfo* slots_dev = (wide::SlotInfo*)h->aux3_dev;
  unsigned long long* counter = (unsigned long long*)((char*)h->aux3_dev + slot_bytes);
  int ncu = 256;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device);
  const int64_t W = rec_words(p);
  // at most 2^28 rows and 16384 blocks per launch (the depth of the merge
  // tree over one launch's blocks stays at most 14)
  const int64_t max_rows = std::max<int64_t>(R, std::min<int64_t>(16384 * R, ((int64_t)1 << 28) / R * R));
  std::vector<wide::SlotInfo> slots(p);
  int64_t done = 0;
  while (done < nrows) {
    const int64_t rows = std::min(nrows - done, max_rows);
    const int64_t nblocks = (rows + R - 1) / R;
    rc = ensure_dev(h, (void**)&h->rec, &h->rec_cap, (size_t)((nblocks * W + merge_slice_words(nblocks, p)) * 8));
    if (rc) return rc;
    for (int c = 0; c < p; ++c) {
      const stats_column& col = h->cols[c];
      wide::SlotInfo& sl = slots[c];
      sl.stride = RS;
      sl.base = (const char*)planes[pl] + 8 * c + done * RS;
      sl.kind = col.dtype;
      sl.chk = (col.flags & STATS_COL_INTEGER) ? 1 : 0;
      sl.isint = h->intf[c];
      sl.pad[0] = sl.pad[1] = 0;
    }
    // ordered after the previous launch, which has read the table
    hipError_t e = hipMemcpyAsync(slots_dev, slots.data(), sizeof(wide::SlotInfo) * (size_t)p,
                                  hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "uploading slot table");
    wide::Args a;
    memset(&a, 0, sizeof a);
    a.slots = slots_dev;
    a.p = p;
    a.nblocks = nblocks;
    a.nrows = rows;
    a.R = R;
    a.rec = h->rec;
    a.status = h->status_dev;
    wide::SegArgs g{nullptr, nullptr, counter, R, rows};
    {
      Timer t;
      t.begin(h, STATS_K_ACCUM);
      launch_seg_aos64(a, g, (int)std::min<int64_t>(nblocks, (int64_t)ncu * 8), h->stream, RS);
      t.end();
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "accumulate kernel launch");
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

// Launch description of the per-lane narrow kernels for the given planes
// (row 0 at the plane bases; nrows, block_rows and rec left for the caller).
AccumLaunch accum_launch_of(const stats_ctx* h, const void* const* planes) {
  AccumLaunch a;
  memset(&a, 0, sizeof a);
  a.p = h->p;
  a.kind = layout_kind(h, planes);
  for (int c = 0; c < h->p; ++c) {
    const stats_column& col = h->cols[c];
    a.colbase[c] = (const char*)planes[col.plane] + col.byte_offset;
    a.colstride[c] = h->row_stride[col.plane];
    a.dtype[c] = col.dtype;
    if (h->intf[c]) a.intmask |= 1u << c;
    if ((col.dtype == STATS_F32 || col.dtype == STATS_F64) && (col.flags & STATS_COL_INTEGER))
      a.chkmask |= 1u << c;
  }
  return a;
}

int64_t block_rows_for(const stats_ctx* h, int64_t nrows) {
  return h->block_rows ? h->block_rows : auto_block_rows(nrows);
}

// Reduce nrows device-resident rows (plane bases already offset to the first
// row) into the handle state.  Small p only (p <= 16).
int accumulate_device_small(stats_ctx* h, const void* const* planes, int64_t nrows) {
  const int p = h->p;
  const int64_t R = block_rows_for(h, nrows);
  if (p >= 11 && aos_rows_layout(h, planes, 128)) return accumulate_aos_rows(h, planes, nrows, R, 128);
  const AccumLaunch a = accum_launch_of(h, planes);
  const int64_t W = rec_words(p);
  // at most 2^28 rows (and 16384 blocks) per launch: plane offsets stay 32-bit
  const int64_t max_rows = std::max<int64_t>(R, std::min<int64_t>(16384 * R, ((int64_t)1 << 28) / R * R));
  int64_t done = 0;
  while (done < nrows) {
    const int64_t rows = std::min(nrows - done, max_rows);
    const int64_t nblocks = (rows + R - 1) / R;
    int rc = ensure_dev(h, (void**)&h->rec, &h->rec_cap, (size_t)((nblocks * W + merge_slice_words(nblocks, p)) * 8));
    if (rc) return rc;
    AccumLaunch b = a;
    for (int c = 0; c < p; ++c) b.colbase[c] = a.colbase[c] + done * a.colstride[c];
    b.nrows = rows;
    b.block_rows = R;
    b.rec = h->rec;
    {
      Timer t;
      t.begin(h, STATS_K_ACCUM);
      launch_accum_small_p(b, h->stream);
      t.end();
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "accumulate kernel launch");
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

int accumulate_device(stats_ctx* h, const void* const* planes, int64_t nrows) {
  if (h->flags & STATS_CFG_PAIRWISE) return accumulate_pairwise(h, planes, nrows);
  if (h->p <= 16) return accumulate_device_small(h, planes, nrows);
  if (h->p <= 32 && h->precision != STATS_PREC_SPLIT && aos_rows_layout(h, planes, 256))
    return accumulate_aos_rows(h, planes, nrows, h->block_rows ? h->block_rows : auto_block_rows(nrows), 256);
  return accumulate_device_wide(h, planes, nrows);
}

// Host input: chunks of staging_rows rows go through two device slots; the
// copy of chunk k+1 (copy stream) overlaps the reduction of chunk k.
// Pageable input is first copied into two pinned host slots by host threads.
// Fills `bytes` bytes at dst from the file at byte offset off with positioned
// reads split over up to kReaders host threads.  false on a read error or end
// of file.
static constexpr int kReaders = 8;
static bool read_file_range(int fd, char* dst, size_t bytes, int64_t off) {
  const size_t piece = std::max<size_t>((size_t)1 << 22, (bytes + kReaders - 1) / kReaders);
  const int n = (int)std::min<size_t>(kReaders, (bytes + piece - 1) / piece);
  std::vector<char> ok(n, 0);
  auto work = [&](int k) {
    size_t a = (size_t)k * piece, b = std::min(bytes, a + piece);
    while (a < b) {
      const ssize_t r = pread(fd, dst + a, b - a, (off_t)(off + (int64_t)a));
      if (r <= 0) {
        if (r < 0 && errno == EINTR) continue;
        return;
      }
      a += (size_t)r;
    }
    ok[k] = 1;
  };
  std::vector<std::thread> th;
  for (int k = 1; k < n; ++k) th.emplace_back(work, k);
  if (n > 0) work(0);
  for (auto& t : th) t.join();
  for (int k = 0; k < n; ++k)
    if (!ok[k]) return false;
  return true;
}

// Copies `bytes` from pageable src to the pinned staging slot dst on up to
// kReaders host threads (one contiguous piece each).
static void copy_to_slot(char* dst, const char* src, size_t bytes) {
  const size_t piece = std::max<size_t>((size_t)1 << 24, (bytes + kReaders - 1) / kReaders);
  const int n = (int)std::min<size_t>(kReaders, (bytes + piece - 1) / piece);
  auto work = [&](int k) {
    const size_t a = (size_t)k * piece, e = std::min(bytes, a + piece);
    if (e > a) memcpy(dst + a, src + a, e - a);
  };
  std::vector<std::thread> th;
  for (int k = 1; k < n; ++k) th.emplace_back(work, k);
  if (n > 0) work(0);
  for (auto& t : th) t.join();
}

int accumulate_host(stats_ctx* h, const void* const* planes, int64_t nrows, bool pinned) {
  return accumulate_host_src(h, planes, -1, 0, nrows, pinned);
}

// Host input from memory planes (fd < 0) or from one file of row-major
// records (fd >= 0, one plane, record r at byte file_off + r * row_stride[0]).
int accumulate_host_src(stats_ctx* h, const void* const* planes, int fd, int64_t file_off, int64_t nrows,
                        bool pinned) {
  const int np = h->n_planes;
  const int64_t S = std::min<int64_t>(h->staging_rows, std::max<int64_t>(nrows, 1));
  if (!h->copy_stream) {
    hipError_t e = hipStreamCreateWithFlags(&h->copy_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamCreate(copy)");
    for (int k = 0; k < 2; ++k) {
      (void)hipEventCreateWithFlags(&h->ev_copy[k], hipEventDisableTiming);
      (void)hipEventCreateWithFlags(&h->ev_free[k], hipEventDisableTiming);
      (void)hipEventRecord(h->ev_free[k], h->stream);
    }
  }
  size_t slot_bytes = 0;
  std::vector<size_t> plane_off(np);
  for (int k = 0; k < np; ++k) {
    plane_off[k] = slot_bytes;
    slot_bytes += (size_t)(((S * h->row_stride[k]) + 255) / 256 * 256);
  }
  for (int k = 0; k < 2; ++k) {
    int rc = ensure_dev(h, &h->stage_dev[k], &h->stage_cap[k], slot_bytes);
    if (rc) return rc;
    if (!pinned && h->stage_host_cap[k] < slot_bytes) {
      if (h->stage_host[k]) {
        (void)hipEventSynchronize(h->ev_copy[k]);
        (void)hipHostFree(h->stage_host[k]);
        h->stage_host[k] = nullptr;
      }
      hipError_t e = hipHostMalloc(&h->stage_host[k], slot_bytes, hipHostMallocDefault);
      if (e != hipSuccess) {
        h->stage_host[k] = nullptr;
        h->stage_host_cap[k] = 0;
        return fail(STATS_E_NOMEM, "hipHostMalloc of the staging slot failed");
      }
      h->stage_host_cap[k] = slot_bytes;
    }
  }
  int64_t done = 0;
  while (done < nrows) {
    const int k = h->slot;
    const int64_t rows = std::min(S, nrows - done);
    // the slot is free once the reduction that last read it has finished
    hipError_t e = hipStreamWaitEvent(h->copy_stream, h->ev_free[k], 0);
    const void* dplanes[STATS_MAX_PLANES];
    for (int q = 0; q < np && e == hipSuccess; ++q) {
      const size_t bytes = (size_t)(rows * h->row_stride[q]);
      char* dst = (char*)h->stage_dev[k] + plane_off[q];
      const char* src = fd >= 0 ? nullptr : (const char*)planes[q] + done * h->row_stride[q];
      if (!pinned) {
        e = hipEventSynchronize(h->ev_copy[k]);  // previous DMA out of the host slot done
        if (e != hipSuccess) break;
        char* hs = (char*)h->stage_host[k] + plane_off[q];
        if (fd >= 0) {
          // the read of this chunk overlaps the copy and reduction of the last
          if (!read_file_range(fd, hs, bytes, file_off + done * h->row_stride[q]))
            return fail(STATS_E_IO, "reading rows " + std::to_string(done) + " .. " +
                                        std::to_string(done + rows) + " of the file failed");
        } else {
          copy_to_slot(hs, src, bytes);
        }
        src = hs;
      }
      Timer t;
      t.begin(h, STATS_K_COPY, h->copy_stream);
      e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->copy_stream);
      t.end();
      dplanes[q] = dst;
    }
    if (e == hipSuccess) e = hipEventRecord(h->ev_copy[k], h->copy_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->ev_copy[k], 0);
    if (e != hipSuccess) return hip_fail(h, e, "staging copy");
    int rc = accumulate_device(h, dplanes, rows);
    if (rc) return rc;
    e = hipEventRecord(h->ev_free[k], h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipEventRecord");
    h->slot ^= 1;
    done += rows;
  }
  if (!pinned) {
    // pageable input may be reused once we return: wait for the last DMA
    for (int k = 0; k < 2; ++k) {
      hipError_t e = hipEventSynchronize(h->ev_copy[k]);
      if (e != hipSuccess) return hip_fail(h, e, "hipEventSynchronize");
    }
  }
  return STATS_OK;
}

}  // namespace st

extern "C" int stats_accumulate(stats_ctx* h, const void* const* planes, int64_t nrows,
                                int32_t mem_kind) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups) return fail(STATS_E_STATE, "groups handle: use stats_accumulate_segmented");
  if (nrows < 0) return fail(STATS_E_ARG, "nrows < 0");
  if (nrows == 0) return STATS_OK;
  if (!planes) return fail(STATS_E_ARG, "planes is NULL");
  for (int k = 0; k < h->n_planes; ++k) {
    bool used = false;
    for (const auto& c : h->cols) used |= c.plane == k;
    if (used && !planes[k]) return fail(STATS_E_ARG, "plane " + std::to_string(k) + " is NULL");
  }
  DeviceGuard g(h->device);
  if (!g.ok) return fail(STATS_E_HIP, "hipSetDevice failed");
  switch (mem_kind) {
    case STATS_MEM_DEVICE: {
      for (int k = 0; k < h->n_planes; ++k)
        if (planes[k] && ((uintptr_t)planes[k] % 16) != 0)
          return fail(STATS_E_ARG, "device planes must be 16-byte aligned");
      return accumulate_device(h, planes, nrows);
    }
    case STATS_MEM_HOST_PINNED: return accumulate_host(h, planes, nrows, true);
    case STATS_MEM_HOST: return accumulate_host(h, planes, nrows, false);
    default: return fail(STATS_E_ARG, "unknown mem_kind");
  }
}

extern "C" int stats_accumulate_file(stats_ctx* h, const char* path, int64_t offset, int64_t nrows) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups) return fail(STATS_E_STATE, "groups handle: use stats_accumulate_segmented");
  if (!path) return fail(STATS_E_ARG, "path is NULL");
  if (h->n_planes != 1) return fail(STATS_E_ARG, "file input needs a handle with one plane of records");
  if (nrows < 0 || offset < 0) return fail(STATS_E_ARG, "nrows or offset < 0");
  if (nrows == 0) return STATS_OK;
  const int fd = open(path, O_RDONLY | O_CLOEXEC);
  if (fd < 0) return fail(STATS_E_IO, std::string("cannot open ") + path + ": " + strerror(errno));
  const off_t end = lseek(fd, 0, SEEK_END);
  if (end < 0 || (int64_t)end < offset + nrows * h->row_stride[0]) {
    close(fd);
    return fail(STATS_E_IO, std::string(path) + " holds fewer than the requested rows");
  }
  int rc;
  {
    DeviceGuard g(h->device);
    rc = g.ok ? accumulate_host_src(h, nullptr, fd, offset, nrows, false)
              : fail(STATS_E_HIP, "hipSetDevice failed");
  }
  close(fd);
  return rc;
}

extern "C" int stats_reset(stats_ctx* h) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  DeviceGuard g(h->device);
  const size_t bytes = (size_t)state_words(h) * 8 * (size_t)(h->ngroups > 0 ? h->ngroups : 1);
  hipError_t e = hipMemsetAsync(h->state[h->cur], 0, bytes, h->stream);
  if (e == hipSuccess) e = clear_status(h);
  if (e != hipSuccess) return hip_fail(h, e, "stats_reset");
  h->text_offset = 0;
  return STATS_OK;
}

extern "C" int stats_sync(stats_ctx* h) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  DeviceGuard g(h->device);
  return sync_handle(h);
}

// ---------------------------------------------------------------------------
// merge

extern "C" int stats_merge(stats_ctx* dst, const stats_ctx* src) {
  if (!dst || !src) return fail(STATS_E_ARG, "handle is NULL");
  if (dst == src) return fail(STATS_E_ARG, "dst and src are the same handle");
  if (dst->poisoned || src->poisoned) return fail(STATS_E_STATE, "handle is poisoned");
  if (dst->ngroups || src->ngroups) return fail(STATS_E_STATE, "merge of groups handles");
  if (dst->p != src->p) return fail(STATS_E_MISMATCH, "different column counts");
  for (int c = 0; c < dst->p; ++c)
    if (dst->intf[c] != src->intf[c]) return fail(STATS_E_MISMATCH, "different column kinds");
  const bool pairwise = (dst->flags & STATS_CFG_PAIRWISE) != 0;
  if (pairwise != ((src->flags & STATS_CFG_PAIRWISE) != 0))
    return fail(STATS_E_MISMATCH, "pairwise and complete-data handles");
  stats_ctx* s = const_cast<stats_ctx*>(src);
  DeviceGuard g(dst->device);
  const int64_t words = state_words(dst);
  const size_t bytes = (size_t)words * 8;
  const uint64_t* src_state = s->state[s->cur];
  const DevStatus* src_status = s->status_dev;
  hipError_t e;
  if (s->device != dst->device) {
    // bring the source state and status word over through the host
    std::vector<uint64_t> tmp(words + sizeof(DevStatus) / 8);
    {
      DeviceGuard gs(s->device);
      e = hipStreamSynchronize(s->stream);
      if (e == hipSuccess) e = hipMemcpy(tmp.data(), src_state, bytes, hipMemcpyDeviceToHost);
      if (e == hipSuccess)
        e = hipMemcpy(tmp.data() + words, s->status_dev, sizeof(DevStatus), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(s, e, "reading source state");
    }
    int rc = ensure_dev(dst, &dst->aux_dev, &dst->aux_cap, bytes + sizeof(DevStatus));
    if (rc) return rc;
    e = hipMemcpyAsync(dst->aux_dev, tmp.data(), bytes + sizeof(DevStatus), hipMemcpyHostToDevice,
                       dst->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(dst->stream);
    if (e != hipSuccess) return hip_fail(dst, e, "uploading source state");
    src_state = (const uint64_t*)dst->aux_dev;
    src_status = (const DevStatus*)((const char*)dst->aux_dev + bytes);
  } else if (s->stream != dst->stream) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, s->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(dst->stream, ev, 0);
    if (e == hipSuccess) e = hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(dst, e, "ordering src before dst");
  }
  if (pairwise)
    launch_pairwise_merge_states(dst->state[dst->cur], src_state, dst->state[dst->cur ^ 1], dst->p, dst->stream);
  else
    launch_merge_states(dst->state[dst->cur], src_state, dst->state[dst->cur ^ 1], dst->p,
                        dst->intf_dev, dst->stream);
  // a deferred error of the source (exactness guard, parse) now holds for dst
  launch_status_or(dst->status_dev, src_status, dst->stream);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(dst, e, "merge kernel launch");
  dst->cur ^= 1;
  // the source must not change under the pending merge: later writes to src
  // are ordered on src's stream, so make src wait for dst
  if (s->device == dst->device && s->stream != dst->stream) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, dst->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, ev, 0);
    if (e == hipSuccess) e = hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(dst, e, "ordering dst before src");
  }
  return STATS_OK;
}

// ---------------------------------------------------------------------------
// raw statistics and finalize

namespace st {

int raw_of_state(stats_ctx* h, const uint64_t* state_dev, int64_t* n, stats_i128* s_int,
                 double* s_f64, stats_i128* C_int, double* C_f64, uint8_t* exact_mask) {
  const int p = h->p;
  const Layout L = Layout::make(p);
  int rc = ensure_dev(h, (void**)&h->raw_out, &h->raw_cap, (size_t)(p + (int64_t)p * p) * 8);
  if (rc) return rc;
  launch_raw(state_dev, p, h->intf_dev, h->raw_out, h->stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "raw kernel launch");
  std::vector<uint64_t> st(L.words);
  std::vector<double> raw(p + (size_t)p * p);
  e = hipMemcpyAsync(st.data(), state_dev, (size_t)L.words * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(raw.data(), h->raw_out, raw.size() * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reading statistics");
  if (n) *n = (int64_t)st[0];
  for (int i = 0; i < p; ++i) {
    if (s_int) {
      if (h->intf[i]) {
        s_int[i].lo = st[L.off_s + 2 * i];
        s_int[i].hi = (int64_t)st[L.off_s + 2 * i + 1];
      } else {
        s_int[i].lo = 0;
        s_int[i].hi = 0;
      }
    }
    if (s_f64) s_f64[i] = raw[i];
    for (int j = 0; j < p; ++j) {
      const int a = std::min(i, j), b = std::max(i, j);
      const bool ex = h->intf[a] && h->intf[b];
      const int64_t t = tri(p, a, b);
      if (C_int) {
        C_int[(int64_t)i * p + j].lo = ex ? st[L.off_C + 2 * t] : 0;
        C_int[(int64_t)i * p + j].hi = ex ? (int64_t)st[L.off_C + 2 * t + 1] : 0;
      }
      if (C_f64) C_f64[(int64_t)i * p + j] = raw[p + (int64_t)i * p + j];
      if (exact_mask) exact_mask[(int64_t)i * p + j] = ex ? 1 : 0;
    }
  }
  return STATS_OK;
}

int selection(const stats_ctx* h, const stats_finalize_opts* o, std::vector<int32_t>* sel) {
  sel->clear();
  bool any = false;
  for (int w = 0; w < STATS_MASK_WORDS; ++w) any |= o->column_mask[w] != 0;
  for (int c = 0; c < h->p; ++c) {
    const bool keep = any ? ((o->column_mask[c / 64] >> (c % 64)) & 1u)
                          : !(h->cols[c].flags & STATS_COL_IDENTIFIER);
    if (keep) sel->push_back(c);
  }
  if (any) {
    for (int c = h->p; c < STATS_MAX_P; ++c)
      if ((o->column_mask[c / 64] >> (c % 64)) & 1u)
        return fail(STATS_E_ARG, "column_mask selects a column >= p");
  }
  if (sel->empty()) return fail(STATS_E_ARG, "no column selected");
  if (o->ddof < 0) return fail(STATS_E_ARG, "ddof < 0");
  if (o->pca_on != 0 && o->pca_on != 1) return fail(STATS_E_ARG, "pca_on must be 0 or 1");
  return STATS_OK;
}

}  // namespace st

extern "C" int stats_raw(stats_ctx* h, int64_t* n, stats_i128* s_int, double* s_f64,
                         stats_i128* C_int, double* C_f64, uint8_t* exact_mask) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups) return fail(STATS_E_STATE, "groups handle: use stats_group_raw");
  if (h->flags & STATS_CFG_PAIRWISE) return fail(STATS_E_STATE, "pairwise handle: use stats_finalize_pairwise");
  DeviceGuard g(h->device);
  int rc = sync_handle(h);
  if (rc) return rc;
  return raw_of_state(h, h->state[h->cur], n, s_int, s_f64, C_int, C_f64, exact_mask);
}

extern "C" int stats_finalize(stats_ctx* h, const stats_finalize_opts* opts, int32_t* p_out,
                              double* mean, double* cov, double* corr, double* eigval,
                              double* eigvec, double* var_pct, double* cum_pct) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups) return fail(STATS_E_STATE, "groups handle: use stats_finalize_groups");
  if (h->flags & STATS_CFG_PAIRWISE) return fail(STATS_E_STATE, "pairwise handle: use stats_finalize_pairwise");
  stats_finalize_opts def;
  memset(&def, 0, sizeof def);
  def.ddof = 1;
  def.want_vectors = 1;
  const stats_finalize_opts* o = opts ? opts : &def;
  std::vector<int32_t> sel;
  int rc = selection(h, o, &sel);
  if (rc) return rc;
  DeviceGuard g(h->device);
  // everything is enqueued behind the pending accumulate work and read back
  // with one synchronization; the status word and N are checked afterwards
  // (the kernel computes nothing when N <= ddof)
  const int q = (int)sel.size();
  const size_t out_words = (size_t)q * 4 + 3 * (size_t)q * q;
  rc = ensure_dev(h, (void**)&h->fin_out, &h->fin_out_cap, out_words * 8);
  const size_t jtab_words = 5 * (size_t)((q + 1) / 2);
  if (!rc) rc = ensure_dev(h, (void**)&h->fin_scratch, &h->fin_scratch_cap, (2 * (size_t)q * q + jtab_words + 2) * 8);
  if (!rc) rc = ensure_dev(h, (void**)&h->sel_dev, &h->sel_cap, (size_t)q * 4);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(h->sel_dev, sel.data(), (size_t)q * 4, hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "uploading selection");
  FinalizeLaunch F;
  F.state = h->state[h->cur];
  F.p = h->p;
  F.sel_dev = h->sel_dev;
  F.q = q;
  F.intflags_dev = h->intf_dev;
  F.ddof = o->ddof;
  F.pca_on = o->pca_on;
  F.want_vectors = o->want_vectors ? 1 : 0;
  F.out = h->fin_out;
  F.scratch = h->fin_scratch;
  F.jtab = h->fin_scratch + 2 * (size_t)q * q;
  F.jc = (unsigned*)(F.jtab + jtab_words);
  {
    Timer t;
    t.begin(h, STATS_K_FINALIZE);
    e = launch_finalize(F, h->stream);
    t.end();
  }
  if (e != hipSuccess) return hip_fail(h, e, "finalize");
  std::vector<double> out(out_words);
  int64_t n = 0;
  DevStatus st;
  e = hipMemcpyAsync(out.data(), h->fin_out, out_words * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&n, h->state[h->cur], 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&st, h->status_dev, sizeof st, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && h->copy_stream) e = hipStreamSynchronize(h->copy_stream);
  if (e != hipSuccess) return hip_fail(h, e, "finalize");
  collect_timings(h);
  rc = status_error(st);
  if (rc) return rc;
  if (n <= o->ddof) return fail(STATS_E_STATE, "N <= ddof: covariance undefined");
  const size_t qq = (size_t)q * q;
  const double* po = out.data();
  if (p_out) *p_out = q;
  if (mean) memcpy(mean, po, q * 8);
  if (cov) memcpy(cov, po + q, qq * 8);
  if (corr) memcpy(corr, po + q + qq, qq * 8);
  if (eigval) memcpy(eigval, po + q + 2 * qq, q * 8);
  if (eigvec && o->want_vectors) memcpy(eigvec, po + 2 * q + 2 * qq, qq * 8);
  if (var_pct) memcpy(var_pct, po + 2 * q + 3 * qq, q * 8);
  if (cum_pct) memcpy(cum_pct, po + 3 * q + 3 * qq, q * 8);
  return STATS_OK;
}

// ---------------------------------------------------------------------------
// checkpoint

static const char kMagic[8] = {'S', 'T', 'S', 'T', 'A', 'T', 'S', '1'};

extern "C" int stats_serialize(stats_ctx* h, void* buf, size_t* len) {
  if (!h || !len) return fail(STATS_E_ARG, "NULL argument");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups) return fail(STATS_E_STATE, "groups handles are not serialized");
  if (h->flags & STATS_CFG_PAIRWISE) return fail(STATS_E_STATE, "pairwise handle: use stats_finalize_pairwise");
  const Layout L = Layout::make(h->p);
  const size_t need = 8 + 8 + (size_t)h->p * 8 + (size_t)L.words * 8;
  if (!buf) {
    *len = need;
    return STATS_OK;
  }
  if (*len < need) return fail(STATS_E_ARG, "buffer too small");
  DeviceGuard g(h->device);
  int rc = sync_handle(h);
  if (rc) return rc;
  char* o = (char*)buf;
  memcpy(o, kMagic, 8);
  const int64_t p = h->p;
  memcpy(o + 8, &p, 8);
  for (int c = 0; c < h->p; ++c) {
    const int32_t sig[2] = {h->cols[c].dtype, (int32_t)(h->intf[c] | (h->cols[c].flags << 1))};
    memcpy(o + 16 + 8 * c, sig, 8);
  }
  hipError_t e = hipMemcpy(o + 16 + 8 * (size_t)h->p, h->state[h->cur], (size_t)L.words * 8,
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "reading state");
  *len = need;
  return STATS_OK;
}

extern "C" int stats_deserialize(const void* buf, size_t len, const stats_config* cfg,
                                 stats_ctx** out) {
  if (out) *out = nullptr;
  if (!buf || !cfg || !out) return fail(STATS_E_ARG, "NULL argument");
  if (len < 16 || memcmp(buf, kMagic, 8) != 0) return fail(STATS_E_ARG, "not a statistics checkpoint");
  int64_t p;
  memcpy(&p, (const char*)buf + 8, 8);
  if (p != cfg->p) return fail(STATS_E_MISMATCH, "checkpoint has a different column count");
  if (cfg->flags & STATS_CFG_PAIRWISE) return fail(STATS_E_STATE, "pairwise handles are not serialized");
  const Layout L = Layout::make((int)p);
  if (len != 16 + 8 * (size_t)p + (size_t)L.words * 8) return fail(STATS_E_ARG, "checkpoint size mismatch");
  stats_ctx* h = nullptr;
  int rc = stats_open(cfg, &h);
  if (rc) return rc;
  for (int c = 0; c < h->p; ++c) {
    int32_t sig[2];
    memcpy(sig, (const char*)buf + 16 + 8 * c, 8);
    if (sig[0] != h->cols[c].dtype || sig[1] != (int32_t)(h->intf[c] | (h->cols[c].flags << 1))) {
      stats_close(h);
      return fail(STATS_E_MISMATCH, "checkpoint column " + std::to_string(c) + " differs");
    }
  }
  DeviceGuard g(h->device);
  hipError_t e = hipMemcpyAsync(h->state[h->cur], (const char*)buf + 16 + 8 * p, (size_t)L.words * 8,
                                hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    rc = hip_fail(h, e, "uploading checkpoint");
    stats_close(h);
    return rc;
  }
  *out = h;
  return STATS_OK;
}

extern "C" int stats_kernel_time(stats_ctx* h, int32_t which, int64_t* launches, double* total_ms) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (which < 0 || which >= STATS_K_COUNT) return fail(STATS_E_ARG, "unknown kernel id");
  if (!(h->flags & STATS_CFG_TIMING)) return fail(STATS_E_STATE, "handle opened without STATS_CFG_TIMING");
  if (launches) *launches = h->kt_n[which];
  if (total_ms) *total_ms = h->kt_ms[which];
  return STATS_OK;
}
