// Allocation-free accumulate for device-resident narrow tables (p <= 16).
//
// The block records that stats_accumulate writes into library-allocated
// memory go here into one fixed device array per GPU, so the call itself
// performs no device allocation (for code under HIP graph capture, serving
// loops and harnesses that forbid hipMalloc).  The handle's state buffers
// were allocated by stats_open; everything else is the existing narrow
// kernels (per-lane accumulation, then the fixed-tree merge).
//
// The array is a file-scope __device__ symbol.  Host code never passes its
// name to a kernel: the device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is used.
#include <mutex>

#include "common.hpp"
#include "runtime.hpp"

namespace {

constexpr size_t kScratchBytes = STATS_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

__device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
uint64_t* g_scratch_dev[kMaxDevices] = {};

// Device address of this GPU's copy of the array (the current device must be
// `dev`).  Returns nullptr and sets the error text on failure.
uint64_t* scratch_of(int dev) {
  std::lock_guard<std::mutex> lk(g_lock);
  if (g_scratch_dev[dev]) return g_scratch_dev[dev];
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    st::fail(STATS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return nullptr;
  }
  g_scratch_dev[dev] = (uint64_t*)ptr;
  return g_scratch_dev[dev];
}

}  // namespace

using namespace st;

extern "C" int stats_accumulate_noalloc(stats_ctx* h, const void* const* planes, int64_t nrows) {
  if (!h) return fail(STATS_E_ARG, "handle is NULL");
  if (h->poisoned) return fail(STATS_E_STATE, "handle is poisoned by an earlier HIP error");
  if (h->ngroups) return fail(STATS_E_STATE, "groups handle: use stats_accumulate_segmented");
  if (h->flags & STATS_CFG_PAIRWISE) return fail(STATS_E_STATE, "pairwise handle: use stats_accumulate");
  if (h->p > 16)
    return fail(STATS_E_ARG, "stats_accumulate_noalloc: p = " + std::to_string(h->p) +
                                 " exceeds 16 (its fixed scratch serves the narrow kernels only)");
  if (nrows < 0) return fail(STATS_E_ARG, "nrows < 0");
  if (nrows == 0) return STATS_OK;
  if (!planes) return fail(STATS_E_ARG, "planes is NULL");
  for (int k = 0; k < h->n_planes; ++k) {
    bool used = false;
    for (const auto& c : h->cols) used |= c.plane == k;
    if (used && !planes[k]) return fail(STATS_E_ARG, "plane " + std::to_string(k) + " is NULL");
    if (planes[k] && ((uintptr_t)planes[k] % 16) != 0)
      return fail(STATS_E_ARG, "device planes must be 16-byte aligned");
  }
  if (h->device < 0 || h->device >= kMaxDevices) return fail(STATS_E_ARG, "device ordinal out of range");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(STATS_E_HIP, "hipSetDevice failed");
  uint64_t* rec = scratch_of(h->device);
  if (!rec) return STATS_E_HIP;

  const int p = h->p;
  const int64_t R = block_rows_for(h, nrows);
  const int64_t W = rec_words(p);
  // blocks per launch: their records fit the array; at most 16384 (the merge
  // tree's depth stays at most 14) and 2^28 rows (32-bit plane offsets)
  const int64_t fit = (int64_t)(kScratchBytes / (size_t)(W * 8));
  const int64_t max_blocks = std::min<int64_t>(fit, 16384);
  const int64_t max_rows = std::max<int64_t>(R, std::min<int64_t>(max_blocks * R, ((int64_t)1 << 28) / R * R));
  if (fit < 1) return fail(STATS_E_ARG, "stats_accumulate_noalloc: one block's record exceeds the fixed scratch");
  const AccumLaunch a = accum_launch_of(h, planes);
  int64_t done = 0;
  while (done < nrows) {
    const int64_t rows = std::min(nrows - done, max_rows);
    const int64_t nblocks = (rows + R - 1) / R;
    AccumLaunch b = a;
    for (int c = 0; c < p; ++c) b.colbase[c] = a.colbase[c] + done * a.colstride[c];
    b.nrows = rows;
    b.block_rows = R;
    b.rec = rec;
    launch_accum_small_p(b, h->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "accumulate kernel launch");
    // reads the records before the next launch (same stream) overwrites them
    launch_merge_records(rec, nblocks, p, h->intf_dev, h->state[h->cur], h->state[h->cur ^ 1],
                         h->status_dev, h->stream);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "merge kernel launch");
    h->cur ^= 1;
    done += rows;
  }
  return STATS_OK;
}
