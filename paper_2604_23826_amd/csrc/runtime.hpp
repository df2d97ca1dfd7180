// Handle structure and runtime helpers of libstats.so (host side).
#pragma once
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

struct stats_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t copy_stream = nullptr;
  int p = 0;
  std::vector<stats_column> cols;
  std::vector<uint8_t> intf;  // 1 = integer column (exact path)
  int n_planes = 0;
  int64_t row_stride[STATS_MAX_PLANES] = {};
  int precision = 0;
  int64_t staging_rows = 0;
  int64_t block_rows = 0;
  uint32_t flags = 0;
  int ngroups = 0;  // 0: single statistics; > 0: groups handle
  bool poisoned = false;

  // device state (double-buffered: merges read state[cur], write state[cur^1])
  uint64_t* state[2] = {nullptr, nullptr};
  int cur = 0;
  uint8_t* intf_dev = nullptr;
  st::DevStatus* status_dev = nullptr;

  // scratch
  uint64_t* rec = nullptr;
  size_t rec_cap = 0;
  double* fin_out = nullptr;
  size_t fin_out_cap = 0;
  double* fin_scratch = nullptr;
  size_t fin_scratch_cap = 0;
  int32_t* sel_dev = nullptr;
  size_t sel_cap = 0;
  double* raw_out = nullptr;
  size_t raw_cap = 0;
  void* aux_dev = nullptr;
  size_t aux_cap = 0;
  void* aux2_dev = nullptr;
  size_t aux2_cap = 0;
  void* aux3_dev = nullptr;
  size_t aux3_cap = 0;
  void* conv_dev = nullptr;  // text -> binary conversion: line counts, status
  size_t conv_cap = 0;

  // host staging ring (two slots)
  void* stage_dev[2] = {nullptr, nullptr};
  size_t stage_cap[2] = {0, 0};
  void* stage_host[2] = {nullptr, nullptr};
  size_t stage_host_cap[2] = {0, 0};
  hipEvent_t ev_copy[2] = {nullptr, nullptr};
  hipEvent_t ev_free[2] = {nullptr, nullptr};
  int slot = 0;

  // segmented launch graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  int graph_nwg = 0;
  int graph_aos64 = -1;  // kernel captured in the graph: 1 = k_seg_aos64
  int64_t seg_tile_rows = 0;
  int seg_wg_per_cu = 0;
  int64_t seg_cap_rt = 0;
  uint64_t* seg_part = nullptr;  // partial states of the segmented merge's first stage
  size_t seg_part_cap = 0;

  // text ingest: bytes consumed so far (offsets in parse errors), and the
  // mean line length of the last chunk measured (0: none yet)
  int64_t text_offset = 0;
  double text_ell = 0.0;

  // kernel timing (STATS_CFG_TIMING)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[STATS_K_COUNT];
  int64_t kt_n[STATS_K_COUNT] = {};
  double kt_ms[STATS_K_COUNT] = {};
};

namespace st {

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);
int hip_fail(stats_ctx* h, hipError_t e, const char* what);
int elem_size(int dtype);
int ensure_dev(stats_ctx* h, void** ptr, size_t* cap, size_t need);
int sync_handle(stats_ctx* h);
void collect_timings(stats_ctx* h);
int accumulate_device(stats_ctx* h, const void* const* planes, int64_t nrows);
int accumulate_device_wide(stats_ctx* h, const void* const* planes, int64_t nrows);
int accumulate_host_src(stats_ctx* h, const void* const* planes, int fd, int64_t file_off, int64_t nrows,
                        bool pinned);
int pairwise_state_words(int p);
int64_t state_words(const stats_ctx* h);
int accumulate_pairwise(stats_ctx* h, const void* const* planes, int64_t nrows);
void launch_pairwise_merge_states(const uint64_t* a, const uint64_t* b, uint64_t* out, int p, hipStream_t s);
AccumLaunch accum_launch_of(const stats_ctx* h, const void* const* planes);
int64_t block_rows_for(const stats_ctx* h, int64_t nrows);
int raw_of_state(stats_ctx* h, const uint64_t* state_dev, int64_t* n, stats_i128* s_int,
                 double* s_f64, stats_i128* C_int, double* C_f64, uint8_t* exact_mask);
int selection(const stats_ctx* h, const stats_finalize_opts* o, std::vector<int32_t>* sel);
hipError_t clear_status(stats_ctx* h);

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

// HIP-event bracket around the launches of one kernel (STATS_CFG_TIMING).
struct Timer {
  stats_ctx* h_ = nullptr;
  int which_ = 0;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  hipStream_t s_ = nullptr;
  void begin(stats_ctx* h, int which, hipStream_t s = nullptr);
  void end();
};

}  // namespace st
