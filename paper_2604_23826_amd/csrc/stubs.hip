// Entry points whose kernels live in their own files (wide tables, batched
// groups, text ingest).
#include "common.hpp"
#include "runtime.hpp"

using namespace st;


extern "C" int stats_accumulate_text(stats_ctx* h, const char* buf, int64_t nbytes, int32_t mem_kind,
                                     int32_t is_last, int64_t* bytes_consumed) {
  (void)h; (void)buf; (void)nbytes; (void)mem_kind; (void)is_last; (void)bytes_consumed;
  return fail(STATS_E_ARG, "text ingest is not supported by this build");
}

extern "C" int stats_accumulate_segmented(stats_ctx* h, const void* const* planes,
                                          const int64_t* row_offsets, int32_t mem_kind) {
  (void)h; (void)planes; (void)row_offsets; (void)mem_kind;
  return fail(STATS_E_ARG, "segmented accumulate is not supported by this build");
}

extern "C" int stats_finalize_groups(stats_ctx* h, const stats_finalize_opts* opts, int32_t* p_out,
                                     int64_t* n_out, double* mean_out, double* cov_out) {
  (void)h; (void)opts; (void)p_out; (void)n_out; (void)mean_out; (void)cov_out;
  return fail(STATS_E_ARG, "groups are not supported by this build");
}

extern "C" int stats_group_raw(stats_ctx* h, int32_t g, int64_t* n, stats_i128* s_int, double* s_f64,
                               stats_i128* C_int, double* C_f64, uint8_t* exact_mask) {
  (void)h; (void)g; (void)n; (void)s_int; (void)s_f64; (void)C_int; (void)C_f64; (void)exact_mask;
  return fail(STATS_E_ARG, "groups are not supported by this build");
}
