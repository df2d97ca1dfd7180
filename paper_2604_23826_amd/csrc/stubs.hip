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



