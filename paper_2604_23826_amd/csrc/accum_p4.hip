// Instantiations of the narrow-table reduction kernels for p = 5 and p = 12.
#include "accum_impl.hpp"

namespace st {
template void launch_accum_p<5>(const acc::Args&, int, int, int64_t, hipStream_t);
template void launch_accum_p<12>(const acc::Args&, int, int, int64_t, hipStream_t);
}  // namespace st
