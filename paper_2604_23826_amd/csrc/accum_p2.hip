// Instantiations of the narrow-table reduction kernels for p = 3 and p = 14.
#include "accum_impl.hpp"

namespace st {
template void launch_accum_p<3>(const acc::Args&, int, int, int64_t, hipStream_t);
template void launch_accum_p<14>(const acc::Args&, int, int, int64_t, hipStream_t);
}  // namespace st
