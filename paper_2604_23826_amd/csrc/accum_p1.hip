// Instantiations of the narrow-table reduction kernels for p = 2 and p = 15.
#include "accum_impl.hpp"

namespace st {
template void launch_accum_p<2>(const acc::Args&, int, int, int64_t, hipStream_t);
template void launch_accum_p<15>(const acc::Args&, int, int, int64_t, hipStream_t);
}  // namespace st
