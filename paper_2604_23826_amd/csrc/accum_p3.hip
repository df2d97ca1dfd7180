// Instantiations of the narrow-table reduction kernels for p = 4 and p = 13.
#include "accum_impl.hpp"

namespace st {
template void launch_accum_p<4>(const acc::Args&, int, int, int64_t, hipStream_t);
template void launch_accum_p<13>(const acc::Args&, int, int, int64_t, hipStream_t);
}  // namespace st
