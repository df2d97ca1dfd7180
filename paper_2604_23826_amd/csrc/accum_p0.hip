// Instantiations of the narrow-table reduction kernels for p = 1 and p = 16.
#include "accum_impl.hpp"

namespace st {
template void launch_accum_p<1>(const acc::Args&, int, int, int64_t, hipStream_t);
template void launch_accum_p<16>(const acc::Args&, int, int, int64_t, hipStream_t);
}  // namespace st
