// Instantiations of the narrow-table reduction kernels for p = 7 and p = 10.
#include "accum_impl.hpp"

namespace st {
template void launch_accum_p<7>(const acc::Args&, int, int, int64_t, hipStream_t);
template void launch_accum_p<10>(const acc::Args&, int, int, int64_t, hipStream_t);
}  // namespace st
