// Instantiations of the narrow-table reduction kernels for p = 6 and p = 11.
#include "accum_impl.hpp"

namespace st {
template void launch_accum_p<6>(const acc::Args&, int, int, int64_t, hipStream_t);
template void launch_accum_p<11>(const acc::Args&, int, int, int64_t, hipStream_t);
}  // namespace st
