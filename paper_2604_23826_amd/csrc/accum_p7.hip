// Instantiations of the narrow-table reduction kernels for p = 8 and p = 9.
#include "accum_impl.hpp"

namespace st {
template void launch_accum_p<8>(const acc::Args&, int, int, int64_t, hipStream_t);
template void launch_accum_p<9>(const acc::Args&, int, int, int64_t, hipStream_t);
}  // namespace st
