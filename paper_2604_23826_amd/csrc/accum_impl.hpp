// Narrow-table reduction (p <= 16): generic kernel and the launcher that picks
// the layout-specialised kernel.
#pragma once
#include "accum_aos.hpp"
#include "accum_common.hpp"
#include "accum_planes.hpp"

namespace st {
namespace acc {

template <int P>
__global__ __launch_bounds__(kThreads, (P <= 12 ? 2 : 1)) void k_generic(Args a) {
  int64_t r0, r1;
  double K[P];
  int64_t Ki[P];
  prologue<P>(a, r0, r1, K, Ki);
  Acc<P> A;
  A.zero();
  uint32_t bad = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kThreads) {
    double d[P];
    generic_row<P>(a, r, K, Ki, d, bad);
    A.add(d);
  }
  finish_block<P>(a, A, K, Ki, bad, r0, r1);
}

}  // namespace acc

// Kind codes for launch_accum_p.
enum { ACC_GENERIC = 0, ACC_AOS = 1, ACC_PLANES = 2 };

template <int P, int NI>
struct PlanesDispatch {
  static void go(const acc::Args& a, int ni, dim3 g, dim3 b, hipStream_t s) {
    if (ni == NI) hipLaunchKernelGGL((acc::k_planes<P, NI>), g, b, 0, s, a);
    else PlanesDispatch<P, NI - 1>::go(a, ni, g, b, s);
  }
};
template <int P>
struct PlanesDispatch<P, -1> {
  static void go(const acc::Args&, int, dim3, dim3, hipStream_t) {}
};

// Launches the block-reduction kernel of width P (explicitly instantiated in
// one accum_p*.hip file per pair of widths, so they compile in parallel).
template <int P>
void launch_accum_p(const acc::Args& a, int kind, int ni, int64_t nblocks, hipStream_t s) {
  const dim3 grid((unsigned)nblocks), block(acc::kThreads);
  if (kind == ACC_AOS) {
    hipLaunchKernelGGL((acc::k_aos_dma<P>), grid, block, 0, s, a);
  } else if (kind == ACC_PLANES && ni >= 0 && ni <= P) {
    PlanesDispatch<P, P>::go(a, ni, grid, block, s);
  } else {
    hipLaunchKernelGGL((acc::k_generic<P>), grid, block, 0, s, a);
  }
}

}  // namespace st
