// F64 burst kernels with the neighbour exchange through LDS: split-mode burst (step (iii)
// on caller-owned patch states).
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
hipError_t launch_burst_ldss_f64(int R, int C, const BurstArgs& a, int blocks,
                                 int threads, size_t lds, hipStream_t s) {
  return launch_family<double, XCH_LDS, MODE_SPLIT>(R, C, a, blocks, threads, lds, s);
}
}  // namespace pdk
