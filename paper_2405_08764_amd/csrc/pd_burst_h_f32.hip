// F32 burst kernels with the hybrid neighbour exchange (DPP inside each wave, band edges
// through LDS).
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
hipError_t launch_burst_h_f32(int R, int C, int mode, const BurstArgs& a, int blocks,
                            int threads, size_t lds, hipStream_t s) {
  return launch_family<float, XCH_HYBRID>(R, C, mode, a, blocks, threads, lds, s);
}
}  // namespace pdk
