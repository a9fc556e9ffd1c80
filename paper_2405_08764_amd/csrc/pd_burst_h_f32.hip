// F32 burst kernels with the hybrid neighbour exchange (DPP inside each wave, band
// edges through LDS): fused macro step (Sec. 3.3 steps (i)-(vi) in one launch).
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
hipError_t launch_burst_h_f32(int R, int C, const BurstArgs& a, int blocks,
                              int threads, size_t lds, hipStream_t s) {
  return launch_family<float, XCH_HYBRID, MODE_FUSED>(R, C, a, blocks, threads, lds, s);
}
}  // namespace pdk
