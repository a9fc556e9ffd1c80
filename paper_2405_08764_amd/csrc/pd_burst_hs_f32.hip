// F32 burst kernels with the hybrid neighbour exchange (DPP inside each wave, band
// edges through LDS): split-mode burst (step (iii) on caller-owned patch states).
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
hipError_t launch_burst_hs_f32(int R, int C, const BurstArgs& a, int blocks,
                               int threads, size_t lds, hipStream_t s) {
  return launch_family<float, XCH_HYBRID, MODE_SPLIT>(R, C, a, blocks, threads, lds, s);
}
}  // namespace pdk
