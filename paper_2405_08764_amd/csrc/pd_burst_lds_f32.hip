// F32 burst kernels with the neighbour exchange through LDS: fused macro step (Sec. 3.3
// steps (i)-(vi) in one launch).
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
hipError_t launch_burst_lds_f32(int R, int C, const BurstArgs& a, int blocks,
                                int threads, size_t lds, hipStream_t s) {
  return launch_family<float, XCH_LDS, MODE_FUSED>(R, C, a, blocks, threads, lds, s);
}
}  // namespace pdk
