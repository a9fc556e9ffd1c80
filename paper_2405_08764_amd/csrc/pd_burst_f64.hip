// FP64 instantiations of the burst kernels.
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
hipError_t launch_burst_f64(int R, int mode, const BurstArgs& a, int blocks, int threads,
                            size_t lds, hipStream_t s) {
  return launch_any_r<double>(R, mode, a, blocks, threads, lds, s);
}
}  // namespace pdk
