// F64 burst kernels with the neighbour exchange through LDS: fused macro step (Sec. 3.3
// steps (i)-(vi) in one launch).
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
hipError_t launch_time_table(const SrcInfo& src, double t_n, double dt, int n_t, double* out,
                             hipStream_t s) {
  const int n = src.ns * n_t;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_time_table, dim3((n + 255) / 256), dim3(256), 0, s, src, t_n, dt, n_t,
                     out);
  return hipGetLastError();
}

hipError_t launch_burst_lds_f64(int R, int C, const BurstArgs& a, int blocks,
                                int threads, size_t lds, hipStream_t s) {
  return launch_family<double, XCH_LDS, MODE_FUSED>(R, C, a, blocks, threads, lds, s);
}
}  // namespace pdk
