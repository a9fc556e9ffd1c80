// Persistent batched burst kernel: many independent grids (uneven macro grids, patch
// sizes, maps, coefficients and time steps) advance one macro step each in one launch.
// Blocks take work items from a device queue (an atomic counter over an item list the
// host sorts by cost, longest first); an item is a group of patches of one instance run
// by the same team bodies as the single-grid kernels, so every patch's arithmetic, and
// therefore its result, is bitwise that of the single-grid path.
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
namespace {

template <int NSB, int XCH, int C, int R>
__device__ __forceinline__ void run_item(const BurstArgs& A, const BatchItem& I,
                                         unsigned char* smem, const double* Uin, double* Uout,
                                         const double* ttab) {
  if constexpr (XCH == XCH_LANES) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const LaneMap L =
        lane_map<R, C>(A, lane, 64, (long long)I.p0 + (long long)w * I.ppb, I.ppb);
    const size_t slice =
        (burst_lds_bytes(PD_F64, R, C, XCH_LANES, 64, I.ppb, L.mx, L.me, NSB) + 15) &
        ~size_t(15);
    const LdsMap M = lds_map<double, R, C, NSB>(A, L, smem + w * slice, 1);
    body_x<double, R, C, NSB, MODE_FUSED>(A, L, M, Uin, Uout, ttab);
  } else {
    const LaneMap L = lane_map<R, C>(A, threadIdx.x, BATCH_THREADS, I.p0, I.ppb);
    const LdsMap M = lds_map<double, R, C, NSB>(A, L, smem, 2);
    body_lds<double, R, C, NSB, MODE_FUSED>(A, L, M, Uin, Uout, ttab);
  }
}

template <int NSB>
__global__ __launch_bounds__(BATCH_THREADS) void k_batch(BatchArgs B) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();  // everyone is done with the previous item and its LDS
    if (threadIdx.x == 0) s_item = atomicAdd(B.head, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= B.n_items) break;
    const BatchItem I = B.items[it];
    const BurstArgs& A = B.inst[I.inst];
    const long long n = B.tuning ? 0 : B.clk->base + B.k;
    const double* Uin = (n & 1) ? A.Unew : A.U;
    double* Uout = (n & 1) ? const_cast<double*>(A.U) : A.Unew;
    const double* ttab = A.ttab + (long long)B.k * A.src.ns * A.n_t;
    if (I.p0 == 0 && A.bvals != nullptr) {  // step (vi)'s Dirichlet nodes, once per instance
      const double* bv = A.bvals + (long long)B.k * A.nb;
      for (int q = threadIdx.x; q < A.nb; q += BATCH_THREADS) {
        int i, j;
        boundary_node(A.g, q, i, j);
        Uout[j * A.g.n_xi + i] = bv[q];
      }
    }
    switch (I.shape) {
#define PD_BITEM(id, xch, C_, R_) \
  case id: run_item<NSB, xch, C_, R_>(A, I, smem, Uin, Uout, ttab); break;
      PD_BATCH_MENU(PD_BITEM)
#undef PD_BITEM
      default: break;
    }
  }
  if (threadIdx.x == 0) {  // the last block out rewinds the queue for the next launch
    __threadfence();
    if (atomicAdd(B.exits, 1u) == gridDim.x - 1) {
      *B.head = 0;
      *B.exits = 0u;
      __threadfence();
    }
  }
}

}  // namespace

hipError_t launch_batch(int nsb, const BatchArgs& a, int blocks, size_t lds, hipStream_t s) {
  if (nsb == 2)
    hipLaunchKernelGGL(k_batch<2>, dim3(blocks), dim3(BATCH_THREADS), lds, s, a);
  else
    hipLaunchKernelGGL(k_batch<1>, dim3(blocks), dim3(BATCH_THREADS), lds, s, a);
  return hipGetLastError();
}

hipError_t batch_blocks_per_cu(int nsb, size_t lds, int* out) {
  if (nsb == 2)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_batch<2>, BATCH_THREADS, lds);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_batch<1>, BATCH_THREADS, lds);
}

}  // namespace pdk
