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
  } else if constexpr (XCH == XCH_HYBRID) {
    const LaneMap L = lane_map_h<R, C>(A, threadIdx.x, BATCH_THREADS, I.p0, I.ppb);
    const int nbt = BATCH_WAVES * (64 / L.Lb);
    const LdsMap M =
        lds_map<double, R, C, NSB>(A, L, smem, 1, hybrid_edge_bytes(8, C, L.Lb, nbt));
    body_h<double, R, C, NSB, MODE_FUSED>(A, L, M, Uin, Uout, ttab, nbt);
  } else {
    const LaneMap L = lane_map<R, C>(A, threadIdx.x, BATCH_THREADS, I.p0, I.ppb);
    const LdsMap M = lds_map<double, R, C, NSB>(A, L, smem, 2);
    body_lds<double, R, C, NSB, MODE_FUSED>(A, L, M, Uin, Uout, ttab);
  }
}

// Three blocks per CU (12 waves, at most 168 registers per lane): the multi-wave teams
// wait on LDS round trips and a barrier every nano step, and a third wave per SIMD hides
// much of that (measured on the mixed batch: 357 -> 315 ms per step; the in-wave shapes
// run as fast as at two waves per SIMD).  Shapes that no longer fit in registers spill
// (the LDS exchange with four columns per lane doubles its time) and lose in the
// autotuner; a fourth wave per SIMD (128 registers) spills everywhere.
template <int NSB>
__global__ __launch_bounds__(BATCH_THREADS, 3) void k_batch(BatchArgs B) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  for (;;) {
    __syncthreads();  // everyone is done with the previous item and its LDS
    if (threadIdx.x == 0) s_item = atomicAdd(B.head, 1);
    __syncthreads();
    const int it = s_item;
    const int n_items = B.n_dev != nullptr ? *B.n_dev : B.n_items;
    if (it >= n_items) break;
    int idx = it;
    if (B.segs != nullptr) {  // segment of `it`: the last with prefix <= it
      int lo = 0, hi = B.n_segs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.segs[mid].w <= it) lo = mid;
        else hi = mid - 1;
      }
      const int4 sg = B.segs[lo];
      idx = sg.x + (it - sg.w) * sg.z;
    }
    const BatchItem I = B.items[idx];
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

// Patches of an item: BATCH_WAVES teams for in-wave shapes, one team otherwise.
__device__ inline int item_patches(const BatchItem& I) {
  switch (I.shape) {
#define PD_XW(id, xch, C_, R_) \
  case id: return (xch == XCH_LANES ? BATCH_WAVES : 1) * I.ppb;
    PD_BATCH_MENU(PD_XW)
#undef PD_XW
    default: return I.ppb;
  }
}

// Exclusive prefix sum over one block of SEG_THREADS threads: v is this thread's value;
// returns the sum of the values of the threads before it and sets total.
constexpr int SEG_THREADS = 256;
__device__ int block_exclusive_scan(int v, int* scratch, int& total) {
  const int t = threadIdx.x;
  scratch[t] = v;
  __syncthreads();
  for (int o = 1; o < SEG_THREADS; o <<= 1) {  // Hillis-Steele inclusive scan
    const int x = t >= o ? scratch[t - o] : 0;
    __syncthreads();
    scratch[t] += x;
    __syncthreads();
  }
  total = scratch[SEG_THREADS - 1];
  const int incl = scratch[t];
  __syncthreads();
  return incl - v;
}

// One block: this step's spot-check segments (per instance, every stride-th item from a
// hashed offset, at least one item), their prefix sums and total; clears the residuals.
// Segment slots follow S.order (instances by descending item cost), so the queue hands
// out the longest spot checks first; each thread takes a contiguous run of slots.
__global__ __launch_bounds__(SEG_THREADS) void k_spot_segments(SpotArgs S) {
  __shared__ int scan[SEG_THREADS];
  const long long step = S.clk->base + S.k;
  const int per = (S.n + SEG_THREADS - 1) / SEG_THREADS;
  const int i0 = threadIdx.x * per, i1 = i0 + per < S.n ? i0 + per : S.n;
  int mine = 0;
  for (int sl = i0; sl < i1; ++sl) {
    const int i = S.order[sl];
    const int cnt = S.count[i];
    unsigned int h = (unsigned int)(step * 2654435761ull) ^ (unsigned int)(i * 40503u + 17u);
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    const int off = (int)(h % (unsigned int)S.stride);
    int c = cnt > off ? (cnt - 1 - off) / S.stride + 1 : 0;
    int f = off;
    if (c == 0 && cnt > 0) {
      c = 1;
      f = (int)(h % (unsigned int)cnt);
    }
    S.spot[sl] = make_int4(S.first[i] + f, c, S.stride, 0);
    S.resid[i] = 0u;
    mine += c;
  }
  int total;
  int run = block_exclusive_scan(mine, scan, total);
  for (int sl = i0; sl < i1; ++sl) {
    S.spot[sl].w = run;
    run += S.spot[sl].y;
  }
  if (threadIdx.x == 0) *S.spot_n = total;
}

// Residuals of the checked patches: |F_hat - F| / s with F from the plain step just
// written, per-instance maximum.  Blocks stride over the spot items.
__global__ void k_spot_residuals(SpotArgs S, const BurstArgs* __restrict__ inst,
                                 const BatchItem* __restrict__ items,
                                 double* const* __restrict__ fhat,
                                 float* const* __restrict__ sres) {
  const int total = *S.spot_n;
  const long long step = S.clk->base + S.k;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    int lo = 0, hi = S.n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (S.spot[mid].w <= it) lo = mid;
      else hi = mid - 1;
    }
    const int4 sg = S.spot[lo];
    const BatchItem I = items[sg.x + (it - sg.w) * sg.z];
    const BurstArgs& A = inst[I.inst];
    const double* Uin = (step & 1) ? A.Unew : A.U;
    const double* Uout = (step & 1) ? A.U : A.Unew;
    const int np = item_patches(I);
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
      const long long p = (long long)I.p0 + q;
      if (p >= A.g.P) continue;
      const int node = A.pmap[11 * p + 6];
      const double F = (Uout[node] - Uin[node]) / A.dt_macro;
      const double r = fabs(fhat[I.inst][p] - F) / (double)sres[I.inst][p];
      const float rf = (float)(r == r ? r : 1e30);
      atomicMax(&S.resid[I.inst], __float_as_uint(rf));
      atomicAdd(&S.stats[0], 1ull);
    }
  }
}

// One block: fallback segments (every item of each instance whose residual exceeds the
// threshold) and their count.
__global__ __launch_bounds__(SEG_THREADS) void k_redo_segments(SpotArgs S) {
  __shared__ int scan[SEG_THREADS];
  const int per = (S.n + SEG_THREADS - 1) / SEG_THREADS;
  const int i0 = threadIdx.x * per, i1 = i0 + per < S.n ? i0 + per : S.n;
  int mine = 0, bad = 0;
  for (int sl = i0; sl < i1; ++sl) {
    const int i = S.order[sl];
    const float r = __uint_as_float(S.resid[i]);
    const bool redo = !((double)r <= S.threshold);
    mine += redo ? S.count[i] : 0;
    bad += redo ? 1 : 0;
  }
  int total;
  int run = block_exclusive_scan(mine, scan, total);
  int nbad;
  (void)block_exclusive_scan(bad, scan, nbad);
  for (int sl = i0; sl < i1; ++sl) {
    const int i = S.order[sl];
    const float r = __uint_as_float(S.resid[i]);
    const bool redo = !((double)r <= S.threshold);
    S.redo[sl] = make_int4(S.first[i], redo ? S.count[i] : 0, 1, run);
    run += redo ? S.count[i] : 0;
  }
  if (threadIdx.x == 0) {
    *S.redo_n = total;
    if (nbad) atomicAdd(&S.stats[1], (unsigned long long)nbad);
  }
}

}  // namespace

hipError_t launch_spot_segments(const SpotArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_spot_segments, dim3(1), dim3(SEG_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_redo_segments(const SpotArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_redo_segments, dim3(1), dim3(SEG_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_spot_residuals(const SpotArgs& a, const BurstArgs* inst,
                                 const BatchItem* items, double* const* fhat,
                                 float* const* sres, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_spot_residuals, dim3(blocks), dim3(256), 0, s, a, inst, items, fhat, sres);
  return hipGetLastError();
}

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
