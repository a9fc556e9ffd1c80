// Full-domain lattice step: the explicit comparator of the paper's full-domain solution
// (Sec. 4.1.2, Table PDvsFDS) -- forward Euler of eq. (Computational_Problem) with the
// bursts' differences on one lattice over the whole box.  The weights are folded once per
// time step size (k_fd_weights); a step reads each weight plane and the field once, so it
// is bound by HBM bandwidth.  One thread per lattice column and FD_ROWS consecutive rows
// (the rows above and below come from registers); a wave spans 64 columns, so every
// plane load is one coalesced 512-byte access.  Waves whose nodes are all interior issue
// every load of their rows before any arithmetic (no branches, so the loads of all rows
// are in flight together); waves touching the boundary take a general path.
#include "pd_internal.h"

namespace pdk {
namespace {

constexpr int FD_ROWS = 2;  // measured: 2 rows 5.53 TB/s, 1 row 5.50, 4 rows 5.43, 8 rows 5.17
constexpr int FD_GROUPS = 4;  // waves per block, stacked in y

template <int NS, int HK>
__global__ __launch_bounds__(64 * FD_GROUPS) void k_fd_step(FdArgs a,
                                                            const double* __restrict__ U,
                                                            double* __restrict__ V, int k) {
  const int nx = a.n_x, ny = a.n_y;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j0 = (blockIdx.y * FD_GROUPS + (threadIdx.x >> 6)) * FD_ROWS;
  const long long P = a.plane;
  double T[NS > 0 ? NS : 1];
#pragma unroll
  for (int s = 0; s < NS; ++s) T[s] = a.ttab[s * FD_CHUNK + k];
  // wave-uniform: all 64 columns and all rows of this wave interior?
  const int ib = blockIdx.x * 64;
  const bool interior = ib >= 1 && ib + 64 <= nx - 1 && j0 >= 1 && j0 + FD_ROWS <= ny - 1;
  if (interior) {
    const long long q0 = (long long)j0 * nx + i;
    double u[FD_ROWS + 2], uw[FD_ROWS], ue[FD_ROWS], w[5 + HK + NS][FD_ROWS];
#pragma unroll
    for (int r = 0; r < FD_ROWS + 2; ++r) u[r] = U[q0 + (long long)(r - 1) * nx];
#pragma unroll
    for (int r = 0; r < FD_ROWS; ++r) {
      uw[r] = U[q0 + (long long)r * nx - 1];
      ue[r] = U[q0 + (long long)r * nx + 1];
    }
#pragma unroll
    for (int p = 0; p < 5 + HK + NS; ++p) {
      const int plane = p < 5 + HK ? p : p + (1 - HK);  // skip the K plane when unused
#pragma unroll
      for (int r = 0; r < FD_ROWS; ++r) w[p][r] = a.W[plane * P + q0 + (long long)r * nx];
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < FD_ROWS; ++r) {
      // fixed order: own value and constant sources, south, north, west, east, then the
      // time-dependent sources
      double k0 = 0.0;
      if constexpr (HK != 0) k0 = w[5][r];
      double acc = fma(w[0][r], u[r + 1], k0);
      acc = fma(w[1][r], u[r], acc);
      acc = fma(w[2][r], u[r + 2], acc);
      acc = fma(w[3][r], uw[r], acc);
      acc = fma(w[4][r], ue[r], acc);
#pragma unroll
      for (int s = 0; s < NS; ++s) acc = fma(T[s], w[5 + HK + s][r], acc);
      V[q0 + (long long)r * nx] = acc;
      bad = bad || !isfinite(acc);
    }
    if (bad) atomicOr(a.flag, 1);
    return;
  }
  if (i >= nx || j0 >= ny) return;
  const bool col_bnd = !a.periodic && (i == 0 || i == nx - 1);
  const int iw = i == 0 ? nx - 1 : i - 1;  // the wrap only matters on a periodic xi axis
  const int ie = i == nx - 1 ? 0 : i + 1;
  double us = j0 > 0 ? U[(long long)(j0 - 1) * nx + i] : 0.0;
  double uc = U[(long long)j0 * nx + i];
  bool bad = false;
  for (int r = 0; r < FD_ROWS; ++r) {
    const int j = j0 + r;
    if (j >= ny) break;
    const long long q = (long long)j * nx + i;
    const double un = j + 1 < ny ? U[q + nx] : 0.0;
    double out;
    if (j == 0 || j == ny - 1 || col_bnd) {
      // Dirichlet node: its index in boundary_node's order
      const int b = j == 0 ? i : (j == ny - 1 ? nx + i : 2 * nx + 2 * (j - 1) + (i == 0 ? 0 : 1));
      out = a.bvals[(long long)k * a.nb + b];
    } else {
      const double uw = U[(long long)j * nx + iw], ue = U[(long long)j * nx + ie];
      double acc = fma(a.W[q], uc, HK ? a.W[5 * P + q] : 0.0);
      acc = fma(a.W[P + q], us, acc);
      acc = fma(a.W[2 * P + q], un, acc);
      acc = fma(a.W[3 * P + q], uw, acc);
      acc = fma(a.W[4 * P + q], ue, acc);
#pragma unroll
      for (int s = 0; s < NS; ++s) acc = fma(T[s], a.W[(6 + s) * P + q], acc);
      out = acc;
      bad = bad || !isfinite(acc);
    }
    V[q] = out;
    us = uc;
    uc = un;
  }
  if (bad) atomicOr(a.flag, 1);
}

}  // namespace

hipError_t launch_fd_step(const FdArgs& a, const double* U, double* V, int k, hipStream_t s) {
  const dim3 grid((a.n_x + 63) / 64, (a.n_y + FD_GROUPS * FD_ROWS - 1) / (FD_GROUPS * FD_ROWS));
  const dim3 block(64 * FD_GROUPS);
#define PD_FD_LAUNCH(NS_, HK_)                                                 \
  if (a.ns == NS_ && (a.has_k != 0) == (HK_ != 0)) {                          \
    hipLaunchKernelGGL((k_fd_step<NS_, HK_>), grid, block, 0, s, a, U, V, k); \
    return hipGetLastError();                                                  \
  }
  PD_FD_LAUNCH(0, 0) PD_FD_LAUNCH(1, 0) PD_FD_LAUNCH(2, 0)
  PD_FD_LAUNCH(0, 1) PD_FD_LAUNCH(1, 1) PD_FD_LAUNCH(2, 1)
#undef PD_FD_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace pdk
