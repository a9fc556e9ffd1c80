// Stage-by-stage kernels of one macro step (Sec. 3.3): lifting and edge data, the
// trapezoidal restriction and the projective update.  The fused hot path does the same
// work inside the burst kernel; these exist so that each step can be checked on its own.
#include "pd_internal.h"
#include "pd_refresh.h"

namespace pdk {
namespace {

// eq. (edge) gradient of edge e (0: xi-, 1: xi+, 2: eta-, 3: eta+) at micro index q from
// the deviations d[b][a] = U(i+a-1, j+b-1) - U(i, j) (the weights sum to zero).
__device__ double edge_value(const double* tab, const TabOff& to, const double (&d)[3][3],
                             int e, int q, double Dxi, double Deta) {
  const double* ew = tab + to.ew + 3 * e;
  double P[3];
  if (e < 2) {
    const double* L = tab + to.L_xe + 3 * q;
    for (int a = 0; a < 3; ++a) P[a] = L[0] * d[0][a] + L[1] * d[1][a] + L[2] * d[2][a];
    return (ew[0] * P[0] + ew[1] * P[1] + ew[2] * P[2]) / Dxi;
  }
  const double* L = tab + to.L_ee + 3 * q;
  for (int b = 0; b < 3; ++b) P[b] = L[0] * d[b][0] + L[1] * d[b][1] + L[2] * d[b][2];
  return (ew[0] * P[0] + ew[1] * P[1] + ew[2] * P[2]) / Deta;
}

__device__ void load_devs(const int* pmap, const double* U, int p, double& c,
                          double (&d)[3][3]) {
  const int* pm = pmap + 11 * p;
  c = U[pm[6]];
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a) d[b][a] = U[pm[2 + 3 * b + a]] - c;
}

// Steps (i)-(ii): one thread per micro point writes the lifted value (unless state is
// null: edge data only); threads with q < 4 M also write one edge value.
__global__ void k_lift_bc(Geo g, const int* __restrict__ pmap, const double* __restrict__ tab,
                          const double* __restrict__ U, double* __restrict__ state,
                          double* __restrict__ edge) {
  const int p = blockIdx.x;
  if (p >= g.P) return;
  const int mx = g.m_xi, me = g.m_eta, pm = mx * me;
  const TabOff to = tab_off(mx, me);
  double c, d[3][3];
  load_devs(pmap, U, p, c, d);
  const double Ux = (d[1][2] - d[1][0]) / (2.0 * g.Dxi);
  const double Ue = (d[2][1] - d[0][1]) / (2.0 * g.Deta);
  const double Uxx = (d[1][2] + d[1][0]) / (g.Dxi * g.Dxi);
  const double Uee = (d[2][1] + d[0][1]) / (g.Deta * g.Deta);
  const double Uxe = (d[2][2] - d[0][2] - d[2][0] + d[0][0]) / (4.0 * g.Dxi * g.Deta);
  const double c0d = -g.kap_xi * Uxx - g.kap_eta * Uee;
  for (int q = threadIdx.x; state != nullptr && q < pm; q += blockDim.x) {
    const int l = q / mx, k = q - l * mx;
    const double s = tab[to.s_xi + k], t = tab[to.s_eta + l];
    const double w = c0d + s * Ux + t * Ue + 0.5 * s * s * Uxx + s * t * Uxe + 0.5 * t * t * Uee;
    state[(long long)p * pm + q] = c + w;
  }
  for (int q = threadIdx.x; q < 4 * g.M; q += blockDim.x) {
    const int e = q / g.M, idx = q - e * g.M;
    const int len = e < 2 ? me : mx;
    edge[(long long)p * 4 * g.M + q] =
        idx < len ? edge_value(tab, to, d, e, idx, g.Dxi, g.Deta) : 0.0;
  }
}

// Step (iv): composite trapezoidal average over the patch's core (the whole patch by
// default), rows first then the row sums (each in index order).  One wave per patch:
// lane l sums row l, lane 0 then sums the rows.
constexpr int RS_WAVES = 4;
__global__ __launch_bounds__(64 * RS_WAVES) void k_restrict(Geo g,
                                                           const double* __restrict__ state,
                                                           double* __restrict__ Ubar) {
  __shared__ double rows[RS_WAVES][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = blockIdx.x * RS_WAVES + w;
  if (p < g.P && lane >= g.ls && lane < g.ls + g.nls)
    rows[w][lane] = restriction_row(g, state, p, lane);
  __syncthreads();
  if (p < g.P && lane == 0) Ubar[p] = restriction_total(g, rows[w]);
}

// Steps (v)-(vi) at the patch nodes.
__global__ void k_macro_update(Geo g, const int* __restrict__ pmap, const double* __restrict__ U,
                               const double* __restrict__ Ubar, double* __restrict__ Unew,
                               double dt_macro, double tau, int* flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  const int node = pmap[11 * p + 6];
  const double v = projective_value(U[node], Ubar[p], dt_macro, tau);
  Unew[node] = v;
  if (!isfinite(v)) atomicOr(flag, 1);
}

// The macro field of a refresh inside a burst: each patch node takes its patch's current
// restriction (boundary nodes are written separately).
__global__ void k_scatter_patch_values(Geo g, const int* __restrict__ pmap,
                                       const double* __restrict__ Ubar, double* __restrict__ U) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  U[pmap[11 * p + 6]] = Ubar[p];
}

}  // namespace

hipError_t launch_scatter_patch_values(const Geo& g, const int* pmap, const double* Ubar,
                                       double* U, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_patch_values, dim3((g.P + 127) / 128), dim3(128), 0, s, g, pmap,
                     Ubar, U);
  return hipGetLastError();
}

hipError_t launch_lift_bc(const Geo& g, const int* pmap, const double* tab, const double* U,
                          double* state, double* edge, hipStream_t s) {
  hipLaunchKernelGGL(k_lift_bc, dim3(g.P), dim3(128), 0, s, g, pmap, tab, U, state, edge);
  return hipGetLastError();
}

hipError_t launch_restrict(const Geo& g, const double* state, double* Ubar, hipStream_t s) {
  hipLaunchKernelGGL(k_restrict, dim3((g.P + RS_WAVES - 1) / RS_WAVES), dim3(64 * RS_WAVES), 0,
                     s, g, state, Ubar);
  return hipGetLastError();
}

hipError_t launch_macro_update(const Geo& g, const int* pmap, const double* U,
                               const double* Ubar, double* Unew, double dt_macro, double tau,
                               int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_macro_update, dim3((g.P + 127) / 128), dim3(128), 0, s, g, pmap, U,
                     Ubar, Unew, dt_macro, tau, flag);
  return hipGetLastError();
}

}  // namespace pdk
