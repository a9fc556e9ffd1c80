// Explicit micro burst with the higher-order upwind first differences of Sec. 4.1.2
// (3-point second differences and forward Euler as in the 2-point burst):
//   3-point  d_p u_i = (3 u_i - 4 u_{i-1} + u_{i-2}) / (2 dp)
//   4-point  d_p u_i = (u_{i+1} - u_{i-1}) / (2 dp) + r / (3 dp) (u_{i-2} - 3 u_{i-1} + 3 u_i - u_{i+1})
// leaning on the upstream side where the velocity component is >= 0 and mirrored where it
// is < 0; points = 2 is the 2-point upwind difference.  The Neumann edge data enter
// through two ghost layers: u_{-1} = u_1 - 2 dp g-, u_{-2} = u_2 - 4 dp g- (and the
// mirror images above the last point).
//
// One block of 256 lanes holds several patches in LDS, each as a (m_xi + 4) x (m_eta + 4)
// tile with its ghost frame, twice (ping-pong).  Every lane owns up to four points and
// keeps their nine folded stencil weights (the 5-point cross along each direction, dt
// folded in) and the source planes in registers for the whole burst.  A lane writing an
// edge-near point also writes the ghost value that point determines, so one barrier per
// nano step suffices.  The tiles hold the increment v = u - u(0) since the lift (the
// scheme is linear): v' = v + dt L_h(v) + [dt L_h(u(0)) + dt s(t)], the lifted part of the
// bracket computed once per point, the ghosts of v homogeneous (v_{-1} = v_1,
// v_{-2} = v_2).  Rounding then acts on |v| ~ tau |F|, not on |u|, which keeps the
// restricted rate (R(u(tau)) - U) / tau accurate for the projective step.
#include "pd_internal.h"

namespace pdk {
namespace {

constexpr int HU_THREADS = 256;
constexpr int HU_PPT = 4;  // points per lane
constexpr int HU_TCH = 256;  // steps per chunk of the source time-factor table

struct HuArgs {
  Geo g;
  SrcInfo src;
  const double* coef;  // [5 + n_src][P][m_eta][m_xi]
  long long plane;
  double* state;       // [P][m_eta][m_xi] in/out
  const double* edge;  // [P][4][M]
  double t_n, dt, r;
  int n_t, points;
  int ppb;             // patches per block
  int* flag;
};

// Coefficients of the upstream-leaning first difference at offsets -2..+2 for a
// non-negative velocity component; the other side is the mirror image c[j] -> -c[-j].
__device__ inline void upwind_coeffs(int points, double r, double d, double c[5]) {
  for (int j = 0; j < 5; ++j) c[j] = 0.0;
  if (points == 2) {
    c[1] = -1.0 / d;
    c[2] = 1.0 / d;
  } else if (points == 3) {
    c[0] = 1.0 / (2.0 * d);
    c[1] = -4.0 / (2.0 * d);
    c[2] = 3.0 / (2.0 * d);
  } else {
    c[0] = r / (3.0 * d);
    c[1] = -1.0 / (2.0 * d) - r / d;
    c[2] = r / d;
    c[3] = 1.0 / (2.0 * d) - r / (3.0 * d);
  }
}

// Weights of u at offsets -2..+2 along one direction for dt (a d2 - b d1), the centre
// entry without the 1 and the reaction.
__device__ inline void dir_stencil(double a, double b, double d, int points, double r,
                                   double dt, double w[5]) {
  double c[5];
  upwind_coeffs(points, r, d, c);
  if (b < 0.0) {
    for (int j = 0; j < 2; ++j) {
      const double t = c[j];
      c[j] = -c[4 - j];
      c[4 - j] = -t;
    }
    c[2] = -c[2];
  }
  const double d2 = a / (d * d);
  for (int j = 0; j < 5; ++j) w[j] = -b * c[j];
  w[1] += d2;
  w[3] += d2;
  w[2] -= 2.0 * d2;
  for (int j = 0; j < 5; ++j) w[j] *= dt;
}

__global__ __launch_bounds__(HU_THREADS) void k_burst_hu(HuArgs A) {
  extern __shared__ __align__(16) double lds[];
  const int mx = A.g.m_xi, me = A.g.m_eta, M = A.g.M;
  const int pm = mx * me, W = mx + 4, ext = W * (me + 4);
  const int per = 2 * ext + 4 * M;  // two tiles with ghost frames, edge data
  double* ttab = lds + A.ppb * per;  // source time factors of HU_TCH steps, [j][step]
  const long long p0 = (long long)blockIdx.x * A.ppb;
  const int npts = A.ppb * pm;
  const double dx = A.g.dxi, de = A.g.deta, dt = A.dt;
  const long long P = A.plane;
  // the patches' fields into the first tile, the edge data after the second
  for (int q = threadIdx.x; q < npts; q += HU_THREADS) {
    const int sl = q / pm, at = q - sl * pm;
    if (p0 + sl >= A.g.P) continue;
    const int l = at / mx, k = at - l * mx;
    lds[sl * per + (l + 2) * W + k + 2] = A.state[(p0 + sl) * pm + at];
  }
  for (int q = threadIdx.x; q < A.ppb * 4 * M; q += HU_THREADS) {
    const int sl = q / (4 * M), e = q - sl * 4 * M;
    if (p0 + sl < A.g.P) lds[sl * per + 2 * ext + e] = A.edge[(p0 + sl) * 4 * M + e];
  }
  // The owned points: weights, tile offset, and the offsets (relative to the point) of
  // the ghost values it determines (0: none; a write of the point's own value to itself).
  // Lanes without a point compute on slot 0's first point with zero weights and store
  // nothing.
  bool ok[HU_PPT];
  int off[HU_PPT], gx[HU_PPT][2], ge[HU_PPT][2];
  double w[HU_PPT][9], sc[HU_PPT], st[HU_PPT][2], gc[HU_PPT];
#pragma unroll
  for (int i = 0; i < HU_PPT; ++i) {
    const int q = threadIdx.x + i * HU_THREADS;
    const int sl = q / pm, at = q - sl * pm;
    ok[i] = q < npts && p0 + sl < A.g.P;
    const int l = ok[i] ? at / mx : 0, k = ok[i] ? at - l * mx : 0;
    off[i] = (ok[i] ? sl * per : 0) + (l + 2) * W + k + 2;
    sc[i] = gc[i] = 0.0;
    st[i][0] = st[i][1] = 0.0;
    for (int j = 0; j < 9; ++j) w[i][j] = 0.0;
    gx[i][0] = gx[i][1] = ge[i][0] = ge[i][1] = 0;
    if (!ok[i]) continue;
    // a point can feed a ghost on each side of a direction only when that side has at
    // most 5 points
    const int xl = k == 1 ? -2 : k == 2 ? -4 : 0, xh = k == mx - 2 ? 2 : k == mx - 3 ? 4 : 0;
    const int el = l == 1 ? -2 * W : l == 2 ? -4 * W : 0;
    const int eh = l == me - 2 ? 2 * W : l == me - 3 ? 4 * W : 0;
    gx[i][0] = xl ? xl : xh;
    gx[i][1] = xl ? xh : 0;
    ge[i][0] = el ? el : eh;
    ge[i][1] = el ? eh : 0;
    const double* Cs = A.coef + (p0 + sl) * pm + at;
    double wx[5], we[5];
    dir_stencil(Cs[0], Cs[2 * P], dx, A.points, A.r, dt, wx);
    dir_stencil(Cs[P], Cs[3 * P], de, A.points, A.r, dt, we);
    w[i][0] = wx[2] + we[2] + dt * Cs[4 * P];
    w[i][1] = wx[0];  // k - 2
    w[i][2] = wx[1];  // k - 1
    w[i][3] = wx[3];  // k + 1
    w[i][4] = wx[4];  // k + 2
    w[i][5] = we[0];  // l - 2
    w[i][6] = we[1];
    w[i][7] = we[3];
    w[i][8] = we[4];
    for (int c = 0; c < A.src.nconst; ++c) sc[i] += A.src.ca[c] * Cs[A.src.plane_c[c] * P];
    for (int j = 0; j < A.src.ns; ++j) st[i][j] = Cs[A.src.plane_t[j] * P];
  }
  // dt L_h applied to tile t around owned point i (no source); c0 the point's own value
  auto apply = [&](int i, const double* t, double& c0) {
    const double* c = t + off[i];
    c0 = c[0];
    double a = w[i][0] * c0;
    a = fma(w[i][1], c[-2], a);
    a = fma(w[i][2], c[-1], a);
    a = fma(w[i][3], c[1], a);
    a = fma(w[i][4], c[2], a);
    a = fma(w[i][5], c[-2 * W], a);
    a = fma(w[i][6], c[-W], a);
    a = fma(w[i][7], c[W], a);
    a = fma(w[i][8], c[2 * W], a);
    return a;
  };
  auto put = [&](int i, double* t, double v) {
    double* c = t + off[i];
    c[0] = v;
    c[gx[i][0]] = v;
    c[ge[i][0]] = v;
    if (mx < 6) c[gx[i][1]] = v;
    if (me < 6) c[ge[i][1]] = v;
  };
  __syncthreads();
  // K0 = dt L_h(u(0)) from the lifted tile with its edge-data ghosts, then v = 0
#pragma unroll
  for (int i = 0; i < HU_PPT; ++i) {
    if (!ok[i]) continue;
    const int q = threadIdx.x + i * HU_THREADS;
    const int sl = q / pm, at = q - sl * pm;
    const int l = at / mx, k = at - l * mx, o = off[i];
    const double* eg = lds + sl * per + 2 * ext;
    const double v = lds[o];
    if (k == 1) lds[o - 2] = v - 2.0 * dx * eg[l];
    if (k == 2) lds[o - 4] = v - 4.0 * dx * eg[l];
    if (k == mx - 2) lds[o + 2] = v + 2.0 * dx * eg[M + l];
    if (k == mx - 3) lds[o + 4] = v + 4.0 * dx * eg[M + l];
    if (l == 1) lds[o - 2 * W] = v - 2.0 * de * eg[2 * M + k];
    if (l == 2) lds[o - 4 * W] = v - 4.0 * de * eg[2 * M + k];
    if (l == me - 2) lds[o + 2 * W] = v + 2.0 * de * eg[3 * M + k];
    if (l == me - 3) lds[o + 4 * W] = v + 4.0 * de * eg[3 * M + k];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < HU_PPT; ++i) {
    double c0;
    gc[i] = ok[i] ? apply(i, lds, c0) : 0.0;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < A.ppb * ext; q += HU_THREADS) {
    const int sl = q / ext;
    lds[sl * per + (q - sl * ext)] = 0.0;
  }
  int cur = 0;
  for (int s = 0; s < A.n_t; ++s) {
    const int sc_ = s % HU_TCH;
    if (sc_ == 0) {  // the next chunk of source time factors, one step per lane
      __syncthreads();
      const int st_ = s + threadIdx.x;
      if (threadIdx.x < HU_TCH && st_ < A.n_t)
        for (int j = 0; j < A.src.ns; ++j)
          ttab[j * HU_TCH + threadIdx.x] = time_factor(A.src, j, A.t_n + st_ * dt);
    }
    __syncthreads();
    const double T0 = A.src.ns > 0 ? ttab[sc_] : 0.0;
    const double T1 = A.src.ns > 1 ? ttab[HU_TCH + sc_] : 0.0;
    const double* u = lds + cur;
    double* nx = lds + (ext - cur);
    double vn[HU_PPT];
#pragma unroll
    for (int i = 0; i < HU_PPT; ++i) {
      double c0;
      const double a = apply(i, u, c0);
      vn[i] = c0 + (a + fma(dt, fma(T1, st[i][1], fma(T0, st[i][0], sc[i])), gc[i]));
    }
#pragma unroll
    for (int i = 0; i < HU_PPT; ++i)
      if (ok[i]) put(i, nx, vn[i]);
    cur = ext - cur;
  }
  __syncthreads();
  bool bad = false;
#pragma unroll
  for (int i = 0; i < HU_PPT; ++i) {
    if (!ok[i]) continue;
    const int q = threadIdx.x + i * HU_THREADS;
    const int sl = q / pm, at = q - sl * pm;
    double* sp = A.state + (p0 + sl) * pm + at;
    const double v = *sp + lds[cur + off[i]];
    *sp = v;
    bad = bad || !isfinite(v);
  }
  if (bad) atomicOr(A.flag, 1);
}

}  // namespace

// Patches per block (at most 1024 points per block, the tiles within HU_LDS_MAX) and LDS
// bytes per block; ppb = 0 when not even one patch fits.
void hu_shape(int mx, int me, int& ppb, size_t& lds) {
  const int M = mx > me ? mx : me;
  const size_t per = (2 * (size_t)(mx + 4) * (me + 4) + 4 * (size_t)M) * sizeof(double);
  const int pm = mx * me;
  const size_t tab = 2 * HU_TCH * sizeof(double);
  ppb = pm > 0 ? HU_THREADS * HU_PPT / pm : 0;
  if ((size_t)ppb * per + tab > HU_LDS_MAX) ppb = (int)((HU_LDS_MAX - tab) / per);
  if (mx < 3 || me < 3) ppb = 0;
  lds = ppb > 0 ? ppb * per + tab : 0;
}

hipError_t launch_burst_hu(const Geo& g, const SrcInfo& src, const double* coef,
                           long long plane, double* state, const double* edge, double t_n,
                           double dt, int n_t, int points, double r, int* flag,
                           hipStream_t s) {
  HuArgs a{};
  a.g = g;
  a.src = src;
  a.coef = coef;
  a.plane = plane;
  a.state = state;
  a.edge = edge;
  a.t_n = t_n;
  a.dt = dt;
  a.r = r;
  a.n_t = n_t;
  a.points = points;
  a.flag = flag;
  size_t lds = 0;
  hu_shape(g.m_xi, g.m_eta, a.ppb, lds);
  if (a.ppb < 1 || points < 2 || points > 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_burst_hu, dim3((g.P + a.ppb - 1) / a.ppb), dim3(HU_THREADS), lds, s,
                     a);
  return hipGetLastError();
}

}  // namespace pdk
