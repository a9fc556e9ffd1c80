// ADI micro burst (Sec. 4.1.1 runs the micro simulation with an alternating-direction
// implicit scheme, n_t = 2): Peaceman-Rachford splitting of the bursts' micro operator
//   L u = alpha d2_xi u + gamma d2_eta u - nu d_xi u - omega d_eta u + phi u + s(t)
// into L_xi = alpha d2_xi - nu d_xi + phi/2 and L_eta = gamma d2_eta - omega d_eta + phi/2
// (the Neumann edge data through ghost points, as in the explicit burst), the source at
// the half step:
//   (I - dt/2 L_xi)  u*      = (I + dt/2 L_eta) u^n + dt/2 s(t + dt/2)
//   (I - dt/2 L_eta) u^{n+1} = (I + dt/2 L_xi)  u*  + dt/2 s(t + dt/2).
// One wave holds several patches in LDS.  Each half step first assembles the tridiagonal
// rows and right-hand sides of every point (all lanes), then lane l eliminates row l (first
// half) or lane k column k (second half) by the Thomas algorithm, the carried factors in
// registers (the ghost-point rows stay tridiagonal: the ghost folds onto the neighbour
// inside the patch).
#include "pd_internal.h"

namespace pdk {
namespace {

struct AdiArgs {
  Geo g;
  SrcInfo src;
  const double* coef;  // [5 + n_src][P][m_eta][m_xi]
  long long plane;
  double* state;       // [P][m_eta][m_xi] in/out
  const double* edge;  // [P][4][M]
  double t_n, dt;
  int n_t;
  int ppb;    // patches per wave
  int* flag;
};

// Neighbour weights of one direction: L x = wm x_- + wp x_+ - (wm + wp - phi/2) x for the
// 3-point second difference (a) and the upwind or central first difference (b).
__device__ inline void dir_weights(double a, double b, double d, bool central, double& wm,
                                   double& wp) {
  const double d2 = a / (d * d);
  if (central) {
    wm = d2 + b / (2.0 * d);
    wp = d2 - b / (2.0 * d);
  } else {
    wm = d2 + (b >= 0.0 ? b / d : 0.0);
    wp = d2 + (b < 0.0 ? -b / d : 0.0);
  }
}

// Row i of (I - h L) along one line for the point at `at`: lo x_{i-1} + di x_i +
// up x_{i+1} = rhs, with the ghost point folded at the line's ends (first, last).
__device__ inline void line_row(double am, double ap, double ph, double h, double r,
                                bool first, bool last, double gfirst, double glast, double d,
                                double& lo, double& di, double& up, double& rhs) {
  lo = -h * am;
  up = -h * ap;
  di = 1.0 + h * (am + ap - 0.5 * ph);
  double cst = 0.0;
  if (first) {  // x_{-1} = x_1 - 2 d g-
    up += lo;
    cst = -2.0 * d * gfirst * am;
    lo = 0.0;
  }
  if (last) {  // x_m = x_{m-2} + 2 d g+
    lo += up;
    cst += 2.0 * d * glast * ap;
    up = 0.0;
  }
  rhs = r + h * cst;
}

// Thomas elimination of one line of n entries with stride `sd` in the row arrays (lo, di,
// up, rh; up and rh are overwritten by the eliminated factors), solution into x.
__device__ inline void thomas_line(const double* lo, const double* di, double* up, double* rh,
                                   double* x, int n, int sd) {
  double c = up[0] / di[0], dd = rh[0] / di[0];
  up[0] = c;
  rh[0] = dd;
  for (int i = 1; i < n; ++i) {
    const int at = i * sd;
    const double l_ = lo[at], den = di[at] - l_ * c;
    c = up[at] / den;
    dd = (rh[at] - l_ * dd) / den;
    up[at] = c;
    rh[at] = dd;
  }
  double v = dd;
  x[(n - 1) * sd] = v;
  for (int i = n - 2; i >= 0; --i) {
    v = rh[i * sd] - up[i * sd] * v;
    x[i * sd] = v;
  }
}

__global__ __launch_bounds__(64) void k_burst_adi(AdiArgs A) {
  extern __shared__ __align__(16) double lds[];
  const int mx = A.g.m_xi, me = A.g.m_eta, M = A.g.M;
  const int pm = mx * me, line = mx > me ? mx : me;
  const int per = 6 * pm + 4 * M;  // u, u*, lo, di, up, rhs, edge data
  const int slot = threadIdx.x / line, lane = threadIdx.x - slot * line;
  const long long p0 = (long long)blockIdx.x * A.ppb;
  const bool live = slot < A.ppb && p0 + slot < A.g.P;
  const double dx = A.g.dxi, de = A.g.deta;
  const bool central = A.g.conv == PD_CONV_CENTRAL;
  const double h = 0.5 * A.dt;
  const long long P = A.plane;
  const int npts = A.ppb * pm;
  // the patches' fields and edge data into LDS
  for (int q = threadIdx.x; q < npts; q += 64) {
    const int sl = q / pm, at = q - sl * pm;
    if (p0 + sl < A.g.P) lds[sl * per + at] = A.state[(p0 + sl) * pm + at];
  }
  for (int q = threadIdx.x; q < A.ppb * 4 * M; q += 64) {
    const int sl = q / (4 * M), e = q - sl * 4 * M;
    if (p0 + sl < A.g.P) lds[sl * per + 6 * pm + e] = A.edge[(p0 + sl) * 4 * M + e];
  }
  __syncthreads();
  bool bad = false;
  for (int s = 0; s < A.n_t; ++s) {
    const double th = A.t_n + s * A.dt + 0.5 * A.dt;
    double T[2] = {0.0, 0.0};
    for (int j = 0; j < A.src.ns; ++j) T[j] = time_factor(A.src, j, th);
    for (int half = 0; half < 2; ++half) {
      // assembly: every point of every patch of the block (all lanes busy)
      for (int q = threadIdx.x; q < npts; q += 64) {
        const int sl = q / pm, at = q - sl * pm;
        if (p0 + sl >= A.g.P) continue;
        double* b = lds + sl * per;
        const double* src = half == 0 ? b : b + pm;  // u^n, then u*
        const double* eg = b + 6 * pm;
        const double* Cs = A.coef + (p0 + sl) * pm;
        const int l = at / mx, k = at - l * mx;
        const double al = Cs[at], ga = Cs[P + at], nu = Cs[2 * P + at], om = Cs[3 * P + at],
                     ph = Cs[4 * P + at];
        double sv = 0.0;
        for (int c = 0; c < A.src.nconst; ++c) sv += A.src.ca[c] * Cs[A.src.plane_c[c] * P + at];
        for (int j = 0; j < A.src.ns; ++j) sv += T[j] * Cs[A.src.plane_t[j] * P + at];
        double am, ap, wm, wp;
        dir_weights(al, nu, dx, central, am, ap);
        dir_weights(ga, om, de, central, wm, wp);
        const double uc = src[at];
        double lo, di, up, rhs;
        if (half == 0) {  // explicit in eta, implicit in xi along row l
          const double uS = l > 0 ? src[at - mx] : src[at + mx] - 2.0 * de * eg[2 * M + k];
          const double uN = l < me - 1 ? src[at + mx] : src[at - mx] + 2.0 * de * eg[3 * M + k];
          const double r = uc + h * (wm * uS + wp * uN - (wm + wp - 0.5 * ph) * uc) + h * sv;
          line_row(am, ap, ph, h, r, k == 0, k == mx - 1, eg[l], eg[M + l], dx, lo, di, up, rhs);
        } else {  // explicit in xi, implicit in eta along column k
          const double uW = k > 0 ? src[at - 1] : src[at + 1] - 2.0 * dx * eg[l];
          const double uE = k < mx - 1 ? src[at + 1] : src[at - 1] + 2.0 * dx * eg[M + l];
          const double r = uc + h * (am * uW + ap * uE - (am + ap - 0.5 * ph) * uc) + h * sv;
          line_row(wm, wp, ph, h, r, l == 0, l == me - 1, eg[2 * M + k], eg[3 * M + k], de,
                   lo, di, up, rhs);
        }
        b[2 * pm + at] = lo;
        b[3 * pm + at] = di;
        b[4 * pm + at] = up;
        b[5 * pm + at] = rhs;
      }
      __syncthreads();
      // the serial part: one lane per line
      if (live) {
        double* b = lds + slot * per;
        if (half == 0 && lane < me) {
          const int o = lane * mx;
          thomas_line(b + 2 * pm + o, b + 3 * pm + o, b + 4 * pm + o, b + 5 * pm + o,
                      b + pm + o, mx, 1);
        } else if (half == 1 && lane < mx) {
          const int o = lane;
          thomas_line(b + 2 * pm + o, b + 3 * pm + o, b + 4 * pm + o, b + 5 * pm + o, b + o,
                      me, mx);
        }
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < npts; q += 64) {
    const int sl = q / pm, at = q - sl * pm;
    if (p0 + sl < A.g.P) {
      const double v = lds[sl * per + at];
      A.state[(p0 + sl) * pm + at] = v;
      bad = bad || !isfinite(v);
    }
  }
  if (bad) atomicOr(A.flag, 1);
}

}  // namespace

// Patches per wave and LDS bytes per block (6 m_xi m_eta + 4 max(m_xi, m_eta) doubles per
// patch); ppb = 0 when not even one patch fits.
void adi_shape(int mx, int me, int& ppb, size_t& lds) {
  const int line = mx > me ? mx : me;
  const size_t per = (6 * (size_t)mx * me + 4 * (size_t)line) * sizeof(double);
  ppb = (int)(ADI_LDS_MAX / per);
  if (ppb > 64 / line) ppb = 64 / line;
  lds = ppb > 0 ? ppb * per : 0;
}

hipError_t launch_burst_adi(const Geo& g, const SrcInfo& src, const double* coef,
                            long long plane, double* state, const double* edge, double t_n,
                            double dt, int n_t, int* flag, hipStream_t s) {
  AdiArgs a{};
  a.g = g;
  a.src = src;
  a.coef = coef;
  a.plane = plane;
  a.state = state;
  a.edge = edge;
  a.t_n = t_n;
  a.dt = dt;
  a.n_t = n_t;
  a.flag = flag;
  size_t lds = 0;
  adi_shape(g.m_xi, g.m_eta, a.ppb, lds);
  if (a.ppb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_burst_adi, dim3((g.P + a.ppb - 1) / a.ppb), dim3(64), lds, s, a);
  return hipGetLastError();
}

}  // namespace pdk
