// ADI micro burst (Sec. 4.1.1 runs the micro simulation with an alternating-direction
// implicit scheme, n_t = 2): Peaceman-Rachford splitting of the bursts' micro operator
//   L u = alpha d2_xi u + gamma d2_eta u - nu d_xi u - omega d_eta u + phi u + s(t)
// into L_xi = alpha d2_xi - nu d_xi + phi/2 and L_eta = gamma d2_eta - omega d_eta + phi/2
// (the Neumann edge data through ghost points, as in the explicit burst), the source at
// the half step:
//   (I - dt/2 L_xi)  u*      = (I + dt/2 L_eta) u^n + dt/2 s(t + dt/2)
//   (I - dt/2 L_eta) u^{n+1} = (I + dt/2 L_xi)  u*  + dt/2 s(t + dt/2).
// One wave per patch, the patch in LDS; lane l solves row l of the first half step and
// lane k column k of the second by the Thomas algorithm (the ghost-point rows stay
// tridiagonal: the ghost folds onto the neighbour inside the patch).
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
  int stage;  // coefficients and source planes staged in LDS
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

__global__ __launch_bounds__(64) void k_burst_adi(AdiArgs A) {
  extern __shared__ __align__(16) double lds[];
  const int mx = A.g.m_xi, me = A.g.m_eta, M = A.g.M;
  const int pm = mx * me, line = mx > me ? mx : me;
  // patch slot and line of this lane (A.ppb patches per wave, `line` lanes each)
  const int slot = threadIdx.x / line, lane = threadIdx.x - slot * line;
  const long long p = (long long)blockIdx.x * A.ppb + slot;
  const bool live = slot < A.ppb && p < A.g.P;
  const int nsp = A.src.nconst + A.src.ns;  // source planes
  const int per = (4 + (A.stage ? 5 + nsp : 0)) * pm + 4 * M;
  double* u = lds + (long long)(slot < A.ppb ? slot : 0) * per;  // [me][mx] u^n, u^{n+1}
  double* us = u + pm;                                            // u*
  double* cp = us + pm;                                           // Thomas scratch
  double* dp = cp + pm;
  double* eg = dp + pm;     // edge data [4][M]
  double* cs = eg + 4 * M;  // staged alpha, gamma, nu, omega, phi, source planes
  const double dx = A.g.dxi, de = A.g.deta;
  const bool central = A.g.conv == PD_CONV_CENTRAL;
  const double h = 0.5 * A.dt;
  const long long P = A.plane;
  const long long pp = live ? p : 0;
  const double* Cg = A.coef + pp * pm;
  const double* gxm = eg;
  const double* gxp = eg + M;
  const double* gem = eg + 2 * M;
  const double* gep = eg + 3 * M;
  double* st = A.state + pp * pm;
  if (live) {
    for (int q = lane; q < pm; q += line) u[q] = st[q];
    for (int q = lane; q < 4 * M; q += line) eg[q] = A.edge[pp * 4 * M + q];
    if (A.stage) {
      for (int f = 0; f < 5; ++f)
        for (int q = lane; q < pm; q += line) cs[f * pm + q] = Cg[f * P + q];
      for (int c = 0; c < A.src.nconst; ++c)
        for (int q = lane; q < pm; q += line) cs[(5 + c) * pm + q] = Cg[A.src.plane_c[c] * P + q];
      for (int j = 0; j < A.src.ns; ++j)
        for (int q = lane; q < pm; q += line)
          cs[(5 + A.src.nconst + j) * pm + q] = Cg[A.src.plane_t[j] * P + q];
    }
  }
  __syncthreads();
  // coefficient f at point `at`: from LDS when staged, else from the planes
  auto cf = [&](int f, int at) { return A.stage ? cs[f * pm + at] : Cg[f * P + at]; };
  bool bad = false;
  for (int s = 0; s < A.n_t; ++s) {
    const double th = A.t_n + s * A.dt + 0.5 * A.dt;
    double T[2] = {0.0, 0.0};
    for (int j = 0; j < A.src.ns; ++j) T[j] = time_factor(A.src, j, th);
    auto source = [&](int at) {
      double v = 0.0;
      if (A.stage) {
        for (int c = 0; c < A.src.nconst; ++c) v += A.src.ca[c] * cs[(5 + c) * pm + at];
        for (int j = 0; j < A.src.ns; ++j) v += T[j] * cs[(5 + A.src.nconst + j) * pm + at];
      } else {
        for (int c = 0; c < A.src.nconst; ++c) v += A.src.ca[c] * Cg[A.src.plane_c[c] * P + at];
        for (int j = 0; j < A.src.ns; ++j) v += T[j] * Cg[A.src.plane_t[j] * P + at];
      }
      return v;
    };
    // first half step: lane l, row l, implicit in xi
    if (live && lane < me) {
      const int l = lane;
      double* c_ = cp + lane * mx;
      double* d_ = dp + lane * mx;
      for (int k = 0; k < mx; ++k) {
        const int at = l * mx + k;
        const double ga = cf(1, at), om = cf(3, at), ph = cf(4, at);
        double wm, wp;
        dir_weights(ga, om, de, central, wm, wp);
        const double uc = u[at];
        const double uS = l > 0 ? u[at - mx] : u[at + mx] - 2.0 * de * gem[k];
        const double uN = l < me - 1 ? u[at + mx] : u[at - mx] + 2.0 * de * gep[k];
        const double Le = wm * uS + wp * uN - (wm + wp - 0.5 * ph) * uc;
        const double r = uc + h * Le + h * source(at);
        const double al = cf(0, at), nu = cf(2, at);
        double am, ap;
        dir_weights(al, nu, dx, central, am, ap);
        // row k of (I - h L_xi): lo x_{k-1} + di x_k + up x_{k+1} = r + h cst
        double lo = -h * am, up = -h * ap, cst = 0.0;
        const double di = 1.0 + h * (am + ap - 0.5 * ph);
        if (k == 0) {  // x_{-1} = x_1 - 2 dx g-
          up += lo;
          cst = -2.0 * dx * gxm[l] * am;
          lo = 0.0;
        }
        if (k == mx - 1) {  // x_m = x_{m-2} + 2 dx g+
          lo += up;
          cst += 2.0 * dx * gxp[l] * ap;
          up = 0.0;
        }
        const double rhs = r + h * cst;
        if (k == 0) {
          c_[0] = up / di;
          d_[0] = rhs / di;
        } else {
          const double den = di - lo * c_[k - 1];
          c_[k] = up / den;
          d_[k] = (rhs - lo * d_[k - 1]) / den;
        }
      }
      double x = d_[mx - 1];
      us[l * mx + mx - 1] = x;
      for (int k = mx - 2; k >= 0; --k) {
        x = d_[k] - c_[k] * x;
        us[l * mx + k] = x;
      }
    }
    __syncthreads();
    // second half step: lane k, column k, implicit in eta
    if (live && lane < mx) {
      const int k = lane;
      double* c_ = cp + lane * me;
      double* d_ = dp + lane * me;
      for (int l = 0; l < me; ++l) {
        const int at = l * mx + k;
        const double al = cf(0, at), nu = cf(2, at), ph = cf(4, at);
        double am, ap;
        dir_weights(al, nu, dx, central, am, ap);
        const double uc = us[at];
        const double uW = k > 0 ? us[at - 1] : us[at + 1] - 2.0 * dx * gxm[l];
        const double uE = k < mx - 1 ? us[at + 1] : us[at - 1] + 2.0 * dx * gxp[l];
        const double Lx = am * uW + ap * uE - (am + ap - 0.5 * ph) * uc;
        const double r = uc + h * Lx + h * source(at);
        const double ga = cf(1, at), om = cf(3, at);
        double wm, wp;
        dir_weights(ga, om, de, central, wm, wp);
        double lo = -h * wm, up = -h * wp, cst = 0.0;
        const double di = 1.0 + h * (wm + wp - 0.5 * ph);
        if (l == 0) {
          up += lo;
          cst = -2.0 * de * gem[k] * wm;
          lo = 0.0;
        }
        if (l == me - 1) {
          lo += up;
          cst += 2.0 * de * gep[k] * wp;
          up = 0.0;
        }
        const double rhs = r + h * cst;
        if (l == 0) {
          c_[0] = up / di;
          d_[0] = rhs / di;
        } else {
          const double den = di - lo * c_[l - 1];
          c_[l] = up / den;
          d_[l] = (rhs - lo * d_[l - 1]) / den;
        }
      }
      double x = d_[me - 1];
      u[(me - 1) * mx + k] = x;
      bad = bad || !isfinite(x);
      for (int l = me - 2; l >= 0; --l) {
        x = d_[l] - c_[l] * x;
        u[l * mx + k] = x;
        bad = bad || !isfinite(x);
      }
    }
    __syncthreads();
  }
  if (live)
    for (int q = lane; q < pm; q += line) st[q] = u[q];
  if (bad) atomicOr(A.flag, 1);
}

}  // namespace

// Patches per wave and LDS bytes per block: with the coefficients staged when a patch's
// field, scratch and planes fit; ppb = 0 when not even one patch's field and scratch fit.
void adi_shape(int mx, int me, int nsp, int& ppb, int& stage, size_t& lds) {
  const int line = mx > me ? mx : me;
  const size_t pm = (size_t)mx * me;
  const int lanes = 64 / line;
  for (stage = 1; stage >= 0; --stage) {
    const size_t per = ((4 + (stage ? 5 + nsp : 0)) * pm + 4 * (size_t)line) * sizeof(double);
    ppb = (int)(ADI_LDS_MAX / per);
    if (ppb > lanes) ppb = lanes;
    if (ppb >= 1) {
      lds = ppb * per;
      return;
    }
  }
  ppb = 0;
  stage = 0;
  lds = 0;
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
  adi_shape(g.m_xi, g.m_eta, src.nconst + src.ns, a.ppb, a.stage, lds);
  if (a.ppb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_burst_adi, dim3((g.P + a.ppb - 1) / a.ppb), dim3(64), lds, s, a);
  return hipGetLastError();
}

}  // namespace pdk
