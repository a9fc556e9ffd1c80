// ADI micro burst with the 2-, 3- or 4-point upwind first differences.  Sec. 4.1.2 runs
// its micro simulations with the alternating-direction implicit solver of Sec. 4.1.1 and
// tries the 3-point form (3 u_i - 4 u_{i-1} + u_{i-2}) / (2 dp) and the 4-point form
// (u_{i+1} - u_{i-1}) / (2 dp) + r/(3 dp) (u_{i-2} - 3 u_{i-1} + 3 u_i - u_{i+1}) in place
// of the 2-point one.  Peaceman-Rachford as in pd_adi.hip:
//   (I - dt/2 L_xi)  u*      = (I + dt/2 L_eta) u^n + dt/2 s(t + dt/2)
//   (I - dt/2 L_eta) u^{n+1} = (I + dt/2 L_xi)  u*  + dt/2 s(t + dt/2),
// L_xi = alpha d2_xi - nu d_xi + phi/2 with the chosen first difference (the printed form
// where the velocity component is >= 0, its mirror image where it is < 0) and the Neumann
// edge data through two ghost layers, u_{-1} = u_1 - 2 dp g-, u_{-2} = u_2 - 4 dp g-,
// u_m = u_{m-2} + 2 dp g+, u_{m+1} = u_{m-3} + 4 dp g+.  Folding the ghosts onto the points
// they mirror keeps every implicit line banded with two neighbours on each side.
//
// One wave holds several patches in LDS.  Each half step first assembles every point's
// five band entries and right-hand side (all lanes, coefficient planes from HBM), then
// lane l eliminates row l (first half) or lane k column k (second half): banded Gaussian
// elimination without pivoting, the two rows below the pivot row carried in registers,
// one reciprocal per row, then the back substitution.  Without pivoting the elimination
// is stable while every line matrix is diagonally dominant; for the 3-point form that
// holds when dt/2 (|nu| / d_xi + phi/2) <= 1 (likewise along eta), e.g. about 0.03 on the
// paper's Sec. 4.1.2 patches.
#include "pd_internal.h"

namespace pdk {

// LDS of one wave's patches (at most 64 KiB).
constexpr size_t ADU_LDS_MAX = 65536;

namespace {

struct AduArgs {
  Geo g;
  SrcInfo src;
  const double* coef;  // [5 + n_src][P][m_eta][m_xi]
  long long plane;
  double* state;       // [P][m_eta][m_xi] in/out
  const double* edge;  // [P][4][M]
  double t_n, dt, r;
  int n_t, points;
  int ppb;             // patches per wave
  int* flag;
};

// Per patch in LDS: u, u*, the five band planes (offsets -2..2), the right-hand sides,
// the edge data.
constexpr int ADU_PLANES = 8;

// Weights of L along one direction at offsets -2..2 (w[0] is offset -2): the 3-point
// second difference with diffusion a, minus velocity b times the first difference of the
// given form on the side the flow comes from, spacing d.  The reaction is added apart.
__device__ inline void dir_stencil(double a, double b, double d, int points, double r,
                                   double (&w)[5]) {
  const double d2 = a / (d * d);
  double c[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // first difference, backward side
  if (points == 2) {
    c[2] = 1.0 / d;
    c[1] = -1.0 / d;
  } else if (points == 3) {
    c[2] = 3.0 / (2.0 * d);
    c[1] = -4.0 / (2.0 * d);
    c[0] = 1.0 / (2.0 * d);
  } else {
    c[3] = 1.0 / (2.0 * d) - r / (3.0 * d);
    c[2] = r / d;
    c[1] = -1.0 / (2.0 * d) - r / d;
    c[0] = r / (3.0 * d);
  }
  const bool back = b >= 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double ck = back ? c[k] : -c[4 - k];  // forward side: the mirror image
    const double dk = (k == 1 || k == 3) ? d2 : (k == 2 ? -2.0 * d2 : 0.0);
    w[k] = dk - b * ck;
  }
}

// Point j of a line of n points, ghosts folded: index of the point it reads and the
// constant added to that point's value (edge gradients gm below, gp above, spacing d).
__device__ inline int fold(int j, int n, double d, double gm, double gp, double& cst) {
  if (j < 0) {
    cst = 2.0 * j * d * gm;
    return -j;
  }
  if (j > n - 1) {
    cst = 2.0 * (j - n + 1) * d * gp;
    return 2 * (n - 1) - j;
  }
  cst = 0.0;
  return j;
}

// Banded elimination of one line of n rows (row i at offset i * sd of each plane): band
// planes B[0..4] (offsets -2..2) and right-hand side Rh; the normalised upper factors and
// right-hand sides are written over B[3], B[4], Rh; the solution goes to x.
__device__ inline void band_line(double* B0, double* B1, double* B2, double* B3, double* B4,
                                 double* Rh, double* x, int n, int sd) {
  // row i (diagonal, +1, +2, rhs), row i + 1 (-1, 0, +1, +2, rhs), row i + 2 (all)
  double a2 = B2[0], a3 = B3[0], a4 = B4[0], ar = Rh[0];
  double b1 = 0.0, b2 = 1.0, b3 = 0.0, b4 = 0.0, br = 0.0;
  double c0 = 0.0, c1 = 0.0, c2 = 1.0, c3 = 0.0, c4 = 0.0, cr = 0.0;
  if (n > 1) b1 = B1[sd], b2 = B2[sd], b3 = B3[sd], b4 = B4[sd], br = Rh[sd];
  if (n > 2) {
    const int at = 2 * sd;
    c0 = B0[at], c1 = B1[at], c2 = B2[at], c3 = B3[at], c4 = B4[at], cr = Rh[at];
  }
  for (int i = 0; i < n; ++i) {
    const int at = i * sd;
    const double inv = 1.0 / a2;
    const double u1 = a3 * inv, u2 = a4 * inv, y = ar * inv;
    B3[at] = u1;
    B4[at] = u2;
    Rh[at] = y;
    // rows i + 1 and i + 2 lose their entries in column i
    b2 = fma(-b1, u1, b2);
    b3 = fma(-b1, u2, b3);
    br = fma(-b1, y, br);
    c1 = fma(-c0, u1, c1);
    c2 = fma(-c0, u2, c2);
    cr = fma(-c0, y, cr);
    a2 = b2, a3 = b3, a4 = b4, ar = br;
    b1 = c1, b2 = c2, b3 = c3, b4 = c4, br = cr;
    if (i + 3 < n) {
      const int nx = (i + 3) * sd;
      c0 = B0[nx], c1 = B1[nx], c2 = B2[nx], c3 = B3[nx], c4 = B4[nx], cr = Rh[nx];
    } else {
      c0 = 0.0, c1 = 0.0, c2 = 1.0, c3 = 0.0, c4 = 0.0, cr = 0.0;
    }
  }
  double x1 = 0.0, x2 = 0.0;  // x_{i+1}, x_{i+2}
  for (int i = n - 1; i >= 0; --i) {
    const int at = i * sd;
    const double v = fma(-B4[at], x2, fma(-B3[at], x1, Rh[at]));
    x[at] = v;
    x2 = x1;
    x1 = v;
  }
}

__global__ __launch_bounds__(64) void k_burst_adi_hu(AduArgs A) {
  extern __shared__ __align__(16) double lds[];
  const int mx = A.g.m_xi, me = A.g.m_eta, M = A.g.M;
  const int pm = mx * me, line = mx > me ? mx : me;
  const int per = ADU_PLANES * pm + 4 * M;
  const int slot = threadIdx.x / line, lane = threadIdx.x - slot * line;
  const long long p0 = (long long)blockIdx.x * A.ppb;
  const bool live = slot < A.ppb && p0 + slot < A.g.P;
  const double dx = A.g.dxi, de = A.g.deta;
  const double h = 0.5 * A.dt;
  const long long P = A.plane;
  const int npts = A.ppb * pm;
  for (int q = threadIdx.x; q < npts; q += 64) {
    const int sl = q / pm, at = q - sl * pm;
    if (p0 + sl < A.g.P) lds[sl * per + at] = A.state[(p0 + sl) * pm + at];
  }
  for (int q = threadIdx.x; q < A.ppb * 4 * M; q += 64) {
    const int sl = q / (4 * M), e = q - sl * 4 * M;
    if (p0 + sl < A.g.P) lds[sl * per + ADU_PLANES * pm + e] = A.edge[(p0 + sl) * 4 * M + e];
  }
  __syncthreads();
  for (int s = 0; s < A.n_t; ++s) {
    const double th = A.t_n + s * A.dt + 0.5 * A.dt;
    double T[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (j < A.src.ns) T[j] = time_factor(A.src, j, th);
    for (int half = 0; half < 2; ++half) {
      for (int q = threadIdx.x; q < npts; q += 64) {
        const int sl = q / pm, at = q - sl * pm;
        if (p0 + sl >= A.g.P) continue;
        double* b = lds + sl * per;
        const double* src = half == 0 ? b : b + pm;  // u^n, then u*
        const double* eg = b + ADU_PLANES * pm;
        const double* Cs = A.coef + (p0 + sl) * pm;
        const int l = at / mx, k = at - l * mx;
        const double al = Cs[at], ga = Cs[P + at], nu = Cs[2 * P + at], om = Cs[3 * P + at],
                     ph = Cs[4 * P + at];
        double sv = 0.0;
        for (int c = 0; c < A.src.nconst; ++c) sv += A.src.ca[c] * Cs[A.src.plane_c[c] * P + at];
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (j < A.src.ns) sv += T[j] * Cs[A.src.plane_t[j] * P + at];
        // implicit weights along the line (xi in the first half), explicit across it
        double wi[5], wc[5];
        dir_stencil(half == 0 ? al : ga, half == 0 ? nu : om, half == 0 ? dx : de, A.points,
                    A.r, wi);
        dir_stencil(half == 0 ? ga : al, half == 0 ? om : nu, half == 0 ? de : dx, A.points,
                    A.r, wc);
        const int ni = half == 0 ? mx : me, nc = half == 0 ? me : mx;
        const int ii = half == 0 ? k : l, ic = half == 0 ? l : k;
        const int sc = half == 0 ? mx : 1;
        const double di = half == 0 ? dx : de, dc = half == 0 ? de : dx;
        // edge data: along the implicit line at this point's crossing index, and across
        const double gim = half == 0 ? eg[l] : eg[2 * M + k];
        const double gip = half == 0 ? eg[M + l] : eg[3 * M + k];
        const double gcm = half == 0 ? eg[2 * M + k] : eg[l];
        const double gcp = half == 0 ? eg[3 * M + k] : eg[M + l];
        const int base_c = at - ic * sc;
        double ex = 0.5 * ph * src[at];
#pragma unroll
        for (int o = 0; o < 5; ++o) {
          double cst;
          const int j = fold(ic + o - 2, nc, dc, gcm, gcp, cst);
          ex = fma(wc[o], src[base_c + j * sc] + cst, ex);
        }
        double rhs = src[at] + h * ex + h * sv;
        double band[5] = {0.0, 0.0, 1.0 - h * 0.5 * ph, 0.0, 0.0};
#pragma unroll
        for (int o = 0; o < 5; ++o) {
          double cst;
          const int t = fold(ii + o - 2, ni, di, gim, gip, cst) - ii + 2;  // in 0..4
#pragma unroll
          for (int q = 0; q < 5; ++q) band[q] -= t == q ? h * wi[o] : 0.0;
          rhs += h * wi[o] * cst;
        }
#pragma unroll
        for (int o = 0; o < 5; ++o) b[(2 + o) * pm + at] = band[o];
        b[7 * pm + at] = rhs;
      }
      __syncthreads();
      if (live) {
        double* b = lds + slot * per;
        if (half == 0 && lane < me) {
          const int o = lane * mx;
          band_line(b + 2 * pm + o, b + 3 * pm + o, b + 4 * pm + o, b + 5 * pm + o,
                    b + 6 * pm + o, b + 7 * pm + o, b + pm + o, mx, 1);
        } else if (half == 1 && lane < mx) {
          const int o = lane;
          band_line(b + 2 * pm + o, b + 3 * pm + o, b + 4 * pm + o, b + 5 * pm + o,
                    b + 6 * pm + o, b + 7 * pm + o, b + o, me, mx);
        }
      }
      __syncthreads();
    }
  }
  bool bad = false;
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

void adu_shape(int mx, int me, int& ppb, size_t& lds) {
  const int line = mx > me ? mx : me;
  const size_t per = ((size_t)ADU_PLANES * mx * me + 4 * (size_t)line) * sizeof(double);
  ppb = line > 64 ? 0 : 64 / line;
  while (ppb > 0 && ppb * per > ADU_LDS_MAX) --ppb;
  lds = ppb * per;
}

hipError_t launch_burst_adi_hu(const Geo& g, const SrcInfo& src, const double* coef,
                               long long plane, double* state, const double* edge, double t_n,
                               double dt, int n_t, int points, double r, int* flag,
                               hipStream_t s) {
  AduArgs a;
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
  adu_shape(g.m_xi, g.m_eta, a.ppb, lds);
  if (a.ppb < 1) return hipErrorInvalidValue;
  const dim3 grid((g.P + a.ppb - 1) / a.ppb);
  hipLaunchKernelGGL(k_burst_adi_hu, grid, dim3(64), lds, s, a);
  return hipGetLastError();
}

}  // namespace pdk
