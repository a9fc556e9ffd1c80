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
// One wave holds several patches; lane j of a patch owns line j (row j in the first half
// step, column j in the second).  It walks its line point by point: loads the point's
// coefficients, forms the five band entries and the right-hand side (the explicit half
// operator across the line reads the other lines' values from LDS), eliminates the
// entries left of the diagonal with the two rows above, already normalised and carried in
// registers, and normalises the row by one reciprocal (banded Gaussian elimination
// without pivoting, fused into the assembly).  The normalised rows go to LDS for the back
// substitution, which writes the line's solution into the other field plane.  Without
// pivoting the elimination is stable while every line matrix is diagonally dominant; for
// the 3-point form that holds when dt/2 (|nu| / d_xi + phi/2) <= 1 (likewise along eta),
// e.g. about 0.03 on the paper's Sec. 4.1.2 patches.
#include "pd_internal.h"

namespace pdk {

// LDS of one wave's patches (at most 64 KiB).
constexpr size_t ADU_LDS_MAX = 65536;
// Per patch in LDS: the field planes u^n / u^{n+1} and u*, the normalised rows (upper
// factors U1, U2 and right-hand side Y), the edge data.
constexpr int ADU_PLANES = 5;

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

// First-difference weights at offsets -2..2 times the spacing, backward side (the
// printed forms).
__device__ inline void d1_unit(int points, double r, double (&c)[5]) {
  c[0] = c[1] = c[2] = c[3] = c[4] = 0.0;
  if (points == 2) {
    c[2] = 1.0;
    c[1] = -1.0;
  } else if (points == 3) {
    c[2] = 1.5;
    c[1] = -2.0;
    c[0] = 0.5;
  } else {
    c[3] = 0.5 - r / 3.0;
    c[2] = r;
    c[1] = -0.5 - r;
    c[0] = r / 3.0;
  }
}

// Weights of L along one direction at offsets -2..2 (w[0] is offset -2): the 3-point
// second difference with diffusion a, minus velocity b times the first difference (unit
// weights cu, on the side the flow comes from: the mirror image where b < 0), spacing
// reciprocals id = 1/d and id2 = 1/d^2.  The reaction is added apart.
__device__ inline void dir_stencil(double a, double b, const double (&cu)[5], double id,
                                   double id2, double (&w)[5]) {
  const double d2 = a * id2;
  const bool back = b >= 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double ck = (back ? cu[k] : -cu[4 - k]) * id;
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

// NC constant and NS time-dependent source terms (compile-time counts, so that the
// source loads of a line's points carry no branches and issue together).
template <int NC, int NS>
__global__ __launch_bounds__(64) void k_burst_adi_hu(AduArgs A) {
  extern __shared__ __align__(16) double lds[];
  const int mx = A.g.m_xi, me = A.g.m_eta, M = A.g.M;
  const int pm = mx * me, line = mx > me ? mx : me;
  const int per = ADU_PLANES * pm + 4 * M;
  const int slot = threadIdx.x / line, lane = threadIdx.x - slot * line;
  const long long p0 = (long long)blockIdx.x * A.ppb;
  const bool live = slot < A.ppb && p0 + slot < A.g.P;
  const double dx = A.g.dxi, de = A.g.deta;
  const double idx = 1.0 / dx, idx2 = 1.0 / (dx * dx), ide = 1.0 / de, ide2 = 1.0 / (de * de);
  double cu[5];
  d1_unit(A.points, A.r, cu);
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
  double* b = lds + (live ? slot : 0) * per;
  double* U1 = b + 2 * pm;
  double* U2 = b + 3 * pm;
  double* Y = b + 4 * pm;
  const double* eg = b + ADU_PLANES * pm;
  for (int s = 0; s < A.n_t; ++s) {
    const double th = A.t_n + s * A.dt + 0.5 * A.dt;
    double T[NS > 0 ? NS : 1] = {0.0};
#pragma unroll
    for (int j = 0; j < NS; ++j) T[j] = time_factor(A.src, j, th);
    for (int half = 0; half < 2; ++half) {
      const bool rows = half == 0;
      const int n = rows ? mx : me, nc = rows ? me : mx;  // points along and across
      if (live && lane < nc) {
        const double* src = b + half * pm;  // u^n, then u*
        double* dst = b + (1 - half) * pm;
        const double* Cs = A.coef + (p0 + slot) * pm;
        const int si = rows ? 1 : mx, sc = rows ? mx : 1;
        const int base = rows ? lane * mx : lane;  // the line's first point
        const double di = rows ? dx : de, dc = rows ? de : dx;
        const double i_id = rows ? idx : ide, i_id2 = rows ? idx2 : ide2;
        const double c_id = rows ? ide : idx, c_id2 = rows ? ide2 : idx2;
        const double gim = rows ? eg[lane] : eg[2 * M + lane];
        const double gip = rows ? eg[M + lane] : eg[3 * M + lane];
        // rows i - 1 and i - 2, normalised: upper factors and right-hand side
        double p1 = 0.0, p2 = 0.0, py = 0.0, q1 = 0.0, q2 = 0.0, qy = 0.0;
#pragma unroll 4
        for (int i = 0; i < n; ++i) {
          const int at = base + i * si;
          const double al = Cs[at], ga = Cs[P + at], nu = Cs[2 * P + at], om = Cs[3 * P + at],
                       ph = Cs[4 * P + at];
          double sv = 0.0;
#pragma unroll
          for (int c = 0; c < NC; ++c) sv += A.src.ca[c] * Cs[A.src.plane_c[c] * P + at];
#pragma unroll
          for (int j = 0; j < NS; ++j) sv += T[j] * Cs[A.src.plane_t[j] * P + at];
          double wi[5], wc[5];  // along the line (implicit), across it (explicit)
          dir_stencil(rows ? al : ga, rows ? nu : om, cu, i_id, i_id2, wi);
          dir_stencil(rows ? ga : al, rows ? om : nu, cu, c_id, c_id2, wc);
          // explicit part: the crossing line through point i, where this line sits at
          // index `lane`, with that line's edge data for its ghosts
          const double gcm = rows ? eg[2 * M + i] : eg[i];
          const double gcp = rows ? eg[3 * M + i] : eg[M + i];
          const int cbase = at - lane * sc;
          double ex = 0.5 * ph * src[at];
#pragma unroll
          for (int o = 0; o < 5; ++o) {
            double cst;
            const int j = fold(lane + o - 2, nc, dc, gcm, gcp, cst);
            ex = fma(wc[o], src[cbase + j * sc] + cst, ex);
          }
          double rhs = src[at] + h * ex + h * sv;
          double band[5] = {0.0, 0.0, 1.0 - h * 0.5 * ph, 0.0, 0.0};
#pragma unroll
          for (int o = 0; o < 5; ++o) {
            double cst;
            const int t = fold(i + o - 2, n, di, gim, gip, cst) - i + 2;  // in 0..4
#pragma unroll
            for (int k = 0; k < 5; ++k) band[k] -= t == k ? h * wi[o] : 0.0;
            rhs += h * wi[o] * cst;
          }
          // entries in columns i - 2 and i - 1 (zero in the first two rows, where the
          // carried rows are zero too) against the rows above, then normalise
          {
            const double f = band[0];
            band[1] = fma(-f, q1, band[1]);
            band[2] = fma(-f, q2, band[2]);
            rhs = fma(-f, qy, rhs);
          }
          {
            const double f = band[1];
            band[2] = fma(-f, p1, band[2]);
            band[3] = fma(-f, p2, band[3]);
            rhs = fma(-f, py, rhs);
          }
          const double inv = 1.0 / band[2];
          q1 = p1, q2 = p2, qy = py;
          p1 = band[3] * inv, p2 = band[4] * inv, py = rhs * inv;
          U1[at] = p1;
          U2[at] = p2;
          Y[at] = py;
        }
        double x1 = 0.0, x2 = 0.0;  // x_{i+1}, x_{i+2}
#pragma unroll 4
        for (int i = n - 1; i >= 0; --i) {
          const int at = base + i * si;
          const double v = fma(-U2[at], x2, fma(-U1[at], x1, Y[at]));
          dst[at] = v;
          x2 = x1;
          x1 = v;
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
  if (src.nconst < 0 || src.nconst > PD_MAXTERM || src.ns < 0 || src.ns > 2)
    return hipErrorInvalidValue;
  static_assert(PD_MAXTERM == 4, "one instance per constant-term count");
  using K = void (*)(AduArgs);
  static const K tab[5][3] = {
      {k_burst_adi_hu<0, 0>, k_burst_adi_hu<0, 1>, k_burst_adi_hu<0, 2>},
      {k_burst_adi_hu<1, 0>, k_burst_adi_hu<1, 1>, k_burst_adi_hu<1, 2>},
      {k_burst_adi_hu<2, 0>, k_burst_adi_hu<2, 1>, k_burst_adi_hu<2, 2>},
      {k_burst_adi_hu<3, 0>, k_burst_adi_hu<3, 1>, k_burst_adi_hu<3, 2>},
      {k_burst_adi_hu<4, 0>, k_burst_adi_hu<4, 1>, k_burst_adi_hu<4, 2>}};
  hipLaunchKernelGGL(tab[src.nconst][src.ns], grid, dim3(64), lds, s, a);
  return hipGetLastError();
}

}  // namespace pdk
