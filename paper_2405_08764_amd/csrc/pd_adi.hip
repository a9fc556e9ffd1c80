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

// ---------------------------------------------------------------- register-line kernel
// Lines of at most ADI_NL points.  The line matrices (I - dt/2 L_xi) of every row and
// (I - dt/2 L_eta) of every column do not change during a burst, so each is factored once
// (the Thomas pivots 1/den_i, the upper factors c_i = up_i/den_i and the lower ones
// lo_i/den_i) and every half step is a divide-free forward and back substitution.  Lane j
// of a patch owns row j in the first half and column j in the second: it keeps both lines'
// factors and explicit weights in registers, pre-scaled by the pivots (the right-hand side
// of point i enters the forward sweep as rhs_i / den_i), with the edge data's ghost terms
// folded into the constant part.  Only the fields go through LDS: the row-to-column
// transposition between the halves.
constexpr int ADI_NL = 12;

// Explicit and implicit data of one line of a lane, pre-scaled by the line's pivots (the
// line's constant and time-dependent source parts, pre-scaled the same way, go to LDS).
struct AdiLine {
  double e0[ADI_NL], em[ADI_NL], ep[ADI_NL];  // own, minus-side and plus-side explicit weights
  double lo[ADI_NL], up[ADI_NL];              // lo_i / den_i and up_i / den_i
};

// Factor one line of n points: (I - h L_line) with implicit weights (im, ip) along the line
// and explicit weights (xm, xp) across it, reaction ph, ghost folds at the line's ends
// (line edge data gf, gl at spacing dl) and across it (edges of the crossing direction:
// cross_first / cross_last, that direction's edge data xgf, xgl at spacing dx).  pt(i)
// returns point i's weights and sources (an LDS read per point, in line order).
struct AdiPoint {
  double im, ip, xm, xp, ph, sv, xgf, xgl;
  double st[2];
};

template <int NS>
__device__ __forceinline__ AdiPoint adi_point(const double* W, int wstride, const double* eg,
                                              int M, bool rows, int at, int i) {
  AdiPoint q;
  const double a0 = W[at], a1 = W[wstride + at], b0 = W[2 * wstride + at],
               b1 = W[3 * wstride + at];
  if (rows) {  // implicit in xi, explicit in eta (ghosts: south / north edge data)
    q.im = a0, q.ip = a1, q.xm = b0, q.xp = b1;
    q.xgf = eg[2 * M + i];
    q.xgl = eg[3 * M + i];
  } else {  // implicit in eta, explicit in xi (ghosts: west / east edge data)
    q.im = b0, q.ip = b1, q.xm = a0, q.xp = a1;
    q.xgf = eg[i];
    q.xgl = eg[M + i];
  }
  q.ph = W[4 * wstride + at];
  q.sv = W[5 * wstride + at];
  q.st[0] = q.st[1] = 0.0;
#pragma unroll
  for (int t = 0; t < NS; ++t) q.st[t] = W[(6 + t) * wstride + at];
  return q;
}

// Point i of the line sits at W[a0 + i as] in the weight planes.  Branch-free over the
// ADI_NL slots (points past the line's end repeat its last point and store zeros), so that
// the factor arrays stay in registers.
template <int NS>
__device__ __forceinline__ void adi_factor(AdiLine& Ln, double (&cs)[ADI_NL],
                                           double (&ts)[NS > 0 ? NS : 1][ADI_NL], int n,
                                           const double* W, int wstride, const double* eg, int M,
                                           bool rows, int a0, int as, double h, double dl,
                                           double gf, double gl, bool cross_first,
                                           bool cross_last, double dx) {
  double cprev = 0.0;
#pragma unroll
  for (int i = 0; i < ADI_NL; ++i) {
    if (i % 4 == 0) __builtin_amdgcn_sched_barrier(0);  // at most 4 points' reads in flight
    const bool in = i < n, first = i == 0, last = i == n - 1;
    const int ii = in ? i : n - 1;
    const AdiPoint q = adi_point<NS>(W, wstride, eg, M, rows, a0 + ii * as, ii);
    double lo = -h * q.im, up = -h * q.ip;
    const double di = 1.0 + h * (q.im + q.ip - 0.5 * q.ph);
    // x_{-1} = x_1 - 2 dl g- at the first point, x_n = x_{n-2} + 2 dl g+ at the last
    double cst = first ? -2.0 * dl * gf * q.im : 0.0;
    up = first ? up + lo : up;
    lo = first ? 0.0 : lo;
    cst = last ? cst + 2.0 * dl * gl * q.ip : cst;
    lo = last ? lo + up : lo;
    up = last ? 0.0 : up;
    const double e0 = 1.0 - h * (q.xm + q.xp - 0.5 * q.ph);
    double em = h * q.xm, ep = h * q.xp;
    // the crossing lines' ghosts: u_- = u_+ - 2 dx g- below, u_+ = u_- + 2 dx g+ above
    double xc = cross_first ? -2.0 * dx * q.xgf * em : 0.0;
    ep = cross_first ? ep + em : ep;
    em = cross_first ? 0.0 : em;
    xc = cross_last ? xc + 2.0 * dx * q.xgl * ep : xc;
    em = cross_last ? em + ep : em;
    ep = cross_last ? 0.0 : ep;
    const double den = di - lo * cprev;
    const double inv = 1.0 / den;
    const double c = up * inv;
    Ln.lo[i] = in ? lo * inv : 0.0;
    Ln.up[i] = in ? c : 0.0;
    Ln.e0[i] = in ? e0 * inv : 0.0;
    Ln.em[i] = in ? em * inv : 0.0;
    Ln.ep[i] = in ? ep * inv : 0.0;
    cs[i] = (h * q.sv + h * cst + xc) * inv;
#pragma unroll
    for (int t = 0; t < NS; ++t) ts[t][i] = h * q.st[t] * inv;
    cprev = in ? c : cprev;
  }
}

// One half step of a line: right-hand sides from the old field (own value, the crossing
// neighbours on both sides) and the line's source parts, forward and back substitution,
// solution to `dst`.  Points are at src[o + i sa] (own), src[om + i sa], src[op + i sa]
// (crossing neighbours), the sources at Cs[ca + i sa] (constant) and Cs[(1 + q) wstride +
// ca + i sa] (time-dependent).  Branch-free over the ADI_NL slots (past the line's end:
// zero weights on a valid point).
template <int NS>
__device__ __forceinline__ void adi_half(const AdiLine& Ln, int n, const double* src, int o,
                                         int om, int op, int sa, double* dst, const double* Cs,
                                         int ca, int wstride,
                                         const double (&T)[NS > 0 ? NS : 1]) {
  double d[ADI_NL];
  double prev = 0.0;
#pragma unroll
  for (int i = 0; i < ADI_NL; ++i) {
    if (i % 4 == 0) __builtin_amdgcn_sched_barrier(0);  // at most 4 points' reads in flight
    const int ii = i < n ? i : n - 1;
    double r = Cs[ca + ii * sa];
    r = i < n ? r : 0.0;
#pragma unroll
    for (int q = 0; q < NS; ++q)
      r = fma(i < n ? T[q] : 0.0, Cs[(1 + q) * wstride + ca + ii * sa], r);
    r = fma(Ln.e0[i], src[o + ii * sa], r);
    r = fma(Ln.em[i], src[om + ii * sa], r);
    r = fma(Ln.ep[i], src[op + ii * sa], r);
    prev = fma(-Ln.lo[i], prev, r);
    d[i] = prev;
  }
  double v = 0.0;
#pragma unroll
  for (int i = ADI_NL - 1; i >= 0; --i) {
    v = i >= n - 1 ? d[i] : fma(-Ln.up[i], v, d[i]);
    if (i < n) dst[o + i * sa] = v;
  }
}

// dir_weights with the spacing's reciprocals precomputed (no division per point).
__device__ inline void dir_weights_r(double a, double b, double id2, double id1, double ih,
                                     bool central, double& wm, double& wp) {
  const double d2 = a * id2;
  if (central) {
    wm = d2 + b * ih;
    wp = d2 - b * ih;
  } else {
    wm = d2 + (b >= 0.0 ? b * id1 : 0.0);
    wp = d2 + (b < 0.0 ? -b * id1 : 0.0);
  }
}

// Two waves per block share ppb patches in LDS: their fields, edge data and the direction
// weights of every point (computed once per point while the coefficient planes stream in,
// coalesced).  Wave 0 owns the rows (lane j of a patch: row j, the implicit xi sweeps of
// the first half step), wave 1 the columns (the implicit eta sweeps of the second); each
// lane factors its line from the LDS weights and keeps only that line's factors.
// With TAB (bursts of at most ADI_TT nano steps) the block tabulates the time factors of
// every nano step in LDS before anything else: evaluated inside the step loop, next to the
// lines' factors, the transcendental code pushed registers to scratch (measured on 16,129
// patches of 11 x 11, n_t = 2: 78 -> 66 us per burst; 64 us with the fresh line offsets
// below).  The values are the same, so are the results.
constexpr int ADI_NW = 6;  // per-point LDS planes: xi weights (2), eta weights (2), phi, source
constexpr int ADI_TT = 64;

template <int NS, bool TAB>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) void k_burst_adi_r(
    AdiArgs A) {
  extern __shared__ __align__(16) double lds[];
  __shared__ double tl[TAB && NS > 0 ? NS * ADI_TT : 1];
  if constexpr (TAB && NS > 0) {
    for (int e = threadIdx.x; e < NS * A.n_t; e += 128) {
      const int q = e / A.n_t, s = e - q * A.n_t;
      tl[q * ADI_TT + s] = time_factor(A.src, q, A.t_n + s * A.dt + 0.5 * A.dt);
    }
  }  // read after the staging barrier below
  const int mx = A.g.m_xi, me = A.g.m_eta, M = A.g.M;
  const int pm = mx * me, line = mx > me ? mx : me;
  const int per = 2 * pm + 4 * M;  // u, u*, edge data
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = lane / line, j = lane - slot * line;
  const long long p0 = (long long)blockIdx.x * A.ppb;
  const int np = (A.g.P - p0) < A.ppb ? (int)(A.g.P - p0) : A.ppb;  // patches of this block
  const bool live = slot < np;
  const double dx = A.g.dxi, de = A.g.deta;
  const bool central = A.g.conv == PD_CONV_CENTRAL;
  const double h = 0.5 * A.dt;
  const long long P = A.plane;
  const int npts = np * pm;
  const int wstride = A.ppb * pm;  // one weight plane
  double* W = lds + A.ppb * per;   // [ADI_NW + NS][ppb pm]
  const double ix2 = 1.0 / (dx * dx), ix1 = 1.0 / dx, ixh = 1.0 / (2.0 * dx);
  const double ie2 = 1.0 / (de * de), ie1 = 1.0 / de, ieh = 1.0 / (2.0 * de);
  const double* C0 = A.coef + p0 * pm;  // the block's patches are contiguous in every plane
  // The requests of ADI_NH points per thread are issued before any is used (ppb pm <= 64
  // ADI_NL points, at most 2 ADI_NH per thread; clamped addresses, masked stores).
  constexpr int ADI_NH = (64 * ADI_NL + 255) / 256;
#pragma unroll
  for (int g2 = 0; g2 < 2; ++g2) {
    double cu[ADI_NH], cal[ADI_NH], cga[ADI_NH], cnu[ADI_NH], com[ADI_NH], cph[ADI_NH],
        csv[ADI_NH], cst[NS > 0 ? NS : 1][ADI_NH];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < ADI_NH; ++r) {
      const int q0 = threadIdx.x + 128 * (g2 * ADI_NH + r), q = q0 < npts ? q0 : npts - 1;
      cu[r] = A.state[p0 * pm + q];
      cal[r] = C0[q];
      cga[r] = C0[P + q];
      cnu[r] = C0[2 * P + q];
      com[r] = C0[3 * P + q];
      cph[r] = C0[4 * P + q];
      double sv = 0.0;
      for (int c = 0; c < A.src.nconst; ++c) sv += A.src.ca[c] * C0[A.src.plane_c[c] * P + q];
      csv[r] = sv;
#pragma unroll
      for (int t = 0; t < NS; ++t) cst[t][r] = C0[A.src.plane_t[t] * P + q];
    }
#pragma unroll
    for (int r = 0; r < ADI_NH; ++r) {
      const int q = threadIdx.x + 128 * (g2 * ADI_NH + r);
      if (q < npts) {
        const int sl = q / pm, at = q - sl * pm;
        lds[sl * per + at] = cu[r];
        double a0, a1, b0, b1;
        dir_weights_r(cal[r], cnu[r], ix2, ix1, ixh, central, a0, a1);
        dir_weights_r(cga[r], com[r], ie2, ie1, ieh, central, b0, b1);
        W[q] = a0;
        W[wstride + q] = a1;
        W[2 * wstride + q] = b0;
        W[3 * wstride + q] = b1;
        W[4 * wstride + q] = cph[r];
        W[5 * wstride + q] = csv[r];
#pragma unroll
        for (int t = 0; t < NS; ++t) W[(ADI_NW + t) * wstride + q] = cst[t][r];
      }
    }
  }
  constexpr int ADI_NE = (4 * 64 + 127) / 128;  // edge values: ppb 4 M <= 4 * 64
  double ce[ADI_NE];
#pragma unroll
  for (int r = 0; r < ADI_NE; ++r) {
    const int q0 = threadIdx.x + 128 * r, q = q0 < np * 4 * M ? q0 : np * 4 * M - 1;
    ce[r] = A.edge[p0 * 4 * M + q];
  }
#pragma unroll
  for (int r = 0; r < ADI_NE; ++r) {
    const int q = threadIdx.x + 128 * r;
    if (q < np * 4 * M) {
      const int sl = q / (4 * M), e = q - sl * 4 * M;
      lds[sl * per + 2 * pm + e] = ce[r];
    }
  }
  __syncthreads();
  const bool rows = wave == 0;
  const int jr = j < me ? j : me - 1, jc = j < mx ? j : mx - 1;
  const int n = rows ? mx : me;  // points on the line
  const int sw = live ? slot : 0;
  const double* eg = lds + sw * per + 2 * pm;
  const int wb = sw * pm;  // the patch's first point in the weight planes
  AdiLine Ln;  // one call site (the line's parameters selected), so Ln stays in registers
  const int la = wb + (rows ? jr * mx : jc), ls = rows ? 1 : mx;  // the line in the planes
  {
    double cs[ADI_NL], ts[NS > 0 ? NS : 1][ADI_NL];
    adi_factor<NS>(Ln, cs, ts, n, W, wstride, eg, M, rows, la, ls, h, rows ? dx : de,
                   rows ? eg[jr] : eg[2 * M + jc], rows ? eg[M + jr] : eg[3 * M + jc],
                   rows ? jr == 0 : jc == 0, rows ? jr == me - 1 : jc == mx - 1,
                   rows ? de : dx);
    __syncthreads();  // every line has read the weight planes: reuse them for the sources
    const bool mine_ = live && (rows ? j < me : j < mx);
    double* Cw = W + (rows ? 0 : 1 + NS) * wstride;
#pragma unroll
    for (int i = 0; i < ADI_NL; ++i)
      if (mine_ && i < n) {
        Cw[la + i * ls] = cs[i];
#pragma unroll
        for (int t = 0; t < NS; ++t) Cw[(1 + t) * wstride + la + i * ls] = ts[t][i];
      }
    __syncthreads();
  }
  // fresh copies of the line's offsets: otherwise the compiler keeps every point's address
  // from the factoring alive through it (and spills them)
  int lh = la;
  asm volatile("" : "+v"(lh));
  const double* Cs = W + (rows ? 0 : 1 + NS) * wstride;
  double* b = lds + sw * per;
  // the line's points and its crossing neighbours on both sides (the folded ghost's weight
  // is zero, so an edge line reads its own inner neighbour there)
  const int o = rows ? jr * mx : jc, sa = rows ? 1 : mx;
  const int om = rows ? (jr > 0 ? jr - 1 : jr + 1) * mx : (jc > 0 ? jc - 1 : jc + 1);
  const int op = rows ? (jr < me - 1 ? jr + 1 : jr - 1) * mx : (jc < mx - 1 ? jc + 1 : jc - 1);
  const bool mine = live && (rows ? j < me : j < mx);
  for (int s = 0; s < A.n_t; ++s) {
    double T[NS > 0 ? NS : 1];
    if constexpr (TAB) {
#pragma unroll
      for (int q = 0; q < NS; ++q) T[q] = tl[q * ADI_TT + s];
    } else {
      const double th = A.t_n + s * A.dt + 0.5 * A.dt;
#pragma unroll
      for (int q = 0; q < NS; ++q) T[q] = time_factor(A.src, q, th);
    }
    // half 1 (wave 0): u -> u*; half 2 (wave 1): u* -> u
    for (int half = 0; half < 2; ++half) {
      if (mine && rows == (half == 0))
        adi_half<NS>(Ln, n, half == 0 ? b : b + pm, o, om, op, sa, half == 0 ? b + pm : b, Cs,
                     lh, wstride, T);
      __syncthreads();
    }
  }
  bool bad = false;
  for (int q = threadIdx.x; q < npts; q += 128) {
    const int sl = q / pm, at = q - sl * pm;
    const double v = lds[sl * per + at];
    A.state[p0 * pm + q] = v;
    bad = bad || !isfinite(v);
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

bool adi_fast(int mx, int me) { return mx <= ADI_NL && me <= ADI_NL; }

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
  if (adi_fast(g.m_xi, g.m_eta) && src.ns <= 1) {
    const int line = g.m_xi > g.m_eta ? g.m_xi : g.m_eta;
    a.ppb = 64 / line < 4 ? 64 / line : 4;  // measured: 4 patches per block beat 5 (LDS)
    const size_t pm = (size_t)g.m_xi * g.m_eta;
    lds = (size_t)a.ppb * ((2 + ADI_NW + src.ns) * pm + 4 * (size_t)g.M) * sizeof(double);
    const dim3 grid((g.P + a.ppb - 1) / a.ppb);
    if (src.ns == 0) hipLaunchKernelGGL((k_burst_adi_r<0, false>), grid, dim3(128), lds, s, a);
    else if (n_t <= ADI_TT) hipLaunchKernelGGL((k_burst_adi_r<1, true>), grid, dim3(128), lds, s, a);
    else hipLaunchKernelGGL((k_burst_adi_r<1, false>), grid, dim3(128), lds, s, a);
    return hipGetLastError();
  }
  adi_shape(g.m_xi, g.m_eta, a.ppb, lds);
  if (a.ppb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_burst_adi, dim3((g.P + a.ppb - 1) / a.ppb), dim3(64), lds, s, a);
  return hipGetLastError();
}

}  // namespace pdk
