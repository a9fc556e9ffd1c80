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
  // the point's value and the ghost copies it determines (offsets 0: none)
  auto put = [&](int i, double* t, double v) {
    double* c = t + off[i];
    c[0] = v;
    if (gx[i][0]) c[gx[i][0]] = v;
    if (ge[i][0]) c[ge[i][0]] = v;
    if (gx[i][1]) c[gx[i][1]] = v;
    if (ge[i][1]) c[ge[i][1]] = v;
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

// ------------------------------------------------------------------ in-wave kernel
// Patches whose lane blocks fit one wave: a lane owns a C x R block (C columns, R rows) of
// one patch and keeps its increment, the folded weights of the 5 x 5 cross and the
// forcing in registers for the whole burst.  The ghost layers of the increment are
// homogeneous mirrors (v_{-k} = v_k below the first point, likewise above the last), so
// a weight reaching past an edge is folded onto the mirrored point inside the patch,
// which keeps every offset within -2..+2.  Values of the two columns next to the block
// arrive from the neighbouring lanes by DPP wave shifts, the two rows above and below by
// ds_bpermute from the bands above and below; no barrier and no LDS traffic in the
// nano-step loop.  The lifted part dt L_h(u(0)) (with the edge data's ghosts) is formed
// once from an LDS tile with its ghost frame.
__device__ __forceinline__ double hx_up(double x) {  // lane i receives lane i - 1
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double hx_down(double x) {  // lane i receives lane i + 1
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double hx_read(int addr, double x) {  // lane addr / 4
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(x));
  return __hiloint2double(hi, lo);
}

// Folded weights along one direction for a point at index i of a line of n points:
// unfolded w[0..4] at offsets -2..+2; an offset reaching index t < 0 or t > n - 1 moves to
// the mirrored index -t or 2 (n - 1) - t.
__device__ inline void hx_fold(const double (&w)[5], int i, int n, double (&f)[5]) {
#pragma unroll
  for (int o = 0; o < 5; ++o) f[o] = 0.0;
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    int t = i + o - 2;
    t = t < 0 ? -t : t;
    t = t > n - 1 ? 2 * (n - 1) - t : t;
    f[t - i + 2] += w[o];
  }
}

constexpr int HX_TCH = 256;  // steps per chunk of the source time-factor table

template <int R, int C, int NS>
__global__ __launch_bounds__(64) void k_burst_hux(HuArgs A) {
  extern __shared__ __align__(16) double lds[];
  const int mx = A.g.m_xi, me = A.g.m_eta, M = A.g.M;
  const int pm = mx * me, W = mx + 4, ext = W * (me + 4);
  const int Lb = (mx + C - 1) / C, B = (me + R - 1) / R, LP = Lb * B;
  const int lane = threadIdx.x;
  const int ps = lane / LP, rl = lane - ps * LP, band = rl / Lb;
  const int k0 = (rl - band * Lb) * C, row0 = band * R;
  const long long p = (long long)blockIdx.x * A.ppb + ps;
  const bool active = ps < A.ppb && p < A.g.P;
  const int slot = active ? ps : 0;
  const long long pa = active ? p : 0;
  const int per = ext + 4 * M;          // lifted tile with ghost frame, edge data
  double* ttab = lds + A.ppb * per;     // [NS][HX_TCH]
  double* tile = lds + slot * per;
  const double* eg = tile + ext;
  const double dx = A.g.dxi, de = A.g.deta, dt = A.dt;
  const long long P = A.plane;
  // the patch states of the block's points and the edge data into LDS
  for (int q = lane; q < A.ppb * 4 * M; q += 64) {
    const int sl = q / (4 * M);
    if ((long long)blockIdx.x * A.ppb + sl < A.g.P)
      lds[sl * per + ext + (q - sl * 4 * M)] = A.edge[((long long)blockIdx.x * A.ppb) * 4 * M + q];
  }
  __syncthreads();  // edge data in LDS
  // the lifted tile with its ghost frame (edge data: u_{-1} = u_1 - 2 d g-,
  // u_{-2} = u_2 - 4 d g-, and mirrored above the last point)
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k = k0 + c, l = row0 + q;
      const bool in = active && k < mx && l < me;
      const double v = A.state[pa * pm + (in ? l * mx + k : 0)];
      if (!in) continue;
      const int o = (l + 2) * W + k + 2;
      tile[o] = v;
      if (k == 1) tile[o - 2] = v - 2.0 * dx * eg[l];
      if (k == 2) tile[o - 4] = v - 4.0 * dx * eg[l];
      if (k == mx - 2) tile[o + 2] = v + 2.0 * dx * eg[M + l];
      if (k == mx - 3) tile[o + 4] = v + 4.0 * dx * eg[M + l];
      if (l == 1) tile[o - 2 * W] = v - 2.0 * de * eg[2 * M + k];
      if (l == 2) tile[o - 4 * W] = v - 4.0 * de * eg[2 * M + k];
      if (l == me - 2) tile[o + 2 * W] = v + 2.0 * de * eg[3 * M + k];
      if (l == me - 3) tile[o + 4 * W] = v + 4.0 * de * eg[3 * M + k];
    }
  __syncthreads();
  // per point: the weights, the lifted part dt L_h(u(0)) + dt (constant sources) from the
  // tile with the unfolded weights, then the weights folded for the increment
  double cw[C][R][9];  // own (with the 1), x-2, x-1, x+1, x+2, e-2, e-1, e+1, e+2
  double K[C][R], sd[NS > 0 ? NS : 1][C][R];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k = k0 + c, l = row0 + q;
      const bool in = active && k < mx && l < me;
      const long long at = pa * pm + (in ? l * mx + k : 0);
      double wx[5], we[5];
      dir_stencil(A.coef[at], A.coef[2 * P + at], dx, A.points, A.r, dt, wx);
      dir_stencil(A.coef[P + at], A.coef[3 * P + at], de, A.points, A.r, dt, we);
      const double ph = dt * A.coef[4 * P + at];
      double sc = 0.0;
      for (int cc = 0; cc < A.src.nconst; ++cc) sc += A.src.ca[cc] * A.coef[A.src.plane_c[cc] * P + at];
#pragma unroll
      for (int j = 0; j < NS; ++j) sd[j][c][q] = in ? dt * A.coef[A.src.plane_t[j] * P + at] : 0.0;
      double kk = 0.0;
      if (in) {
        const double* t = tile + (l + 2) * W + k + 2;
        kk = (wx[2] + we[2] + ph) * t[0];
        kk = fma(wx[0], t[-2], kk);
        kk = fma(wx[1], t[-1], kk);
        kk = fma(wx[3], t[1], kk);
        kk = fma(wx[4], t[2], kk);
        kk = fma(we[0], t[-2 * W], kk);
        kk = fma(we[1], t[-W], kk);
        kk = fma(we[3], t[W], kk);
        kk = fma(we[4], t[2 * W], kk);
        kk += dt * sc;
      }
      K[c][q] = kk;
      double fx[5], fe[5];
      hx_fold(wx, k < mx ? k : mx - 1, mx, fx);
      hx_fold(we, l < me ? l : me - 1, me, fe);
      const double zc = in ? 1.0 : 0.0;
      cw[c][q][0] = zc * (1.0 + fx[2] + fe[2] + ph);
      cw[c][q][1] = zc * fx[0];
      cw[c][q][2] = zc * fx[1];
      cw[c][q][3] = zc * fx[3];
      cw[c][q][4] = zc * fx[4];
      cw[c][q][5] = zc * fe[0];
      cw[c][q][6] = zc * fe[1];
      cw[c][q][7] = zc * fe[3];
      cw[c][q][8] = zc * fe[4];
    }
  // the nano steps on the increment v (starts at zero)
  double v[C][R], y[C][R];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < R; ++q) v[c][q] = 0.0;
  const int aN = ((lane + Lb) & 63) << 2, aS = ((lane - Lb) & 63) << 2;
  auto step = [&](const double (&s)[C][R], double (&d)[C][R], int st) {
    if (NS > 0 && st % HX_TCH == 0) {  // the next chunk of source time factors
      __syncthreads();
      for (int e = lane; e < NS * HX_TCH; e += 64) {
        const int j = e / HX_TCH, ss = st + (e - j * HX_TCH);
        ttab[e] = ss < A.n_t ? time_factor(A.src, j, A.t_n + ss * dt) : 0.0;
      }
      __syncthreads();
    }
    double T[NS > 0 ? NS : 1];
#pragma unroll
    for (int j = 0; j < NS; ++j) T[j] = ttab[j * HX_TCH + st % HX_TCH];
    // rows above (first two of the band above) and below (last two of the band below)
    double n1[C], n2[C], s1[C], s2[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      n1[c] = hx_read(aN, s[c][0]);
      n2[c] = hx_read(aN, s[c][R > 1 ? 1 : 0]);
      s1[c] = hx_read(aS, s[c][R - 1]);
      s2[c] = hx_read(aS, s[c][R > 1 ? R - 2 : 0]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      // the two columns east of the block (first two of lane + 1), west (last two of lane - 1)
      const double e1 = hx_down(s[0][q]), e2 = hx_down(s[C > 1 ? 1 : 0][q]);
      const double w1 = hx_up(s[C - 1][q]), w2 = hx_up(s[C > 1 ? C - 2 : 0][q]);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double xm2 = c >= 2 ? s[c - 2][q] : (c == 1 ? w1 : w2);
        const double xm1 = c >= 1 ? s[c - 1][q] : w1;
        const double xp1 = c + 1 < C ? s[c + 1][q] : e1;
        const double xp2 = c + 2 < C ? s[c + 2][q] : (c + 1 < C ? e1 : e2);
        const double em2 = q >= 2 ? s[c][q - 2] : (q == 1 ? s1[c] : s2[c]);
        const double em1 = q >= 1 ? s[c][q - 1] : s1[c];
        const double ep1 = q + 1 < R ? s[c][q + 1] : n1[c];
        const double ep2 = q + 2 < R ? s[c][q + 2] : (q + 1 < R ? n1[c] : n2[c]);
        // fixed order: own value, eta -2 .. +2, xi -2 .. +2, then the forcing
        double a = fma(cw[c][q][0], s[c][q], K[c][q]);
        a = fma(cw[c][q][5], em2, a);
        a = fma(cw[c][q][6], em1, a);
        a = fma(cw[c][q][7], ep1, a);
        a = fma(cw[c][q][8], ep2, a);
        a = fma(cw[c][q][1], xm2, a);
        a = fma(cw[c][q][2], xm1, a);
        a = fma(cw[c][q][3], xp1, a);
        a = fma(cw[c][q][4], xp2, a);
#pragma unroll
        for (int j = 0; j < NS; ++j) a = fma(T[j], sd[j][c][q], a);
        d[c][q] = a;
      }
    }
  };
  int st = 0;
  for (; st + 1 < A.n_t; st += 2) {
    step(v, y, st);
    step(y, v, st + 1);
  }
  if (st < A.n_t) {
    step(v, y, st);
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < R; ++q) v[c][q] = y[c][q];
  }
  bool bad = false;
  double un[C][R];  // u(0) again (not kept in registers through the nano steps)
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k = k0 + c, l = row0 + q;
      const bool in = active && k < mx && l < me;
      un[c][q] = A.state[pa * pm + (in ? l * mx + k : 0)];
    }
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k = k0 + c, l = row0 + q;
      if (active && k < mx && l < me) {
        const double u = un[c][q] + v[c][q];
        A.state[p * pm + l * mx + k] = u;
        bad = bad || !isfinite(u);
      }
    }
  if (bad) atomicOr(A.flag, 1);
}

// Lane blocks of the in-wave kernel and the patches per wave they give (0: the patch does
// not fit one wave).
#define PD_HUX_SHAPES(X) X(3, 2) X(2, 3) X(2, 2)

int hux_ppb(int R, int C, int mx, int me) {
  const int LP = ((mx + C - 1) / C) * ((me + R - 1) / R);
  return LP <= 64 ? 64 / LP : 0;
}

// The lane block with the most useful lane slots (ties: fewer exchanged values per point).
bool hux_pick(int mx, int me, int& R, int& C) {
  double best = 0.0;
  R = C = 0;
#define PD_HUX_TRY(R_, C_)                                                      \
  {                                                                             \
    const int pp = hux_ppb(R_, C_, mx, me);                                     \
    const double u = pp * (double)mx * me / (64.0 * R_ * C_) + 1e-3 * (R_ + C_); \
    if (pp > 0 && u > best) best = u, R = R_, C = C_;                           \
  }
  PD_HUX_SHAPES(PD_HUX_TRY)
#undef PD_HUX_TRY
  return R > 0;
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
                           bool lds_only, hipStream_t s) {
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
  if (points < 2 || points > 4) return hipErrorInvalidValue;
  int R = 0, C = 0;
  if (!lds_only && hux_pick(g.m_xi, g.m_eta, R, C)) {
    a.ppb = hux_ppb(R, C, g.m_xi, g.m_eta);
    const size_t lds = ((size_t)a.ppb * ((g.m_xi + 4) * (size_t)(g.m_eta + 4) + 4 * (size_t)g.M) +
                        2 * HX_TCH) * sizeof(double);
    const dim3 grid((g.P + a.ppb - 1) / a.ppb);
#define PD_HUX_LAUNCH(R_, C_)                                                         \
    if (R == R_ && C == C_) {                                                         \
      if (src.ns == 0) hipLaunchKernelGGL((k_burst_hux<R_, C_, 0>), grid, dim3(64), lds, s, a); \
      else if (src.ns == 1) hipLaunchKernelGGL((k_burst_hux<R_, C_, 1>), grid, dim3(64), lds, s, a); \
      else hipLaunchKernelGGL((k_burst_hux<R_, C_, 2>), grid, dim3(64), lds, s, a);  \
      return hipGetLastError();                                                       \
    }
    PD_HUX_SHAPES(PD_HUX_LAUNCH)
#undef PD_HUX_LAUNCH
  }
  size_t lds = 0;
  hu_shape(g.m_xi, g.m_eta, a.ppb, lds);
  if (a.ppb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_burst_hu, dim3((g.P + a.ppb - 1) / a.ppb), dim3(HU_THREADS), lds, s,
                     a);
  return hipGetLastError();
}

}  // namespace pdk
