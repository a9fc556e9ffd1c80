// Coefficients of the transformed operator, boundary data and explicit bounds.
//
// Sec. 2.1, eq. (Computational_Problem): for an orthogonal map (beta = 0) the operator
// div(D grad u - v u) + f u becomes
//   alpha u_xixi + gamma u_etaeta - nu u_xi - omega u_eta + phi u
// and, with the scale factors h1 = |r_xi|, h2 = |r_eta| and D = diag(D11, D22),
//   alpha = D11 / h1^2,  gamma = D22 / h2^2,
//   nu    = (v . r_xi)  / h1^2 - d_xi (D11 h2 / h1) / (h1 h2),
//   omega = (v . r_eta) / h2^2 - d_eta(D22 h1 / h2) / (h1 h2),
//   phi   = f - div v,
// which reproduces the worked lists of Sec. 4.1.1 (eq. P1_C), 4.1.2 (eq. P1_C_Vari_Diff)
// and 4.2 (eq. Ann_Diff_Computational).  Maps: eq. (Stretching_Transformation),
// tanh stretching clustered at x = 1, eq. (Transformation_Annulus) with xi = theta.
// Source term k: T_k(t) (c_k S_k - L[S_k]), L the same operator applied to S_k.
#include "pd_internal.h"
#include "pd_refresh.h"

namespace pdk {
namespace {

struct Metric {
  double x, y;
  double x_s, y_s, x_e, y_e;         // first derivatives (s = xi, e = eta)
  double x_ss, y_ss, x_ee, y_ee;     // second derivatives
  double x_se, y_se;                 // mixed
};

__device__ void metric_at(const Geo& g, double xi, double eta, Metric& m) {
  m = Metric{};
  if (g.geometry == PD_GEOM_SINE) {
    const double l = g.gparam;
    double sx, cx, se, ce;
    sincospi(xi, &sx, &cx);
    sincospi(eta, &se, &ce);
    m.x = xi + (l / M_PI) * sx;
    m.y = eta + (l / M_PI) * se;
    m.x_s = 1.0 + l * cx;
    m.y_e = 1.0 + l * ce;
    m.x_ss = -l * M_PI * sx;
    m.y_ee = -l * M_PI * se;
  } else if (g.geometry == PD_GEOM_TANH && g.gparam != 0.0) {
    const double b = g.gparam, tb = tanh(b);
    const double tx = tanh(b * xi), ty = tanh(b * eta);
    const double qx = 1.0 - tx * tx, qy = 1.0 - ty * ty;   // sech^2
    m.x = tx / tb;
    m.y = ty / tb;
    m.x_s = b * qx / tb;
    m.y_e = b * qy / tb;
    m.x_ss = -2.0 * b * b * tx * qx / tb;
    m.y_ee = -2.0 * b * b * ty * qy / tb;
  } else if (g.geometry == PD_GEOM_ANNULUS) {
    double s, c;
    sincos(xi, &s, &c);
    m.x = eta * c;
    m.y = eta * s;
    m.x_s = -eta * s;
    m.y_s = eta * c;
    m.x_e = c;
    m.y_e = s;
    m.x_ss = -eta * c;
    m.y_ss = -eta * s;
    m.x_se = -s;
    m.y_se = c;
  } else {
    m.x = xi;
    m.y = eta;
    m.x_s = 1.0;
    m.y_e = 1.0;
  }
}

// Value and Cartesian gradient of a field; polar terms use r = eta, theta = xi.
__device__ void field_at(const pd_field& F, double x, double y, bool annulus, double r,
                         double th, double& v, double& vx, double& vy) {
  v = F.c0 + F.cx * x + F.cy * y;
  vx = F.cx;
  vy = F.cy;
  for (int k = 0; k < F.nmode; ++k) {
    double s, c;
    sincos(F.kx[k] * x + F.ky[k] * y + F.ph[k], &s, &c);
    v += F.amp[k] * c;
    vx -= F.amp[k] * F.kx[k] * s;
    vy -= F.amp[k] * F.ky[k] * s;
  }
  if (annulus && F.npolar > 0) {
    double st, ct;
    sincos(th, &st, &ct);
    for (int k = 0; k < F.npolar; ++k) {
      const double P = F.pc0[k] + F.pc1[k] * r + F.pc2[k] * r * r;
      const double dP = F.pc1[k] + 2.0 * F.pc2[k] * r;
      double s, c;
      sincos(F.pn[k] * th + F.pph[k], &s, &c);
      const double fr = F.pamp[k] * dP * c;             // dF/dr
      const double ft = -F.pamp[k] * P * F.pn[k] * s;   // dF/dtheta
      v += F.pamp[k] * P * c;
      vx += ct * fr - st / r * ft;
      vy += st * fr + ct / r * ft;
    }
  }
}

__device__ void fn1_at(const pd_fn1& f, double s, double& v, double& d1, double& d2) {
  if (f.type == PD_FN_SIN || f.type == PD_FN_COS) {
    double sn, cs;
    sincos(f.a * s + f.b, &sn, &cs);
    if (f.type == PD_FN_SIN) {
      v = sn;
      d1 = f.a * cs;
      d2 = -f.a * f.a * sn;
    } else {
      v = cs;
      d1 = -f.a * sn;
      d2 = -f.a * f.a * cs;
    }
  } else if (f.type == PD_FN_EXP) {
    v = exp(f.a * s + f.b);
    d1 = f.a * v;
    d2 = f.a * f.a * v;
  } else {
    v = f.a + f.b * s + f.c * s * s + f.d * s * s * s;
    d1 = f.b + 2.0 * f.c * s + 3.0 * f.d * s * s;
    d2 = 2.0 * f.c + 6.0 * f.d * s;
  }
}

// S and its derivatives in the computational coordinates: S, S_xi, S_eta, S_xixi, S_etaeta.
__device__ void sfun_at(const pd_sfun& S, const Metric& m, double xi, double eta, double* o) {
  double f, f1, f2, q, q1, q2;
  if (S.kind == 1) {  // amp f(r) g(theta), r = eta, theta = xi
    fn1_at(S.f, eta, f, f1, f2);
    fn1_at(S.g, xi, q, q1, q2);
    o[0] = S.amp * f * q;
    o[1] = S.amp * f * q1;
    o[2] = S.amp * f1 * q;
    o[3] = S.amp * f * q2;
    o[4] = S.amp * f2 * q;
    return;
  }
  fn1_at(S.f, m.x, f, f1, f2);
  fn1_at(S.g, m.y, q, q1, q2);
  const double Sx = S.amp * f1 * q, Sy = S.amp * f * q1;
  const double Sxx = S.amp * f2 * q, Syy = S.amp * f * q2, Sxy = S.amp * f1 * q1;
  o[0] = S.amp * f * q;
  o[1] = Sx * m.x_s + Sy * m.y_s;
  o[2] = Sx * m.x_e + Sy * m.y_e;
  o[3] = Sxx * m.x_s * m.x_s + 2.0 * Sxy * m.x_s * m.y_s + Syy * m.y_s * m.y_s + Sx * m.x_ss +
         Sy * m.y_ss;
  o[4] = Sxx * m.x_e * m.x_e + 2.0 * Sxy * m.x_e * m.y_e + Syy * m.y_e * m.y_e + Sx * m.x_ee +
         Sy * m.y_ee;
}

__device__ double tfun_at(const pd_tfun& T, double t) {
  if (T.type == PD_T_EXP) return T.a * exp(T.b * t);
  if (T.type == PD_T_SIN) return T.a + T.b * sin(T.c * t);
  return T.a;
}

// alpha, gamma, nu, omega, phi and the source parts at (xi, eta).
__device__ void coefficients_at(const Geo& g, const pd_coeff_desc& c, int n_src, double xi,
                                double eta, double* out) {
  Metric m;
  metric_at(g, xi, eta, m);
  const bool ann = g.geometry == PD_GEOM_ANNULUS;
  const double h1 = sqrt(m.x_s * m.x_s + m.y_s * m.y_s);
  const double h2 = sqrt(m.x_e * m.x_e + m.y_e * m.y_e);
  const double h1_s = (m.x_s * m.x_ss + m.y_s * m.y_ss) / h1;
  const double h1_e = (m.x_s * m.x_se + m.y_s * m.y_se) / h1;
  const double h2_s = (m.x_e * m.x_se + m.y_e * m.y_se) / h2;
  const double h2_e = (m.x_e * m.x_ee + m.y_e * m.y_ee) / h2;
  double a, ax, ay, b, bx, by, v1, v1x, v1y, v2, v2x, v2y, f, fx, fy;
  field_at(c.D11, m.x, m.y, ann, eta, xi, a, ax, ay);
  field_at(c.D22, m.x, m.y, ann, eta, xi, b, bx, by);
  field_at(c.v1, m.x, m.y, ann, eta, xi, v1, v1x, v1y);
  field_at(c.v2, m.x, m.y, ann, eta, xi, v2, v2x, v2y);
  field_at(c.f, m.x, m.y, ann, eta, xi, f, fx, fy);
  const double a_s = ax * m.x_s + ay * m.y_s;   // d D11 / d xi
  const double b_e = bx * m.x_e + by * m.y_e;   // d D22 / d eta
  const double alpha = a / (h1 * h1);
  const double gamma = b / (h2 * h2);
  const double nu = (v1 * m.x_s + v2 * m.y_s) / (h1 * h1) -
                    (a_s * h2 / h1 + a * (h2_s * h1 - h2 * h1_s) / (h1 * h1)) / (h1 * h2);
  const double omega = (v1 * m.x_e + v2 * m.y_e) / (h2 * h2) -
                       (b_e * h1 / h2 + b * (h1_e * h2 - h1 * h2_e) / (h2 * h2)) / (h1 * h2);
  const double phi = f - (v1x + v2y);
  out[0] = alpha;
  out[1] = gamma;
  out[2] = nu;
  out[3] = omega;
  out[4] = phi;
  for (int k = 0; k < n_src; ++k) {
    double S[5];
    sfun_at(c.src_s[k], m, xi, eta, S);
    const double LS = alpha * S[3] + gamma * S[4] - nu * S[1] - omega * S[2] + phi * S[0];
    out[5 + k] = c.src_c[k] * S[0] - LS;
  }
}

__device__ double boundary_at(const Geo& g, const pd_coeff_desc& c, double xi, double eta,
                              double t) {
  Metric m;
  metric_at(g, xi, eta, m);
  double u = 0.0;
  for (int q = 0; q < c.n_bc; ++q) {
    double S[5];
    sfun_at(c.bc_s[q], m, xi, eta, S);
    u += tfun_at(c.bc_t[q], t) * S[0];
  }
  return u;
}

__device__ inline double micro_offset(double h, int m, int k) {
  return (double)(2 * k - (m - 1)) * (h / (2.0 * (m - 1)));
}

__device__ inline void patch_node(const Geo& g, int p, int& i, int& j) {
  i = g.i_first + p % g.npx;
  j = 1 + p / g.npx;
}

__global__ void k_coefficients(Geo g, const pd_coeff_desc* __restrict__ desc, int n_src,
                               double* __restrict__ coef) {
  const long long npts = (long long)g.P * g.m_xi * g.m_eta;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= npts) return;
  const int pm = g.m_xi * g.m_eta;
  const int p = (int)(q / pm), r = (int)(q - (long long)p * pm);
  const int l = r / g.m_xi, k = r - l * g.m_xi;
  int i, j;
  patch_node(g, p, i, j);
  const double xi = (g.xi0 + i * g.Dxi) + micro_offset(g.h_xi, g.m_xi, k);
  const double eta = (g.eta0 + j * g.Deta) + micro_offset(g.h_eta, g.m_eta, l);
  double out[5 + PD_MAXTERM];
  coefficients_at(g, *desc, n_src, xi, eta, out);
  for (int c = 0; c < 5 + n_src; ++c) coef[c * npts + q] = out[c];
}

__device__ inline double fe_bound(double a, double c, double nu, double om, double ph,
                                  double dx, double de) {
  return 1.0 / (2.0 * a / (dx * dx) + 2.0 * c / (de * de) + fabs(nu) / dx + fabs(om) / de +
                fabs(ph));
}

// Block minima of the explicit forward-Euler bound over the micro points (slot 0) and
// over the patch nodes at macro spacing (slot 1); 0 where diffusion is not positive.
__global__ void k_limits(Geo g, const pd_coeff_desc* __restrict__ desc, int n_src,
                         const double* __restrict__ coef, double* __restrict__ partial) {
  __shared__ double red[2][256];
  const long long npts = (long long)g.P * g.m_xi * g.m_eta;
  double lo = INFINITY, hi = INFINITY;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < npts; q += stride) {
    const double a = coef[q], c = coef[npts + q];
    const double b = (a > 0.0 && c > 0.0)
                         ? fe_bound(a, c, coef[2 * npts + q], coef[3 * npts + q],
                                    coef[4 * npts + q], g.dxi, g.deta)
                         : 0.0;
    lo = fmin(lo, b);
  }
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < g.P; p += stride) {
    int i, j;
    patch_node(g, (int)p, i, j);
    double out[5 + PD_MAXTERM];
    coefficients_at(g, *desc, 0, g.xi0 + i * g.Dxi, g.eta0 + j * g.Deta, out);
    const double b = (out[0] > 0.0 && out[1] > 0.0)
                         ? fe_bound(out[0], out[1], out[2], out[3], out[4], g.Dxi, g.Deta)
                         : 0.0;
    hi = fmin(hi, b);
  }
  red[0][threadIdx.x] = lo;
  red[1][threadIdx.x] = hi;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = fmin(red[1][threadIdx.x], red[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = red[0][0];
    partial[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_limits_final(const double* __restrict__ partial, int nblocks,
                               double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double lo = INFINITY, hi = INFINITY;
  for (int b = 0; b < nblocks; ++b) {
    lo = fmin(lo, partial[2 * b]);
    hi = fmin(hi, partial[2 * b + 1]);
  }
  out[0] = lo;
  out[1] = hi;
}


// Dirichlet data u_b(t) on the boundary nodes (eq. CDR_Com_IC_BCs, eq. Ann_C_IC_BCs).
__global__ void k_boundary(Geo g, const pd_coeff_desc* __restrict__ desc, double* U, double t) {
  const int nb = boundary_count(g);
  for (int q = threadIdx.x; q < nb; q += blockDim.x) {
    int i, j;
    boundary_node(g, q, i, j);
    U[j * g.n_xi + i] = boundary_at(g, *desc, g.xi0 + i * g.Dxi, g.eta0 + j * g.Deta, t);
  }
}

// Start time t_n + s0 dt of a sub-burst: one rounded product and one rounded sum (the
// library is built without floating-point contraction), the value the host computes for
// the same sub-burst, so its table equals the one a separate burst from there would use.
__device__ double sub_burst_start(double t_n, int s0, double dt) {
  return t_n + (double)s0 * dt;
}

// Time factors of the Q sub-bursts of a refreshed macro step, one thread per entry of the
// ns n_t entries: sub-burst q's table [ns][s1 - s0] sits at out + ns s0, so entry E lies
// in the sub-burst whose steps hold x = E / ns, i.e. the last q with floor(n_t q / Q) <= x.
__global__ void k_refresh_tables(SrcInfo src, double t_n, double dt, int n_t, int Q,
                                 double* __restrict__ out) {
  const long long E = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (E >= (long long)src.ns * n_t) return;
  const long long x = E / src.ns;
  const int q = (int)(((x + 1) * Q - 1) / n_t);
  const int s0 = (int)((long long)n_t * q / Q), s1 = (int)((long long)n_t * (q + 1) / Q);
  const int len = s1 - s0;
  const int r = (int)(E - (long long)src.ns * s0);
  const int j = r / len, s = r - j * len;
  const double t_q = sub_burst_start(t_n, s0, dt);
  out[E] = time_factor(src, j, t_q + (double)s * dt);
}

// Set-up of a resident refreshed macro step: the Dirichlet values at the ends of sub-bursts
// 0 .. Q - 2, out[q][nb] = u_b(t_n + s1 dt) with s1 = floor(n_t (q + 1) / Q) (the time
// rounded as the host rounds it), row Q - 1 at t_end (the macro step's end), and the
// waves' flags cleared.
__global__ void k_refresh_setup(Geo g, const pd_coeff_desc* __restrict__ desc, double t_n,
                                double dt, int n_t, int Q, double t_end,
                                double* __restrict__ out, long long* __restrict__ flags,
                                int nflags) {
  const int nb = boundary_count(g);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nflags) flags[e] = 0;
  if (e >= (long long)Q * nb) return;
  const int q = (int)(e / nb), b = (int)(e - (long long)q * nb);
  const int s1 = (int)((long long)n_t * (q + 1) / Q);
  int i, j;
  boundary_node(g, b, i, j);
  out[e] = boundary_at(g, *desc, g.xi0 + i * g.Dxi, g.eta0 + j * g.Deta,
                       q + 1 < Q ? sub_burst_start(t_n, s1, dt) : t_end);
}

// Blocks of the two refresh kernels below: the first RF_WAVES-patch groups restrict (one
// wave per patch, as k_restrict), the blocks after them write the Dirichlet nodes.
constexpr int RF_WAVES = 4;
constexpr int RF_THREADS = 64 * RF_WAVES;

__device__ double refresh_restrict(const Geo& g, const double* state, double* Ubar, int p,
                                   int w, int lane, double (&rows)[RF_WAVES][64]) {
  if (p < g.P && lane >= g.ls && lane < g.ls + g.nls)
    rows[w][lane] = restriction_row(g, state, p, lane);
  __syncthreads();
  double v = 0.0;
  if (p < g.P && lane == 0) {
    v = restriction_total(g, rows[w]);
    Ubar[p] = v;
  }
  return v;
}

__device__ void refresh_boundary(const Geo& g, const pd_coeff_desc& desc, double* U,
                                 double t, int q) {
  if (q >= boundary_count(g)) return;
  int i, j;
  boundary_node(g, q, i, j);
  U[j * g.n_xi + i] = boundary_at(g, desc, g.xi0 + i * g.Dxi, g.eta0 + j * g.Deta, t);
}

__global__ __launch_bounds__(RF_THREADS) void k_refresh_field(
    Geo g, const int* __restrict__ pmap, const pd_coeff_desc* __restrict__ desc,
    const double* __restrict__ state, double* __restrict__ Ubar, double* __restrict__ U,
    double t) {
  __shared__ double rows[RF_WAVES][64];
  const int groups = (g.P + RF_WAVES - 1) / RF_WAVES;
  if ((int)blockIdx.x >= groups) {
    refresh_boundary(g, *desc, U, t, ((int)blockIdx.x - groups) * RF_THREADS + threadIdx.x);
    return;
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = blockIdx.x * RF_WAVES + w;
  const double v = refresh_restrict(g, state, Ubar, p, w, lane, rows);
  if (p < g.P && lane == 0) U[pmap[11 * p + 6]] = v;
}

__global__ __launch_bounds__(RF_THREADS) void k_refresh_final(
    Geo g, const int* __restrict__ pmap, const pd_coeff_desc* __restrict__ desc,
    const double* __restrict__ state, double* __restrict__ Ubar,
    const double* __restrict__ U_n, double* __restrict__ U_np1, double dt_macro, double tau,
    int* flag, double t) {
  __shared__ double rows[RF_WAVES][64];
  const int groups = (g.P + RF_WAVES - 1) / RF_WAVES;
  if ((int)blockIdx.x >= groups) {
    refresh_boundary(g, *desc, U_np1, t, ((int)blockIdx.x - groups) * RF_THREADS + threadIdx.x);
    return;
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = blockIdx.x * RF_WAVES + w;
  const double ub = refresh_restrict(g, state, Ubar, p, w, lane, rows);
  if (p < g.P && lane == 0) {
    const int node = pmap[11 * p + 6];
    const double v = projective_value(U_n[node], ub, dt_macro, tau);
    U_np1[node] = v;
    if (!isfinite(v)) atomicOr(flag, 1);
  }
}

// First node of a graph replay of S macro steps: macro steps base .. base+S-1 with base =
// the clock's step count.  Fills the time factors of their bursts,
// ttab[k][j][s] = T_j(t_n + s dt_micro) with t_n = t0 + (base + k) dt, and the Dirichlet
// values at their end times, bvals[k][q] = u_b(node q, t0 + (base + k + 1) dt); the burst
// of step k reads entry k of both.  The last block to finish advances the clock by S (every
// block has read it by then).
__global__ void k_replay(Geo g, SrcInfo src, const pd_coeff_desc* __restrict__ desc,
                         Clock* clk, int S, int n_t, double dt_micro, double* __restrict__ ttab,
                         double* __restrict__ bvals) {
  const long long base = clk->next;
  const double t0 = clk->t0, dt = clk->dt;
  const int per = src.ns * n_t, nb = boundary_count(g);
  const int stride = gridDim.x * blockDim.x, first = blockIdx.x * blockDim.x + threadIdx.x;
  for (int e = first; e < S * per; e += stride) {
    const int k = e / per, r = e - k * per;
    const int j = r / n_t, s = r - j * n_t;
    const double t_n = t0 + (double)(base + k) * dt;
    ttab[e] = time_factor(src, j, t_n + (double)s * dt_micro);
  }
  for (int e = first; e < S * nb; e += stride) {
    const int k = e / nb, q = e - k * nb;
    int i, j;
    boundary_node(g, q, i, j);
    bvals[e] = boundary_at(g, *desc, g.xi0 + i * g.Dxi, g.eta0 + j * g.Deta,
                           t0 + (double)(base + k + 1) * dt);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&clk->done, 1u) == gridDim.x - 1) {
      clk->base = base;
      clk->next = base + S;
      clk->done = 0u;
      __threadfence();
    }
  }
}

// k_replay for a batch: block i fills instance i's time factors and Dirichlet values for
// macro steps base .. base+S-1 (base = the shared clock's step count), in the same
// arithmetic as k_replay (t0 = the instance's t_n field, dt = its dt_macro); the last
// block advances the clock.
__global__ void k_batch_replay(const BurstArgs* __restrict__ inst,
                               const pd_coeff_desc* const* __restrict__ descs, int n, Clock* clk,
                               int S) {
  const long long base = clk->next;
  for (int b = blockIdx.x; b < n; b += gridDim.x) {
    const BurstArgs& A = inst[b];
    const int per = A.src.ns * A.n_t, nb = A.nb;
    const double t0 = A.t_n, dtm = A.dt_macro;
    double* ttab = const_cast<double*>(A.ttab);
    double* bv = const_cast<double*>(A.bvals);
    for (int e = threadIdx.x; e < S * per; e += blockDim.x) {
      const int k = e / per, r = e - k * per;
      const int j = r / A.n_t, s = r - j * A.n_t;
      const double t_n = t0 + (double)(base + k) * dtm;
      ttab[e] = time_factor(A.src, j, t_n + (double)s * A.dt);
    }
    for (int e = threadIdx.x; e < S * nb; e += blockDim.x) {
      const int k = e / nb, q = e - k * nb;
      int i, j;
      boundary_node(A.g, q, i, j);
      bv[e] = boundary_at(A.g, *descs[b], A.g.xi0 + i * A.g.Dxi, A.g.eta0 + j * A.g.Deta,
                          t0 + (double)(base + k + 1) * dtm);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&clk->done, 1u) == gridDim.x - 1) {
      clk->base = base;
      clk->next = base + S;
      clk->done = 0u;
      __threadfence();
    }
  }
}

// Static inputs of the learned closure per patch: the coefficients at the patch centre
// as rates on the macro spacing (alpha/Dxi^2, gamma/Deta^2, nu/Dxi, omega/Deta), phi, the
// micro-to-macro spacing ratios, and the source's spatial parts at the centre.
__global__ void k_closure_static(Geo g, SrcInfo src, const int* __restrict__ pmap,
                                 const double* __restrict__ coef, long long plane,
                                 double* __restrict__ st) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  const int i = pmap[11 * p], j = pmap[11 * p + 1];
  const long long at =
      (long long)p * g.m_xi * g.m_eta + (long long)(g.m_eta / 2) * g.m_xi + g.m_xi / 2;
  double* o = st + (long long)p * CL_NST;
  o[0] = i;
  o[1] = j;
  o[2] = coef[at] / (g.Dxi * g.Dxi);
  o[3] = coef[plane + at] / (g.Deta * g.Deta);
  o[4] = coef[2 * plane + at] / g.Dxi;
  o[5] = coef[3 * plane + at] / g.Deta;
  o[6] = coef[4 * plane + at];
  o[7] = g.dxi / g.Dxi;
  o[8] = g.deta / g.Deta;
  double gc = 0.0;
  for (int c = 0; c < src.nconst; ++c) gc += src.ca[c] * coef[src.plane_c[c] * plane + at];
  o[9] = gc;
  o[10] = src.ns > 0 ? coef[src.plane_t[0] * plane + at] : 0.0;
  o[11] = src.ns > 1 ? coef[src.plane_t[1] * plane + at] : 0.0;
}

__global__ void k_initial(Geo g, const pd_coeff_desc* __restrict__ desc, double* U, double t) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n_xi * g.n_eta) return;
  const int j = q / g.n_xi, i = q - j * g.n_xi;
  U[q] = boundary_at(g, *desc, g.xi0 + i * g.Dxi, g.eta0 + j * g.Deta, t);
}

__global__ void k_clock_init(Clock* clk, double t0, double dt, double* b0, double* b1) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    clk->t0 = t0;
    clk->dt = dt;
    clk->base = 0;
    clk->next = 0;
    clk->done = 0u;
    clk->buf[0] = b0;
    clk->buf[1] = b1;
  }
}

// ------------------------------------------------------------ full-domain lattice
// The lattice Geo: n_xi x n_eta nodes over the box with spacings Dxi, Deta (the box
// divided into n_xi intervals when xi is periodic, n_xi - 1 otherwise).

// Folded forward-Euler weights of every lattice node for the step dt: the operator of
// eq. (Computational_Problem) with 3-point second differences and 2-point upwind (the
// side the convection comes from) or central first differences, written as
//   u' = cC u + cS u_S + cN u_N + cW u_W + cE u_E + K + sum_j T_j(t) sd_j,
// cC = 1 + dt phi - (((E + W) + N) + S): the first-difference parts are differences of
// neighbours, so the weights of a row sum to 1 + dt phi.  Planes [cC, cS, cN, cW, cE, K,
// sd_0, sd_1] of `plane` doubles each; K holds the constant-in-time source terms.  Block
// minima of the explicit bound (0 where diffusion is not positive) go to partial.
__global__ void k_fd_weights(Geo g, const pd_coeff_desc* __restrict__ desc, SrcInfo src,
                             int n_src, double dt, double* __restrict__ W, long long plane,
                             double* __restrict__ partial) {
  __shared__ double red[256];
  double lim = INFINITY;
  const double hx = g.Dxi, hy = g.Deta;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < plane;
       q += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(q / g.n_xi), i = (int)(q - (long long)j * g.n_xi);
    double c[5 + PD_MAXTERM];
    coefficients_at(g, *desc, n_src, g.xi0 + i * hx, g.eta0 + j * hy, c);
    const double ax = c[0] / (hx * hx), ay = c[1] / (hy * hy);
    double e, w, n, so;
    if (g.conv == PD_CONV_CENTRAL) {
      e = ax - c[2] / (2.0 * hx);
      w = ax + c[2] / (2.0 * hx);
      n = ay - c[3] / (2.0 * hy);
      so = ay + c[3] / (2.0 * hy);
    } else {
      e = c[2] >= 0.0 ? ax : ax - c[2] / hx;
      w = c[2] >= 0.0 ? ax + c[2] / hx : ax;
      n = c[3] >= 0.0 ? ay : ay - c[3] / hy;
      so = c[3] >= 0.0 ? ay + c[3] / hy : ay;
    }
    const double E = dt * e, Wt = dt * w, N = dt * n, S = dt * so;
    W[q] = 1.0 + dt * c[4] - (((E + Wt) + N) + S);
    W[plane + q] = S;
    W[2 * plane + q] = N;
    W[3 * plane + q] = Wt;
    W[4 * plane + q] = E;
    double K = 0.0;
    for (int k = 0; k < src.nconst; ++k) K += src.ca[k] * c[src.plane_c[k]];
    W[5 * plane + q] = dt * K;
    for (int j2 = 0; j2 < src.ns; ++j2) W[(6 + j2) * plane + q] = dt * c[src.plane_t[j2]];
    const double b = (c[0] > 0.0 && c[1] > 0.0)
                         ? fe_bound(c[0], c[1], c[2], c[3], c[4], hx, hy)
                         : 0.0;
    lim = fmin(lim, b);
  }
  red[threadIdx.x] = lim;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_fd_limit_final(const double* __restrict__ partial, int nblocks,
                                 double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double lim = INFINITY;
  for (int b = 0; b < nblocks; ++b) lim = fmin(lim, partial[b]);
  out[0] = lim;
}

// Time factors and Dirichlet data of lattice steps s0 .. s0 + S - 1 (S <= FD_CHUNK; step
// s starts at t0 + s dt): ttab[j][k] = T_j(t0 + (s0 + k) dt) with rows of FD_CHUNK,
// bvals[k][q] = u_b(node q) at the end of step s0 + k.
__global__ void k_fd_tables(Geo g, SrcInfo src, const pd_coeff_desc* __restrict__ desc,
                            double t0, double dt, long long s0, int S,
                            double* __restrict__ ttab, double* __restrict__ bvals) {
  const int nb = boundary_count(g);
  const int stride = gridDim.x * blockDim.x, first = blockIdx.x * blockDim.x + threadIdx.x;
  for (int e = first; e < src.ns * S; e += stride) {
    const int j = e / S, k = e - j * S;
    ttab[j * FD_CHUNK + k] = time_factor(src, j, t0 + (double)(s0 + k) * dt);
  }
  for (int e = first; e < S * nb; e += stride) {
    const int k = e / nb, q = e - k * nb;
    int i, j;
    boundary_node(g, q, i, j);
    bvals[e] = boundary_at(g, *desc, g.xi0 + i * g.Dxi, g.eta0 + j * g.Deta,
                           (t0 + (double)(s0 + k) * dt) + dt);
  }
}

}  // namespace

hipError_t launch_coefficients(const Geo& g, const pd_coeff_desc* dev_desc, int n_src,
                               double* coef, hipStream_t s) {
  const long long npts = (long long)g.P * g.m_xi * g.m_eta;
  const int threads = 256;
  const long long blocks = (npts + threads - 1) / threads;
  hipLaunchKernelGGL(k_coefficients, dim3((unsigned)blocks), dim3(threads), 0, s, g, dev_desc,
                     n_src, coef);
  return hipGetLastError();
}

hipError_t launch_limits(const Geo& g, const pd_coeff_desc* dev_desc, int n_src,
                         const double* coef, double* partial, int nblocks, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_limits, dim3(nblocks), dim3(256), 0, s, g, dev_desc, n_src, coef,
                     partial);
  hipLaunchKernelGGL(k_limits_final, dim3(1), dim3(64), 0, s, partial, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_boundary(const Geo& g, const pd_coeff_desc* dev_desc, double* U, double t,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_boundary, dim3(1), dim3(256), 0, s, g, dev_desc, U, t);
  return hipGetLastError();
}

hipError_t launch_refresh_tables(const SrcInfo& src, double t_n, double dt, int n_t, int Q,
                                 double* out, hipStream_t s) {
  if (src.ns == 0) return hipSuccess;
  const int blocks = (src.ns * n_t + 255) / 256;
  hipLaunchKernelGGL(k_refresh_tables, dim3(blocks), dim3(256), 0, s, src, t_n, dt, n_t, Q, out);
  return hipGetLastError();
}

hipError_t launch_refresh_setup(const Geo& g, const pd_coeff_desc* dev_desc, double t_n,
                                double dt, int n_t, int Q, double t_end, double* out,
                                long long* flags, int nflags, hipStream_t s) {
  long long n = (long long)Q * boundary_count(g);
  if (n < nflags) n = nflags;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refresh_setup, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                     dev_desc, t_n, dt, n_t, Q, t_end, out, flags, nflags);
  return hipGetLastError();
}

static int refresh_blocks(const Geo& g) {
  return (g.P + RF_WAVES - 1) / RF_WAVES + (boundary_count(g) + RF_THREADS - 1) / RF_THREADS;
}

hipError_t launch_refresh_field(const Geo& g, const int* pmap, const pd_coeff_desc* dev_desc,
                                const double* state, double* Ubar, double* U, double t,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_refresh_field, dim3(refresh_blocks(g)), dim3(RF_THREADS), 0, s, g, pmap,
                     dev_desc, state, Ubar, U, t);
  return hipGetLastError();
}

hipError_t launch_refresh_final(const Geo& g, const int* pmap, const pd_coeff_desc* dev_desc,
                                const double* state, double* Ubar, const double* U_n,
                                double* U_np1, double dt_macro, double tau, int* flag,
                                double t, hipStream_t s) {
  hipLaunchKernelGGL(k_refresh_final, dim3(refresh_blocks(g)), dim3(RF_THREADS), 0, s, g, pmap,
                     dev_desc, state, Ubar, U_n, U_np1, dt_macro, tau, flag, t);
  return hipGetLastError();
}

hipError_t launch_closure_static(const Geo& g, const SrcInfo& src, const int* pmap,
                                 const double* coef, long long plane, double* st,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_closure_static, dim3((g.P + 255) / 256), dim3(256), 0, s, g, src, pmap,
                     coef, plane, st);
  return hipGetLastError();
}

hipError_t launch_batch_replay(const BurstArgs* inst, const pd_coeff_desc* const* descs, int n,
                               Clock* clk, int S, hipStream_t s) {
  const int blocks = n < 1024 ? n : 1024;
  hipLaunchKernelGGL(k_batch_replay, dim3(blocks), dim3(256), 0, s, inst, descs, n, clk, S);
  return hipGetLastError();
}

hipError_t launch_replay(const Geo& g, const SrcInfo& src, const pd_coeff_desc* dev_desc,
                         Clock* clk, int S, int n_t, double dt_micro, double* ttab,
                         double* bvals, hipStream_t s) {
  const long long work = (long long)S * (src.ns * n_t + boundary_count(g));
  long long blocks = (work + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 128 ? 128 : blocks);
  hipLaunchKernelGGL(k_replay, dim3((unsigned)blocks), dim3(256), 0, s, g, src, dev_desc, clk,
                     S, n_t, dt_micro, ttab, bvals);
  return hipGetLastError();
}

hipError_t launch_initial(const Geo& g, const pd_coeff_desc* dev_desc, double* U, double t,
                          hipStream_t s) {
  const int n = g.n_xi * g.n_eta;
  hipLaunchKernelGGL(k_initial, dim3((n + 255) / 256), dim3(256), 0, s, g, dev_desc, U, t);
  return hipGetLastError();
}

hipError_t launch_clock_init(Clock* clk, double t0, double dt, double* b0, double* b1,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_clock_init, dim3(1), dim3(64), 0, s, clk, t0, dt, b0, b1);
  return hipGetLastError();
}

hipError_t launch_fd_weights(const Geo& lat, const pd_coeff_desc* dev_desc, const SrcInfo& src,
                             int n_src, double dt, double* W, double* partial, int nblocks,
                             double* lim, hipStream_t s) {
  const long long plane = (long long)lat.n_xi * lat.n_eta;
  hipLaunchKernelGGL(k_fd_weights, dim3(nblocks), dim3(256), 0, s, lat, dev_desc, src, n_src,
                     dt, W, plane, partial);
  hipLaunchKernelGGL(k_fd_limit_final, dim3(1), dim3(64), 0, s, partial, nblocks, lim);
  return hipGetLastError();
}

hipError_t launch_fd_tables(const Geo& lat, const SrcInfo& src, const pd_coeff_desc* dev_desc,
                            double t0, double dt, long long s0, int S, double* ttab,
                            double* bvals, hipStream_t s) {
  const long long work = (long long)S * (boundary_count(lat) > src.ns ? boundary_count(lat)
                                                                       : src.ns);
  long long blocks = (work + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(k_fd_tables, dim3((unsigned)blocks), dim3(256), 0, s, lat, src, dev_desc,
                     t0, dt, s0, S, ttab, bvals);
  return hipGetLastError();
}

}  // namespace pdk
