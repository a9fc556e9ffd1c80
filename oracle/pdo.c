/*
 * pdo.c -- plain, slow FP64 CPU oracle of the curvilinear patch dynamics scheme
 * (arXiv 2405.08764).  TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product path.
 *
 * Written from the paper; shares nothing with the HIP library.  Build:
 *   gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared pdo.c -o libpdo.so -lm
 * and, for the extended-precision reference of the same steps,
 *   gcc ... -DPDO_REAL="long double" pdo.c -o libpdo_ld.so -lm
 *
 * Parity pins (each checked by a CPU test against something other than this file):
 *   coefficients      Sec. 4.1.1, 4.1.2 and 4.2 closed-form coefficient lists; on every
 *                     other map and field kind (tanh map, Fourier D11 != D22 and v, polar
 *                     k(r, theta), Fourier fields on the annulus) the transformed operator
 *                     of eq. (Computational_Problem) against eq. (Physical_Problem)
 *                     differentiated symbolically, with the source planes and the map
 *                     derivatives, and planted mistakes in these branches rejected
 *   source            the printed sources of Sec. 4.1.1 / 4.1.2 (exact solution e^{x+y+t})
 *   edge gradients    exact derivative of quadratic macro fields; eq. (edge) weights
 *   lift              quadratic exactness; restriction of the lift returns U
 *   restriction       trapezoid moments of 1, s, s^2 (closed forms)
 *   burst             quadratic fields evolve exactly; constant fields stay constant;
 *                     mirror symmetry of the upwind direction; brute-force full-domain
 *   macro step        closed-form 9-point macro stencil for constant diffusion (any n_t)
 *   whole scheme      manufactured-solution convergence on square and annulus; the
 *                     Fourier-Bessel series of Sec. 4.2 (ballpark of Table P2_PerErr)
 *   full domain       quadratic (central) and linear (upwind) steady states with the
 *                     manufactured source; constants kept on a mapped box;
 *                     manufactured convergence (central order 2, upwind order 1);
 *                     it is also the brute-force reference patch dynamics converges to
 * The readings taken where the paper is silent are listed where they are used.
 */
#include "pdo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Arithmetic type of the edge data, lift, burst, restriction and projective step.  The
 * default build is FP64; building with -DPDO_REAL="long double" gives the same algorithm
 * in x87 extended precision, which measures the FP64 build's own round-off floor. */
#ifndef PDO_REAL
#define PDO_REAL double
#endif
typedef PDO_REAL real;

static int g_threads = 1;

void pdo_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int pdo_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------ grid, Sec. 3 -- */

/* Macro spacing, Sec. 3: Delta = (b - a)/N with N intervals; a periodic axis has N
 * unique nodes. */
static double dxi(const pdo_grid* g) {
  return g->periodic_xi ? (g->xi1 - g->xi0) / g->n_xi : (g->xi1 - g->xi0) / (g->n_xi - 1);
}
static double deta(const pdo_grid* g) { return (g->eta1 - g->eta0) / (g->n_eta - 1); }

/* Micro spacing: m points span the patch edge h, edges included. */
static double micro_off(double h, int m, int k) {
  return (double)(2 * k - (m - 1)) * (h / (2.0 * (m - 1)));
}

/* Patches sit on interior nodes, Sec. 3 (every node along a periodic axis). */
static int first_pi(const pdo_grid* g) { return g->periodic_xi ? 0 : 1; }
static int npatch_xi(const pdo_grid* g) { return g->periodic_xi ? g->n_xi : g->n_xi - 2; }
static int npatch_eta(const pdo_grid* g) { return g->n_eta - 2; }

int pdo_num_patches(const pdo_grid* g) { return npatch_xi(g) * npatch_eta(g); }

static void patch_ij(const pdo_grid* g, int p, int* i, int* j) {
  int nx = npatch_xi(g);
  *i = first_pi(g) + p % nx;
  *j = 1 + p / nx;
}

static int wrap_i(const pdo_grid* g, int i) {
  if (!g->periodic_xi) return i;
  if (i < 0) return i + g->n_xi;
  if (i >= g->n_xi) return i - g->n_xi;
  return i;
}

void pdo_patch_map(const pdo_grid* g, int* out) {
  int P = pdo_num_patches(g);
  for (int p = 0; p < P; ++p) {
    int i, j;
    patch_ij(g, p, &i, &j);
    int* o = out + 11 * p;
    o[0] = i;
    o[1] = j;
    int c = 2;
    for (int b = -1; b <= 1; ++b)
      for (int a = -1; a <= 1; ++a) o[c++] = (j + b) * g->n_xi + wrap_i(g, i + a);
  }
}

static int is_sq_box01(const pdo_grid* g) {
  return g->xi0 == 0.0 && g->xi1 == 1.0 && g->eta0 == 0.0 && g->eta1 == 1.0;
}

static int field_ok(const pdo_field* f, int polar_ok) {
  if (f->nmode < 0 || f->nmode > PDO_MAXMODE) return 0;
  if (f->npolar < 0 || f->npolar > PDO_MAXPOLAR) return 0;
  if (f->npolar > 0 && !polar_ok) return 0;
  return 1;
}

int pdo_check(const pdo_grid* g, const pdo_problem* pr) {
  if (g->n_xi < 3 || g->n_eta < 3 || g->m_xi < 3 || g->m_eta < 3) return PDO_EINVAL;
  if (!(g->xi1 > g->xi0) || !(g->eta1 > g->eta0)) return PDO_EINVAL;
  if (!(g->h_xi > 0.0) || !(g->h_eta > 0.0)) return PDO_EINVAL;
  /* Sec. 3: h / Delta < 1, so patches never overlap. */
  if (!(g->h_xi < dxi(g)) || !(g->h_eta < deta(g))) return PDO_EINVAL;
  if (g->conv != PDO_CONV_UPWIND && g->conv != PDO_CONV_CENTRAL) return PDO_EINVAL;
  if (g->c0mode != PDO_C0_TRAPEZOID && g->c0mode != PDO_C0_PRINTED) return PDO_EINVAL;
  if (g->core_points != 0 &&
      (g->core_points < 2 || g->core_points > g->m_xi || g->core_points > g->m_eta ||
       (g->m_xi - g->core_points) % 2 != 0 || (g->m_eta - g->core_points) % 2 != 0))
    return PDO_EINVAL;
  int annulus = g->geometry == PDO_GEOM_ANNULUS;
  switch (g->geometry) {
    case PDO_GEOM_IDENTITY: break;
    case PDO_GEOM_SINE:
      if (!is_sq_box01(g) || !(g->gparam >= 0.0 && g->gparam < 1.0)) return PDO_EINVAL;
      break;
    case PDO_GEOM_TANH:
      if (!is_sq_box01(g) || !(g->gparam >= 0.0)) return PDO_EINVAL;
      break;
    case PDO_GEOM_ANNULUS:
      if (!(g->eta0 > 0.0) || !g->periodic_xi) return PDO_EINVAL;
      break;
    default: return PDO_EINVAL;
  }
  if (!field_ok(&pr->D11, annulus) || !field_ok(&pr->D22, annulus) ||
      !field_ok(&pr->v1, annulus) || !field_ok(&pr->v2, annulus) || !field_ok(&pr->f, annulus))
    return PDO_EINVAL;
  /* A diagonal tensor in the Cartesian frame keeps eq. (Computational_Problem) free of a
   * mixed derivative only for maps with x = x(xi), y = y(eta); the annulus takes the
   * paper's scalar D. */
  if (annulus && memcmp(&pr->D11, &pr->D22, sizeof(pdo_field)) != 0) return PDO_EINVAL;
  if (pr->n_bc < 0 || pr->n_bc > PDO_MAXTERM || pr->n_src < 0 || pr->n_src > PDO_MAXTERM)
    return PDO_EINVAL;
  for (int m = 0; m < pr->n_bc; ++m)
    if (pr->bc_s[m].kind == 1 && !annulus) return PDO_EINVAL;
  for (int k = 0; k < pr->n_src; ++k)
    if (pr->src_s[k].kind == 1 && !annulus) return PDO_EINVAL;
  return PDO_OK;
}

/* --------------------------------------------- Lagrange basis, eq. (Lagrange_2D) -- */

/* L_beta(t) = prod_{r != beta} (t - o_r) / (o_beta - o_r), nodes o = (-D, 0, +D)
 * relative to the patch centre; numerator and denominator multiplied in r order. */
static double lagrange(int beta, double t, double D) {
  const double o[3] = {-D, 0.0, D};
  double num = 1.0, den = 1.0;
  int first = 1;
  for (int r = 0; r < 3; ++r) {
    if (r == beta) continue;
    if (first) {
      num = t - o[r];
      den = o[beta] - o[r];
      first = 0;
    } else {
      num = num * (t - o[r]);
      den = den * (o[beta] - o[r]);
    }
  }
  return num / den;
}

/* eq. (edge) weights on (U_{i-1}, U_i, U_{i+1}) for the edge at xi_i + side h/2,
 * side = -1 or +1, r = h / (2 Delta). */
static void edge_weights(double r, int side, double* w) {
  if (side < 0) {
    w[0] = -0.5 - r;
    w[1] = 2.0 * r;
    w[2] = 0.5 - r;
  } else {
    w[0] = -0.5 + r;
    w[1] = -2.0 * r;
    w[2] = 0.5 + r;
  }
}

/* The restriction's core: the central n of the m micro points of a side (n = m, the whole
 * patch, unless core_points is set), first index k0.  Sec. 2 of the paper leaves the
 * averaging region open ("core average"); a smaller core is the buffer idea of gap-tooth
 * schemes, kept here as an option. */
static void core_range(const pdo_grid* g, int m, int* k0, int* n) {
  *n = g->core_points > 0 ? g->core_points : m;
  *k0 = (m - *n) / 2;
}

/* eq. (C_0): C0 = U - kappa_xi U_xixi - kappa_eta U_etaeta.  The paper obtains C0 from
 * the averaging property of eq. (Averaging); with the composite trapezoidal rule that it
 * uses for the restriction, the discrete average of s^2/2 over the n core points (spanning
 * hc = (n - 1) delta, the whole patch h by default) is hc^2/24 + delta^2/12, so the
 * trapezoid reading keeps R(lift) = U exactly.  The printed hc^2/24 is PDO_C0_PRINTED. */
static double kappa(const pdo_grid* g, double h, int m) {
  double d = h / (m - 1);
  int k0, n;
  core_range(g, m, &k0, &n);
  double hc = (n - 1) * d;
  if (g->c0mode == PDO_C0_PRINTED) return hc * hc / 24.0;
  return hc * hc / 24.0 + d * d / 12.0;
}

int pdo_tables_size(const pdo_grid* g) {
  return g->m_xi + g->m_eta + 3 * g->m_eta + 3 * g->m_xi + 12 + g->m_xi + g->m_eta + 8;
}

/* Layout: s_xi[m_xi], s_eta[m_eta], Lq for the xi edges [m_eta][3] (interpolation in eta),
 * Lq for the eta edges [m_xi][3], edge weights xi (minus 3, plus 3), eta (minus 3, plus 3),
 * trapezoid weights c_k [m_xi], [m_eta], then Dxi, Deta, dxi, deta, r_xi, r_eta,
 * kappa_xi, kappa_eta. */
void pdo_tables(const pdo_grid* g, double* out) {
  int mx = g->m_xi, me = g->m_eta;
  double Dx = dxi(g), De = deta(g);
  double* o = out;
  for (int k = 0; k < mx; ++k) *o++ = micro_off(g->h_xi, mx, k);
  for (int l = 0; l < me; ++l) *o++ = micro_off(g->h_eta, me, l);
  for (int l = 0; l < me; ++l)
    for (int q = 0; q < 3; ++q) *o++ = lagrange(q, micro_off(g->h_eta, me, l), De);
  for (int k = 0; k < mx; ++k)
    for (int q = 0; q < 3; ++q) *o++ = lagrange(q, micro_off(g->h_xi, mx, k), Dx);
  double rx = g->h_xi / (2.0 * Dx), re = g->h_eta / (2.0 * De);
  edge_weights(rx, -1, o); o += 3;
  edge_weights(rx, +1, o); o += 3;
  edge_weights(re, -1, o); o += 3;
  edge_weights(re, +1, o); o += 3;
  int kx0, nx, le0, ne;
  core_range(g, mx, &kx0, &nx);
  core_range(g, me, &le0, &ne);
  for (int k = 0; k < mx; ++k)
    *o++ = (k < kx0 || k > kx0 + nx - 1) ? 0.0 : ((k == kx0 || k == kx0 + nx - 1) ? 0.5 : 1.0);
  for (int l = 0; l < me; ++l)
    *o++ = (l < le0 || l > le0 + ne - 1) ? 0.0 : ((l == le0 || l == le0 + ne - 1) ? 0.5 : 1.0);
  *o++ = Dx;
  *o++ = De;
  *o++ = g->h_xi / (mx - 1);
  *o++ = g->h_eta / (me - 1);
  *o++ = rx;
  *o++ = re;
  *o++ = kappa(g, g->h_xi, mx);
  *o++ = kappa(g, g->h_eta, me);
}

/* ------------------------------------------------- metric, Sec. 2.1, 4.1.1, 4.2 -- */

typedef struct {
  double x, y, xs, ys, xe, ye, xss, yss, xee, yee, xse, yse;
} mapv;

static void map_eval(const pdo_grid* g, double xi, double eta, mapv* m) {
  memset(m, 0, sizeof(*m));
  switch (g->geometry) {
    case PDO_GEOM_SINE: { /* eq. (Stretching_Transformation) */
      double l = g->gparam;
      m->x = xi + (l / M_PI) * sin(M_PI * xi);
      m->y = eta + (l / M_PI) * sin(M_PI * eta);
      m->xs = 1.0 + l * cos(M_PI * xi);
      m->ye = 1.0 + l * cos(M_PI * eta);
      m->xss = -l * M_PI * sin(M_PI * xi);
      m->yee = -l * M_PI * sin(M_PI * eta);
      break;
    }
    case PDO_GEOM_TANH: { /* x = tanh(b xi)/tanh b: clusters nodes at x = 1 */
      double b = g->gparam;
      if (b == 0.0) {
        m->x = xi;
        m->y = eta;
        m->xs = 1.0;
        m->ye = 1.0;
        break;
      }
      double tb = tanh(b);
      double Tx = tanh(b * xi), Ty = tanh(b * eta);
      double sx = 1.0 - Tx * Tx, sy = 1.0 - Ty * Ty;
      m->x = Tx / tb;
      m->y = Ty / tb;
      m->xs = b * sx / tb;
      m->ye = b * sy / tb;
      m->xss = -2.0 * b * b * Tx * sx / tb;
      m->yee = -2.0 * b * b * Ty * sy / tb;
      break;
    }
    case PDO_GEOM_ANNULUS: { /* eq. (Transformation_Annulus): xi = theta, eta = r */
      double c = cos(xi), s = sin(xi);
      m->x = eta * c;
      m->y = eta * s;
      m->xs = -eta * s;
      m->ys = eta * c;
      m->xe = c;
      m->ye = s;
      m->xss = -eta * c;
      m->yss = -eta * s;
      m->xse = -s;
      m->yse = c;
      break;
    }
    default:
      m->x = xi;
      m->y = eta;
      m->xs = 1.0;
      m->ye = 1.0;
      break;
  }
}

void pdo_metric(const pdo_grid* g, double xi, double eta, double* out) {
  mapv m;
  map_eval(g, xi, eta, &m);
  out[0] = m.x; out[1] = m.y;
  out[2] = m.xs; out[3] = m.ys; out[4] = m.xe; out[5] = m.ye;
  out[6] = m.xss; out[7] = m.yss; out[8] = m.xee; out[9] = m.yee;
  out[10] = m.xse; out[11] = m.yse;
  out[12] = sqrt(m.xs * m.xs + m.ys * m.ys);
  out[13] = sqrt(m.xe * m.xe + m.ye * m.ye);
  out[14] = m.xs * m.ye - m.xe * m.ys;
  out[15] = 0.0;
}

/* ------------------------------------------------------------- physical fields -- */

static void field_eval(const pdo_field* F, double x, double y, int polar, double r, double th,
                       double* val, double* gx, double* gy) {
  double v = F->c0 + F->cx * x + F->cy * y;
  double fx = F->cx, fy = F->cy;
  for (int k = 0; k < F->nmode; ++k) {
    double a = F->kx[k] * x + F->ky[k] * y + F->ph[k];
    double c = cos(a), s = sin(a);
    v += F->amp[k] * c;
    fx -= F->amp[k] * F->kx[k] * s;
    fy -= F->amp[k] * F->ky[k] * s;
  }
  if (polar) {
    double ct = cos(th), st = sin(th);
    for (int p = 0; p < F->npolar; ++p) {
      double P = F->pc0[p] + F->pc1[p] * r + F->pc2[p] * r * r;
      double Pr = F->pc1[p] + 2.0 * F->pc2[p] * r;
      double a = F->pn[p] * th + F->pph[p];
      double C = cos(a), S = sin(a);
      double Fr = F->pamp[p] * Pr * C;
      double Ft = -F->pamp[p] * P * F->pn[p] * S;
      v += F->pamp[p] * P * C;
      fx += ct * Fr - st / r * Ft;
      fy += st * Fr + ct / r * Ft;
    }
  }
  *val = v;
  *gx = fx;
  *gy = fy;
}

static void fn1_eval(const pdo_fn1* f, double s, double* v, double* d1, double* d2) {
  switch (f->type) {
    case PDO_FN_SIN: {
      double a = f->a * s + f->b;
      *v = sin(a);
      *d1 = f->a * cos(a);
      *d2 = -f->a * f->a * sin(a);
      break;
    }
    case PDO_FN_COS: {
      double a = f->a * s + f->b;
      *v = cos(a);
      *d1 = -f->a * sin(a);
      *d2 = -f->a * f->a * cos(a);
      break;
    }
    case PDO_FN_EXP: {
      double e = exp(f->a * s + f->b);
      *v = e;
      *d1 = f->a * e;
      *d2 = f->a * f->a * e;
      break;
    }
    default: {
      *v = f->a + f->b * s + f->c * s * s + f->d * s * s * s;
      *d1 = f->b + 2.0 * f->c * s + 3.0 * f->d * s * s;
      *d2 = 2.0 * f->c + 6.0 * f->d * s;
      break;
    }
  }
}

static double tfun_eval(const pdo_tfun* T, double t) {
  switch (T->type) {
    case PDO_T_EXP: return T->a * exp(T->b * t);
    case PDO_T_SIN: return T->a + T->b * sin(T->c * t);
    default: return T->a;
  }
}

/* A separable function and its derivatives in the computational coordinates. */
typedef struct { double v, s, e, ss, ee; } sder;

static void sfun_eval(const pdo_sfun* S, const mapv* m, double xi, double eta, sder* o) {
  double f, f1, f2, q, q1, q2;
  if (S->kind == 1) { /* amp f(r) g(theta) on the annulus: r = eta, theta = xi */
    fn1_eval(&S->f, eta, &f, &f1, &f2);
    fn1_eval(&S->g, xi, &q, &q1, &q2);
    o->v = S->amp * f * q;
    o->s = S->amp * f * q1;
    o->ss = S->amp * f * q2;
    o->e = S->amp * f1 * q;
    o->ee = S->amp * f2 * q;
    return;
  }
  fn1_eval(&S->f, m->x, &f, &f1, &f2);
  fn1_eval(&S->g, m->y, &q, &q1, &q2);
  double Sx = S->amp * f1 * q, Sy = S->amp * f * q1;
  double Sxx = S->amp * f2 * q, Syy = S->amp * f * q2, Sxy = S->amp * f1 * q1;
  o->v = S->amp * f * q;
  o->s = Sx * m->xs + Sy * m->ys;
  o->e = Sx * m->xe + Sy * m->ye;
  o->ss = Sxx * m->xs * m->xs + 2.0 * Sxy * m->xs * m->ys + Syy * m->ys * m->ys +
          Sx * m->xss + Sy * m->yss;
  o->ee = Sxx * m->xe * m->xe + 2.0 * Sxy * m->xe * m->ye + Syy * m->ye * m->ye +
          Sx * m->xee + Sy * m->yee;
}

/* Coefficients of eq. (Computational_Problem) for an orthogonal map (beta = 0), written
 * with the scale factors h1 = |dr/dxi|, h2 = |dr/deta|:
 *   div(D grad u) = (1/(h1 h2)) [ d_xi(D11 h2/h1 u_xi) + d_eta(D22 h1/h2 u_eta) ],
 *   v . grad u   = (v . r_xi)/h1^2 u_xi + (v . r_eta)/h2^2 u_eta,
 *   div(v u)     = v . grad u + (div v) u,
 * so alpha = D11/h1^2, gamma = D22/h2^2,
 *    nu    = (v . r_xi)/h1^2  - (1/(h1 h2)) d_xi (D11 h2/h1),
 *    omega = (v . r_eta)/h2^2 - (1/(h1 h2)) d_eta(D22 h1/h2),
 *    phi   = f - div v.
 * This is the sign convention of eq. (Computational_Problem) (u_t = ... - nu u_xi ...);
 * it reproduces the worked coefficient lists of Sec. 4.1.1, 4.1.2 and 4.2 exactly,
 * while the general nu, omega printed under eq. (Computational_Problem), read literally,
 * give their negatives; the worked examples decide. */
typedef struct { double alpha, gamma, nu, omega, phi; } coefv;

static void coef_eval(const pdo_grid* g, const pdo_problem* pr, double xi, double eta,
                      mapv* m, coefv* c) {
  map_eval(g, xi, eta, m);
  int polar = g->geometry == PDO_GEOM_ANNULUS;
  double r = eta, th = xi;
  double h1 = sqrt(m->xs * m->xs + m->ys * m->ys);
  double h2 = sqrt(m->xe * m->xe + m->ye * m->ye);
  double h1s = (m->xs * m->xss + m->ys * m->yss) / h1;
  double h1e = (m->xs * m->xse + m->ys * m->yse) / h1;
  double h2s = (m->xe * m->xse + m->ye * m->yse) / h2;
  double h2e = (m->xe * m->xee + m->ye * m->yee) / h2;
  double D11, D11x, D11y, D22, D22x, D22y, v1, v1x, v1y, v2, v2x, v2y, f, fx, fy;
  field_eval(&pr->D11, m->x, m->y, polar, r, th, &D11, &D11x, &D11y);
  field_eval(&pr->D22, m->x, m->y, polar, r, th, &D22, &D22x, &D22y);
  field_eval(&pr->v1, m->x, m->y, polar, r, th, &v1, &v1x, &v1y);
  field_eval(&pr->v2, m->x, m->y, polar, r, th, &v2, &v2x, &v2y);
  field_eval(&pr->f, m->x, m->y, polar, r, th, &f, &fx, &fy);
  double D11s = D11x * m->xs + D11y * m->ys;
  double D22e = D22x * m->xe + D22y * m->ye;
  c->alpha = D11 / (h1 * h1);
  c->gamma = D22 / (h2 * h2);
  c->nu = (v1 * m->xs + v2 * m->ys) / (h1 * h1) -
          (D11s * h2 / h1 + D11 * (h2s * h1 - h2 * h1s) / (h1 * h1)) / (h1 * h2);
  c->omega = (v1 * m->xe + v2 * m->ye) / (h2 * h2) -
             (D22e * h1 / h2 + D22 * (h1e * h2 - h1 * h2e) / (h2 * h2)) / (h1 * h2);
  c->phi = f - (v1x + v2y);
}

/* Spatial part of source term k: sigma = c S - L[S] with L the operator of
 * eq. (Computational_Problem) (equal to the physical operator of
 * eq. (Physical_Problem) under the map).  A manufactured solution T(t) S(x,y) has source
 * T' S - T L[S] = T (c S - L[S]) with c = T'/T. */
static double source_sigma(const pdo_problem* pr, int k, const mapv* m, const coefv* c,
                           double xi, double eta) {
  sder S;
  sfun_eval(&pr->src_s[k], m, xi, eta, &S);
  double L = c->alpha * S.ss + c->gamma * S.ee - c->nu * S.s - c->omega * S.e + c->phi * S.v;
  return pr->src_c[k] * S.v - L;
}

void pdo_coeffs_at(const pdo_grid* g, const pdo_problem* pr, double xi, double eta,
                   double* out) {
  mapv m;
  coefv c;
  coef_eval(g, pr, xi, eta, &m, &c);
  out[0] = c.alpha;
  out[1] = c.gamma;
  out[2] = c.nu;
  out[3] = c.omega;
  out[4] = c.phi;
  for (int k = 0; k < pr->n_src; ++k) out[5 + k] = source_sigma(pr, k, &m, &c, xi, eta);
}

static double node_xi(const pdo_grid* g, int i) { return g->xi0 + i * dxi(g); }
static double node_eta(const pdo_grid* g, int j) { return g->eta0 + j * deta(g); }

void pdo_coefficients_masked(const pdo_grid* g, const pdo_problem* pr,
                             const unsigned char* mask, double* coef) {
  int P = pdo_num_patches(g), mx = g->m_xi, me = g->m_eta;
  int nc = PDO_NCOEF(pr);
  size_t plane = (size_t)P * mx * me;
  double out[5 + PDO_MAXTERM];
  for (int p = 0; p < P; ++p) {
    if (mask && !mask[p]) continue;
    int i, j;
    patch_ij(g, p, &i, &j);
    for (int l = 0; l < me; ++l)
      for (int k = 0; k < mx; ++k) {
        double xi = node_xi(g, i) + micro_off(g->h_xi, mx, k);
        double eta = node_eta(g, j) + micro_off(g->h_eta, me, l);
        pdo_coeffs_at(g, pr, xi, eta, out);
        size_t at = ((size_t)p * me + l) * mx + k;
        for (int q = 0; q < nc; ++q) coef[q * plane + at] = out[q];
      }
  }
}

void pdo_coefficients(const pdo_grid* g, const pdo_problem* pr, double* coef) {
  pdo_coefficients_masked(g, pr, NULL, coef);
}

static double sfun_value(const pdo_sfun* S, const mapv* m, double xi, double eta) {
  sder d;
  sfun_eval(S, m, xi, eta, &d);
  return d.v;
}

double pdo_boundary_value(const pdo_grid* g, const pdo_problem* pr, double xi, double eta,
                          double t) {
  mapv m;
  map_eval(g, xi, eta, &m);
  double u = 0.0;
  for (int q = 0; q < pr->n_bc; ++q)
    u += tfun_eval(&pr->bc_t[q], t) * sfun_value(&pr->bc_s[q], &m, xi, eta);
  return u;
}

void pdo_initial(const pdo_grid* g, const pdo_problem* pr, double t, double* U) {
  for (int j = 0; j < g->n_eta; ++j)
    for (int i = 0; i < g->n_xi; ++i)
      U[j * g->n_xi + i] = pdo_boundary_value(g, pr, node_xi(g, i), node_eta(g, j), t);
}

/* ---------------------------------------------------- step (i): eq. (edge) -------- */

static int mmax(const pdo_grid* g) { return g->m_xi > g->m_eta ? g->m_xi : g->m_eta; }

/* Gradients of the bi-quadratic interpolant of the 3x3 macro neighbourhood normal to the
 * four patch edges, at the micro points of each edge (kept fixed over the burst: the
 * Q = 1 case). */
static void edge_patch(const pdo_grid* g, const double* U, int p, real* e) {
  int i, j;
  patch_ij(g, p, &i, &j);
  int nx = g->n_xi, mx = g->m_xi, me = g->m_eta, M = mmax(g);
  double Dx = dxi(g), De = deta(g);
  double rx = g->h_xi / (2.0 * Dx), re = g->h_eta / (2.0 * De);
  int im = wrap_i(g, i - 1), ip = wrap_i(g, i + 1);
  int ii[3] = {im, i, ip};
  double wm[3], wp[3];
  /* xi edges: interpolate along eta (L_q^j) at every micro row. */
  edge_weights(rx, -1, wm);
  edge_weights(rx, +1, wp);
  for (int l = 0; l < me; ++l) {
    double t = micro_off(g->h_eta, me, l);
    double L[3] = {lagrange(0, t, De), lagrange(1, t, De), lagrange(2, t, De)};
    real Pc[3];
    for (int a = 0; a < 3; ++a) {
      Pc[a] = (real)L[0] * U[(j - 1) * nx + ii[a]] + (real)L[1] * U[j * nx + ii[a]] +
              (real)L[2] * U[(j + 1) * nx + ii[a]];
    }
    e[0 * M + l] = ((real)wm[0] * Pc[0] + (real)wm[1] * Pc[1] + (real)wm[2] * Pc[2]) / Dx;
    e[1 * M + l] = ((real)wp[0] * Pc[0] + (real)wp[1] * Pc[1] + (real)wp[2] * Pc[2]) / Dx;
  }
  /* eta edges: interpolate along xi (L_p^i) at every micro column. */
  edge_weights(re, -1, wm);
  edge_weights(re, +1, wp);
  for (int k = 0; k < mx; ++k) {
    double s = micro_off(g->h_xi, mx, k);
    double L[3] = {lagrange(0, s, Dx), lagrange(1, s, Dx), lagrange(2, s, Dx)};
    real Pr[3];
    for (int b = 0; b < 3; ++b) {
      int jj = j - 1 + b;
      Pr[b] = (real)L[0] * U[jj * nx + im] + (real)L[1] * U[jj * nx + i] +
              (real)L[2] * U[jj * nx + ip];
    }
    e[2 * M + k] = ((real)wm[0] * Pr[0] + (real)wm[1] * Pr[1] + (real)wm[2] * Pr[2]) / De;
    e[3 * M + k] = ((real)wp[0] * Pr[0] + (real)wp[1] * Pr[1] + (real)wp[2] * Pr[2]) / De;
  }
}

void pdo_edge(const pdo_grid* g, const double* U, double* edge) {
  int P = pdo_num_patches(g), M = mmax(g);
  real* e = (real*)calloc(4 * M, sizeof(real)); /* entries past an edge's length stay 0 */
  for (int p = 0; p < P; ++p) {
    edge_patch(g, U, p, e);
    for (int q = 0; q < 4 * M; ++q) edge[(size_t)p * 4 * M + q] = (double)e[q];
  }
  free(e);
}

/* ------------------------------------------------ step (ii): eq. (Lifting) -------- */

/* Derivatives in eq. (Lifting) and eq. (C_0) by central differences at the node, which
 * are the derivatives of the bi-quadratic interpolant eq. (Lagrange_2D) there. */
static void lift_patch(const pdo_grid* g, const double* U, int p, real* u) {
  int i, j;
  patch_ij(g, p, &i, &j);
  int nx = g->n_xi, mx = g->m_xi, me = g->m_eta;
  double Dx = dxi(g), De = deta(g);
  int im = wrap_i(g, i - 1), ip = wrap_i(g, i + 1);
  real Uc = U[j * nx + i];
  real Ux = ((real)U[j * nx + ip] - U[j * nx + im]) / (2.0 * Dx);
  real Ue = ((real)U[(j + 1) * nx + i] - U[(j - 1) * nx + i]) / (2.0 * De);
  real Uxx = ((real)U[j * nx + ip] - 2.0 * Uc + U[j * nx + im]) / (Dx * Dx);
  real Uee = ((real)U[(j + 1) * nx + i] - 2.0 * Uc + U[(j - 1) * nx + i]) / (De * De);
  real Uxe = ((real)U[(j + 1) * nx + ip] - U[(j - 1) * nx + ip] - U[(j + 1) * nx + im] +
              U[(j - 1) * nx + im]) / (4.0 * Dx * De);
  real C0 = Uc - kappa(g, g->h_xi, mx) * Uxx - kappa(g, g->h_eta, me) * Uee;
  for (int l = 0; l < me; ++l) {
    real t = micro_off(g->h_eta, me, l);
    for (int k = 0; k < mx; ++k) {
      real s = micro_off(g->h_xi, mx, k);
      u[l * mx + k] =
          C0 + s * Ux + t * Ue + 0.5 * s * s * Uxx + s * t * Uxe + 0.5 * t * t * Uee;
    }
  }
}

void pdo_lift(const pdo_grid* g, const double* U, double* u) {
  int P = pdo_num_patches(g);
  size_t pm = (size_t)g->m_xi * g->m_eta;
  real* w = (real*)malloc(pm * sizeof(real));
  for (int p = 0; p < P; ++p) {
    lift_patch(g, U, p, w);
    for (size_t q = 0; q < pm; ++q) u[p * pm + q] = (double)w[q];
  }
  free(w);
}

/* ----------------------------------------------- step (iii): the micro burst ------ */

/* Explicit forward Euler (Sec. 4.2) on eq. (Computational_Problem) inside one patch:
 * 3-point central second differences, first derivatives by the 2-point upwind formula of
 * Sec. 4.1.1 (backward when nu >= 0, forward when nu < 0, since the paper's formula
 * assumes a non-negative velocity) or by central differences as in eq. (MOL_Diff_Annu).
 * The Neumann edge data enter through ghost points: (u_1 - u_{-1})/(2 delta) = g^- and
 * (u_m - u_{m-2})/(2 delta) = g^+, used by every difference that reaches past an edge;
 * corners take both ghosts independently.  Every point advances from the old level. */
static int burst_patch(const pdo_grid* g, const pdo_problem* pr, const double* coef,
                       size_t plane, int p, real* u, const real* e, double t_n, double dt,
                       int n_t, real* w) {
  int mx = g->m_xi, me = g->m_eta, M = mmax(g), nsrc = pr->n_src;
  real dx = g->h_xi / (mx - 1), de = g->h_eta / (me - 1);
  size_t pm = (size_t)mx * me;
  const double* A = coef + 0 * plane + p * pm;
  const double* G = coef + 1 * plane + p * pm;
  const double* N = coef + 2 * plane + p * pm;
  const double* W = coef + 3 * plane + p * pm;
  const double* F = coef + 4 * plane + p * pm;
  const real* gxm = e + 0 * M;
  const real* gxp = e + 1 * M;
  const real* gem = e + 2 * M;
  const real* gep = e + 3 * M;
  real* cur = u;
  real* nxt = w;
  for (int step = 0; step < n_t; ++step) {
    double t = t_n + step * dt;
    double T[PDO_MAXTERM];
    for (int q = 0; q < nsrc; ++q) T[q] = tfun_eval(&pr->src_t[q], t);
    for (int l = 0; l < me; ++l)
      for (int k = 0; k < mx; ++k) {
        size_t at = (size_t)l * mx + k;
        real uc = cur[at];
        real uW = k > 0 ? cur[at - 1] : cur[at + 1] - 2.0 * dx * gxm[l];
        real uE = k < mx - 1 ? cur[at + 1] : cur[at - 1] + 2.0 * dx * gxp[l];
        real uS = l > 0 ? cur[at - mx] : cur[at + mx] - 2.0 * de * gem[k];
        real uN = l < me - 1 ? cur[at + mx] : cur[at - mx] + 2.0 * de * gep[k];
        real dxx = (uE - 2.0 * uc + uW) / (dx * dx);
        real dee = (uN - 2.0 * uc + uS) / (de * de);
        real nu = N[at], om = W[at], dx1, de1;
        if (g->conv == PDO_CONV_CENTRAL) {
          dx1 = (uE - uW) / (2.0 * dx);
          de1 = (uN - uS) / (2.0 * de);
        } else {
          dx1 = nu >= 0.0 ? (uc - uW) / dx : (uE - uc) / dx;
          de1 = om >= 0.0 ? (uc - uS) / de : (uN - uc) / de;
        }
        real src = 0.0;
        for (int q = 0; q < nsrc; ++q) src += (real)T[q] * coef[(5 + q) * plane + p * pm + at];
        real rhs = A[at] * dxx + G[at] * dee - nu * dx1 - om * de1 + F[at] * uc + src;
        nxt[at] = uc + (real)dt * rhs;
      }
    real* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  int ok = 1;
  for (size_t q = 0; q < pm; ++q) {
    if (cur != u) u[q] = cur[q];
    if (!isfinite(u[q])) ok = 0;
  }
  return ok;
}

int pdo_burst(const pdo_grid* g, const pdo_problem* pr, const double* coef, double* u,
              const double* edge, double t_n, double dt, int n_t) {
  int P = pdo_num_patches(g), M = mmax(g);
  size_t pm = (size_t)g->m_xi * g->m_eta, plane = (size_t)P * pm;
  int bad = 0;
#pragma omp parallel for schedule(static) num_threads(g_threads) reduction(+ : bad)
  for (int p = 0; p < P; ++p) {
    real* v = (real*)malloc((2 * pm + 4 * M) * sizeof(real));
    real* e = v + 2 * pm;
    for (size_t q = 0; q < pm; ++q) v[q] = u[p * pm + q];
    for (int q = 0; q < 4 * M; ++q) e[q] = edge[(size_t)p * 4 * M + q];
    if (!burst_patch(g, pr, coef, plane, p, v, e, t_n, dt, n_t, v + pm)) bad++;
    for (size_t q = 0; q < pm; ++q) u[p * pm + q] = (double)v[q];
    free(v);
  }
  return bad ? PDO_ENONFINITE : PDO_OK;
}

/* ---------------------------------------- step (iv): eq. (Restriction) ----------- */

/* Composite trapezoidal rule over the patch (or its core) in the computational
 * coordinates divided by the region's area: weights 1/2 at the region's edges, the delta^2
 * factors cancel against (n - 1) delta. */
static real restrict_patch(const pdo_grid* g, const real* u) {
  int mx = g->m_xi, me = g->m_eta, kx0, nx, le0, ne;
  core_range(g, mx, &kx0, &nx);
  core_range(g, me, &le0, &ne);
  real sum = 0.0;
  for (int l = le0; l < le0 + ne; ++l) {
    real row = 0.0;
    for (int k = kx0; k < kx0 + nx; ++k)
      row += ((k == kx0 || k == kx0 + nx - 1) ? 0.5 : 1.0) * u[l * mx + k];
    sum += ((l == le0 || l == le0 + ne - 1) ? 0.5 : 1.0) * row;
  }
  return sum / ((real)(nx - 1) * (real)(ne - 1));
}

void pdo_restrict(const pdo_grid* g, const double* u, double* Ubar) {
  int P = pdo_num_patches(g);
  size_t pm = (size_t)g->m_xi * g->m_eta;
  real* w = (real*)malloc(pm * sizeof(real));
  for (int p = 0; p < P; ++p) {
    for (size_t q = 0; q < pm; ++q) w[q] = u[p * pm + q];
    Ubar[p] = (double)restrict_patch(g, w);
  }
  free(w);
}

/* ------------------------------- steps (v)-(vi): eq. (Time_Derivative), (Extrapolation) */

static void set_boundary(const pdo_grid* g, const pdo_problem* pr, double* U, double t) {
  int nx = g->n_xi, ne = g->n_eta;
  for (int j = 0; j < ne; ++j)
    for (int i = 0; i < nx; ++i) {
      int bnd = (j == 0 || j == ne - 1) || (!g->periodic_xi && (i == 0 || i == nx - 1));
      if (bnd) U[j * nx + i] = pdo_boundary_value(g, pr, node_xi(g, i), node_eta(g, j), t);
    }
}

void pdo_macro_update(const pdo_grid* g, const pdo_problem* pr, const double* Un,
                      const double* Ubar, double* Unp1, double t_n, double Dt, double tau) {
  int P = pdo_num_patches(g), nx = g->n_xi;
  memcpy(Unp1, Un, sizeof(double) * (size_t)nx * g->n_eta);
  for (int p = 0; p < P; ++p) {
    int i, j;
    patch_ij(g, p, &i, &j);
    double F = (Ubar[p] - Un[j * nx + i]) / tau; /* U^{0,n} read as the macro value */
    Unp1[j * nx + i] = Un[j * nx + i] + Dt * F;
  }
  set_boundary(g, pr, Unp1, t_n + Dt);
}

int pdo_step(const pdo_grid* g, const pdo_problem* pr, const double* coef, const double* Un,
             double* Unp1, double t_n, double Dt, double dt, int n_t, const unsigned char* mask) {
  int P = pdo_num_patches(g), M = mmax(g), nx = g->n_xi;
  size_t pm = (size_t)g->m_xi * g->m_eta, plane = (size_t)P * pm;
  real tau = n_t * dt;
  memcpy(Unp1, Un, sizeof(double) * (size_t)nx * g->n_eta);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) num_threads(g_threads) reduction(+ : bad)
  for (int p = 0; p < P; ++p) {
    if (mask && !mask[p]) continue;
    real* u = (real*)malloc((2 * pm + 4 * M) * sizeof(real));
    real* w = u + pm;
    real* e = w + pm;
    edge_patch(g, Un, p, e);                                            /* (i)   */
    lift_patch(g, Un, p, u);                                            /* (ii)  */
    if (!burst_patch(g, pr, coef, plane, p, u, e, t_n, dt, n_t, w)) bad++; /* (iii) */
    real Ub = restrict_patch(g, u);                                     /* (iv)  */
    int i, j;
    patch_ij(g, p, &i, &j);
    real F = (Ub - Un[j * nx + i]) / tau;                               /* (v)   */
    Unp1[j * nx + i] = (double)(Un[j * nx + i] + (real)Dt * F);         /* (vi)  */
    free(u);
  }
  set_boundary(g, pr, Unp1, t_n + Dt);
  return bad ? PDO_ENONFINITE : PDO_OK;
}

int pdo_solve(const pdo_grid* g, const pdo_problem* pr, const double* coef, double* U,
              double t0, double Dt, int n_steps, double dt, int n_t) {
  size_t n = (size_t)g->n_xi * g->n_eta;
  double* V = (double*)malloc(n * sizeof(double));
  int rc = PDO_OK;
  for (int s = 0; s < n_steps && rc == PDO_OK; ++s) {
    double t_n = t0 + s * Dt;
    rc = pdo_step(g, pr, coef, U, V, t_n, Dt, dt, n_t, NULL);
    memcpy(U, V, n * sizeof(double));
  }
  free(V);
  return rc;
}

/* ----------------------------------------------------------- stability bounds ----- */

static double fe_bound(double a, double c, double nu, double om, double ph, double dx,
                       double de) {
  return 1.0 / (2.0 * a / (dx * dx) + 2.0 * c / (de * de) + fabs(nu) / dx + fabs(om) / de +
                fabs(ph));
}

double pdo_dt_micro_limit(const pdo_grid* g, const double* coef, int ncoef) {
  (void)ncoef;
  int P = pdo_num_patches(g);
  size_t pm = (size_t)g->m_xi * g->m_eta, plane = (size_t)P * pm;
  double dx = g->h_xi / (g->m_xi - 1), de = g->h_eta / (g->m_eta - 1);
  double lim = INFINITY;
  for (size_t q = 0; q < plane; ++q) {
    if (!(coef[q] > 0.0) || !(coef[plane + q] > 0.0)) return 0.0;
    double b = fe_bound(coef[q], coef[plane + q], coef[2 * plane + q], coef[3 * plane + q],
                        coef[4 * plane + q], dx, de);
    if (b < lim) lim = b;
  }
  return lim;
}

double pdo_dt_macro_limit(const pdo_grid* g, const pdo_problem* pr) {
  int P = pdo_num_patches(g);
  double lim = INFINITY, out[5 + PDO_MAXTERM];
  for (int p = 0; p < P; ++p) {
    int i, j;
    patch_ij(g, p, &i, &j);
    pdo_coeffs_at(g, pr, node_xi(g, i), node_eta(g, j), out);
    double b = fe_bound(out[0], out[1], out[2], out[3], out[4], dxi(g), deta(g));
    if (b < lim) lim = b;
  }
  return lim;
}

/* ---------------------------------------------------- full-domain explicit run ---- */
/* The operator of eq. (Computational_Problem) on one lattice over the whole box, with the
 * micro differences of a burst (3-point second differences; 2-point upwind or central
 * first differences) and forward Euler; the boundary rows (and columns unless xi is
 * periodic) take the Dirichlet data u_b at the end of each step. */

static void fd_spacing(const pdo_grid* g, int n_x, int n_y, double* hx, double* hy) {
  *hx = g->periodic_xi ? (g->xi1 - g->xi0) / n_x : (g->xi1 - g->xi0) / (n_x - 1);
  *hy = (g->eta1 - g->eta0) / (n_y - 1);
}

static int fd_is_boundary(const pdo_grid* g, int n_x, int n_y, int i, int j) {
  return (j == 0 || j == n_y - 1) || (!g->periodic_xi && (i == 0 || i == n_x - 1));
}

/* Forward-Euler update of interior node (i, j) from U at time t: c are the operator's
 * coefficients and source parts at the node, T the source time factors at t. */
static double fd_update(const pdo_grid* g, const pdo_problem* pr, const double* c,
                        const double* T, const double* U, int n_x, double hx, double hy,
                        int i, int j, double dt) {
  int iw = i - 1 < 0 ? n_x - 1 : i - 1, ie = i + 1 >= n_x ? 0 : i + 1;
  double uc = U[j * n_x + i], uW = U[j * n_x + iw], uE = U[j * n_x + ie];
  double uS = U[(j - 1) * n_x + i], uN = U[(j + 1) * n_x + i];
  double dxx = (uE - 2.0 * uc + uW) / (hx * hx);
  double dee = (uN - 2.0 * uc + uS) / (hy * hy);
  double dx1, de1;
  if (g->conv == PDO_CONV_CENTRAL) {
    dx1 = (uE - uW) / (2.0 * hx);
    de1 = (uN - uS) / (2.0 * hy);
  } else {
    dx1 = c[2] >= 0.0 ? (uc - uW) / hx : (uE - uc) / hx;
    de1 = c[3] >= 0.0 ? (uc - uS) / hy : (uN - uc) / hy;
  }
  double src = 0.0;
  for (int q = 0; q < pr->n_src; ++q) src += T[q] * c[5 + q];
  double rhs = c[0] * dxx + c[1] * dee - c[2] * dx1 - c[3] * de1 + c[4] * uc + src;
  return uc + dt * rhs;
}

int pdo_full_domain(const pdo_grid* g, const pdo_problem* pr, int n_x, int n_y, double* U,
                    double t0, double dt, int n_steps) {
  if (n_x < 3 || n_y < 3) return PDO_EINVAL;
  double hx, hy;
  fd_spacing(g, n_x, n_y, &hx, &hy);
  int nc = PDO_NCOEF(pr);
  size_t n = (size_t)n_x * n_y;
  double* C = (double*)malloc(n * nc * sizeof(double));
  double* V = (double*)malloc(n * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n_y; ++j) {
    double out[5 + PDO_MAXTERM];
    for (int i = 0; i < n_x; ++i) {
      pdo_coeffs_at(g, pr, g->xi0 + i * hx, g->eta0 + j * hy, out);
      for (int q = 0; q < nc; ++q) C[((size_t)j * n_x + i) * nc + q] = out[q];
    }
  }
  int rc = PDO_OK;
  for (int s = 0; s < n_steps; ++s) {
    double t = t0 + s * dt;
    double T[PDO_MAXTERM];
    for (int q = 0; q < pr->n_src; ++q) T[q] = tfun_eval(&pr->src_t[q], t);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n_y; ++j)
      for (int i = 0; i < n_x; ++i) {
        if (fd_is_boundary(g, n_x, n_y, i, j))
          V[j * n_x + i] = pdo_boundary_value(g, pr, g->xi0 + i * hx, g->eta0 + j * hy, t + dt);
        else
          V[j * n_x + i] = fd_update(g, pr, C + ((size_t)j * n_x + i) * nc, T, U, n_x, hx, hy,
                                     i, j, dt);
      }
    memcpy(U, V, n * sizeof(double));
    for (size_t q = 0; q < n; ++q)
      if (!isfinite(U[q])) rc = PDO_ENONFINITE;
    if (rc != PDO_OK) break;
  }
  free(C);
  free(V);
  return rc;
}

double pdo_full_domain_point(const pdo_grid* g, const pdo_problem* pr, int n_x, int n_y,
                             const double* U, double t, double dt, int i, int j) {
  double hx, hy;
  fd_spacing(g, n_x, n_y, &hx, &hy);
  if (fd_is_boundary(g, n_x, n_y, i, j))
    return pdo_boundary_value(g, pr, g->xi0 + i * hx, g->eta0 + j * hy, t + dt);
  double c[5 + PDO_MAXTERM], T[PDO_MAXTERM];
  pdo_coeffs_at(g, pr, g->xi0 + i * hx, g->eta0 + j * hy, c);
  for (int q = 0; q < pr->n_src; ++q) T[q] = tfun_eval(&pr->src_t[q], t);
  return fd_update(g, pr, c, T, U, n_x, hx, hy, i, j, dt);
}
