/*
 * pdo.h -- plain, slow FP64 CPU oracle of the curvilinear patch dynamics scheme of
 * Karmakar & Dalal, "A Generalised Curvilinear Coordinate system-based Patch Dynamics
 * Scheme in Equation-free Multiscale Modelling" (arXiv 2405.08764).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header, table or
 * constant generator with the HIP library; both are written independently from the
 * paper.  Every function follows the paper's steps in its order and notation:
 *
 *   Sec. 2      eq. (Physical_Problem), eq. (Computational_Problem) and its coefficient
 *               list: the CDR equation and its orthogonal-curvilinear form;
 *   Sec. 3      the equidistant macro mesh and the patches centred on interior nodes,
 *               eq. (Averaging) the restriction;
 *   Sec. 3.1    eq. (Lagrange_2D) and eq. (edge): Neumann patch-edge gradients;
 *   Sec. 3.2    eq. (Lifting) and eq. (C_0): the lifting operator;
 *   Sec. 3.3    steps (i)-(vi): edge data, lifting, evolution, restriction,
 *               eq. (Time_Derivative) and eq. (Extrapolation);
 *   Sec. 4.1    eq. (Stretching_Transformation), 2-point upwind / 3-point central
 *               differences, trapezoidal restriction;
 *   Sec. 4.2    eq. (Transformation_Annulus), eq. (MOL_Diff_Annu), explicit forward
 *               Euler micro stepping, periodic macro boundary in xi.
 *
 * Everything is double precision, compiled with -ffp-contract=off.
 * Parity status of each function is listed in the header of pdo.c.
 */
#ifndef PDO_H
#define PDO_H

#ifdef __cplusplus
extern "C" {
#endif

#define PDO_MAXMODE 16
#define PDO_MAXPOLAR 4
#define PDO_MAXTERM 4

enum { PDO_OK = 0, PDO_EINVAL = -1, PDO_EUNSTABLE = -3, PDO_ENONFINITE = -5 };

/* Geometry of the map x(xi,eta), y(xi,eta). */
enum {
  PDO_GEOM_IDENTITY = 0, /* x = xi, y = eta on any box                               */
  PDO_GEOM_SINE = 1,     /* x = xi + (l/pi) sin(pi xi), same in y; box [0,1]^2 (Sec 4.1) */
  PDO_GEOM_TANH = 2,     /* x = tanh(b xi)/tanh(b), same in y; box [0,1]^2             */
  PDO_GEOM_ANNULUS = 3   /* x = eta cos xi, y = eta sin xi; xi periodic (Sec 4.2)      */
};
enum { PDO_CONV_UPWIND = 0, PDO_CONV_CENTRAL = 1 };
enum { PDO_C0_TRAPEZOID = 0, PDO_C0_PRINTED = 1 };

typedef struct {
  int geometry;
  double gparam;            /* lambda (sine) or beta (tanh)                      */
  double xi0, xi1, eta0, eta1;
  int n_xi, n_eta;          /* macro node counts; periodic axis: unique nodes    */
  int periodic_xi;
  double h_xi, h_eta;       /* patch edge lengths in the computational domain    */
  int m_xi, m_eta;          /* micro points per patch side (edges included)      */
  int conv;                 /* first-derivative micro scheme                     */
  int c0mode;               /* reading of eq. (C_0)                              */
  int core_points;          /* restriction over the central core_points micro     */
                            /* points per side (0: the whole patch)               */
} pdo_grid;

/* A scalar physical field F(x,y) =
 *   c0 + cx x + cy y + sum_k amp_k cos(kx_k x + ky_k y + ph_k)
 *      + sum_p pamp_p (pc0_p + pc1_p r + pc2_p r^2) cos(pn_p theta + pph_p)
 * (polar terms only on the annulus, where r = eta and theta = xi). */
typedef struct {
  double c0, cx, cy;
  int nmode;
  double amp[PDO_MAXMODE], kx[PDO_MAXMODE], ky[PDO_MAXMODE], ph[PDO_MAXMODE];
  int npolar;
  double pamp[PDO_MAXPOLAR], pc0[PDO_MAXPOLAR], pc1[PDO_MAXPOLAR], pc2[PDO_MAXPOLAR];
  double pn[PDO_MAXPOLAR], pph[PDO_MAXPOLAR];
} pdo_field;

/* One-dimensional function s -> value. */
enum { PDO_FN_SIN = 0, PDO_FN_COS = 1, PDO_FN_EXP = 2, PDO_FN_POLY = 3 };
typedef struct { int type; double a, b, c, d; } pdo_fn1;
/* SIN: sin(a s + b); COS: cos(a s + b); EXP: exp(a s + b); POLY: a + b s + c s^2 + d s^3 */

/* Separable spatial function: kind 0: amp f(x) g(y); kind 1 (annulus): amp f(r) g(theta). */
typedef struct { int kind; double amp; pdo_fn1 f, g; } pdo_sfun;

/* Time factor: CONST: a; EXP: a exp(b t); SIN: a + b sin(c t). */
enum { PDO_T_CONST = 0, PDO_T_EXP = 1, PDO_T_SIN = 2 };
typedef struct { int type; double a, b, c; } pdo_tfun;

/* The physical problem, eq. (Physical_Problem): u_t = div(D grad u - v u) + f u + g.
 * D = diag(D11, D22) (D11 = D22 on the annulus), v = (v1, v2), reaction f.
 * Initial and Dirichlet data: u_b(x,y,t) = sum_m bc_t[m](t) bc_s[m](x,y).
 * Source: g = sum_k src_t[k](t) (src_c[k] S_k - L[S_k]) with S_k = src_s[k] and L the
 * spatial operator; a manufactured solution sum_m T_m S_m gives src_c = T'/T. */
typedef struct {
  pdo_field D11, D22, v1, v2, f;
  int n_bc;
  pdo_tfun bc_t[PDO_MAXTERM];
  pdo_sfun bc_s[PDO_MAXTERM];
  int n_src;
  pdo_tfun src_t[PDO_MAXTERM];
  double src_c[PDO_MAXTERM];
  pdo_sfun src_s[PDO_MAXTERM];
} pdo_problem;

/* Number of coefficient planes stored per micro point: alpha, gamma, nu, omega, phi,
 * then one source plane per source term. */
#define PDO_NCOEF(prob) (5 + (prob)->n_src)

int pdo_check(const pdo_grid* g, const pdo_problem* prob);
int pdo_num_patches(const pdo_grid* g);
/* Per patch: i, j, then the 9 node indices (j+b)*n_xi + (i+a) for b, a in -1..1
 * (b outer, a inner).  Layout [P][11]. */
void pdo_patch_map(const pdo_grid* g, int* out);
/* Micro offsets and stencil tables; layout documented in pdo.c (pdo_tables). */
void pdo_tables(const pdo_grid* g, double* out);
int pdo_tables_size(const pdo_grid* g);

/* Map and metric at (xi, eta): out[0..15] =
 * x, y, x_xi, y_xi, x_eta, y_eta, x_xixi, y_xixi, x_etaeta, y_etaeta, x_xieta, y_xieta,
 * h1, h2 (scale factors), J = x_xi y_eta - x_eta y_xi. */
void pdo_metric(const pdo_grid* g, double xi, double eta, double* out);
/* Computational coefficients at one point: out = alpha, gamma, nu, omega, phi,
 * then sigma_k (spatial part of source term k). */
void pdo_coeffs_at(const pdo_grid* g, const pdo_problem* prob, double xi, double eta, double* out);
/* All coefficient planes at every micro point: layout [NCOEF][P][m_eta][m_xi]. */
void pdo_coefficients(const pdo_grid* g, const pdo_problem* prob, double* coef);
/* The same planes for the patches with mask[p] != 0 only (the others are left as they
 * are): a sampled check of a large grid needs the coefficients of a few patches. */
void pdo_coefficients_masked(const pdo_grid* g, const pdo_problem* prob,
                             const unsigned char* mask, double* coef);
/* u_b at one point and time. */
double pdo_boundary_value(const pdo_grid* g, const pdo_problem* prob, double xi, double eta, double t);
/* Macro field at t from u_b at every node; layout [n_eta][n_xi]. */
void pdo_initial(const pdo_grid* g, const pdo_problem* prob, double t, double* U);

/* Step (i): eq. (edge) gradients, layout [P][4][mmax] with edge order
 * (xi-, xi+, eta-, eta+); xi edges hold m_eta values, eta edges m_xi values;
 * mmax = max(m_xi, m_eta). */
void pdo_edge(const pdo_grid* g, const double* U, double* edge);
/* Step (ii): eq. (Lifting), layout [P][m_eta][m_xi]. */
void pdo_lift(const pdo_grid* g, const double* U, double* u);
/* Step (iii): n_t forward-Euler nano steps of size dt from time t_n. */
int pdo_burst(const pdo_grid* g, const pdo_problem* prob, const double* coef, double* u,
              const double* edge, double t_n, double dt, int n_t);
/* Step (iv): eq. (Restriction) by the composite trapezoidal rule; Ubar[P]. */
void pdo_restrict(const pdo_grid* g, const double* u, double* Ubar);
/* Steps (v)-(vi) and the Dirichlet boundary at t_n + Dt. */
void pdo_macro_update(const pdo_grid* g, const pdo_problem* prob, const double* Un,
                      const double* Ubar, double* Unp1, double t_n, double Dt, double tau);
/* One whole macro step; mask (may be NULL) marks the patches to advance (others keep Un). */
int pdo_step(const pdo_grid* g, const pdo_problem* prob, const double* coef, const double* Un,
             double* Unp1, double t_n, double Dt, double dt, int n_t, const unsigned char* mask);
/* n_steps macro steps from t0; U in/out. */
int pdo_solve(const pdo_grid* g, const pdo_problem* prob, const double* coef, double* U,
              double t0, double Dt, int n_steps, double dt, int n_t);

/* Explicit stability bounds: micro (over micro points) and macro (over patch nodes). */
double pdo_dt_micro_limit(const pdo_grid* g, const double* coef, int ncoef);
double pdo_dt_macro_limit(const pdo_grid* g, const pdo_problem* prob);

/* Full-domain explicit scheme on the whole computational box at micro resolution
 * (same operator and differences as a burst, Dirichlet data from u_b): n_x by n_y
 * lattice points including the boundary, U in/out [n_y][n_x]. */
int pdo_full_domain(const pdo_grid* g, const pdo_problem* prob, int n_x, int n_y, double* U,
                    double t0, double dt, int n_steps);
/* The value one step of pdo_full_domain from time t gives at node (i, j) alone (the
 * Dirichlet value at t + dt on a boundary node): spot checks of large lattices. */
double pdo_full_domain_point(const pdo_grid* g, const pdo_problem* prob, int n_x, int n_y,
                             const double* U, double t, double dt, int i, int j);

void pdo_set_threads(int n);
int pdo_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
