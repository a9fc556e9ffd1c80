/*
 * pd.h -- C ABI of the MI355X-native curvilinear patch dynamics library (libpd.so).
 *
 * The scheme is that of Karmakar & Dalal, "A Generalised Curvilinear Coordinate
 * system-based Patch Dynamics Scheme in Equation-free Multiscale Modelling"
 * (arXiv 2405.08764):  the CDR equation eq. (Physical_Problem) is mapped to a rectangle
 * (eq. Computational_Problem), patches sit on the interior nodes of an equidistant macro
 * mesh (Sec. 3), and one macro step is steps (i)-(vi) of Sec. 3.3: Neumann edge data
 * eq. (edge), lifting eq. (Lifting)/(C_0), a burst of explicit finite-difference nano
 * steps inside every patch, the trapezoidal restriction eq. (Restriction), the time
 * derivative eq. (Time_Derivative) and the projective step eq. (Extrapolation).
 *
 * Conventions for every call:
 *  - Pointers named dev_* / U / Ubar / patch_state / edge are DEVICE pointers on the
 *    grid's device; host_* pointers are host memory.  The caller owns all of them; the
 *    library never allocates or frees caller memory.  The only device memory the library
 *    uses beyond the arguments is the caller-provided workspace (pd_bind_workspace).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Every call
 *    except create/query/destroy/bind/get_* is asynchronous on that stream, except
 *    pd_set_coefficients, which synchronises the stream once to read back the explicit
 *    stability bounds.
 *  - Macro fields U are FP64, row-major [n_eta][n_xi] (node (i, j) at j*n_xi + i).
 *    Patch p sits on node (i, j) = (i_first + p % npx, 1 + p / npx) with npx patches per
 *    row, i_first = 0 on a periodic xi axis and 1 otherwise.
 *  - Micro fields are FP64 [P][m_eta][m_xi]; edge data FP64 [P][4][max(m_xi, m_eta)]
 *    in the edge order (xi-, xi+, eta-, eta+).
 *  - Return values: PD_OK or a negative pd_status; pd_last_error() gives a message
 *    (thread-local).  No C++ exception crosses this interface.
 */
#ifndef PD_H
#define PD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pd_status;
#define PD_OK 0
#define PD_EINVAL (-1)      /* invalid descriptor or argument                          */
#define PD_ESTATE (-2)      /* workspace or coefficients not set                       */
#define PD_EUNSTABLE (-3)   /* time step above the explicit bound (see pd_set_option)  */
#define PD_EDEVICE (-4)     /* HIP runtime error; message carries hipGetErrorString    */
#define PD_ENONFINITE (-5)  /* a non-finite macro value was produced                   */
#define PD_ENOMEM (-6)      /* workspace too small                                     */

#define PD_MAXMODE 16
#define PD_MAXPOLAR 4
#define PD_MAXTERM 4

/* Map x(xi, eta), y(xi, eta) of eq. (Transformtion_Inv). */
#define PD_GEOM_IDENTITY 0 /* x = xi, y = eta                                           */
#define PD_GEOM_SINE 1     /* eq. (Stretching_Transformation), box [0,1]^2, 0 <= l < 1  */
#define PD_GEOM_TANH 2     /* x = tanh(b xi)/tanh(b), y likewise, box [0,1]^2, b >= 0    */
#define PD_GEOM_ANNULUS 3  /* eq. (Transformation_Annulus): xi = theta (periodic),      */
                           /* eta = r in [eta0, eta1], eta0 > 0                          */
#define PD_CONV_UPWIND 0   /* 2-point upwind first differences (Sec. 4.1.1)            */
#define PD_CONV_CENTRAL 1  /* central first differences (eq. MOL_Diff_Annu)            */
#define PD_C0_TRAPEZOID 0  /* C0 consistent with the trapezoid restriction            */
#define PD_C0_PRINTED 1    /* C0 with the printed h^2/24 of eq. (C_0)                  */
#define PD_F64 0           /* burst arithmetic in FP64                                 */
#define PD_F32 1           /* burst in FP32 on deviations from the patch's macro value */

typedef struct {
  int32_t geometry;
  double gparam;                  /* lambda (sine) or beta (tanh)                      */
  double xi0, xi1, eta0, eta1;    /* computational box Omega_c                         */
  int32_t n_xi, n_eta;            /* macro node counts; periodic axis: unique nodes    */
  int32_t periodic_xi;            /* 1: xi periodic (annulus), Sec. 4.2                */
  double h_xi, h_eta;             /* patch edge lengths, 0 < h < Delta (Sec. 3)        */
  int32_t m_xi, m_eta;            /* micro points per patch side incl. edges, 3..64    */
  int32_t conv;                   /* PD_CONV_*                                          */
  int32_t c0mode;                 /* PD_C0_*                                            */
  int32_t precision;              /* PD_F64 / PD_F32                                    */
  int32_t device;                 /* HIP device ordinal                                 */
  int32_t max_sources;            /* source terms the workspace holds planes for        */
                                  /* (0 = PD_MAXTERM); pd_set_coefficients checks it    */
  int32_t core_points;            /* restriction (eq. Restriction) over the central     */
                                  /* core_points micro points per side, C0 from their   */
                                  /* trapezoid average; 0 = the whole patch.  Otherwise */
                                  /* 2 <= core_points <= m_xi, m_eta, same parity       */
} pd_grid_desc;

/* Scalar field F(x, y) = c0 + cx x + cy y + sum amp cos(kx x + ky y + ph)
 *   + sum pamp (pc0 + pc1 r + pc2 r^2) cos(pn theta + pph)   (polar terms: annulus). */
typedef struct {
  double c0, cx, cy;
  int32_t nmode;
  double amp[PD_MAXMODE], kx[PD_MAXMODE], ky[PD_MAXMODE], ph[PD_MAXMODE];
  int32_t npolar;
  double pamp[PD_MAXPOLAR], pc0[PD_MAXPOLAR], pc1[PD_MAXPOLAR], pc2[PD_MAXPOLAR];
  double pn[PD_MAXPOLAR], pph[PD_MAXPOLAR];
} pd_field;

/* 1-D function: SIN sin(a s + b), COS cos(a s + b), EXP exp(a s + b),
 * POLY a + b s + c s^2 + d s^3. */
#define PD_FN_SIN 0
#define PD_FN_COS 1
#define PD_FN_EXP 2
#define PD_FN_POLY 3
typedef struct { int32_t type; double a, b, c, d; } pd_fn1;
/* kind 0: amp f(x) g(y);  kind 1 (annulus): amp f(r) g(theta). */
typedef struct { int32_t kind; double amp; pd_fn1 f, g; } pd_sfun;
/* Time factor: CONST a;  EXP a exp(b t);  SIN a + b sin(c t). */
#define PD_T_CONST 0
#define PD_T_EXP 1
#define PD_T_SIN 2
typedef struct { int32_t type; double a, b, c; } pd_tfun;

/* eq. (Physical_Problem): u_t = div(D grad u - v u) + f u + g with D = diag(D11, D22)
 * (D11 == D22 on the annulus), v = (v1, v2), reaction f.  Initial/Dirichlet data
 * u_b = sum_m bc_t[m](t) bc_s[m](x, y); source g = sum_k src_t[k](t) (src_c[k] S_k - L[S_k])
 * with S_k = src_s[k] and L the spatial operator (a manufactured solution T S has
 * c = T'/T).  At most PD_MAXTERM terms each. */
typedef struct {
  pd_field D11, D22, v1, v2, f;
  int32_t n_bc;
  pd_tfun bc_t[PD_MAXTERM];
  pd_sfun bc_s[PD_MAXTERM];
  int32_t n_src;
  pd_tfun src_t[PD_MAXTERM];
  double src_c[PD_MAXTERM];
  pd_sfun src_s[PD_MAXTERM];
} pd_coeff_desc;

typedef struct {
  int32_t n_patches, m_xi, m_eta, n_xi, n_eta;
  int64_t n_points;          /* n_patches * m_xi * m_eta                              */
  size_t workspace_bytes;    /* device bytes pd_bind_workspace needs                  */
  double dt_micro_limit;     /* explicit bound over micro points (after coefficients)  */
  double dt_macro_limit;     /* explicit bound at macro spacing over patch nodes       */
  int32_t coefficients_set;
  int32_t n_time_sources;    /* source terms with a non-constant time factor           */
  int32_t rows_per_lane, patches_per_block, block_threads; /* current launch shape     */
  int32_t cols_per_lane;
  int32_t exchange;          /* 1: neighbours through LDS, 2: inside one wave (DPP),  */
                             /* 3: DPP inside each wave, band edges through LDS        */
  int32_t tuned;             /* 1 once pd_autotune chose the launch shape               */
  double tuned_ms;           /* its measured time per fused step (ms), else 0           */
  int32_t resident_solve;    /* 1 if the last pd_solve ran resident launches           */
  int32_t resident_refresh;  /* 1 if the last pd_macro_step_refresh ran resident       */
} pd_info;

typedef struct pd_grid_s* pd_grid;

/* Sec. 3: build the macro mesh, the patch index map and the stencil tables (Lagrange
 * weights eq. (Lagrange_2D) at the micro edge points, eq. (edge) weights, trapezoid
 * weights, micro offsets) on the host.  Allocates no device memory.
 * Errors: PD_EINVAL for out-of-range fields (h >= Delta, m < 3 or m > 64, n < 3, bad
 * geometry or box), PD_EDEVICE if the device cannot be selected. */
pd_status pd_create_grid(const pd_grid_desc* desc, pd_grid* out);
pd_status pd_destroy_grid(pd_grid g);
pd_status pd_query(pd_grid g, pd_info* out);
/* Give the grid `bytes` of device memory at dev (>= pd_info.workspace_bytes, 256-byte
 * aligned) for its coefficients, tables, ping-pong macro buffer and flags.  The memory
 * must stay valid until the grid is destroyed or rebound.  PD_ENOMEM if too small. */
pd_status pd_bind_workspace(pd_grid g, void* dev, size_t bytes);
/* Sec. 2.1 coefficient list of eq. (Computational_Problem) (alpha, gamma, nu, omega,
 * phi and the source parts) at every micro point, computed on the device in the
 * scale-factor form for orthogonal maps; also the explicit stability bounds.
 * PD_EINVAL on a bad descriptor or non-positive diffusion, PD_ESTATE without workspace. */
pd_status pd_set_coefficients(pd_grid g, const pd_coeff_desc* c, void* stream);
/* U at every node from u_b(t) (initial data, Sec. 3.2). */
pd_status pd_initial(pd_grid g, double* U, double t, void* stream);

/* Steps (i) and (ii) of Sec. 3.3: eq. (edge) gradients into edge [P][4][M] and the lifted
 * micro field eq. (Lifting) into patch_state [P][m_eta][m_xi], both FP64. */
pd_status pd_lift_bc(pd_grid g, const double* U, double* patch_state, double* edge,
                     void* stream);
/* Step (iii): n_t explicit forward-Euler nano steps of size dt_micro from time t_n inside
 * every patch with the edge gradients held fixed (tau = n_t dt_micro, 1 <= n_t <= 65536).
 * patch_state is updated in place.  PD_EUNSTABLE if dt_micro exceeds the explicit bound. */
pd_status pd_micro_burst(pd_grid g, double* patch_state, const double* edge, double t_n,
                         double dt_micro, int32_t n_t, void* stream);
/* Step (iii) with the alternating-direction implicit micro solver of Sec. 4.1.1 (there
 * n_t = 2): n_t Peaceman-Rachford steps of size dt_micro from t_n in every patch.  The
 * bursts' micro operator (same differences and ghost-point edge data as pd_micro_burst)
 * is split into its xi part (alpha, nu, phi/2) and eta part (gamma, omega, phi/2); each
 * step solves (I - dt/2 L_xi) u* = (I + dt/2 L_eta) u + dt/2 s and
 * (I - dt/2 L_eta) u' = (I + dt/2 L_xi) u* + dt/2 s, s the source at the step's half time,
 * by tridiagonal sweeps along rows, then columns.  No explicit stability bound applies.
 * patch_state is updated in place.  PD_EINVAL for dt_micro <= 0, n_t < 1, or patches with
 * 6 m_xi m_eta + 4 max(m_xi, m_eta) > 8192 (a patch, its sweeps' rows and its edge data
 * live in 64 KiB of LDS; m up to 36 for square patches). */
pd_status pd_micro_burst_adi(pd_grid g, double* patch_state, const double* edge, double t_n,
                             double dt_micro, int32_t n_t, void* stream);
/* Step (iii) with the higher-order upwind convection differences of Sec. 4.1.2: n_t
 * forward-Euler nano steps of size dt_micro from t_n in every patch, the 3-point second
 * differences and the source as in pd_micro_burst, the first differences by
 *   points = 3: (3 u_i - 4 u_{i-1} + u_{i-2}) / (2 dp),
 *   points = 4: (u_{i+1} - u_{i-1}) / (2 dp) + r/(3 dp) (u_{i-2} - 3 u_{i-1} + 3 u_i - u_{i+1})
 *               (r = 1/2 is third order, r = 0 the central difference),
 *   points = 2: (u_i - u_{i-1}) / dp (the 2-point upwind difference),
 * each taken as printed where the velocity component is >= 0 and mirrored (i -> -i, sign
 * flipped) where it is < 0, whatever the grid's convection option.  The edge gradients
 * g-, g+ of edge [P][4][M] enter through two ghost layers: u_{-1} = u_1 - 2 dp g-,
 * u_{-2} = u_2 - 4 dp g-, u_m = u_{m-2} + 2 dp g+, u_{m+1} = u_{m-3} + 4 dp g+.
 * patch_state [P][m_eta][m_xi] FP64 is updated in place.  No stability bound is checked
 * (the 2-point bound of pd_query is a guide for diffusion-dominated patches); a
 * non-finite result sets the flag pd_sync reports as PD_EUNSTABLE.  PD_EINVAL for
 * dt_micro <= 0, n_t < 1, points outside 2..4, non-finite r, or patches with m_xi or
 * m_eta < 3 or m_xi m_eta > 1024; PD_ESTATE before coefficients are set. */
pd_status pd_micro_burst_upwind(pd_grid g, double* patch_state, const double* edge,
                                double t_n, double dt_micro, int32_t n_t, int32_t points,
                                double r, void* stream);
/* Step (iii) with the ADI micro solver of pd_micro_burst_adi and the first differences of
 * pd_micro_burst_upwind (Sec. 4.1.2 ran its micro simulations with that solver and tried
 * the 3- and 4-point upwind forms in it): n_t Peaceman-Rachford nano steps of size
 * dt_micro from t_n,
 *   (I - dt/2 L_xi)  u*      = (I + dt/2 L_eta) u^n + dt/2 s(t + dt/2),
 *   (I - dt/2 L_eta) u^{n+1} = (I + dt/2 L_xi)  u*  + dt/2 s(t + dt/2),
 * L_xi = alpha d2_xi - nu d_xi + phi/2 and L_eta likewise, d_xi and d_eta of the given
 * form (points 2, 3 or 4, parameter r, mirrored where the velocity component is < 0,
 * whatever the grid's convection option), the edge gradients of edge [P][4][M] through the
 * two ghost layers of pd_micro_burst_upwind.  The implicit lines are banded (two
 * neighbours on each side) and are eliminated without pivoting: stable while every line
 * matrix is diagonally dominant (3-point form: dt/2 (|nu| / d_xi + phi/2) <= 1, likewise
 * along eta); a non-finite result sets the flag pd_sync reports.  patch_state
 * [P][m_eta][m_xi] FP64 is updated in place.  PD_EINVAL for dt_micro <= 0, n_t < 1,
 * points outside 2..4, non-finite r, or 5 m_xi m_eta + 4 max(m_xi, m_eta) > 8192 (a patch's
 * two field planes, its eliminated rows and its edge data in 64 KiB of LDS; m up to 40
 * for square patches); PD_ESTATE before coefficients are set. */
pd_status pd_micro_burst_adi_upwind(pd_grid g, double* patch_state, const double* edge,
                                    double t_n, double dt_micro, int32_t n_t, int32_t points,
                                    double r, void* stream);
/* Step (iv): eq. (Restriction) by the composite trapezoidal rule, Ubar[P]. */
pd_status pd_restrict(pd_grid g, const double* patch_state, double* Ubar, void* stream);
/* Steps (v)-(vi): U_np1 = U_n + dt_macro (Ubar - U_n)/tau at patch nodes, Dirichlet data
 * at t_n + dt_macro on boundary nodes.  With Ubar == NULL the whole macro step (i)-(vi)
 * runs fused on the device (the hot path).  U_n and U_np1 must not alias. */
pd_status pd_macro_step(pd_grid g, const double* U_n, double* U_np1, double t_n,
                        double dt_macro, double dt_micro, int32_t n_t, const double* Ubar,
                        void* stream);
/* Steps (i)-(vi) fused on the device for the patch nodes only (U_np1's boundary nodes are
 * left untouched); pd_macro_step with Ubar == NULL is this call followed by
 * pd_apply_boundary.  U_n and U_np1 must not alias. */
pd_status pd_patch_step(pd_grid g, const double* U_n, double* U_np1, double t_n,
                        double dt_macro, double dt_micro, int32_t n_t, void* stream);
/* One macro step with the edge data refreshed during the burst (the refinement the paper
 * names after freezing the edge gradients for the whole burst, Sec. 3.3 step (ii)): the
 * n_t nano steps run as n_refresh sub-bursts (sub-burst q takes nano steps
 * n_t q / n_refresh .. n_t (q + 1) / n_refresh - 1, integer division, starting at
 * t_n + (n_t q / n_refresh) dt_micro); between sub-bursts every patch is restricted
 * (eq. Restriction), U_work takes the patch averages at the patch nodes and the Dirichlet
 * data at the next sub-burst's start time on the boundary nodes, and the eq. (edge)
 * gradients are recomputed from U_work.  Then (iv)-(vi) as pd_macro_step.  n_refresh = 1
 * is the split form of pd_macro_step.  Caller buffers: patch_state [P][m_eta][m_xi], edge
 * [P][4][M], Ubar [P], U_work [n_eta][n_xi] (distinct from U_n and U_np1); their
 * contents afterwards are unspecified.  PD_EINVAL unless 1 <= n_refresh <= n_t;
 * PD_EUNSTABLE as pd_macro_step. */
pd_status pd_macro_step_refresh(pd_grid g, const double* U_n, double* U_np1, double t_n,
                                double dt_macro, double dt_micro, int32_t n_t,
                                int32_t n_refresh, double* patch_state, double* edge,
                                double* Ubar, double* U_work, void* stream);
/* Dirichlet data u_b(t) on every boundary node of U (eq. CDR_Com_IC_BCs, eq. Ann_C_IC_BCs:
 * all four sides of a square, the two circles of the annulus). */
pd_status pd_apply_boundary(pd_grid g, double* U, double t, void* stream);
/* Repeat the fused macro step n_steps times from t0 (Sec. 3.3 "until the final time"),
 * replayed from a captured HIP graph; U is in/out.  Runs on `stream` (a private stream
 * ordered after the caller's when stream is NULL, since the null stream cannot be
 * captured). */
pd_status pd_solve(pd_grid g, double* U, double t0, double dt_macro, int32_t n_steps,
                   double dt_micro, int32_t n_t, void* stream);
/* Synchronise the stream and report PD_ENONFINITE if a kernel saw a non-finite value
 * since the last call (the flag is then cleared). */
pd_status pd_sync(pd_grid g, void* stream);

/* Host copies of the index map [P][11] (i, j, then the 9 node indices, eta offset outer)
 * and of the stencil tables (same layout as documented in pd_get_tables_size). */
pd_status pd_get_patch_map(pd_grid g, int32_t* host_out);
/* Tables: s_xi[m_xi], s_eta[m_eta], L_q at the xi-edge points [m_eta][3], at the eta-edge
 * points [m_xi][3], edge weights (xi-, xi+, eta-, eta+) x 3, trapezoid weights [m_xi],
 * [m_eta], then Dxi, Deta, dxi, deta, r_xi, r_eta, kappa_xi, kappa_eta. */
int32_t pd_get_tables_size(pd_grid g);
pd_status pd_get_tables(pd_grid g, double* host_out);
/* Device copy of the coefficient planes [5 + n_src][P][m_eta][m_xi] (alpha, gamma, nu,
 * omega, phi, then each source term's spatial part in descriptor order). */
pd_status pd_copy_coefficients(pd_grid g, double* dev_out, void* stream);

/* Options: PD_OPT_ALLOW_UNSTABLE (0/1) skips the stability guard; PD_OPT_ROWS_PER_LANE,
 * PD_OPT_COLS_PER_LANE (1..4), PD_OPT_PATCHES_PER_BLOCK, PD_OPT_BLOCK_THREADS (upper bound,
 * 64..256) and PD_OPT_EXCHANGE (1 LDS, 2 in-wave, 3 hybrid) set the fused burst's launch shape
 * (0 = automatic).  Results do not depend on the launch shape (bitwise).
 * PD_OPT_RESIDENT_SOLVE (default 1): pd_solve runs each replay of its in-wave FP64 steps
 * as one launch whose waves stay resident across the steps (when they all fit on the
 * device at once, a patch block has at most 7 patches and at most one source term depends
 * on time), else one launch per step;
 * the results are bitwise the same.  The same option lets pd_macro_step_refresh (n_refresh
 * of 2 .. 16) run its sub-bursts in one such launch, the edge data refreshed between them
 * through U_work and the workspace's second macro buffer (same results up to rounding
 * order).  The resident launch assumes the device is otherwise
 * idle: if work on another stream holds the slots some of its waves need, their
 * neighbours stop waiting after a bounded time and pd_sync returns PD_EDEVICE (turn the
 * option off for grids that share the device with concurrent kernels). */
#define PD_OPT_ALLOW_UNSTABLE 1
#define PD_OPT_ROWS_PER_LANE 2
#define PD_OPT_PATCHES_PER_BLOCK 3
#define PD_OPT_BLOCK_THREADS 4
#define PD_OPT_COLS_PER_LANE 5
#define PD_OPT_EXCHANGE 6
#define PD_OPT_RESIDENT_SOLVE 7
pd_status pd_set_option(pd_grid g, int32_t option, int64_t value);

/* Launch-shape autotuner of the fused step (not in the paper: a property of this library).
 * Times every launch shape allowed by the current options (exchange, columns and rows per
 * lane, patches per block, block size) on the actual problem with HIP events: `reps`
 * fused steps from U (read only; results go to the workspace's second macro buffer, so no
 * pd_solve of this grid may be in flight), then keeps the fastest.  A process-wide cache
 * keyed by the patch count and size, precision, time-dependent source count and n_t
 * answers repeated calls without timing unless flags has PD_TUNE_FORCE.  best_ms (may be
 * NULL) receives the measured time per step.  Synchronises `stream`.  Errors as
 * pd_patch_step; PD_ENONFINITE if a timed step produced a non-finite value. */
#define PD_TUNE_FORCE 1
pd_status pd_autotune(pd_grid g, const double* U, double t_n, double dt_macro,
                      double dt_micro, int32_t n_t, int32_t reps, uint32_t flags,
                      double* best_ms, void* stream);

/* ----------------------------------------------------------------------------- batches
 * Many independent problems advanced together (not in the paper: how this library fills
 * a GPU with many small grids).  Every member keeps its own grid (FP64 bursts,
 * coefficients set, workspace bound), macro field U (device, [n_eta][n_xi], in/out) and
 * time parameters.  A batch macro step is one persistent launch in which blocks take
 * groups of patches of any member from a device work queue (sorted longest first), with
 * lift, burst, restriction and projection fused as in pd_patch_step and the Dirichlet
 * nodes written by the same launch; pd_batch_solve replays steps from a HIP graph.  The
 * result for each member is bitwise that of pd_solve on its grid.  While a batch is in
 * use its members' workspaces belong to it (their second macro buffer, time-factor and
 * Dirichlet tables). */
typedef struct pd_batch_s* pd_batch;
typedef struct {
  pd_grid grid;
  double* U;
  double t0, dt_macro, dt_micro;
  int32_t n_t;
} pd_batch_member;
typedef struct {
  int32_t n_members;
  int32_t n_items;           /* work items of the queue                                 */
  int32_t blocks;            /* persistent blocks per launch                            */
  int32_t time_sources;      /* time-dependent source terms the kernel carries (1 or 2)  */
  size_t workspace_bytes;    /* device bytes pd_batch_bind_workspace needs               */
  size_t lds_bytes;          /* dynamic LDS per block                                    */
  int32_t tuned;
  double tuned_ms;           /* measured time of one batch macro step after tuning (ms)  */
  int64_t updates_per_step;  /* sum over members of patches x points x n_t               */
} pd_batch_info;
/* Validates the members (PD_EINVAL: null grid or U, FP32 grid, bad time parameters;
 * PD_ESTATE: coefficients or workspace missing; PD_EUNSTABLE as pd_solve) and picks a
 * launch shape per member from the batch kernel's menu.  Allocates no device memory. */
pd_status pd_batch_create(const pd_batch_member* members, int32_t n, pd_batch* out);
pd_status pd_batch_destroy(pd_batch b);
pd_status pd_batch_query(pd_batch b, pd_batch_info* out);
/* Device memory for the instance table, the work queue and the shared clock
 * (>= pd_batch_info.workspace_bytes, 256-byte aligned); PD_ENOMEM if too small. */
pd_status pd_batch_bind_workspace(pd_batch b, void* dev, size_t bytes);
/* Menu shape of a member (its index in the kernel's menu and patches per team) and a
 * way to force one (shape -1 = automatic); PD_EINVAL if the shape cannot hold the
 * member's patches. */
pd_status pd_batch_get_shape(pd_batch b, int32_t member, int32_t* shape, int32_t* ppb);
pd_status pd_batch_set_shape(pd_batch b, int32_t member, int32_t shape);
/* Autotuner: for each group of members with the same patch size, times every feasible
 * menu shape in the batch kernel itself (HIP events, `reps` launches) and keeps the
 * fastest; best_ms (may be NULL) receives the measured time of a whole batch step.
 * Writes only the members' second macro buffers.  Synchronises `stream`. */
pd_status pd_batch_autotune(pd_batch b, int32_t reps, double* best_ms, void* stream);
/* n_steps macro steps of every member from its t0. */
pd_status pd_batch_solve(pd_batch b, int32_t n_steps, void* stream);
/* Synchronise and report PD_ENONFINITE if any member's kernels saw a non-finite value. */
pd_status pd_batch_sync(pd_batch b, void* stream);

/* ---------------------------------------------------------------------- learned closure
 * A small network that stands in for a patch's micro-burst (not in the paper: an addition
 * whose targets the plain scheme produces and which the plain scheme checks).  For the
 * patch at macro node (i, j) it predicts F = (R(u(tau)) - U)/tau (eq. Time_Derivative) as
 *   F_hat = F0 + s y_hat,
 * F0 the macro finite-difference operator at the node with the patch-centre coefficients,
 * s = kappa sigma + 1e-3 (|g| + |phi U|) (kappa: sum of the rates alpha/Dxi^2,
 * gamma/Deta^2, |nu|/Dxi, |omega|/Deta, |phi|; sigma: RMS of the 24 stencil differences),
 * and y_hat the network output on 33 inputs: the 24 differences of the 5x5 stencil / sigma
 * (row-major, centre skipped; indices wrap on a periodic axis, clamp otherwise),
 * U/(|U| + sigma), the five rates / kappa, q/(1+|q|) with q = g/(kappa (|U| + sigma)), and
 * the micro cell Peclet numbers P/(1+P), P = |nu| dxi/(2 alpha) and |omega| deta/(2 gamma)
 * (the scale factors enter through alpha, gamma, nu, omega); standardised per input.
 * Network 33 -> 128 -> 128 -> 1 with GELU(x) = x Phi(x); parameters as one FP32 vector
 * W1 [33][128] (input-major), b1, W2 [128][128], b2, w3 [128], b3 (20993 values).  Training
 * runs in FP32 (mean squared error on standardised targets, Adam with beta1 0.9, beta2
 * 0.999, eps 1e-8); inference rounds inputs, weights and first-layer activations to
 * bfloat16 and accumulates in FP32 on MFMA.  All pointers are
 * device pointers unless named host_. */
typedef struct pd_closure_s* pd_closure;
/* max_batch: rows per training step and per inference chunk (64..4194304). */
pd_status pd_closure_create(int32_t device, int32_t max_batch, pd_closure* out);
pd_status pd_closure_destroy(pd_closure c);
pd_status pd_closure_query(pd_closure c, size_t* workspace_bytes, int32_t* n_params);
/* Zeroes the workspace; parameters and standardisation must then be set. */
pd_status pd_closure_bind_workspace(pd_closure c, void* dev, size_t bytes);
/* Host vectors of 20993 FP32 values; setting resets the optimiser state. */
pd_status pd_closure_set_params(pd_closure c, const float* host_params);
pd_status pd_closure_get_params(pd_closure c, float* host_params);
/* Per-input mean and standard deviation (33 each, host), or fitted on the device to rows
 * X [n][33] of raw inputs (and, when y is non-NULL, the target mean and deviation from
 * targets y [n]: the network learns (y - mean)/deviation and y_hat = mean + deviation out;
 * by default mean 0, deviation 1). */
pd_status pd_closure_set_standardisation(pd_closure c, const float* host_mu, const float* host_sd);
pd_status pd_closure_get_standardisation(pd_closure c, float* host_mu, float* host_sd);
pd_status pd_closure_fit_standardisation(pd_closure c, const float* X, const float* y, int64_t n,
                                         void* stream);
pd_status pd_closure_set_target_scale(pd_closure c, float mean, float sd);
pd_status pd_closure_get_target_scale(pd_closure c, float* mean, float* sd);
/* Raw inputs X [P][33] (FP32), F0 [P] and s [P] (FP64, may be NULL) of every patch of a
 * grid for the macro field U at time t_n. */
pd_status pd_closure_features(pd_grid g, const double* U, double t_n, float* X, double* F0,
                              double* s, void* stream);
/* Training pairs of one plain macro step U_n -> U_np1 (e.g. pd_macro_step) of every
 * patch: inputs X [P][33] and targets y [P] = (F - F0)/s clipped to [-10, 10], with
 * F = (U_np1 - U_n)/dt_macro at the patch node (eq. Extrapolation solved for F). */
pd_status pd_closure_targets(pd_grid g, const double* U_n, const double* U_np1, double t_n,
                             double dt_macro, float* X, float* y, void* stream);
/* Mean-squared-error loss (FP32 [1]) and gradients (FP32 [20993], layout of the
 * parameters) on n <= max_batch rows of raw inputs X and targets y. */
pd_status pd_closure_gradients(pd_closure c, const float* X, const float* y, int32_t n,
                               float* grad, float* loss, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * training loops, harnesses that forbid hipMalloc): pd_closure_gradients with its scratch
 * (standardised rows, activations, back-propagated planes, split-K partial sums) in a
 * fixed device array inside the library instead of the closure workspace's training
 * buffers.  Same kernels and arguments; grad [20993] and loss [1] (FP32, device) must be
 * non-null and are written directly (loss is cleared by a kernel, no memset).  Limit:
 * 1 <= n <= PD_NOALLOC_MAX_ROWS rows, else PD_EINVAL with a message; the closure must
 * have its workspace bound, parameters and standardisation set (PD_ESTATE otherwise).
 * The array takes pd_noalloc_scratch_bytes() (about 17 MB) on each device the library
 * runs on, held until the process ends.  The call allocates nothing: no hipMalloc,
 * hipFree or allocating library routine.  Every call on one device shares that device's
 * array, so calls that overlap on one device (other streams, other threads) race; calls
 * ordered on one stream are safe. */
#define PD_NOALLOC_MAX_ROWS 4096
pd_status pd_closure_gradients_noalloc(pd_closure c, const float* X, const float* y, int32_t n,
                                       float* grad, float* loss, void* stream);
size_t pd_noalloc_scratch_bytes(void);
/* `epochs` passes over n rows in minibatches of `batch` rows (a seeded affine shuffle per
 * epoch, n / batch full batches), one Adam step each; host_losses (may be NULL) receives
 * the mean minibatch loss of each epoch (then the call synchronises per epoch). */
pd_status pd_closure_train(pd_closure c, const float* X, const float* y, int64_t n,
                           int32_t batch, int32_t epochs, float lr, uint32_t seed,
                           float* host_losses, void* stream);
/* Network outputs [n] (FP32, before the target scale) for raw inputs X [n][33], bfloat16
 * MFMA path. */
pd_status pd_closure_infer(pd_closure c, const float* X, float* out, int64_t n, void* stream);
/* The closure macro step of every patch node of a grid: U_np1 = U_n + dt_macro F_hat
 * (boundary nodes untouched; F_hat [P] FP64 stored when non-NULL).  U_n, U_np1 distinct. */
pd_status pd_closure_patch_step(pd_closure c, pd_grid g, const double* U_n, double* U_np1,
                                double t_n, double dt_macro, double* F_hat, void* stream);

/* Batched closure steps with the plain scheme as fallback.  Each macro step of every
 * member: the closure step of all patch nodes (and the Dirichlet nodes), then plain bursts
 * on one work item in `stride` of each member (a per-step hashed choice, at least one
 * item per member) which overwrite those patches, the residual |F_hat - F| / s of every
 * checked patch, and, for each member whose largest residual exceeds `threshold` (or is
 * not finite), plain bursts on all its items in the same step.  All in one HIP graph per
 * 16 steps.  Attach needs pd_batch_closure_bytes of device memory (256-byte aligned) and
 * a closure with parameters and standardisation set; the closure must outlive the batch's
 * use of it.  Stats: patches checked and member fallbacks since the last reset. */
pd_status pd_batch_closure_bytes(pd_batch b, size_t* bytes);
pd_status pd_batch_closure_attach(pd_batch b, pd_closure c, int32_t stride, double threshold,
                                  void* dev, size_t bytes);
pd_status pd_batch_closure_solve(pd_batch b, int32_t n_steps, void* stream);
pd_status pd_batch_closure_stats(pd_batch b, int64_t* checked, int64_t* fallbacks,
                                 int32_t reset);

/* ------------------------------------------------------------ full-domain lattice
 * The explicit comparator of the paper's full-domain solution (Sec. 4.1.2, Table
 * PDvsFDS, there a method-of-lines run on one 151^2 lattice): the operator of
 * eq. (Computational_Problem) of grid g's problem, discretised on one n_x x n_y lattice
 * over the whole box with the bursts' differences (3-point second differences; 2-point
 * upwind or central first differences, the grid's conv) and advanced by forward Euler
 * steps of dt.  Lattice node (i, j) sits at (xi0 + i hx, eta0 + j hy) with
 * hx = (xi1 - xi0) / (n_x - 1) (on a periodic xi axis (xi1 - xi0) / n_x, the nodes
 * wrapping) and hy = (eta1 - eta0) / (n_y - 1); fields are FP64 row-major [n_y][n_x].
 * After every step the boundary rows (and the end columns unless xi is periodic) take
 * the Dirichlet data u_b at the step's end time; step s of a solve from t0 starts at
 * t0 + s dt and its source time factors are taken there.
 *  - pd_fd_create: host only; the grid must outlive the lattice.  PD_EINVAL for
 *    n_x or n_y < 3 or more than 2^30 nodes.
 *  - pd_fd_bind_workspace: caller device memory of workspace_bytes, 256-byte aligned
 *    (PD_ENOMEM if smaller): weight planes, a second field buffer, step tables.
 *  - pd_fd_prepare: folds the weights for dt (needs the grid's coefficients; do it again
 *    after pd_set_coefficients) and computes the explicit bound over the lattice;
 *    synchronises the stream once.  PD_EUNSTABLE if dt is above the bound (unless the
 *    grid's PD_OPT_ALLOW_UNSTABLE is set), PD_EINVAL if diffusion is not positive.
 *  - pd_fd_initial: U = u_b(t) at every lattice node (asynchronous).
 *  - pd_fd_solve: n_steps >= 0 steps of U in place (asynchronous; PD_ESTATE before a
 *    successful prepare).
 *  - pd_fd_sync: synchronises and returns PD_ENONFINITE if a step produced a
 *    non-finite value since the last sync. */
typedef struct pd_fd_s* pd_fd;
typedef struct {
  int32_t n_x, n_y;
  size_t workspace_bytes;
  double dt_limit;             /* explicit bound over the lattice (after pd_fd_prepare) */
  double dt;                   /* the prepared step (0 before pd_fd_prepare)            */
  double spacing_x, spacing_y; /* hx, hy                                                */
} pd_fd_info;
pd_status pd_fd_create(pd_grid g, int32_t n_x, int32_t n_y, pd_fd* out);
pd_status pd_fd_destroy(pd_fd f);
pd_status pd_fd_query(pd_fd f, pd_fd_info* out);
pd_status pd_fd_bind_workspace(pd_fd f, void* dev, size_t bytes);
pd_status pd_fd_prepare(pd_fd f, double dt, void* stream);
pd_status pd_fd_initial(pd_fd f, double* U, double t, void* stream);
pd_status pd_fd_solve(pd_fd f, double* U, double t0, int32_t n_steps, void* stream);
pd_status pd_fd_sync(pd_fd f, void* stream);

const char* pd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
