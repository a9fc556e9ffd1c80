// Internal declarations shared by the host API (pd_host.hip) and the kernels
// (pd_coeff.hip, pd_burst.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/pd.h"

namespace pdk {

// Grid constants as the kernels see them (copied by value into kernel arguments).
struct Geo {
  int geometry;
  double gparam;
  double xi0, xi1, eta0, eta1;
  int n_xi, n_eta, periodic;
  double h_xi, h_eta;
  int m_xi, m_eta;
  int conv, c0mode;
  double Dxi, Deta;     // macro spacings
  double dxi, deta;     // micro spacings h/(m-1)
  double kap_xi, kap_eta;
  int P, npx, i_first, M;
  int ks, nks, ls, nls;  // restriction core: first index and points, xi and eta
};

// Trapezoid weight of index i within the core [i0, i0 + n).
__host__ __device__ inline double core_w(int i, int i0, int n) {
  return (i == i0 || i == i0 + n - 1) ? 0.5 : 1.0;
}

// Offsets (in doubles) of the pieces of the stencil table: the same layout that
// pd_get_tables documents.
struct TabOff {
  int s_xi, s_eta, L_xe, L_ee, ew, c_xi, c_eta, scal, size;
};

// Stencil-table values each thread of a team stages in registers during the burst
// prologue (the team copies at most TAB_STAGE * team threads values to LDS): with
// m_xi, m_eta <= 64 the tables hold 5 (m_xi + m_eta) + 20 <= 660 values, and a 64-thread
// team holds a patch only if ceil(m_xi / C) ceil(m_eta / R) <= 64 with C R <= 12, so
// m_xi + m_eta <= 85 and at most 445 values; launch-shape choices check it anyway.
constexpr int TAB_STAGE = 7;

__host__ __device__ inline TabOff tab_off(int mx, int me) {
  TabOff t;
  t.s_xi = 0;
  t.s_eta = mx;
  t.L_xe = mx + me;           // [m_eta][3]: interpolation along eta at the xi edges
  t.L_ee = t.L_xe + 3 * me;   // [m_xi][3]:  interpolation along xi at the eta edges
  t.ew = t.L_ee + 3 * mx;     // xi-, xi+, eta-, eta+ (3 each)
  t.c_xi = t.ew + 12;
  t.c_eta = t.c_xi + mx;
  t.scal = t.c_eta + me;      // Dxi, Deta, dxi, deta, r_xi, r_eta, kappa_xi, kappa_eta
  t.size = t.scal + 8;
  return t;
}

// Device-side clock of pd_solve.  A replay of the captured steps starts with k_replay,
// which sets base = next (macro steps done so far) and advances next; step k of the
// replay is macro step n = base + k at time t0 + n dt, reading the macro field from
// buf[n & 1] and writing buf[(n + 1) & 1].
struct Clock {
  double t0, dt;
  long long base, next;
  double* buf[2];
  unsigned int done;  // blocks of k_replay finished (the last one advances the clock)
};

// Time factors and the constant part of the source, packed for kernel arguments.
struct SrcInfo {
  int ns;                 // time-dependent terms (<= 2)
  int plane_t[2];         // their coefficient planes
  int ttype[2];
  double ta[2], tb[2], tc[2];
  int nconst;             // constant terms folded into the static forcing
  int plane_c[PD_MAXTERM];
  double ca[PD_MAXTERM];
};

// Time factor T_j(t) of time-dependent source term j.
__device__ inline double time_factor(const SrcInfo& src, int j, double t) {
  if (src.ttype[j] == PD_T_EXP) return src.ta[j] * exp(src.tb[j] * t);
  if (src.ttype[j] == PD_T_SIN) return src.ta[j] + src.tb[j] * sin(src.tc[j] * t);
  return src.ta[j];
}

// Dirichlet nodes in a fixed order: the eta = eta0 and eta = eta1 rows, then (when xi is
// not periodic) the xi = xi0 and xi = xi1 columns between them, alternating.
__host__ __device__ inline int boundary_count(const Geo& g) {
  return 2 * g.n_xi + (g.periodic ? 0 : 2 * (g.n_eta - 2));
}
__host__ __device__ inline void boundary_node(const Geo& g, int q, int& i, int& j) {
  const int nb_rows = 2 * g.n_xi;
  const int r = q - nb_rows;
  i = q < nb_rows ? q % g.n_xi : ((r & 1) ? g.n_xi - 1 : 0);
  j = q < nb_rows ? (q < g.n_xi ? 0 : g.n_eta - 1) : 1 + r / 2;
}

enum { MODE_SPLIT = 0, MODE_FUSED = 1 };
// Neighbour exchange of the burst: through LDS (any block size), inside one wave (DPP
// wave shifts and ds_bpermute, single-wave blocks), or hybrid (DPP inside each wave, band
// edges through LDS, blocks of several waves).
enum { XCH_LDS = 1, XCH_LANES = 2, XCH_HYBRID = 3 };

struct BurstArgs {
  Geo g;
  SrcInfo src;
  const double* coef;     // planes [5 + n_src][P][m_eta][m_xi]
  const int* pmap;        // [P][11]
  const double* tab;      // stencil tables
  long long plane;        // P * m_xi * m_eta
  // split mode
  double* state;          // [P][m_eta][m_xi] in/out
  const double* edge;     // [P][4][M]
  // fused mode
  const double* U;        // U_n
  double* Unew;           // U_{n+1} (patch nodes)
  const Clock* clk;       // non-null: macro step clk->base + k, buffers from the clock
  int k;                  //   (step within the graph replay)
  const double* ttab;     // [ns][n_t] time factors T_j(t_n + s dt)
  const double* bvals;    // non-null: Dirichlet values at t_n + dt_macro, written to Unew
  int nb;                 //   (boundary_count entries)
  double t_n, dt, dt_macro, tau;
  int n_t;
  int ppb;                // patches per block
  int* flag;              // non-finite flag
  int balance;            // in-wave kernels: every block is resident at once, so waves
                          // lower their issue priority as they progress (set at launch)
};

// Launchers implemented in the kernel translation units.
hipError_t launch_coefficients(const Geo& g, const pd_coeff_desc* dev_desc, int n_src,
                               double* coef, hipStream_t s);
hipError_t launch_limits(const Geo& g, const pd_coeff_desc* dev_desc, int n_src,
                         const double* coef, double* partial, int nblocks, double* out,
                         hipStream_t s);
hipError_t launch_boundary(const Geo& g, const pd_coeff_desc* dev_desc, double* U, double t,
                           hipStream_t s);
// Start of a graph replay of S macro steps: advances the clock and fills the time factors
// ttab[S][ns][n_t] and the Dirichlet values bvals[S][nb] of those steps.
hipError_t launch_replay(const Geo& g, const SrcInfo& src, const pd_coeff_desc* dev_desc,
                         Clock* clk, int S, int n_t, double dt_micro, double* ttab,
                         double* bvals, hipStream_t s);
hipError_t launch_initial(const Geo& g, const pd_coeff_desc* dev_desc, double* U, double t,
                          hipStream_t s);
// ADI micro burst (split mode): one wave holds ppb patches (max(m_xi, m_eta) lanes each),
// 6 m_xi m_eta + 4 max(m_xi, m_eta) doubles of LDS per patch; ppb = 0 when no patch fits
// in ADI_LDS_MAX.
constexpr size_t ADI_LDS_MAX = 65536;
void adi_shape(int mx, int me, int& ppb, size_t& lds);
hipError_t launch_burst_adi(const Geo& g, const SrcInfo& src, const double* coef,
                            long long plane, double* state, const double* edge, double t_n,
                            double dt, int n_t, int* flag, hipStream_t s);

// Explicit burst with the 2-, 3- or 4-point upwind first differences (pd_upwind.hip): up to
// 1024 micro points per block, the patches' ghost-framed tiles within HU_LDS_MAX.
constexpr size_t HU_LDS_MAX = 65536;
void hu_shape(int mx, int me, int& ppb, size_t& lds);
// lds_only: the LDS-tile kernel even where a patch fits the in-wave kernel's lane blocks.
hipError_t launch_burst_hu(const Geo& g, const SrcInfo& src, const double* coef,
                           long long plane, double* state, const double* edge, double t_n,
                           double dt, int n_t, int points, double r, int* flag,
                           bool lds_only, hipStream_t s);

// ---------------------------------------------------------------- full-domain lattice
// The explicit comparator on one lattice over the whole box: a Geo whose n_xi x n_eta
// nodes are the lattice (spacings Dxi, Deta), weight planes [cC, cS, cN, cW, cE, K,
// sd_0, sd_1] (see k_fd_weights), time-factor and Dirichlet tables per chunk of steps.
constexpr int FD_CHUNK = 256;  // steps per table chunk
constexpr int FD_NB = 1024;    // blocks of the weight pass (and its bound reduction)
struct FdArgs {
  int n_x, n_y, periodic;
  int ns;             // time-dependent source terms (0..2)
  int has_k;          // constant source terms present (K plane non-zero)
  int nb;             // Dirichlet nodes
  long long plane;    // n_x * n_y
  const double* W;    // weight planes
  const double* ttab; // [ns][FD_CHUNK]
  const double* bvals;// [FD_CHUNK][nb]
  int* flag;          // set to 1 on a non-finite value
};
hipError_t launch_fd_weights(const Geo& lat, const pd_coeff_desc* dev_desc, const SrcInfo& src,
                             int n_src, double dt, double* W, double* partial, int nblocks,
                             double* lim, hipStream_t s);
hipError_t launch_fd_tables(const Geo& lat, const SrcInfo& src, const pd_coeff_desc* dev_desc,
                            double t0, double dt, long long s0, int S, double* ttab,
                            double* bvals, hipStream_t s);
// One lattice step: V = step(U) with the tables' entry k.
hipError_t launch_fd_step(const FdArgs& a, const double* U, double* V, int k, hipStream_t s);

hipError_t launch_clock_init(Clock* clk, double t0, double dt, double* b0, double* b1,
                             hipStream_t s);
hipError_t launch_lift_bc(const Geo& g, const int* pmap, const double* tab, const double* U,
                          double* state, double* edge, hipStream_t s);
hipError_t launch_restrict(const Geo& g, const double* state, double* Ubar, hipStream_t s);
hipError_t launch_scatter_patch_values(const Geo& g, const int* pmap, const double* Ubar,
                                       double* U, hipStream_t s);
hipError_t launch_macro_update(const Geo& g, const int* pmap, const double* U,
                               const double* Ubar, double* Unew, double dt_macro, double tau,
                               int* flag, hipStream_t s);
// Time factors of the time-dependent source terms for one burst.
hipError_t launch_time_table(const SrcInfo& src, double t_n, double dt, int n_t, double* out,
                             hipStream_t s);
constexpr int MAX_NT = 65536;  // nano steps per burst (size of the time-factor table)
// Burst kernels: precision PD_F64/PD_F32, C columns x R rows per lane, exchange, mode.
hipError_t launch_burst(int precision, int R, int C, int xch, int mode, const BurstArgs& a,
                        int blocks, int threads, size_t lds, hipStream_t s);
bool burst_shape_supported(int R, int C);

// Dynamic LDS bytes of a burst launch: the lane-major exchange tiles (double-buffered,
// guard of lanes-per-band + 1 words on both sides) or the FP64 lifted tile of the
// prologue, whichever is larger, then the time-factor chunk, the restriction rows, a
// copy of the stencil tables and the edge data of each patch slot.
__host__ __device__ inline size_t burst_lds_bytes(int precision, int R, int C, int xch,
                                                  int threads, int ppb, int mx, int me,
                                                  int ns) {
  const size_t rs = precision == PD_F32 ? 4 : 8;
  const int Lb = (mx + C - 1) / C;
  const size_t nbuf = xch == XCH_LDS ? 2 : 1;
  size_t exch = nbuf * R * C * (size_t)(threads + 2 * (Lb + 1)) * rs;
  if (xch == XCH_HYBRID) {  // band-edge planes: 2 buffers x (top, bottom) x (bands + 3)
    const size_t edges = (size_t)4 * ((threads / 64) * (64 / Lb) + 3) * C * Lb * rs;
    if (edges > exch) exch = edges;
  }
  const size_t lift = (size_t)ppb * (mx + 2) * (me + 2) * 8;
  const size_t region = ((exch > lift ? exch : lift) + 15) & ~size_t(15);
  const int TCH = 256;
  return region + (size_t)(ns > 0 ? ns : 1) * TCH * 8 + (size_t)ppb * me * 8 +
         (size_t)tab_off(mx, me).size * 8 + (size_t)ppb * 2 * (mx + me) * 8 + 64;
}

// ---------------------------------------------------------------- batched bursts
// Launch shapes the persistent batch kernel can run: (id, exchange, columns, rows per
// lane).  In-wave shapes run four single-wave teams per block; LDS and hybrid shapes one
// team of the whole block.
#define PD_BATCH_MENU(X)                                                                 \
  X(0, XCH_LANES, 1, 3) X(1, XCH_LANES, 1, 5) X(2, XCH_LANES, 1, 6) X(3, XCH_LANES, 1, 7) \
  X(4, XCH_LANES, 2, 3) X(5, XCH_LDS, 1, 5) X(6, XCH_LDS, 2, 3) X(7, XCH_LDS, 3, 2)       \
  X(8, XCH_LDS, 4, 2) X(9, XCH_HYBRID, 2, 4) X(10, XCH_HYBRID, 3, 2)                     \
  X(11, XCH_HYBRID, 2, 3)
constexpr int BATCH_MENU = 12;
constexpr int BATCH_THREADS = 256;
constexpr int BATCH_WAVES = BATCH_THREADS / 64;

// One unit of the device work queue: ppb patches per team from patch p0 of instance inst
// (in-wave shapes: BATCH_WAVES teams, p0 + w * ppb for wave w).
struct BatchItem {
  int inst, shape, p0, ppb;
};

struct BatchArgs {
  const BurstArgs* inst;    // per instance: grid constants, planes, tables, U (buffer 0),
                            // Unew (buffer 1), t_n = t0, dt, dt_macro, tau, n_t, ttab, bvals
  const BatchItem* items;   // in queue order
  int n_items;
  int* head;                // next item (the last block to finish resets it)
  unsigned int* exits;      // blocks finished
  const Clock* clk;         // macro step = clk->base + k (buffers by its parity)
  int k;                    // step within the graph replay
  int tuning;               // 1: read buffer 0, write buffer 1, whatever the clock says
  // segment mode (device-built lists): item j of the launch is
  // items[seg.first + (j - seg.prefix) seg.stride] of the segment holding j, with the
  // item count read from n_dev
  const int4* segs;         // {first, count, stride, prefix} per segment, or nullptr
  int n_segs;
  const int* n_dev;
};

// Spot checks and fallback of the batched closure (device-side state, one entry per
// instance).  first/count: the instance's items in the instance-ordered item list.
struct SpotArgs {
  const int* first;
  const int* count;
  const int* order;         // instances by descending item cost: segment slot s is order[s]
  int n;                    // instances
  int stride;               // one item in `stride` is checked per step
  const Clock* clk;
  int k;
  int4* spot;               // spot-check segments, and their item count in spot_n
  int* spot_n;
  int4* redo;               // fallback segments and count
  int* redo_n;
  unsigned int* resid;      // per-instance maximum residual (float bits)
  double threshold;
  unsigned long long* stats;  // [0] patches checked, [1] instance fallbacks
};
hipError_t launch_spot_segments(const SpotArgs& a, hipStream_t s);
hipError_t launch_redo_segments(const SpotArgs& a, hipStream_t s);
hipError_t launch_spot_residuals(const SpotArgs& a, const BurstArgs* inst,
                                 const BatchItem* items, double* const* fhat,
                                 float* const* sres, int blocks, hipStream_t s);

// Persistent batch kernel, nsb = 1 or 2 time-dependent source terms at most.
hipError_t launch_batch(int nsb, const BatchArgs& a, int blocks, size_t lds, hipStream_t s);
hipError_t batch_blocks_per_cu(int nsb, size_t lds, int* out);
// Time factors and Dirichlet values of S steps for every instance (one block per
// instance); the last block advances the clock.
hipError_t launch_batch_replay(const BurstArgs* inst, const pd_coeff_desc* const* descs, int n,
                               Clock* clk, int S, hipStream_t s);

// ------------------------------------------------------------------ learned closure
constexpr int CL_FEAT = 33;     // network inputs
constexpr int CL_HID = 128;     // hidden width
constexpr int CL_NPAR = CL_FEAT * CL_HID + CL_HID + CL_HID * CL_HID + CL_HID + CL_HID + 1;
// offsets of the parameters in the flat FP32 vector: W1 [33][128], b1, W2 [128][128], b2,
// w3 [128], b3
constexpr int CL_OW1 = 0, CL_OB1 = CL_OW1 + CL_FEAT * CL_HID, CL_OW2 = CL_OB1 + CL_HID,
              CL_OB2 = CL_OW2 + CL_HID * CL_HID, CL_OW3 = CL_OB2 + CL_HID,
              CL_OB3 = CL_OW3 + CL_HID;
// per-patch static closure data (doubles): node i, j; rates a, b, c, d; phi; micro-to-macro
// spacing ratios dxi/Dxi, deta/Deta; constant source at the centre; time-dependent source
// parts at the centre (2)
constexpr int CL_SPLITK = 64;  // row chunks of the weight-gradient products
constexpr int CL_NST = 12;
hipError_t launch_closure_static(const Geo& g, const SrcInfo& src, const int* pmap,
                                 const double* coef, long long plane, double* st,
                                 hipStream_t s);
constexpr int CL_K1P = 40;  // first-layer depth padded to a multiple of 8 (bfloat16 MFMA)

struct MlpW {
  const unsigned short *w1t, *w2t, *w3;
  const float* par;  // FP32 biases b1, b2, b3 live in the master vector
};

struct ClosureArgs {
  BurstArgs one;                  // single grid
  const double* st_one;
  double* fhat_one;
  const BurstArgs* inst;          // batch: instance table (nullptr for a single grid)
  const double* const* st_tab;    // batch: per-instance static closure data
  double* const* fhat_tab;        // batch: per-instance F_hat
  const int* items;               // batch: (instance, first patch) pairs
  int n_items;                    // units of 64 patches (batch items, or ceil(P / 64))
  int k;                          // batch: step within the graph replay
  float* const* sres_tab;         // batch: per-instance closure scale s (spot residuals)
  MlpW W;
  const float *mu, *sd;
  const float* ys;                // target mean and deviation: y = ys[0] + ys[1] out
};

hipError_t launch_closure_features(const Geo& g, const SrcInfo& src, const double* st,
                                   const double* U, double t_n, float* X, double* F0,
                                   double* sc, const double* Unp1, double dtm, float* y,
                                   hipStream_t s);
hipError_t launch_mlp_grads(int nb, const float* Xn, const float* y, const float* par,
                            float* H1, float* A1, float* H2, float* A2, float* dH2,
                            float* dH1, float* out, float* dout, float* grad, float* loss,
                            float* part, hipStream_t s);
hipError_t launch_adam(float* par, float* m, float* v, const float* g, int step, float lr,
                       hipStream_t s);
hipError_t launch_fill_f32(float* x, long long n, float v, hipStream_t s);
hipError_t launch_colstats(long long n, const float* X, float* mu, float* sd, hipStream_t s);
hipError_t launch_standardise(long long n, const float* X, long long n_src, long long a,
                              long long c, const float* mu, const float* sd, float* Xn,
                              const float* y, float* yb, const float* ys, hipStream_t s);
hipError_t launch_target_stats(long long n, const float* y, float* ys, hipStream_t s);
hipError_t launch_pack(const float* par, unsigned short* w1t, unsigned short* w2t,
                       unsigned short* w3, hipStream_t s);
hipError_t launch_mlp_infer(long long n, const float* Xn, const unsigned short* w1t,
                            const unsigned short* w2t, const unsigned short* w3, const float* par,
                            float* out, hipStream_t s);
hipError_t launch_closure_step(const ClosureArgs& a, hipStream_t s);

}  // namespace pdk
