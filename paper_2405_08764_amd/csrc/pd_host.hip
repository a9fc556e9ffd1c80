// Host side of the C ABI in include/pd.h: validation, the macro mesh and patch index
// map (Sec. 3), the stencil tables (eq. Lagrange_2D at the micro edge points, eq. edge
// weights, trapezoid weights, the eq. C_0 constants), the caller-owned workspace, launch
// shapes and the HIP graph that replays whole macro steps (Sec. 3.3 "until the final
// time T").
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pd_internal.h"
#include "pd_refresh.h"

namespace pdk {
#define PD_DECL(tag)                                                                      \
  hipError_t launch_burst_##tag(int R, int C, const BurstArgs& a, int blocks, int threads, \
                                size_t lds, hipStream_t s);
PD_DECL(lds_f64)
PD_DECL(lds_f32)
PD_DECL(x_f64)
PD_DECL(x_f32)
PD_DECL(h_f64)
PD_DECL(h_f32)
PD_DECL(ldss_f64)
PD_DECL(ldss_f32)
PD_DECL(xs_f64)
PD_DECL(xs_f32)
PD_DECL(hs_f64)
PD_DECL(hs_f32)
#undef PD_DECL

// Resident fused solve with the in-wave exchange (pd_solve_x_f64.hip).
size_t solve_x_extra_lds(int ppb, int mx, int me, int nconst);
hipError_t launch_zero_flags(long long* f, int n, hipStream_t s);
hipError_t launch_solve_x_f64(int R, int C, const BurstArgs& a, long long* flags, int* err,
                              int steps, const double* ttab0, const double* bval0, int per,
                              int blocks, size_t lds, hipStream_t s, int* resident);
// Resident refreshed macro step with the in-wave exchange (pd_solve_x_f64.hip).
size_t refresh_x_extra_lds(int ppb, int mx, int me, int nconst);
hipError_t launch_refresh_x_f64(int R, int C, const BurstArgs& a, long long* flags, int* err,
                                int Q, double* Uw0, double* Uw1, const double* bvq,
                                int blocks, size_t lds, hipStream_t s, int* resident);

// ADI burst with the higher-order upwind differences (pd_adi_upwind.hip): patches per
// wave and LDS bytes for m_xi x m_eta patches (ppb = 0 when none fits), and the launcher.
void adu_shape(int mx, int me, int& ppb, size_t& lds);
hipError_t launch_burst_adi_hu(const Geo& g, const SrcInfo& src, const double* coef,
                               long long plane, double* state, const double* edge, double t_n,
                               double dt, int n_t, int points, double r, int* flag,
                               hipStream_t s);

// The burst kernel of one exchange family, precision and mode (fused macro step or
// split-mode burst on caller-owned patch states); every family runs both modes.
hipError_t launch_burst(int precision, int R, int C, int xch, int mode, const BurstArgs& a,
                        int blocks, int threads, size_t lds, hipStream_t s) {
  const bool f32 = precision == PD_F32, split = mode == MODE_SPLIT;
  decltype(&launch_burst_lds_f64) fn;
  if (xch == XCH_LANES)
    fn = split ? (f32 ? launch_burst_xs_f32 : launch_burst_xs_f64)
               : (f32 ? launch_burst_x_f32 : launch_burst_x_f64);
  else if (xch == XCH_HYBRID)
    fn = split ? (f32 ? launch_burst_hs_f32 : launch_burst_hs_f64)
               : (f32 ? launch_burst_h_f32 : launch_burst_h_f64);
  else
    fn = split ? (f32 ? launch_burst_ldss_f32 : launch_burst_ldss_f64)
               : (f32 ? launch_burst_lds_f32 : launch_burst_lds_f64);
  return fn(R, C, a, blocks, threads, lds, s);
}

bool burst_shape_supported(int R, int C) {
  if (C == 1) return R == 3 || R == 4 || R == 5 || R == 6 || R == 7 || R == 8 || R == 9 || R == 11;
  if (C == 2) return R >= 2 && R <= 6;
  if (C == 3) return R >= 2 && R <= 4;
  if (C == 4) return R == 2 || R == 3;
  return false;
}
}  // namespace pdk

using namespace pdk;

namespace {

thread_local std::string g_err;

pd_status fail(pd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

pd_status hip_fail(hipError_t e, const char* where) {
  return fail(PD_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int NB_LIM = 512;  // blocks of the stability-bound reduction
constexpr int MAX_REPLAY = 16;                 // macro steps per pd_solve graph replay
constexpr size_t TT_CAP = 2 * (size_t)MAX_NT;  // time-factor table entries

// Micro offsets: m points span the edge h symmetrically, edges included.
double micro_off(double h, int m, int k) {
  return (double)(2 * k - (m - 1)) * (h / (2.0 * (m - 1)));
}

// Lagrange basis eq. (Lagrange_2D) on the nodes (-D, 0, +D) relative to the patch centre:
// product over the other nodes r in increasing order of (t - o_r) / (o_beta - o_r).
double lagrange_basis(int beta, double t, double D) {
  const double nodes[3] = {-D, 0.0, D};
  double num = 0.0, den = 0.0;
  bool started = false;
  for (int r = 0; r < 3; ++r) {
    if (r == beta) continue;
    const double fn = t - nodes[r], fd = nodes[beta] - nodes[r];
    if (!started) {
      num = fn;
      den = fd;
      started = true;
    } else {
      num = num * fn;
      den = den * fd;
    }
  }
  return num / den;
}

}  // namespace

struct pd_grid_s {
  pd_grid_desc d{};
  Geo g{};
  std::vector<int32_t> pmap;
  std::vector<double> tab;
  TabOff to{};
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t off_coef = 0, off_pmap = 0, off_tab = 0, off_desc = 0, off_V = 0, off_flag = 0,
         off_clock = 0, off_part = 0, off_lim = 0, off_ttab = 0, off_bval = 0, off_cst = 0,
         off_pflag = 0, need = 0;
  bool cst_ok = false;  // static closure data computed for the current coefficients
  // coefficients
  bool coeffs_set = false;
  pd_coeff_desc cd{};
  int n_src = 0;
  int max_src = PD_MAXTERM;  // source planes the workspace holds
  SrcInfo src{};
  double lim_micro = 0.0, lim_macro = 0.0;
  // options
  int allow_unstable = 0, opt_R = 0, opt_C = 0, opt_ppb = 0, opt_threads = 0, opt_xch = 0;
  int opt_resident = 1, last_resident = 0, last_refresh_resident = 0;
  // launch shape of the burst, fused and split mode alike
  int R = 0, C = 0, xch = 0, ppb = 0, threads = 0, blocks = 0;
  size_t lds = 0;
  // graph replay of pd_solve
  hipStream_t cap = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int g_steps = 0;
  double g_dtm = 0, g_dt = 0;
  int g_nt = 0;
  double* g_U = nullptr;
  int g_R = 0, g_C = 0, g_ppb = 0, g_threads = 0, g_xch = 0, g_res = 0;
  int g_res_ran = 0;  // the captured replay launches the resident solve
  // autotuner result
  int tuned = 0;
  double tuned_ms = 0.0;
  // what the time-factor table holds (single-step layout), so repeated steps from the
  // same time on the same stream skip recomputing it
  bool tt_ok = false;
  double tt_t = 0.0, tt_dt = 0.0;
  int tt_nt = 0;
  hipStream_t tt_s = nullptr;

  double* coef() { return reinterpret_cast<double*>(ws + off_coef); }
  int* dpmap() { return reinterpret_cast<int*>(ws + off_pmap); }
  double* dtab() { return reinterpret_cast<double*>(ws + off_tab); }
  pd_coeff_desc* ddesc() { return reinterpret_cast<pd_coeff_desc*>(ws + off_desc); }
  double* V() { return reinterpret_cast<double*>(ws + off_V); }
  int* flag() { return reinterpret_cast<int*>(ws + off_flag); }
  Clock* clock() { return reinterpret_cast<Clock*>(ws + off_clock); }
  long long* pflags() { return reinterpret_cast<long long*>(ws + off_pflag); }
  double* part() { return reinterpret_cast<double*>(ws + off_part); }
  double* lim() { return reinterpret_cast<double*>(ws + off_lim); }
  double* ttab() { return reinterpret_cast<double*>(ws + off_ttab); }
  double* bvals() { return reinterpret_cast<double*>(ws + off_bval); }
  double* cst() { return reinterpret_cast<double*>(ws + off_cst); }
};

namespace {

void drop_graph(pd_grid g) {
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->gexec = nullptr;
  g->graph = nullptr;
  g->g_steps = 0;
}

// Launch shape of the burst: C columns x R rows per lane, ppb patches per block, and the
// neighbour exchange.  Candidates are ranked by the useful fraction of the lane slots
// (idle lanes and padding points are wasted VALU issue), weighted 1.5x for the in-wave
// exchange (no LDS traffic and no barrier in the nano-step loop; measured about that much
// faster per lane slot) and 1.2x for the hybrid one (measured on 17 x 17 patches: slower
// per nano step than the in-wave kernel and close to the LDS one); on ties, wider lane
// blocks (fewer exchanged values per point), more rows, then smaller blocks.  The same
// shape serves the fused step and the split-mode burst.  pd_autotune replaces this guess
// by measurement.
struct Shape {
  int R, C, xch, ppb, threads;
  double score;
};

bool next_shape(pd_grid g, int xch_only, std::vector<Shape>& out) {
  const int mx = g->g.m_xi, me = g->g.m_eta;
  const int candR[] = {2, 3, 4, 5, 6, 7, 8, 9, 11};
  out.clear();
  for (int xch = XCH_LDS; xch <= XCH_HYBRID; ++xch) {
    if (xch_only && xch != xch_only) continue;
    for (int C = 1; C <= 4; ++C) {
      if (g->opt_C && C != g->opt_C) continue;
      for (int R : candR) {
        if (!burst_shape_supported(R, C) || (g->opt_R && R != g->opt_R)) continue;
        const int Lb = (mx + C - 1) / C, B = (me + R - 1) / R;
        const int LP = Lb * B;
        for (int cap = 64; cap <= 256; cap += 64) {
          if (xch == XCH_LANES && cap != 64) break;
          if (xch == XCH_HYBRID && cap == 64) continue;  // one wave: the in-wave kernel
          if (g->opt_threads && cap > g->opt_threads) break;
          int ppb, threads;
          if (xch == XCH_HYBRID) {  // whole bands per wave; patches take B bands
            if (Lb > 64) continue;
            ppb = (cap / 64) * (64 / Lb) / B;
            if (ppb < 1) continue;
            if (g->opt_ppb) ppb = g->opt_ppb < ppb ? g->opt_ppb : ppb;
            threads = cap;
          } else {
            if (LP > cap) continue;
            ppb = cap / LP;
            if (g->opt_ppb) ppb = g->opt_ppb < ppb ? g->opt_ppb : ppb;
            threads = ((ppb * LP + 63) / 64) * 64;
          }
          if (burst_lds_bytes(g->d.precision, R, C, xch, threads, ppb, mx, me, g->src.ns) > 65536)
            continue;
          // the prologue stages the stencil tables at TAB_STAGE values per team thread
          if (tab_off(mx, me).size > TAB_STAGE * (xch == XCH_LANES ? 64 : threads)) continue;
          const double eff = (double)ppb * mx * me / ((double)threads * R * C);
          const double w = xch == XCH_LANES ? 1.5 : (xch == XCH_HYBRID ? 1.2 : 1.0);
          const double score = eff * w + 1e-3 * (C - 1) + 1e-4 * R - 1e-5 * threads;
          out.push_back({R, C, xch, ppb, threads, score});
        }
      }
    }
  }
  return !out.empty();
}

void apply_shape(pd_grid g, const Shape& b) {
  g->R = b.R;
  g->C = b.C;
  g->xch = b.xch;
  g->ppb = b.ppb;
  g->threads = b.threads;
  g->blocks = (g->g.P + b.ppb - 1) / b.ppb;
  g->lds = burst_lds_bytes(g->d.precision, b.R, b.C, b.xch, b.threads, b.ppb, g->g.m_xi,
                           g->g.m_eta, g->src.ns);
}

// Process-wide cache of autotuned shapes.
struct TuneKey {
  int P, mx, me, precision, ns, n_t, conv, xch, C, R, ppb, threads;
  bool operator<(const TuneKey& o) const {
    return std::tie(P, mx, me, precision, ns, n_t, conv, xch, C, R, ppb, threads) <
           std::tie(o.P, o.mx, o.me, o.precision, o.ns, o.n_t, o.conv, o.xch, o.C, o.R, o.ppb,
                    o.threads);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<Shape, double>> g_tune;

void choose_shape(pd_grid g) {
  std::vector<Shape> c;
  g->R = 0;
  if (next_shape(g, g->opt_xch, c)) {
    const Shape* b = &c[0];
    for (const Shape& x : c)
      if (x.score > b->score) b = &x;
    apply_shape(g, *b);
  }
}

pd_status check_field(const pd_field& f, bool annulus, const char* name) {
  if (f.nmode < 0 || f.nmode > PD_MAXMODE || f.npolar < 0 || f.npolar > PD_MAXPOLAR)
    return fail(PD_EINVAL, std::string(name) + ": term count out of range");
  if (f.npolar > 0 && !annulus)
    return fail(PD_EINVAL, std::string(name) + ": polar terms need the annulus geometry");
  return PD_OK;
}

pd_status check_fn1(const pd_fn1& f) {
  if (f.type < PD_FN_SIN || f.type > PD_FN_POLY) return fail(PD_EINVAL, "bad 1-D function type");
  return PD_OK;
}

pd_status check_tfun(const pd_tfun& t) {
  if (t.type < PD_T_CONST || t.type > PD_T_SIN) return fail(PD_EINVAL, "bad time factor type");
  return PD_OK;
}

pd_status check_sfun(const pd_sfun& s, bool annulus) {
  if (s.kind != 0 && s.kind != 1) return fail(PD_EINVAL, "bad spatial function kind");
  if (s.kind == 1 && !annulus) return fail(PD_EINVAL, "polar spatial function needs the annulus");
  pd_status st = check_fn1(s.f);
  if (st) return st;
  return check_fn1(s.g);
}

pd_status need_ws(pd_grid g) {
  if (!g) return fail(PD_EINVAL, "null grid");
  if (!g->ws) return fail(PD_ESTATE, "no workspace bound");
  return PD_OK;
}

pd_status need_coeffs(pd_grid g) {
  pd_status s = need_ws(g);
  if (s) return s;
  if (!g->coeffs_set) return fail(PD_ESTATE, "coefficients not set");
  if (!g->R) return fail(PD_EINVAL, "no supported burst launch shape for this patch size");
  return PD_OK;
}

pd_status guard_micro(pd_grid g, double dt, int n_t) {
  if (!(dt > 0.0) || n_t < 1) return fail(PD_EINVAL, "dt_micro must be > 0 and n_t >= 1");
  if (n_t > MAX_NT) return fail(PD_EINVAL, "n_t above the supported 65536 nano steps per burst");
  if (!g->allow_unstable && dt > g->lim_micro * (1.0 + 1e-12)) {
    char b[160];
    snprintf(b, sizeof b, "dt_micro %.6g above the explicit bound %.6g", dt, g->lim_micro);
    return fail(PD_EUNSTABLE, b);
  }
  return PD_OK;
}

pd_status guard_macro(pd_grid g, double dtm, double dt, int n_t) {
  pd_status s = guard_micro(g, dt, n_t);
  if (s) return s;
  if (!(dtm > 0.0)) return fail(PD_EINVAL, "dt_macro must be > 0");
  if (!g->allow_unstable && dtm > g->lim_macro * (1.0 + 1e-12)) {
    char b[160];
    snprintf(b, sizeof b, "dt_macro %.6g above the explicit bound %.6g", dtm, g->lim_macro);
    return fail(PD_EUNSTABLE, b);
  }
  return PD_OK;
}

hipError_t ensure_time_table(pd_grid g, double t_n, double dt, int n_t, hipStream_t s) {
  if (g->tt_ok && g->tt_t == t_n && g->tt_dt == dt && g->tt_nt == n_t && g->tt_s == s)
    return hipSuccess;
  g->tt_ok = false;
  const hipError_t e = launch_time_table(g->src, t_n, dt, n_t, g->ttab(), s);
  if (e == hipSuccess) {
    g->tt_ok = true;
    g->tt_t = t_n;
    g->tt_dt = dt;
    g->tt_nt = n_t;
    g->tt_s = s;
  }
  return e;
}

BurstArgs base_args(pd_grid g, double t_n, double dt, int n_t) {
  BurstArgs a{};
  a.g = g->g;
  a.src = g->src;
  a.coef = g->coef();
  a.pmap = g->dpmap();
  a.tab = g->dtab();
  a.plane = (long long)g->g.P * g->g.m_xi * g->g.m_eta;
  a.t_n = t_n;
  a.dt = dt;
  a.n_t = n_t;
  a.ppb = g->ppb;
  a.flag = g->flag();
  a.ttab = g->ttab();
  return a;
}

}  // namespace

extern "C" {

const char* pd_last_error(void) { return g_err.c_str(); }

pd_status pd_create_grid(const pd_grid_desc* d, pd_grid* out) {
  if (!d || !out) return fail(PD_EINVAL, "null argument");
  *out = nullptr;
  const pd_grid_desc& D = *d;
  if (D.n_xi < 3 || D.n_eta < 3) return fail(PD_EINVAL, "need at least 3 macro nodes per axis");
  if (D.m_xi < 3 || D.m_eta < 3 || D.m_xi > 64 || D.m_eta > 64)
    return fail(PD_EINVAL, "micro points per side must be in 3..64");
  if (!(D.xi1 > D.xi0) || !(D.eta1 > D.eta0)) return fail(PD_EINVAL, "empty computational box");
  const double Dxi = D.periodic_xi ? (D.xi1 - D.xi0) / D.n_xi : (D.xi1 - D.xi0) / (D.n_xi - 1);
  const double Deta = (D.eta1 - D.eta0) / (D.n_eta - 1);
  if (!(D.h_xi > 0.0) || !(D.h_eta > 0.0) || !(D.h_xi < Dxi) || !(D.h_eta < Deta))
    return fail(PD_EINVAL, "patch edges must satisfy 0 < h < Delta (patches may not overlap)");
  if (D.conv != PD_CONV_UPWIND && D.conv != PD_CONV_CENTRAL) return fail(PD_EINVAL, "bad conv");
  if (D.c0mode != PD_C0_TRAPEZOID && D.c0mode != PD_C0_PRINTED) return fail(PD_EINVAL, "bad c0mode");
  if (D.core_points != 0 &&
      (D.core_points < 2 || D.core_points > D.m_xi || D.core_points > D.m_eta ||
       (D.m_xi - D.core_points) % 2 != 0 || (D.m_eta - D.core_points) % 2 != 0))
    return fail(PD_EINVAL, "core_points must be 0 or 2..m with the parity of m_xi and m_eta");
  if (D.precision != PD_F64 && D.precision != PD_F32) return fail(PD_EINVAL, "bad precision");
  const bool box01 = D.xi0 == 0.0 && D.xi1 == 1.0 && D.eta0 == 0.0 && D.eta1 == 1.0;
  switch (D.geometry) {
    case PD_GEOM_IDENTITY: break;
    case PD_GEOM_SINE:
      if (!box01 || !(D.gparam >= 0.0 && D.gparam < 1.0))
        return fail(PD_EINVAL, "sine stretching needs the unit box and 0 <= lambda < 1");
      break;
    case PD_GEOM_TANH:
      if (!box01 || !(D.gparam >= 0.0)) return fail(PD_EINVAL, "tanh stretching needs the unit box and beta >= 0");
      break;
    case PD_GEOM_ANNULUS:
      if (!(D.eta0 > 0.0) || !D.periodic_xi)
        return fail(PD_EINVAL, "the annulus needs eta0 > 0 and a periodic xi axis");
      break;
    default: return fail(PD_EINVAL, "bad geometry");
  }
  if (D.device < 0) return fail(PD_EINVAL, "negative device ordinal");
  if (D.max_sources < 0 || D.max_sources > PD_MAXTERM)
    return fail(PD_EINVAL, "max_sources must be in 0..PD_MAXTERM");

  pd_grid g = new pd_grid_s();
  g->d = D;
  g->max_src = D.max_sources > 0 ? D.max_sources : PD_MAXTERM;
  Geo& G = g->g;
  G.geometry = D.geometry;
  G.gparam = D.gparam;
  G.xi0 = D.xi0; G.xi1 = D.xi1; G.eta0 = D.eta0; G.eta1 = D.eta1;
  G.n_xi = D.n_xi; G.n_eta = D.n_eta; G.periodic = D.periodic_xi ? 1 : 0;
  G.h_xi = D.h_xi; G.h_eta = D.h_eta;
  G.m_xi = D.m_xi; G.m_eta = D.m_eta;
  G.conv = D.conv; G.c0mode = D.c0mode;
  G.Dxi = Dxi;
  G.Deta = Deta;
  G.dxi = D.h_xi / (D.m_xi - 1);
  G.deta = D.h_eta / (D.m_eta - 1);
  // the restriction's core: the central points (the whole patch by default)
  G.nks = D.core_points > 0 ? D.core_points : D.m_xi;
  G.nls = D.core_points > 0 ? D.core_points : D.m_eta;
  G.ks = (D.m_xi - G.nks) / 2;
  G.ls = (D.m_eta - G.nls) / 2;
  // eq. (C_0): C0 = U - kappa U_xixi - kappa U_etaeta with kappa the average of s^2/2 over
  // the core (span hc): hc^2/24, plus delta^2/12 under the trapezoid reading so that the
  // trapezoidal restriction of the lift returns U.
  {
    const double hx = (G.nks - 1) * G.dxi, he = (G.nls - 1) * G.deta;
    G.kap_xi = D.c0mode == PD_C0_PRINTED ? hx * hx / 24.0 : hx * hx / 24.0 + G.dxi * G.dxi / 12.0;
    G.kap_eta = D.c0mode == PD_C0_PRINTED ? he * he / 24.0 : he * he / 24.0 + G.deta * G.deta / 12.0;
  }
  G.npx = D.periodic_xi ? D.n_xi : D.n_xi - 2;
  G.i_first = D.periodic_xi ? 0 : 1;
  G.P = G.npx * (D.n_eta - 2);
  G.M = D.m_xi > D.m_eta ? D.m_xi : D.m_eta;

  // Patch index map: node (i, j) and its 3x3 neighbourhood, wrapped on a periodic axis.
  g->pmap.resize((size_t)G.P * 11);
  for (int p = 0; p < G.P; ++p) {
    const int i = G.i_first + p % G.npx, j = 1 + p / G.npx;
    int32_t* o = &g->pmap[(size_t)p * 11];
    o[0] = i;
    o[1] = j;
    for (int b = -1; b <= 1; ++b)
      for (int a = -1; a <= 1; ++a) {
        int ii = i + a;
        if (D.periodic_xi) ii = (ii + D.n_xi) % D.n_xi;
        o[2 + 3 * (b + 1) + (a + 1)] = (j + b) * D.n_xi + ii;
      }
  }

  // Stencil tables.
  const int mx = D.m_xi, me = D.m_eta;
  g->to = tab_off(mx, me);
  g->tab.assign(g->to.size, 0.0);
  double* T = g->tab.data();
  for (int k = 0; k < mx; ++k) T[g->to.s_xi + k] = micro_off(D.h_xi, mx, k);
  for (int l = 0; l < me; ++l) T[g->to.s_eta + l] = micro_off(D.h_eta, me, l);
  for (int l = 0; l < me; ++l)
    for (int q = 0; q < 3; ++q) T[g->to.L_xe + 3 * l + q] = lagrange_basis(q, micro_off(D.h_eta, me, l), Deta);
  for (int k = 0; k < mx; ++k)
    for (int q = 0; q < 3; ++q) T[g->to.L_ee + 3 * k + q] = lagrange_basis(q, micro_off(D.h_xi, mx, k), Dxi);
  const double rx = D.h_xi / (2.0 * Dxi), re = D.h_eta / (2.0 * Deta);
  const double ew[12] = {-0.5 - rx, 2.0 * rx, 0.5 - rx, -0.5 + rx, -2.0 * rx, 0.5 + rx,
                         -0.5 - re, 2.0 * re, 0.5 - re, -0.5 + re, -2.0 * re, 0.5 + re};
  for (int q = 0; q < 12; ++q) T[g->to.ew + q] = ew[q];
  for (int k = 0; k < mx; ++k)
    T[g->to.c_xi + k] = (k < G.ks || k >= G.ks + G.nks) ? 0.0 : core_w(k, G.ks, G.nks);
  for (int l = 0; l < me; ++l)
    T[g->to.c_eta + l] = (l < G.ls || l >= G.ls + G.nls) ? 0.0 : core_w(l, G.ls, G.nls);
  const double sc[8] = {Dxi, Deta, G.dxi, G.deta, rx, re, G.kap_xi, G.kap_eta};
  for (int q = 0; q < 8; ++q) T[g->to.scal + q] = sc[q];

  // Workspace layout.
  size_t o = 0;
  const size_t npts = (size_t)G.P * mx * me;
  g->off_coef = o; o = align256(o + (5 + g->max_src) * npts * sizeof(double));
  g->off_pmap = o; o = align256(o + g->pmap.size() * sizeof(int32_t));
  g->off_tab = o; o = align256(o + g->tab.size() * sizeof(double));
  g->off_desc = o; o = align256(o + sizeof(pd_coeff_desc));
  g->off_V = o; o = align256(o + (size_t)D.n_xi * D.n_eta * sizeof(double));
  g->off_flag = o; o = align256(o + 16);
  g->off_clock = o; o = align256(o + sizeof(Clock));
  g->off_part = o; o = align256(o + 2 * NB_LIM * sizeof(double));
  g->off_lim = o; o = align256(o + 2 * sizeof(double));
  g->off_ttab = o; o = align256(o + TT_CAP * sizeof(double));
  g->off_bval = o; o = align256(o + (size_t)MAX_REPLAY * boundary_count(G) * sizeof(double));
  g->off_cst = o; o = align256(o + (size_t)G.P * CL_NST * sizeof(double));
  g->off_pflag = o; o = align256(o + (size_t)G.P * sizeof(long long));
  g->need = o;
  choose_shape(g);
  *out = g;
  return PD_OK;
}

pd_status pd_destroy_grid(pd_grid g) {
  if (!g) return PD_OK;
  (void)hipSetDevice(g->d.device);
  drop_graph(g);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  if (g->ev_in) (void)hipEventDestroy(g->ev_in);
  if (g->ev_out) (void)hipEventDestroy(g->ev_out);
  delete g;
  return PD_OK;
}

pd_status pd_query(pd_grid g, pd_info* out) {
  if (!g || !out) return fail(PD_EINVAL, "null argument");
  pd_info& I = *out;
  I = pd_info{};
  I.n_patches = g->g.P;
  I.m_xi = g->g.m_xi;
  I.m_eta = g->g.m_eta;
  I.n_xi = g->g.n_xi;
  I.n_eta = g->g.n_eta;
  I.n_points = (int64_t)g->g.P * g->g.m_xi * g->g.m_eta;
  I.workspace_bytes = g->need;
  I.dt_micro_limit = g->lim_micro;
  I.dt_macro_limit = g->lim_macro;
  I.coefficients_set = g->coeffs_set ? 1 : 0;
  I.n_time_sources = g->src.ns;
  I.rows_per_lane = g->R;
  I.cols_per_lane = g->C;
  I.exchange = g->xch;
  I.patches_per_block = g->ppb;
  I.block_threads = g->threads;
  out->tuned = g->tuned;
  out->tuned_ms = g->tuned_ms;
  out->resident_solve = g->last_resident;
  out->resident_refresh = g->last_refresh_resident;
  return PD_OK;
}

pd_status pd_bind_workspace(pd_grid g, void* dev, size_t bytes) {
  if (!g || !dev) return fail(PD_EINVAL, "null argument");
  if (bytes < g->need) return fail(PD_ENOMEM, "workspace smaller than pd_info.workspace_bytes");
  if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(PD_EINVAL, "workspace must be 256-byte aligned");
  HIPCHK(hipSetDevice(g->d.device));
  drop_graph(g);
  g->ws = static_cast<char*>(dev);
  g->ws_bytes = bytes;
  g->coeffs_set = false;
  HIPCHK(hipMemcpy(g->dpmap(), g->pmap.data(), g->pmap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(g->dtab(), g->tab.data(), g->tab.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(g->flag(), 0, 16));
  return PD_OK;
}

pd_status pd_set_coefficients(pd_grid g, const pd_coeff_desc* c, void* stream) {
  pd_status st = need_ws(g);
  if (st) return st;
  if (!c) return fail(PD_EINVAL, "null coefficient descriptor");
  const bool ann = g->d.geometry == PD_GEOM_ANNULUS;
  if ((st = check_field(c->D11, ann, "D11")) || (st = check_field(c->D22, ann, "D22")) ||
      (st = check_field(c->v1, ann, "v1")) || (st = check_field(c->v2, ann, "v2")) ||
      (st = check_field(c->f, ann, "f")))
    return st;
  if (ann && std::memcmp(&c->D11, &c->D22, sizeof(pd_field)) != 0)
    return fail(PD_EINVAL, "the annulus takes a scalar diffusion coefficient (D11 == D22)");
  if (c->n_src > g->max_src)
    return fail(PD_EINVAL, "more source terms than the grid was created for (max_sources)");
  if (c->n_bc < 0 || c->n_bc > PD_MAXTERM || c->n_src < 0 || c->n_src > PD_MAXTERM)
    return fail(PD_EINVAL, "term count out of range");
  SrcInfo si{};
  for (int q = 0; q < c->n_bc; ++q)
    if ((st = check_tfun(c->bc_t[q])) || (st = check_sfun(c->bc_s[q], ann))) return st;
  for (int k = 0; k < c->n_src; ++k) {
    if ((st = check_tfun(c->src_t[k])) || (st = check_sfun(c->src_s[k], ann))) return st;
    if (c->src_t[k].type == PD_T_CONST) {
      si.plane_c[si.nconst] = 5 + k;
      si.ca[si.nconst] = c->src_t[k].a;
      si.nconst++;
    } else {
      if (si.ns == 2) return fail(PD_EINVAL, "at most 2 time-dependent source terms");
      si.plane_t[si.ns] = 5 + k;
      si.ttype[si.ns] = c->src_t[k].type;
      si.ta[si.ns] = c->src_t[k].a;
      si.tb[si.ns] = c->src_t[k].b;
      si.tc[si.ns] = c->src_t[k].c;
      si.ns++;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(g->d.device));
  drop_graph(g);
  HIPCHK(hipMemcpyAsync(g->ddesc(), c, sizeof(pd_coeff_desc), hipMemcpyHostToDevice, s));
  HIPCHK(launch_coefficients(g->g, g->ddesc(), c->n_src, g->coef(), s));
  HIPCHK(launch_limits(g->g, g->ddesc(), c->n_src, g->coef(), g->part(), NB_LIM, g->lim(), s));
  double lim[2];
  HIPCHK(hipMemcpyAsync(lim, g->lim(), sizeof lim, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!(lim[0] > 0.0) || !(lim[1] > 0.0))
    return fail(PD_EINVAL, "diffusion must be positive at every micro point and patch node");
  g->cd = *c;
  g->n_src = c->n_src;
  g->src = si;
  g->lim_micro = lim[0];
  g->lim_macro = lim[1];
  g->coeffs_set = true;
  g->tt_ok = false;
  g->cst_ok = false;
  choose_shape(g);
  return PD_OK;
}

pd_status pd_initial(pd_grid g, double* U, double t, void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!U) return fail(PD_EINVAL, "null U");
  HIPCHK(hipSetDevice(g->d.device));
  HIPCHK(launch_initial(g->g, g->ddesc(), U, t, static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_lift_bc(pd_grid g, const double* U, double* state, double* edge, void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!U || !state || !edge) return fail(PD_EINVAL, "null argument");
  HIPCHK(hipSetDevice(g->d.device));
  HIPCHK(launch_lift_bc(g->g, g->dpmap(), g->dtab(), U, state, edge,
                        static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_micro_burst(pd_grid g, double* state, const double* edge, double t_n, double dt,
                         int32_t n_t, void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!state || !edge) return fail(PD_EINVAL, "null argument");
  if ((st = guard_micro(g, dt, n_t))) return st;
  HIPCHK(hipSetDevice(g->d.device));
  BurstArgs a = base_args(g, t_n, dt, n_t);
  a.state = state;
  a.edge = edge;
  HIPCHK(ensure_time_table(g, t_n, dt, n_t, static_cast<hipStream_t>(stream)));
  HIPCHK(launch_burst(g->d.precision, g->R, g->C, g->xch, MODE_SPLIT, a, g->blocks,
                      g->threads, g->lds, static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_micro_burst_adi(pd_grid g, double* state, const double* edge, double t_n,
                             double dt, int32_t n_t, void* stream) {
  pd_status st = need_ws(g);  // no explicit-burst launch shape needed
  if (st) return st;
  if (!g->coeffs_set) return fail(PD_ESTATE, "coefficients not set");
  if (!state || !edge) return fail(PD_EINVAL, "null argument");
  if (!(dt > 0.0) || n_t < 1) return fail(PD_EINVAL, "dt_micro must be > 0 and n_t >= 1");
  {
    int ppb = 0;
    size_t lds = 0;
    adi_shape(g->g.m_xi, g->g.m_eta, ppb, lds);
    if (ppb < 1)
      return fail(PD_EINVAL, "the ADI burst needs 6 m_xi m_eta + 4 max(m_xi, m_eta) <= 8192");
  }
  HIPCHK(hipSetDevice(g->d.device));
  HIPCHK(launch_burst_adi(g->g, g->src, g->coef(), (long long)g->g.P * g->g.m_xi * g->g.m_eta,
                          state, edge, t_n, dt, n_t, g->flag(), static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_micro_burst_adi_upwind(pd_grid g, double* state, const double* edge,
                                    double t_n, double dt, int32_t n_t, int32_t points,
                                    double r, void* stream) {
  pd_status st = need_ws(g);  // no explicit-burst launch shape needed
  if (st) return st;
  if (!g->coeffs_set) return fail(PD_ESTATE, "coefficients not set");
  if (!state || !edge) return fail(PD_EINVAL, "null argument");
  if (!(dt > 0.0) || n_t < 1) return fail(PD_EINVAL, "dt_micro must be > 0 and n_t >= 1");
  if (points < 2 || points > 4) return fail(PD_EINVAL, "points must be 2, 3 or 4");
  if (!std::isfinite(r)) return fail(PD_EINVAL, "r must be finite");
  {
    int ppb = 0;
    size_t lds = 0;
    adu_shape(g->g.m_xi, g->g.m_eta, ppb, lds);
    if (ppb < 1)
      return fail(PD_EINVAL,
                  "the ADI upwind burst needs 5 m_xi m_eta + 4 max(m_xi, m_eta) <= 8192");
  }
  HIPCHK(hipSetDevice(g->d.device));
  HIPCHK(launch_burst_adi_hu(g->g, g->src, g->coef(),
                             (long long)g->g.P * g->g.m_xi * g->g.m_eta, state, edge, t_n, dt,
                             n_t, points, r, g->flag(), static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_micro_burst_upwind(pd_grid g, double* state, const double* edge, double t_n,
                                double dt, int32_t n_t, int32_t points, double r,
                                void* stream) {
  pd_status st = need_ws(g);  // no explicit-burst launch shape needed
  if (st) return st;
  if (!g->coeffs_set) return fail(PD_ESTATE, "coefficients not set");
  if (!state || !edge) return fail(PD_EINVAL, "null argument");
  if (!(dt > 0.0) || n_t < 1) return fail(PD_EINVAL, "dt_micro must be > 0 and n_t >= 1");
  if (points < 2 || points > 4) return fail(PD_EINVAL, "points must be 2, 3 or 4");
  if (!std::isfinite(r)) return fail(PD_EINVAL, "r must be finite");
  {
    int ppb = 0;
    size_t lds = 0;
    hu_shape(g->g.m_xi, g->g.m_eta, ppb, lds);
    if (ppb < 1)
      return fail(PD_EINVAL, "the upwind burst needs 3 <= m_xi, m_eta and m_xi m_eta <= 1024");
  }
  HIPCHK(hipSetDevice(g->d.device));
  HIPCHK(launch_burst_hu(g->g, g->src, g->coef(), (long long)g->g.P * g->g.m_xi * g->g.m_eta,
                         state, edge, t_n, dt, n_t, points, r, g->flag(),
                         g->opt_xch == XCH_LDS, static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_restrict(pd_grid g, const double* state, double* Ubar, void* stream) {
  pd_status st = need_ws(g);
  if (st) return st;
  if (!state || !Ubar) return fail(PD_EINVAL, "null argument");
  HIPCHK(hipSetDevice(g->d.device));
  HIPCHK(launch_restrict(g->g, state, Ubar, static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_macro_step(pd_grid g, const double* U_n, double* U_np1, double t_n,
                        double dt_macro, double dt, int32_t n_t, const double* Ubar,
                        void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!U_n || !U_np1 || U_n == U_np1) return fail(PD_EINVAL, "U_n, U_np1 must be distinct non-null buffers");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(g->d.device));
  const double tau = n_t * dt;
  if (Ubar) {
    if (!(dt_macro > 0.0) || !(tau > 0.0)) return fail(PD_EINVAL, "dt_macro and tau must be > 0");
    HIPCHK(launch_macro_update(g->g, g->dpmap(), U_n, Ubar, U_np1, dt_macro, tau, g->flag(), s));
  } else {
    if ((st = guard_macro(g, dt_macro, dt, n_t))) return st;
    BurstArgs a = base_args(g, t_n, dt, n_t);
    a.U = U_n;
    a.Unew = U_np1;
    a.dt_macro = dt_macro;
    a.tau = tau;
    HIPCHK(ensure_time_table(g, t_n, dt, n_t, s));
    HIPCHK(launch_burst(g->d.precision, g->R, g->C, g->xch, MODE_FUSED, a, g->blocks, g->threads, g->lds, s));
  }
  HIPCHK(launch_boundary(g->g, g->ddesc(), U_np1, t_n + dt_macro, s));
  return PD_OK;
}

pd_status pd_patch_step(pd_grid g, const double* U_n, double* U_np1, double t_n,
                        double dt_macro, double dt, int32_t n_t, void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!U_n || !U_np1 || U_n == U_np1) return fail(PD_EINVAL, "U_n, U_np1 must be distinct non-null buffers");
  if ((st = guard_macro(g, dt_macro, dt, n_t))) return st;
  HIPCHK(hipSetDevice(g->d.device));
  BurstArgs a = base_args(g, t_n, dt, n_t);
  a.U = U_n;
  a.Unew = U_np1;
  a.dt_macro = dt_macro;
  a.tau = n_t * dt;
  HIPCHK(ensure_time_table(g, t_n, dt, n_t, static_cast<hipStream_t>(stream)));
  HIPCHK(launch_burst(g->d.precision, g->R, g->C, g->xch, MODE_FUSED, a, g->blocks, g->threads, g->lds,
                      static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_macro_step_refresh(pd_grid g, const double* U_n, double* U_np1, double t_n,
                                double dt_macro, double dt, int32_t n_t, int32_t n_refresh,
                                double* state, double* edge, double* Ubar, double* U_work,
                                void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!U_n || !U_np1 || U_n == U_np1) return fail(PD_EINVAL, "U_n, U_np1 must be distinct non-null buffers");
  if (!state || !edge || !Ubar || !U_work) return fail(PD_EINVAL, "null work buffer");
  if (U_work == U_n || U_work == U_np1) return fail(PD_EINVAL, "U_work must be its own buffer");
  if (n_refresh < 1 || n_refresh > n_t) return fail(PD_EINVAL, "need 1 <= n_refresh <= n_t");
  if ((st = guard_macro(g, dt_macro, dt, n_t))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(hipSetDevice(g->d.device));
  if (n_refresh > 1 && g->opt_resident && g->xch == XCH_LANES && g->d.precision == PD_F64 &&
      g->threads == 64 && 9 * g->ppb <= 64 && g->src.ns <= 1 && n_refresh <= MAX_REPLAY) {
    // every wave resident for the whole step: the sub-bursts in registers, the refreshed
    // fields exchanged through U_work and the workspace's second macro buffer
    HIPCHK(ensure_time_table(g, t_n, dt, n_t, s));
    HIPCHK(launch_refresh_setup(g->g, g->ddesc(), t_n, dt, n_t, n_refresh, t_n + dt_macro,
                                g->bvals(), g->pflags(), g->blocks, s));
    BurstArgs a = base_args(g, t_n, dt, n_t);
    a.U = U_n;
    a.Unew = U_np1;
    a.dt_macro = dt_macro;
    a.tau = n_t * dt;
    a.nb = boundary_count(g->g);  // row length of the Dirichlet table
    int resident = 0;
    HIPCHK(launch_refresh_x_f64(
        g->R, g->C, a, g->pflags(), g->flag() + 1, n_refresh, U_work, g->V(), g->bvals(),
        g->blocks, g->lds + refresh_x_extra_lds(g->ppb, g->g.m_xi, g->g.m_eta, g->src.nconst),
        s, &resident));
    g->last_refresh_resident = resident;
    if (resident) return PD_OK;
  }
  g->last_refresh_resident = 0;
  HIPCHK(launch_lift_bc(g->g, g->dpmap(), g->dtab(), U_n, state, edge, s));
  // the time factors of every sub-burst in one launch (the sub-burst tables tile the
  // n_t-step table's space, so the single-burst table cached on the grid is gone)
  g->tt_ok = false;
  HIPCHK(launch_refresh_tables(g->src, t_n, dt, n_t, n_refresh, g->ttab(), s));
  for (int q = 0; q < n_refresh; ++q) {
    const int s0 = (int)((long long)n_t * q / n_refresh);
    const int s1 = (int)((long long)n_t * (q + 1) / n_refresh);
    BurstArgs a = base_args(g, t_n + s0 * dt, dt, s1 - s0);
    a.state = state;
    a.edge = edge;
    a.ttab = g->ttab() + (size_t)g->src.ns * s0;
    HIPCHK(launch_burst(g->d.precision, g->R, g->C, g->xch, MODE_SPLIT, a, g->blocks,
                        g->threads, g->lds, s));
    if (q + 1 < n_refresh) {
      // the macro field at the sub-burst's end (patch averages at the patch nodes,
      // Dirichlet data on the boundary nodes), then eq. (edge) gradients from it
      HIPCHK(launch_refresh_field(g->g, g->dpmap(), g->ddesc(), state, Ubar, U_work,
                                  t_n + s1 * dt, s));
      HIPCHK(launch_lift_bc(g->g, g->dpmap(), g->dtab(), U_work, nullptr, edge, s));
    }
  }
  HIPCHK(launch_refresh_final(g->g, g->dpmap(), g->ddesc(), state, Ubar, U_n, U_np1, dt_macro,
                              n_t * dt, g->flag(), t_n + dt_macro, s));
  return PD_OK;
}

pd_status pd_apply_boundary(pd_grid g, double* U, double t, void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!U) return fail(PD_EINVAL, "null U");
  HIPCHK(hipSetDevice(g->d.device));
  HIPCHK(launch_boundary(g->g, g->ddesc(), U, t, static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_solve(pd_grid g, double* U, double t0, double dt_macro, int32_t n_steps,
                   double dt, int32_t n_t, void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!U || n_steps < 0) return fail(PD_EINVAL, "null U or negative step count");
  if (n_steps == 0) return PD_OK;
  if ((st = guard_macro(g, dt_macro, dt, n_t))) return st;
  HIPCHK(hipSetDevice(g->d.device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool own = s == nullptr;  // the null stream cannot be captured
  if (own && !g->cap) {
    HIPCHK(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming));
  }
  hipStream_t w = own ? g->cap : s;
  const double tau = n_t * dt;
  BurstArgs a = base_args(g, t0, dt, n_t);
  a.dt_macro = dt_macro;
  a.tau = tau;
  a.clk = g->clock();
  // Macro steps per graph replay: one k_replay node (clock, time factors and Dirichlet
  // values of all S steps), then one fused burst per step.
  const size_t per = (size_t)g->src.ns * n_t;
  // Graph replays are always S steps long; a shorter request, or the remainder of a
  // longer one, runs as direct launches, so short runs (warm-ups) never rebuild the graph.
  int S = MAX_REPLAY;
  while (S > 1 && S * per > TT_CAP) --S;
  const int reps = n_steps / S, rem = n_steps - reps * S;
  const int nb = boundary_count(g->g);
  a.nb = nb;
  // resident solve: in-wave FP64 steps, every wave's neighbour list within one wave
  const bool res = g->opt_resident && g->xch == XCH_LANES && g->d.precision == PD_F64 &&
                   g->threads == 64 && 9 * g->ppb <= 64;
  const bool reuse = g->gexec && g->g_steps == S && g->g_dtm == dt_macro && g->g_dt == dt &&
                     g->g_nt == n_t && g->g_U == U && g->g_R == g->R && g->g_C == g->C &&
                     g->g_ppb == g->ppb && g->g_threads == g->threads && g->g_xch == g->xch &&
                     g->g_res == (int)res;
  if (own) {
    HIPCHK(hipEventRecord(g->ev_in, s));
    HIPCHK(hipStreamWaitEvent(w, g->ev_in, 0));
  }
  g->tt_ok = false;  // k_replay rewrites the time-factor table
  HIPCHK(launch_clock_init(g->clock(), t0, dt_macro, U, g->V(), w));
  if (res) HIPCHK(launch_zero_flags(g->pflags(), g->blocks, w));
  g->last_resident = 0;
  auto steps = [&](int count) -> hipError_t {
    hipError_t e = launch_replay(g->g, g->src, g->ddesc(), g->clock(), count, n_t, dt,
                                 g->ttab(), g->bvals(), w);
    if (res && e == hipSuccess) {
      int resident = 0;
      a.k = 0;
      a.ttab = g->ttab();
      a.bvals = nullptr;  // written by the owning waves step by step
      e = launch_solve_x_f64(g->R, g->C, a, g->pflags(), g->flag() + 1, count, g->ttab(),
                             g->bvals(), (int)per, g->blocks,
                             g->lds + solve_x_extra_lds(g->ppb, g->g.m_xi, g->g.m_eta, g->src.nconst), w,
                             &resident);
      g->last_resident = resident;
      if (e != hipSuccess || resident) return e;
    }
    for (int k = 0; k < count && e == hipSuccess; ++k) {
      a.k = k;
      a.ttab = g->ttab() + k * per;
      a.bvals = g->bvals() + (size_t)k * nb;
      e = launch_burst(g->d.precision, g->R, g->C, g->xch, MODE_FUSED, a, g->blocks,
                       g->threads, g->lds, w);
    }
    return e;
  };
  if (reps > 0 && !reuse) {
    drop_graph(g);
    HIPCHK(hipStreamBeginCapture(w, hipStreamCaptureModeThreadLocal));
    const hipError_t e = steps(S);
    if (e != hipSuccess) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(w, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      return hip_fail(e, "graph capture");
    }
    HIPCHK(hipStreamEndCapture(w, &g->graph));
    HIPCHK(hipGraphInstantiate(&g->gexec, g->graph, nullptr, nullptr, 0));
    g->g_steps = S;
    g->g_dtm = dt_macro;
    g->g_dt = dt;
    g->g_nt = n_t;
    g->g_U = U;
    g->g_R = g->R;
    g->g_C = g->C;
    g->g_ppb = g->ppb;
    g->g_threads = g->threads;
    g->g_xch = g->xch;
    g->g_res = (int)res;
    g->g_res_ran = g->last_resident;
  }
  if (reps > 0) g->last_resident = g->g_res_ran;
  for (int r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(g->gexec, w));
  if (rem) HIPCHK(steps(rem));
  if (n_steps & 1)
    HIPCHK(hipMemcpyAsync(U, g->V(), (size_t)g->g.n_xi * g->g.n_eta * sizeof(double),
                          hipMemcpyDeviceToDevice, w));
  if (own) {
    HIPCHK(hipEventRecord(g->ev_out, w));
    HIPCHK(hipStreamWaitEvent(s, g->ev_out, 0));
  }
  return PD_OK;
}

pd_status pd_autotune(pd_grid g, const double* U, double t_n, double dt_macro, double dt,
                      int32_t n_t, int32_t reps, uint32_t flags, double* best_ms,
                      void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!U) return fail(PD_EINVAL, "null U");
  if ((st = guard_macro(g, dt_macro, dt, n_t))) return st;
  if (reps < 1) reps = 5;
  HIPCHK(hipSetDevice(g->d.device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const TuneKey key{g->g.P, g->g.m_xi, g->g.m_eta, g->d.precision, g->src.ns, n_t,
                    g->g.conv, g->opt_xch, g->opt_C, g->opt_R, g->opt_ppb, g->opt_threads};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end() && !(flags & PD_TUNE_FORCE)) {
      apply_shape(g, it->second.first);
      g->tuned = 1;
      g->tuned_ms = it->second.second;
      if (best_ms) *best_ms = g->tuned_ms;
      return PD_OK;
    }
  }
  std::vector<Shape> cand;
  if (!next_shape(g, g->opt_xch, cand)) return fail(PD_EINVAL, "no launch shape to tune");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto cleanup = [&]() {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  };
  const Shape keep{g->R, g->C, g->xch, g->ppb, g->threads, 0.0};
  double best = 1e300;
  Shape bs = keep;
  hipError_t e = ensure_time_table(g, t_n, dt, n_t, s);
  for (size_t q = 0; q < cand.size() && e == hipSuccess; ++q) {
    apply_shape(g, cand[q]);
    BurstArgs a = base_args(g, t_n, dt, n_t);
    a.U = U;
    a.Unew = g->V();
    a.dt_macro = dt_macro;
    a.tau = n_t * dt;
    auto launch = [&]() {
      return launch_burst(g->d.precision, g->R, g->C, g->xch, MODE_FUSED, a, g->blocks,
                          g->threads, g->lds, s);
    };
    if ((e = launch()) != hipSuccess) break;  // warm-up (code load, caches)
    // best of three trials of `reps` launches each (the first also sizes later trials)
    double best_trial = 1e300;
    int n = reps;
    for (int trial = 0; trial < 3 && e == hipSuccess; ++trial) {
      if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
      for (int r = 0; r < n && e == hipSuccess; ++r) e = launch();
      if (e != hipSuccess || (e = hipEventRecord(e1, s)) != hipSuccess) break;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
      float f = 0.f;
      if ((e = hipEventElapsedTime(&f, e0, e1)) != hipSuccess) break;
      const double per_launch = (double)f / n;
      if (per_launch < best_trial) best_trial = per_launch;
      if (trial == 0 && per_launch * n < 0.5) {  // trials of at least ~0.5 ms
        const int want = (int)(0.5 / (per_launch > 1e-6 ? per_launch : 1e-6)) + 1;
        n = want > 64 ? 64 : want;
      }
    }
    if (e != hipSuccess) break;
    float ms = (float)best_trial;
    const double per = (double)ms;
    if (per < best) {
      best = per;
      bs = cand[q];
    }
  }
  cleanup();
  apply_shape(g, e == hipSuccess ? bs : keep);
  if (e != hipSuccess) return hip_fail(e, "pd_autotune");
  g->tuned = 1;
  g->tuned_ms = best;
  if (best_ms) *best_ms = best;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {bs, best};
  }
  int flag = 0;
  HIPCHK(hipMemcpy(&flag, g->flag(), sizeof(int), hipMemcpyDeviceToHost));
  if (flag) {
    HIPCHK(hipMemset(g->flag(), 0, sizeof(int)));
    return fail(PD_ENONFINITE, "a timed step produced a non-finite value");
  }
  return PD_OK;
}

pd_status pd_sync(pd_grid g, void* stream) {
  pd_status st = need_ws(g);
  if (st) return st;
  HIPCHK(hipSetDevice(g->d.device));
  HIPCHK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  int flag[2] = {0, 0};
  HIPCHK(hipMemcpy(flag, g->flag(), 2 * sizeof(int), hipMemcpyDeviceToHost));
  if (flag[1]) {
    HIPCHK(hipMemset(g->flag(), 0, 2 * sizeof(int)));
    return fail(PD_EDEVICE, "a resident solve's wait for neighbouring waves gave up");
  }
  if (flag[0]) {
    HIPCHK(hipMemset(g->flag(), 0, sizeof(int)));
    return fail(PD_ENONFINITE, "a kernel produced a non-finite value");
  }
  return PD_OK;
}

pd_status pd_get_patch_map(pd_grid g, int32_t* out) {
  if (!g || !out) return fail(PD_EINVAL, "null argument");
  std::memcpy(out, g->pmap.data(), g->pmap.size() * sizeof(int32_t));
  return PD_OK;
}

int32_t pd_get_tables_size(pd_grid g) { return g ? g->to.size : 0; }

pd_status pd_get_tables(pd_grid g, double* out) {
  if (!g || !out) return fail(PD_EINVAL, "null argument");
  std::memcpy(out, g->tab.data(), g->tab.size() * sizeof(double));
  return PD_OK;
}

pd_status pd_copy_coefficients(pd_grid g, double* dev_out, void* stream) {
  pd_status st = need_coeffs(g);
  if (st) return st;
  if (!dev_out) return fail(PD_EINVAL, "null argument");
  HIPCHK(hipSetDevice(g->d.device));
  const size_t n = (size_t)(5 + g->n_src) * g->g.P * g->g.m_xi * g->g.m_eta;
  HIPCHK(hipMemcpyAsync(dev_out, g->coef(), n * sizeof(double), hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  return PD_OK;
}

pd_status pd_set_option(pd_grid g, int32_t option, int64_t value) {
  if (!g) return fail(PD_EINVAL, "null grid");
  switch (option) {
    case PD_OPT_ALLOW_UNSTABLE: g->allow_unstable = value ? 1 : 0; return PD_OK;
    case PD_OPT_RESIDENT_SOLVE: g->opt_resident = value ? 1 : 0; return PD_OK;
    case PD_OPT_ROWS_PER_LANE:
      if (value < 0 || value > 11) return fail(PD_EINVAL, "unsupported rows per lane");
      g->opt_R = (int)value;
      break;
    case PD_OPT_COLS_PER_LANE:
      if (value < 0 || value > 4) return fail(PD_EINVAL, "columns per lane must be 1 to 4");
      g->opt_C = (int)value;
      break;
    case PD_OPT_EXCHANGE:
      if (value < 0 || value > 3)
        return fail(PD_EINVAL, "exchange must be 0, 1 (LDS), 2 (in-wave) or 3 (hybrid)");
      g->opt_xch = (int)value;
      break;
    case PD_OPT_PATCHES_PER_BLOCK:
      if (value < 0 || value > 256) return fail(PD_EINVAL, "patches per block out of range");
      g->opt_ppb = (int)value;
      break;
    case PD_OPT_BLOCK_THREADS:
      if (value != 0 && (value < 64 || value > 256 || value % 64))
        return fail(PD_EINVAL, "block threads must be 64, 128, 192 or 256");
      g->opt_threads = (int)value;
      break;
    default: return fail(PD_EINVAL, "unknown option");
  }
  g->tuned = 0;
  g->tuned_ms = 0.0;
  choose_shape(g);
  if (!g->R) {
    g->opt_R = 0;
    g->opt_C = 0;
    g->opt_ppb = 0;
    g->opt_threads = 0;
    g->opt_xch = 0;
    choose_shape(g);
    return fail(PD_EINVAL, "no launch shape with these options; reverted to automatic");
  }
  return PD_OK;
}

}  // extern "C"

#include "pd_batch_host.inc"
#include "pd_closure_host.inc"
#include "pd_fd_host.inc"
