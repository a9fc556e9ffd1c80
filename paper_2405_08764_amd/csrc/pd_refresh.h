// The stage kernels of a macro step with the edge data refreshed between sub-bursts
// (Sec. 3.3, steps (ii)-(vi) with step (ii) repeated inside the burst), and the pieces of
// arithmetic they share with the one-stage-per-kernel path (k_restrict, k_macro_update):
// both use these helpers, so the fused and the separate forms agree bit for bit.
#pragma once

#include "pd_internal.h"

namespace pdk {

// Step (iv), first half: the trapezoid sum of row l of patch p over the restriction core
// (index order).  Only rows l in [ls, ls + nls) take part.
__device__ inline double restriction_row(const Geo& g, const double* state, int p, int l) {
  const double* u = state + ((long long)p * g.m_eta + l) * g.m_xi;
  double row = 0.0;
  for (int k = g.ks; k < g.ks + g.nks; ++k) row += core_w(k, g.ks, g.nks) * u[k];
  return row;
}

// Step (iv), second half: the trapezoid sum of the row sums (index order), divided by the
// core's cell count: the patch average of eq. (Restriction).
__device__ inline double restriction_total(const Geo& g, const double* rows) {
  double tot = 0.0;
  for (int l = g.ls; l < g.ls + g.nls; ++l) tot += core_w(l, g.ls, g.nls) * rows[l];
  return tot / ((double)(g.nks - 1) * (double)(g.nls - 1));
}

// Steps (v)-(vi) at one patch node: the time-derivative estimate over the burst and the
// projective step of eq. (Macro_Update).
__device__ inline double projective_value(double Un, double Ubar, double dt_macro,
                                          double tau) {
  const double F = (Ubar - Un) / tau;
  return Un + dt_macro * F;
}

// Time factors of all Q sub-bursts of a refreshed macro step in one launch.  Sub-burst q
// takes nano steps s0 .. s1 - 1 (s0 = floor(n_t q / Q), s1 = floor(n_t (q + 1) / Q)); its
// table [ns][s1 - s0] starts at out + ns s0 and holds T_j(t_q + s dt) with
// t_q = t_n + s0 dt, which is what one burst from t_q would read.
hipError_t launch_refresh_tables(const SrcInfo& src, double t_n, double dt, int n_t, int Q,
                                 double* out, hipStream_t s);
// Set-up of the resident refreshed step: Dirichlet values at the ends of sub-bursts
// 0 .. Q - 2 (out[q][nb] at t_n + s1 dt) and at t_end (row Q - 1), flags[0 .. nflags) = 0.
hipError_t launch_refresh_setup(const Geo& g, const pd_coeff_desc* dev_desc, double t_n,
                                double dt, int n_t, int Q, double t_end, double* out,
                                long long* flags, int nflags, hipStream_t s);
// The macro field between two sub-bursts: every patch restricted (Ubar[p]), U at the
// patch nodes set to those averages, U at the Dirichlet nodes set to u_b(t).
hipError_t launch_refresh_field(const Geo& g, const int* pmap, const pd_coeff_desc* dev_desc,
                                const double* state, double* Ubar, double* U, double t,
                                hipStream_t s);
// The end of a refreshed macro step: restriction (Ubar), projective step from U_n at the
// patch nodes of U_np1 (flag set on a non-finite value), u_b(t) at its Dirichlet nodes.
hipError_t launch_refresh_final(const Geo& g, const int* pmap, const pd_coeff_desc* dev_desc,
                                const double* state, double* Ubar, const double* U_n,
                                double* U_np1, double dt_macro, double tau, int* flag,
                                double t, hipStream_t s);

}  // namespace pdk
