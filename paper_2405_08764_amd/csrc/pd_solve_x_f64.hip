// Resident fused solve with the in-wave exchange (FP64): the waves of one launch carry out
// S macro steps (Sec. 3.3 steps (i)-(vi), repeated), keeping the folded stencil weights of
// their patches in registers from the first step on.  Between steps no grid-wide barrier
// is needed: a patch's next burst reads only the 3 x 3 macro nodes around it, so a wave
// waits for the waves that wrote those nodes (and the Dirichlet values among them), each
// of which publishes a per-wave flag, the number of the last macro step it finished.  The
// wait is bounded: a wave that sees no progress for about half a second sets an error flag
// (pd_sync reports it) and carries on, so the launch always ends.  The launch requires
// every wave to be resident at once (the host checks it with the occupancy API).
//
// The exchanged values (each wave's patch nodes and the Dirichlet nodes it owns) and the
// flags go through device-scope loads and stores, so that waves on different XCDs see each
// other's writes without flushing or invalidating whole caches.
//
// Later steps skip the coefficient loads and the weight formation; they form the edge
// data, the lifted tile, R(w0) and the forcing K0 again from the new macro field, with the
// same arithmetic as the first step (the reaction and constant-source parts reloaded, the
// ghost-point factors of the edge points kept in LDS), so the results are bitwise those of
// one fused launch per step.
#include "pd_internal.h"
#include "pd_burst.inc"

namespace pdk {
namespace {

// Polls of the neighbours' flags (each after a short sleep) before giving up.
constexpr int SOLVE_SPIN = 1 << 19;

struct SolveArgs {
  long long* flags;     // per block: macro steps finished (zeroed at the start of a solve)
  int* err;             // set when a wait gave up
  int steps;            // macro steps of this launch
  const double* ttab0;  // time factors of step 0 ([ns][n_t] per step)
  const double* bval0;  // Dirichlet values of step 0 (nb per step)
  int per;              // ns * n_t
};

// Patch whose wave writes node (i, j): the patch at that node, or for a Dirichlet node the
// patch at the nearest interior node (it lies within the 3 x 3 neighbourhood of every
// patch that reads the node).
__device__ inline int owner_patch(const Geo& g, int i, int j) {
  const int jj = j < 1 ? 1 : (j > g.n_eta - 2 ? g.n_eta - 2 : j);
  int ii = i;
  if (!g.periodic) ii = i < 1 ? 1 : (i > g.n_xi - 2 ? g.n_xi - 2 : i);
  return (jj - 1) * g.npx + (ii - g.i_first);
}

__device__ inline bool is_boundary(const Geo& g, int i, int j) {
  return j == 0 || j == g.n_eta - 1 || (!g.periodic && (i == 0 || i == g.n_xi - 1));
}

// Index of Dirichlet node (i, j) in the boundary order of boundary_node.
__device__ inline int boundary_index(const Geo& g, int i, int j) {
  if (j == 0) return i;
  if (j == g.n_eta - 1) return g.n_xi + i;
  return 2 * g.n_xi + 2 * (j - 1) + (i == g.n_xi - 1 ? 1 : 0);
}

// Lanes 0 .. 9 ppb - 1 of a block: neighbour node (lane % 9) of patch slot lane / 9, the
// block of the wave that writes it (-1: this block, or no such patch), and whether this
// block writes it as a Dirichlet node (its node and boundary index).
struct Neighbours {
  int block, bnode, bq;
};

__device__ inline Neighbours neighbours(const BurstArgs& A) {
  const Geo& G = A.g;
  const int lane = threadIdx.x;
  const long long pb = (long long)blockIdx.x * A.ppb + lane / 9;
  Neighbours n{-1, -1, 0};
  if (lane < 9 * A.ppb && pb < G.P) {
    const int nd = A.pmap[11 * pb + 2 + lane % 9];
    const int i = nd % G.n_xi, j = nd / G.n_xi;
    const int ow = owner_patch(G, i, j);
    const int ob = ow / A.ppb;
    n.block = ob == (int)blockIdx.x ? -1 : ob;
    if (is_boundary(G, i, j) && ow == pb) {
      n.bnode = nd;
      n.bq = boundary_index(G, i, j);
    }
  }
  return n;
}

// Bounded wait until every neighbouring block's flag has reached `target` (polls after a
// short sleep); gives up with the error flag set after SOLVE_SPIN polls.
__device__ inline void wait_for_neighbours(const long long* flags, int nb_block,
                                           long long target, int* err) {
  int spins = 0;
  for (;;) {
    const bool ok =
        nb_block < 0 ||
        __hip_atomic_load(flags + nb_block, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target;
    if (__all(ok)) break;
    if (++spins > SOLVE_SPIN) {
      if (threadIdx.x == 0) atomicOr(err, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(4);
  }
}

// Per-step constants of the forcing K0 kept in LDS from the first step: the ghost-point
// factors of the patch edges (the pre-fold outer weight times -2 dxi, 2 dxi, -2 deta,
// 2 deta on the west, east, south and north edges), per patch slot [west me][east me]
// [south mx][north mx]; dt phi at every point (pr, per slot [m_eta][m_xi]); with constant
// source terms, their sum at every point (cs).  The same expressions as the prologue's.
template <int R, int C>
__device__ __forceinline__ void save_step_constants(const BurstArgs& A, const LaneMap& L,
                                                    double* gs, double* pr, double* cs) {
  const int mx = L.mx, me = L.me;
  const long long pm = (long long)mx * me, plane = A.plane;
  const double dt = A.dt, dxi = A.g.dxi, deta = A.g.deta;
  const double kx2 = dt / (dxi * dxi), ke2 = dt / (deta * deta);
  const double kx1 = dt / dxi, ke1 = dt / deta;
  const double kxh = dt / (2.0 * dxi), keh = dt / (2.0 * deta);
  const bool upwind = A.g.conv == PD_CONV_UPWIND;
  const bool one_const = A.src.nconst == 1;
  double* g = gs + L.slot * 2 * (mx + me);
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int k = L.k0 + c, l = L.row0 + q;
      if (!L.active || k >= mx || l >= me) continue;
      const long long at = L.p * pm + (long long)l * mx + k;
      const int li = L.slot * (int)pm + l * mx + k;
      pr[li] = dt * A.coef[4 * plane + at];
      if (A.src.nconst > 0) {
        double st = one_const ? A.coef[A.src.plane_c[0] * plane + at] : 0.0;
        for (int cc = 0; A.src.nconst > 1 && cc < A.src.nconst; ++cc)
          st += A.src.ca[cc] * A.coef[A.src.plane_c[cc] * plane + at];
        cs[li] = one_const ? 0.0 + A.src.ca[0] * st : st;
      }
      if (k != 0 && k != mx - 1 && l != 0 && l != me - 1) continue;
      const double al = A.coef[at], ga = A.coef[plane + at], nu = A.coef[2 * plane + at],
                   om = A.coef[3 * plane + at];
      const double ax = al * kx2, ay = ga * ke2;
      double e_, w_, n_, s_;
      if (upwind) {
        e_ = ax + (nu < 0.0 ? -nu * kx1 : 0.0);
        w_ = ax + (nu >= 0.0 ? nu * kx1 : 0.0);
        n_ = ay + (om < 0.0 ? -om * ke1 : 0.0);
        s_ = ay + (om >= 0.0 ? om * ke1 : 0.0);
      } else {
        e_ = ax - nu * kxh;
        w_ = ax + nu * kxh;
        n_ = ay - om * keh;
        s_ = ay + om * keh;
      }
      if (k == 0) {
        g[l] = -2.0 * dxi * w_;
        e_ += w_;
      }
      if (k == mx - 1) g[me + l] = 2.0 * dxi * e_;
      if (l == 0) {
        g[2 * me + k] = -2.0 * deta * s_;
        n_ += s_;
      }
      if (l == me - 1) g[2 * me + mx + k] = 2.0 * deta * n_;
    }
}

// Steps (i)-(ii) of a later macro step: the edge data and the lifted tile from U_n, R(w0),
// the forcing K0 with the weights already in registers, v = 0.  Same arithmetic as the
// first step's prologue.
template <int R, int C, int NS>
__device__ __forceinline__ void step_prologue(const BurstArgs& A, const LaneMap& L,
                                              const LdsMap& M, const double* Uin,
                                              const double* gs, const double* prl,
                                              const double* csl, BlockRegs<double, R, C, NS>& X,
                                              double& cref, double& R0) {
  const int mx = L.mx, me = L.me, TW = M.TW, TS = M.TS;
  const TabOff to = tab_off(mx, me);
  double Dxi = A.g.Dxi, Deta = A.g.Deta, dt = A.dt;
  asm volatile("" : "+s"(Dxi), "+s"(Deta), "+s"(dt));  // not hoisted out of the step loop
  const long long p = L.p;
  const int* pmp = A.pmap + 11 * (L.active ? p : 0);
  // the other waves' values of U_n, read at device scope (not from this XCD's L2)
  auto ld = [&](int node) {
    return __hip_atomic_load(Uin + node, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  const double cr = ld(pmp[6]);
  double d[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) d[b][a] = ld(pmp[2 + 3 * b + a]);
  cref = L.active ? cr : 0.0;
  double* dtile = reinterpret_cast<double*>(M.region);
  for (int q = L.tid; q < M.nreg; q += L.nthr) dtile[q] = 0.0;
  __syncthreads();
  const double* tab = M.tab;
  const double iDxi = 1.0 / Dxi, iDeta = 1.0 / Deta;
  const int ne = 2 * (mx + me);
  double* edg = M.edge + L.slot * ne;
  if (L.active) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) d[b][a] = d[b][a] - cref;
    for (int j = L.rl; j < ne; j += L.LP) {
      const int side = j < 2 * me ? (j < me ? 0 : 1) : (j < 2 * me + mx ? 2 : 3);
      const int at = side < 2 ? j - side * me : j - 2 * me - (side - 2) * mx;
      double P[3];
      if (side < 2) {
        const double* Lq = tab + to.L_xe + 3 * at;
#pragma unroll
        for (int a = 0; a < 3; ++a) P[a] = Lq[0] * d[0][a] + Lq[1] * d[1][a] + Lq[2] * d[2][a];
      } else {
        const double* Lq = tab + to.L_ee + 3 * at;
#pragma unroll
        for (int b = 0; b < 3; ++b) P[b] = Lq[0] * d[b][0] + Lq[1] * d[b][1] + Lq[2] * d[b][2];
      }
      const double* ew = tab + to.ew + 3 * side;
      edg[j] = (ew[0] * P[0] + ew[1] * P[1] + ew[2] * P[2]) * (side < 2 ? iDxi : iDeta);
    }
    const double Ux = (d[1][2] - d[1][0]) / (2.0 * Dxi);
    const double Ue = (d[2][1] - d[0][1]) / (2.0 * Deta);
    const double Uxx = (d[1][2] + d[1][0]) / (Dxi * Dxi);
    const double Uee = (d[2][1] + d[0][1]) / (Deta * Deta);
    const double Uxe = (d[2][2] - d[0][2] - d[2][0] + d[0][0]) / (4.0 * Dxi * Deta);
    const double c0d = -A.g.kap_xi * Uxx - A.g.kap_eta * Uee;
    for (int c = 0; c < C; ++c) {
      const int k = L.k0 + c;
      if (k >= mx) break;
      const double s = tab[to.s_xi + k];
      for (int q = 0; q < R; ++q) {
        const int l = L.row0 + q;
        if (l >= me) break;
        const double t = tab[to.s_eta + l];
        dtile[L.slot * TS + (l + 1) * TW + k + 1] =
            c0d + s * Ux + t * Ue + 0.5 * s * s * Uxx + s * t * Uxe + 0.5 * t * t * Uee;
      }
    }
  }
  __syncthreads();
  const double* dt0 = dtile + L.slot * TS;
  const int ks = A.g.ks, nks = A.g.nks, ls = A.g.ls, nls = A.g.nls;
  if (L.active) {
    for (int l = ls + L.rl; l < ls + nls; l += L.LP) {
      double acc = 0.0;
      for (int kk = ks; kk < ks + nks; ++kk)
        acc += core_w(kk, ks, nks) * dt0[(l + 1) * TW + kk + 1];
      M.rows[L.slot * me + l] = acc;
    }
  }
  const double* g = gs + L.slot * ne;
  const int pm = mx * me;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int l = L.row0 + q;
    __builtin_amdgcn_sched_barrier(0);  // one row's LDS reads in flight at a time
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int k = L.k0 + c;
      const bool in = L.active && k < mx && l < me;
      X.v[c][q] = 0.0;
      X.K[c][q] = 0.0;  // points outside the patch (as in the first step)
      if (in) {
        const int li = L.slot * pm + l * mx + k;
        const double pr = prl[li];
        const double sq = A.src.nconst > 0 ? csl[li] : 0.0;
        double G = 0.0;
        if (k == 0) G += g[l] * edg[l];
        if (k == mx - 1) G += g[me + l] * edg[me + l];
        if (l == 0) G += g[2 * me + k] * edg[2 * me + k];
        if (l == me - 1) G += g[2 * me + mx + k] * edg[2 * me + mx + k];
        const int ci = (l + 1) * TW + k + 1;
        const double w0 = dt0[ci];
        const double Lw0 = X.cE[c][q] * (dt0[ci + 1] - w0) + X.cW[c][q] * (dt0[ci - 1] - w0) +
                           X.cN[c][q] * (dt0[ci + TW] - w0) + X.cS[c][q] * (dt0[ci - TW] - w0);
        X.K[c][q] = Lw0 + pr * (cref + w0) + G + dt * sq;
      }
    }
  }
  __syncthreads();
  R0 = 0.0;
  if (L.active && L.rl == 0) {
    for (int l = ls; l < ls + nls; ++l) R0 += core_w(l, ls, nls) * M.rows[L.slot * me + l];
    R0 = R0 / ((double)(nks - 1) * (double)(nls - 1));
  }
  for (int q = L.tid; q < M.nreg; q += L.nthr) dtile[q] = 0.0;
  __syncthreads();
}

// The nano-step loop of body_x (priority bands included), nt steps from ttab.
template <int R, int C, int NS>
__device__ __forceinline__ void nano_loop(const BurstArgs& A, const LaneMap& L, const LdsMap& M,
                                          BlockRegs<double, R, C, NS>& X, const double* ttab,
                                          int nt) {
  const int lane = L.tid;
  const int aN = ((lane + L.Lb) & 63) << 2;
  const int aS = ((lane - L.Lb) & 63) << 2;
  double Y[C][R];
  int st = 0;
  int band = A.balance ? 0 : 4;
  if (band == 0) __builtin_amdgcn_s_setprio(3);
  for (; st + 1 < nt; st += 2) {
    if (band < 4 && st * 4 >= (band + 1) * nt) {
      band = (st * 4) / nt;
      if (band == 1) __builtin_amdgcn_s_setprio(2);
      else if (band == 2) __builtin_amdgcn_s_setprio(1);
      else __builtin_amdgcn_s_setprio(0);
    }
    nano_step_x<double, R, C, NS>(A, L, M, X, X.v, Y, st, aN, aS, ttab);
    nano_step_x<double, R, C, NS>(A, L, M, X, Y, X.v, st + 1, aN, aS, ttab);
  }
  if (A.balance) __builtin_amdgcn_s_setprio(0);
  if (st < nt) {
    nano_step_x<double, R, C, NS>(A, L, M, X, X.v, Y, st, aN, aS, ttab);
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < R; ++q) X.v[c][q] = Y[c][q];
  }
}

template <int R, int C, int NS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_solve_x(BurstArgs A, SolveArgs S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LaneMap L = lane_map<R, C>(A, threadIdx.x, 64, (long long)blockIdx.x * A.ppb, A.ppb);
  const LdsMap M = lds_map<double, R, C, NS>(A, L, smem, 1);
  // step constants (save_step_constants) after the burst's own LDS
  double* gs = M.edge + A.ppb * 2 * (L.mx + L.me);
  double* prl = gs + A.ppb * 2 * (L.mx + L.me);
  double* csl = prl + A.ppb * L.mx * L.me;
  const int lane = threadIdx.x;
  const Neighbours Nb = neighbours(A);
  const int nb_block = Nb.block, bnode = Nb.bnode, bq = Nb.bq;
  BlockRegs<double, R, C, NS> X;
  double cref = 0.0, R0 = 0.0;
  int node = 0;
  // macro step k: the buffers from the clock, the Dirichlet nodes this block writes, the
  // flag that tells the neighbours U_{n+1} is written
  // The new values go to device scope (write-through, not held in this XCD's L2), and the
  // flag is stored only once they have all completed; readers load the flag and then the
  // values at device scope, so no cache-wide release or acquire is needed.
  auto finish = [&](int k, long long n, double* Uout) {
    burst_epilogue<double, R, C, NS, MODE_FUSED>(A, L, M, reinterpret_cast<double*>(M.region),
                                                 X, cref, node, R0, Uout);
    if (L.active && L.rl == 0)  // the patch node the epilogue just stored
      __hip_atomic_store(Uout + node, Uout[node], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bnode >= 0)
      __hip_atomic_store(Uout + bnode, S.bval0[(size_t)k * A.nb + bq], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);  // every store of the wave has completed
    __syncthreads();
    if (lane == 0)
      __hip_atomic_store(S.flags + blockIdx.x, n + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  {
    const long long n = A.clk->base;
    burst_prologue<double, R, C, NS, MODE_FUSED>(A, L, M, A.clk->buf[n & 1], X, cref, node, R0);
    save_step_constants<R, C>(A, L, gs, prl, csl);
    __syncthreads();
    nano_loop<R, C, NS>(A, L, M, X, S.ttab0, A.n_t);
    finish(0, n, A.clk->buf[(n + 1) & 1]);
  }
  for (int k = 1; k < S.steps; ++k) {
    const long long n = A.clk->base + k;
    // the neighbours have finished macro step n - 1 (U_n written, U_{n-1} read)
    wait_for_neighbours(S.flags, nb_block, n, S.err);
    // the lane's block position passed through an empty asm per step: the compiler would
    // otherwise hoist every address and constant of the step prologue out of the step
    // loop and spill them (the weights already fill the registers)
    LaneMap Lk = L;
    asm volatile("" : "+v"(Lk.k0), "+v"(Lk.row0), "+v"(Lk.slot), "+v"(Lk.rl));
    step_prologue<R, C, NS>(A, Lk, M, A.clk->buf[n & 1], gs, prl, csl, X, cref, R0);
    nano_loop<R, C, NS>(A, L, M, X, S.ttab0 + (size_t)k * S.per, A.n_t);
    finish(k, n, A.clk->buf[(n + 1) & 1]);
  }
}

// ---------------------------------------------------------------------------------------
// Resident refreshed macro step (the edge data refreshed during the burst, Sec. 3.3 step
// (ii) repeated): the waves of one launch run the Q sub-bursts of one macro step with the
// patch states and the weights in registers.  After sub-burst q (q < Q - 1) each wave
// publishes its patches' restrictions (and the Dirichlet values at the sub-burst's end for
// the boundary nodes it owns) into refresh field q & 1 and raises its flag to q + 1; after
// its neighbours have done the same it forms the eq. (edge) data of the refreshed field and
// moves the forcing by the change of the ghost-point terms (the state carries on, the lift
// is not redone).  Two alternating fields suffice: a wave is never more than one sub-burst
// ahead of a neighbour.  The time factors come from the whole burst's table.

struct RefreshArgs {
  long long* flags;   // per block: sub-bursts finished (zeroed before the launch)
  int* err;           // set when a wait gave up
  int Q;              // sub-bursts
  double* Uw0;        // refresh field of even q (macro-field layout)
  double* Uw1;        // refresh field of odd q
  const double* bvq;  // Dirichlet values at the ends of sub-bursts 0 .. Q - 1, [Q][nb]
                      // (the last row at the macro step's end)
};

// R(u) - U of every patch of the block (returned on its lanes with rl == 0): R(w0) plus the
// restriction of the increment, in the order of the burst epilogue.
template <int R, int C, int NS>
__device__ __forceinline__ double state_average(const BurstArgs& A, const LaneMap& L,
                                                const LdsMap& M,
                                                const BlockRegs<double, R, C, NS>& X,
                                                double R0) {
  double* fin = reinterpret_cast<double*>(M.region);
  const int me = L.me, S = M.S, my = M.OFF + L.vl;
  if (L.active) {
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (L.row0 + q < me) {
#pragma unroll
        for (int c = 0; c < C; ++c) fin[(q * C + c) * S + my] = X.v[c][q];
      }
  }
  __syncthreads();
  const int ks = A.g.ks, nks = A.g.nks, ls = A.g.ls, nls = A.g.nls;
  if (L.active) {
    const int base = M.OFF + L.slot * L.LP;
    for (int l = ls + L.rl; l < ls + nls; l += L.LP) {
      const int bl = l / R, ql = l - bl * R;
      double acc = 0.0;
      for (int kk = ks; kk < ks + nks; ++kk) {
        const int lane = base + bl * L.Lb + kk / C;
        acc += core_w(kk, ks, nks) * fin[(ql * C + kk % C) * S + lane];
      }
      M.rows[L.slot * me + l] = acc;
    }
  }
  __syncthreads();
  double tot = 0.0;
  if (L.active && L.rl == 0) {
    for (int l = ls; l < ls + nls; ++l) tot += core_w(l, ls, nls) * M.rows[L.slot * me + l];
    tot = tot / ((double)(nks - 1) * (double)(nls - 1));
  }
  return R0 + tot;
}

// The eq. (edge) data of the refreshed field Uw into en (per slot, the layout of M.edge),
// then each point's forcing moved by its ghost-point factors times the change from eo.
template <int R, int C, int NS>
__device__ __forceinline__ void refresh_edges(const BurstArgs& A, const LaneMap& L,
                                              const LdsMap& M, const double* Uw,
                                              const int* nodes, const double* gs,
                                              const double* eo, double* en,
                                              BlockRegs<double, R, C, NS>& X) {
  const int mx = L.mx, me = L.me, ne = 2 * (mx + me);
  const TabOff to = tab_off(mx, me);
  const double* tab = M.tab;
  double Dxi = A.g.Dxi, Deta = A.g.Deta;
  asm volatile("" : "+s"(Dxi), "+s"(Deta));  // not hoisted out of the sub-burst loop
  const int* nd = nodes + 9 * (L.active ? L.slot : 0);  // the 3 x 3 nodes, centre at 4
  auto ld = [&](int n) {
    return __hip_atomic_load(Uw + n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  double d[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) d[b][a] = ld(nd[3 * b + a]);
  const double c0 = d[1][1];
  const double iDxi = 1.0 / Dxi, iDeta = 1.0 / Deta;
  double* e_new = en + L.slot * ne;
  if (L.active) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) d[b][a] = d[b][a] - c0;
    for (int j = L.rl; j < ne; j += L.LP) {
      const int side = j < 2 * me ? (j < me ? 0 : 1) : (j < 2 * me + mx ? 2 : 3);
      const int at = side < 2 ? j - side * me : j - 2 * me - (side - 2) * mx;
      double P[3];
      if (side < 2) {
        const double* Lq = tab + to.L_xe + 3 * at;
#pragma unroll
        for (int a = 0; a < 3; ++a) P[a] = Lq[0] * d[0][a] + Lq[1] * d[1][a] + Lq[2] * d[2][a];
      } else {
        const double* Lq = tab + to.L_ee + 3 * at;
#pragma unroll
        for (int b = 0; b < 3; ++b) P[b] = Lq[0] * d[b][0] + Lq[1] * d[b][1] + Lq[2] * d[b][2];
      }
      const double* ew = tab + to.ew + 3 * side;
      e_new[j] = (ew[0] * P[0] + ew[1] * P[1] + ew[2] * P[2]) * (side < 2 ? iDxi : iDeta);
    }
  }
  __syncthreads();
  const double* e_old = eo + L.slot * ne;
  const double* g = gs + L.slot * ne;
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int k = L.k0 + c, l = L.row0 + q;
      if (!L.active || k >= mx || l >= me) continue;
      double dG = 0.0;
      if (k == 0) dG += g[l] * (e_new[l] - e_old[l]);
      if (k == mx - 1) dG += g[me + l] * (e_new[me + l] - e_old[me + l]);
      if (l == 0) dG += g[2 * me + k] * (e_new[2 * me + k] - e_old[2 * me + k]);
      if (l == me - 1) dG += g[2 * me + mx + k] * (e_new[2 * me + mx + k] - e_old[2 * me + mx + k]);
      X.K[c][q] += dG;
    }
}

template <int R, int C, int NS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_refresh_x(
    BurstArgs A, RefreshArgs F) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LaneMap L = lane_map<R, C>(A, threadIdx.x, 64, (long long)blockIdx.x * A.ppb, A.ppb);
  const LdsMap M = lds_map<double, R, C, NS>(A, L, smem, 1);
  const int ne = 2 * (L.mx + L.me);
  double* gs = M.edge + A.ppb * ne;  // ghost-point factors, then the other step constants
  double* prl = gs + A.ppb * ne;
  double* csl = prl + A.ppb * L.mx * L.me;
  double* eg2 = csl + (A.src.nconst > 0 ? A.ppb * L.mx * L.me : 0);  // second edge-data set
  int* nodes = reinterpret_cast<int*>(eg2 + A.ppb * ne);  // each slot's 3 x 3 macro nodes
  const Neighbours Nb = neighbours(A);
  if (threadIdx.x < 9 * A.ppb) {  // read after the prologue's barriers
    const long long pb = (long long)blockIdx.x * A.ppb + threadIdx.x / 9;
    nodes[threadIdx.x] = pb < A.g.P ? A.pmap[11 * pb + 2 + threadIdx.x % 9] : 0;
  }
  BlockRegs<double, R, C, NS> X;
  double cref = 0.0, R0 = 0.0;
  int node = 0;
  burst_prologue<double, R, C, NS, MODE_FUSED>(A, L, M, A.U, X, cref, node, R0);
  save_step_constants<R, C>(A, L, gs, prl, csl);
  __syncthreads();
  double* eo = M.edge;
  double* en = eg2;
  int s0 = 0;
  for (int q = 0; q < F.Q; ++q) {
    const int s1 = (int)((long long)A.n_t * (q + 1) / F.Q);
    nano_loop<R, C, NS>(A, L, M, X, A.ttab + s0, s1 - s0);
    s0 = s1;
    if (q + 1 == F.Q) break;
    double* Uw = (q & 1) ? F.Uw1 : F.Uw0;
    // the lane's block position through an empty asm (as in k_solve_x): otherwise the
    // compiler keeps the refresh's addresses alive across the nano loop and spills them
    LaneMap Lk = L;
    asm volatile("" : "+v"(Lk.k0), "+v"(Lk.row0), "+v"(Lk.slot), "+v"(Lk.rl), "+v"(Lk.vl));
    const double avg = state_average<R, C, NS>(A, Lk, M, X, R0);
    if (L.active && L.rl == 0)
      __hip_atomic_store(Uw + node, cref + avg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (Nb.bnode >= 0)
      __hip_atomic_store(Uw + Nb.bnode, F.bvq[(size_t)q * A.nb + Nb.bq], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);  // every store of the wave has completed
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(F.flags + blockIdx.x, (long long)(q + 1), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    wait_for_neighbours(F.flags, Nb.block, q + 1, F.err);
    refresh_edges<R, C, NS>(A, Lk, M, Uw, nodes, gs, eo, en, X);
    double* t = eo;
    eo = en;
    en = t;
  }
  burst_epilogue<double, R, C, NS, MODE_FUSED>(A, L, M, reinterpret_cast<double*>(M.region),
                                               X, cref, node, R0, A.Unew);
  if (Nb.bnode >= 0) A.Unew[Nb.bnode] = F.bvq[(size_t)(F.Q - 1) * A.nb + Nb.bq];  // step (vi)
}

__global__ void k_zero_flags(long long* f, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) f[i] = 0;
}

}  // namespace

// LDS bytes the resident solve needs beyond the in-wave burst's: the step constants.
size_t solve_x_extra_lds(int ppb, int mx, int me, int nconst) {
  return (size_t)ppb * (2 * (mx + me) + (nconst > 0 ? 2 : 1) * mx * me) * 8;
}

hipError_t launch_zero_flags(long long* f, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_flags, dim3((n + 255) / 256), dim3(256), 0, s, f, n);
  return hipGetLastError();
}

size_t refresh_x_extra_lds(int ppb, int mx, int me, int nconst) {
  return solve_x_extra_lds(ppb, mx, me, nconst) + (size_t)ppb * 2 * (mx + me) * 8 +
         (((size_t)ppb * 9 * 4 + 15) & ~size_t(15));
}

// Launches the resident refreshed macro step when every block fits on the device at once
// and at most one source term depends on time; *resident = 0 (nothing launched) otherwise.
hipError_t launch_refresh_x_f64(int R, int C, const BurstArgs& a, long long* flags, int* err,
                                int Q, double* Uw0, double* Uw1, const double* bvq,
                                int blocks, size_t lds, hipStream_t s, int* resident) {
  RefreshArgs F{flags, err, Q, Uw0, Uw1, bvq};
  *resident = 0;
  if (a.src.ns > 1) return hipSuccess;
#define PD_RONE(R_, C_, NS_)                                                              \
  {                                                                                       \
    const void* kf = reinterpret_cast<const void*>(k_refresh_x<R_, C_, NS_>);             \
    if (!all_resident(kf, blocks, 64, lds)) return hipSuccess;                            \
    BurstArgs b = a;                                                                      \
    b.balance = 1;                                                                        \
    *resident = 1;                                                                        \
    hipLaunchKernelGGL((k_refresh_x<R_, C_, NS_>), dim3(blocks), dim3(64), lds, s, b, F); \
  }
#define PD_RCASE(R_, C_)                          \
  if (R == R_ && C == C_) {                       \
    if (a.src.ns == 0) PD_RONE(R_, C_, 0)         \
    else PD_RONE(R_, C_, 1)                       \
    return hipGetLastError();                     \
  }
  PD_SHAPES(PD_RCASE)
#undef PD_RCASE
#undef PD_RONE
  return hipErrorInvalidValue;
}

// Launches the resident solve of `steps` macro steps when every block fits on the device
// at once; *resident = 0 (and nothing launched) otherwise.
hipError_t launch_solve_x_f64(int R, int C, const BurstArgs& a, long long* flags, int* err,
                              int steps, const double* ttab0, const double* bval0, int per,
                              int blocks, size_t lds, hipStream_t s, int* resident) {
  SolveArgs S{flags, err, steps, ttab0, bval0, per};
  const int ns = a.src.ns;
  *resident = 0;
#define PD_SONE(R_, C_, NS_)                                                              \
  {                                                                                       \
    const void* kf = reinterpret_cast<const void*>(k_solve_x<R_, C_, NS_>);               \
    if (!all_resident(kf, blocks, 64, lds)) return hipSuccess;                            \
    BurstArgs b = a;                                                                      \
    b.balance = 1;                                                                        \
    *resident = 1;                                                                        \
    hipLaunchKernelGGL((k_solve_x<R_, C_, NS_>), dim3(blocks), dim3(64), lds, s, b, S);   \
  }
  // Two time-dependent sources stay on one launch per step: the step prologue's extra
  // per-source state spills hundreds of registers in this kernel.
  if (ns > 1) return hipSuccess;
#define PD_SCASE(R_, C_)                          \
  if (R == R_ && C == C_) {                       \
    if (ns == 0) PD_SONE(R_, C_, 0)               \
    else PD_SONE(R_, C_, 1)                       \
    return hipGetLastError();                     \
  }
  PD_SHAPES(PD_SCASE)
#undef PD_SCASE
#undef PD_SONE
  return hipErrorInvalidValue;
}

}  // namespace pdk
