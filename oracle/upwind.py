"""Oracle of the explicit micro burst with the higher-order upwind first differences
(TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's CPU baseline, never by the
product path; shares no code with the HIP library).

Sec. 4.1.2 replaces the bursts' 2-point upwind convection difference by two second-order
alternatives, keeping the 3-point central second differences and forward Euler:
    3-point:  d_p u_i = (3 u_i - 4 u_{i-1} + u_{i-2}) / (2 dp)
    4-point:  d_p u_i = (u_{i+1} - u_{i-1}) / (2 dp)
                        + r / (3 dp) (u_{i-2} - 3 u_{i-1} + 3 u_i - u_{i+1}),
r a free parameter the paper does not fix (r = 1/2 makes the 4-point form exact on cubics;
r = 0 is the central difference).  Readings taken here:
  - the printed forms lean on the side the flow comes from, so they apply where the
    velocity component is >= 0; where it is < 0 the mirror image (i -> -i, sign flipped)
    applies, as for the 2-point formula;
  - the Neumann edge data enter through two ghost layers, each the central reading of the
    edge gradient g at its distance: u_{-1} = u_1 - 2 dp g-, u_{-2} = u_2 - 4 dp g-, and
    u_m = u_{m-2} + 2 dp g+, u_{m+1} = u_{m-3} + 4 dp g+ above the last point u_{m-1}
    (both are exact for quadratics, like the single ghost layer of the 2-point burst).
points = 2 gives the bursts' own 2-point upwind difference.
"""
import numpy as np


def extend(u, gm, gp, d):
    """Rows of u [n][m] with two ghost points on each side: [n][m + 4] (the Neumann edge
    data of eq. (edge) at one and two spacings past the edge)."""
    n, m = u.shape
    e = np.empty((n, m + 4))
    e[:, 2:m + 2] = u
    e[:, 1] = u[:, 1] - 2.0 * d * gm
    e[:, 0] = u[:, 2] - 4.0 * d * gm
    e[:, m + 2] = u[:, m - 2] + 2.0 * d * gp
    e[:, m + 3] = u[:, m - 3] + 4.0 * d * gp
    return e


def first_difference(e, nu, d, points, r):
    """Upwind first difference along the rows of an extended field e [n][m + 4] at its m
    inner points; nu [n][m] selects the side (the 2-, 3- and 4-point formulas of
    Sec. 4.1.2)."""
    um2, um1, u0, up1, up2 = e[:, :-4], e[:, 1:-3], e[:, 2:-2], e[:, 3:-1], e[:, 4:]
    if points == 2:
        back = (u0 - um1) / d
        fwd = (up1 - u0) / d
    elif points == 3:
        back = (3.0 * u0 - 4.0 * um1 + um2) / (2.0 * d)
        fwd = -(3.0 * u0 - 4.0 * up1 + up2) / (2.0 * d)
    elif points == 4:
        back = (up1 - um1) / (2.0 * d) + r / (3.0 * d) * (um2 - 3.0 * um1 + 3.0 * u0 - up1)
        fwd = (up1 - um1) / (2.0 * d) - r / (3.0 * d) * (up2 - 3.0 * up1 + 3.0 * u0 - um1)
    else:
        raise ValueError("points must be 2, 3 or 4")
    return np.where(nu >= 0.0, back, fwd)


def second_difference(e, d):
    """3-point central second difference of the bursts' diffusion terms (Sec. 4.1.1)."""
    return (e[:, 3:-1] - 2.0 * e[:, 2:-2] + e[:, 1:-3]) / (d * d)


def operator(u, alpha, gamma, nu, om, phi, src, edge, dx, de, points, r):
    """alpha u_xixi + gamma u_etaeta - nu u_xi - omega u_eta + phi u + src on one patch
    u [m_eta][m_xi] (eq. (Computational_Problem) discretised); edge = (g_xi-, g_xi+,
    g_eta-, g_eta+), each of length >= the side."""
    me, mx = u.shape
    gxm, gxp, gem, gep = edge
    ex = extend(u, gxm[:me], gxp[:me], dx)
    ee = extend(u.T, gem[:mx], gep[:mx], de)
    d2x = second_difference(ex, dx)
    d2e = second_difference(ee, de).T
    d1x = first_difference(ex, nu, dx, points, r)
    d1e = first_difference(ee, om.T, de, points, r).T
    return alpha * d2x + gamma * d2e - nu * d1x - om * d1e + phi * u + src


def burst(grid, coef, u, edge, t_n, dt, n_t, tfac, points, r=0.5):
    """n_t forward-Euler nano steps of every patch, step (iii) of Sec. 3.3 (source at the
    old time level, as in the 2-point burst).  coef [5 + n_src][P][me][mx]; u [P][me][mx] (not modified); edge
    [P][4][M]; tfac(t) -> the source terms' time factors."""
    mx, me = grid["m_xi"], grid["m_eta"]
    dx, de = grid["h_xi"] / (mx - 1), grid["h_eta"] / (me - 1)
    out = np.array(u, dtype=np.float64)
    for p in range(out.shape[0]):
        c = coef[:, p]
        al, ga, nu, om, ph, S = c[0], c[1], c[2], c[3], c[4], c[5:]
        v = out[p]
        for s in range(n_t):
            T = tfac(t_n + s * dt)
            src = sum((T[q] * S[q] for q in range(len(S))), np.zeros_like(v))
            v = v + dt * operator(v, al, ga, nu, om, ph, src, edge[p], dx, de, points, r)
        out[p] = v
    return out
