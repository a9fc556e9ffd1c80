"""Oracle of the ADI micro solver (TEST INFRASTRUCTURE ONLY: used by the tests and the
benchmark's CPU baseline, never by the product path; shares no code with the HIP library).

Sec. 4.1.1 runs the micro simulation in every patch with an alternating-direction
implicit scheme (n_t = 2 nano steps per burst) and does not spell it out.  The reading
taken here is the Peaceman-Rachford splitting of the bursts' micro operator
    L u = alpha d2_xi u + gamma d2_eta u - nu d_xi u - omega d_eta u + phi u + s(t)
(3-point second differences, 2-point upwind or central first differences, the Neumann
edge data through ghost points exactly as in the explicit burst) into
    L_xi  = alpha d2_xi - nu d_xi + phi/2   (with its ghost constants),
    L_eta = gamma d2_eta - omega d_eta + phi/2,
with the source at the half step:
    (I - dt/2 L_xi)  u*      = (I + dt/2 L_eta) u^n + dt/2 s(t + dt/2)
    (I - dt/2 L_eta) u^{n+1} = (I + dt/2 L_xi)  u*  + dt/2 s(t + dt/2).
Each implicit half step is a set of 1-D systems (rows, then columns); here they are built
by applying the affine operator to unit vectors and solved densely (numpy), which is slow
and plainly what the equations say.

Sec. 4.1.2 runs the same micro solver with the 3-point and 4-point upwind first
differences in place of the 2-point one.  With `points` given, each half operator takes
the first difference of that form (oracle/upwind.py: the printed formula where the
velocity component is >= 0, its mirror image where it is < 0, the edge data through two
ghost layers); the implicit lines are then banded (two neighbours on each side) and are
solved densely like the tridiagonal ones.
"""
import numpy as np

from oracle import upwind


def _parts(coef, p, mx, me):
    """alpha, gamma, nu, omega, phi and the source planes of patch p, [me][mx] each (the
    coefficient list of eq. (Computational_Problem))."""
    c = coef[:, p]
    return c[0], c[1], c[2], c[3], c[4], c[5:]


def op_xi(u, alpha, nu, phi, gxm, gxp, dx, central):
    """L_xi u for a patch field u [me][mx] (affine: includes the ghost constants): the xi
    half of the split operator, Sec. 4.1.1."""
    me, mx = u.shape
    uW = np.empty_like(u)
    uE = np.empty_like(u)
    uW[:, 1:] = u[:, :-1]
    uE[:, :-1] = u[:, 1:]
    uW[:, 0] = u[:, 1] - 2.0 * dx * gxm[:me]
    uE[:, -1] = u[:, -2] + 2.0 * dx * gxp[:me]
    d2 = (uE - 2.0 * u + uW) / (dx * dx)
    if central:
        d1 = (uE - uW) / (2.0 * dx)
    else:
        d1 = np.where(nu >= 0.0, (u - uW) / dx, (uE - u) / dx)
    return alpha * d2 - nu * d1 + 0.5 * phi * u


def op_eta(u, gamma, om, phi, gem, gep, de, central):
    """L_eta u, the eta half of the split operator (Sec. 4.1.1), by transposition."""
    return op_xi(u.T, gamma.T, om.T, phi.T, gem, gep, de, central).T


def op_xi_p(u, alpha, nu, phi, gxm, gxp, dx, points, r):
    """L_xi u with the p-point upwind first difference of Sec. 4.1.2 (affine: the two
    ghost layers of edge data included): alpha d2_xi u - nu d_xi u + phi/2 u."""
    me = u.shape[0]
    e = upwind.extend(u, gxm[:me], gxp[:me], dx)
    return (alpha * upwind.second_difference(e, dx)
            - nu * upwind.first_difference(e, nu, dx, points, r) + 0.5 * phi * u)


def op_eta_p(u, gamma, om, phi, gem, gep, de, points, r):
    """L_eta u with the p-point upwind first difference, by transposition."""
    return op_xi_p(u.T, gamma.T, om.T, phi.T, gem, gep, de, points, r).T


def _solve_lines(apply, rhs, h):
    """Solve (I - h A) x = rhs for the affine line operator apply(x) = A x + c, line by
    line (rows of rhs): the matrix from unit vectors, then a dense solve."""
    n_lines, n = rhs.shape
    out = np.empty_like(rhs)
    zero = apply(np.zeros_like(rhs))
    cols = []
    for j in range(n):
        e = np.zeros_like(rhs)
        e[:, j] = 1.0
        cols.append(apply(e) - zero)
    for r in range(n_lines):
        A = np.stack([cols[j][r] for j in range(n)], axis=1)
        out[r] = np.linalg.solve(np.eye(n) - h * A, rhs[r] + h * zero[r])
    return out


def adi_burst(grid, coef, u, edge, t_n, dt, n_t, tfac, points=None, r=0.5):
    """n_t Peaceman-Rachford nano steps of every patch (the ADI micro solver of
    Sec. 4.1.1).  grid: dict with h_xi, h_eta,
    m_xi, m_eta, conv; coef [5 + n_src][P][me][mx]; u [P][me][mx] (not modified);
    edge [P][4][M] (xi-, xi+, eta-, eta+); tfac(t) -> the source time factors.
    points = 2, 3 or 4: the first differences of that upwind form (Sec. 4.1.2; r is the
    4-point form's parameter) whatever the grid's convection option; None: the grid's own
    2-point upwind or central differences."""
    mx, me = grid["m_xi"], grid["m_eta"]
    dx, de = grid["h_xi"] / (mx - 1), grid["h_eta"] / (me - 1)
    central = grid["conv"] == "central"
    out = np.array(u, dtype=np.float64)
    for p in range(out.shape[0]):
        al, ga, nu, om, ph, S = _parts(coef, p, mx, me)
        gxm, gxp, gem, gep = edge[p]
        v = out[p]
        for s in range(n_t):
            th = t_n + s * dt + 0.5 * dt
            T = tfac(th)
            src = sum((T[q] * S[q] for q in range(len(S))), np.zeros_like(v))
            if points is None:
                Lx = lambda w: op_xi(w, al, nu, ph, gxm, gxp, dx, central)
                Le = lambda w: op_eta(w, ga, om, ph, gem, gep, de, central)
            else:
                Lx = lambda w: op_xi_p(w, al, nu, ph, gxm, gxp, dx, points, r)
                Le = lambda w: op_eta_p(w, ga, om, ph, gem, gep, de, points, r)
            r1 = v + 0.5 * dt * Le(v) + 0.5 * dt * src
            ustar = _solve_lines(Lx, r1, 0.5 * dt)
            r2 = ustar + 0.5 * dt * Lx(ustar) + 0.5 * dt * src
            v = _solve_lines(lambda w: Le(w.T).T, r2.T, 0.5 * dt).T
        out[p] = v
    return out


def fe_burst(grid, coef, u, edge, t_n, dt, n_t, tfac, points=None, r=0.5):
    """Forward Euler with the same operator, step (iii) of Sec. 3.3 (cross-check of the
    operator against the C oracle's explicit burst, and with `points` against the
    explicit burst of the higher-order upwind forms)."""
    mx, me = grid["m_xi"], grid["m_eta"]
    dx, de = grid["h_xi"] / (mx - 1), grid["h_eta"] / (me - 1)
    central = grid["conv"] == "central"
    out = np.array(u, dtype=np.float64)
    for p in range(out.shape[0]):
        al, ga, nu, om, ph, S = _parts(coef, p, mx, me)
        gxm, gxp, gem, gep = edge[p]
        v = out[p]
        for s in range(n_t):
            T = tfac(t_n + s * dt)
            src = sum((T[q] * S[q] for q in range(len(S))), np.zeros_like(v))
            if points is None:
                Lv = (op_xi(v, al, nu, ph, gxm, gxp, dx, central)
                      + op_eta(v, ga, om, ph, gem, gep, de, central))
            else:
                Lv = (op_xi_p(v, al, nu, ph, gxm, gxp, dx, points, r)
                      + op_eta_p(v, ga, om, ph, gem, gep, de, points, r))
            v = v + dt * (Lv + src)
        out[p] = v
    return out


def time_factors(prob):
    """T(t) of every source term of a problem description (constant a; a e^{b t};
    a + b sin(c t)), the time factors of the worked sources of Sec. 4."""
    terms = [tf for (tf, _, _) in prob["src"]]

    def T(t):
        out = []
        for tf in terms:
            if tf[0] == "exp":
                out.append(tf[1] * np.exp(tf[2] * t))
            elif tf[0] == "sin":
                out.append(tf[1] + tf[2] * np.sin(tf[3] * t))
            else:
                out.append(tf[1])
        return out
    return T
