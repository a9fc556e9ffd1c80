"""The ADI micro solver with the higher-order upwind differences of Sec. 4.1.2
(oracle/adi.py with `points`) pinned: the 2-point form and the 4-point form at r = 0 are
the plain ADI solver bit for bit, one forward-Euler step of its operator is the explicit
higher-order upwind burst, a field that varies along one direction is advanced by
Crank-Nicolson of a banded 1-D matrix built here from the printed stencils (both ghost
layers folded by hand, both signs of the velocity), linear fields move exactly, and the
error falls at second order in time."""
import math

import numpy as np
import pytest

from oracle import adi, upwind
from paper_2405_08764_amd import workloads as W


def const_problem(a=0.7, c=1.3, v=(0.0, 0.0), f=0.0, conv="upwind", n=6, m=9):
    g = W.grid("identity", n, n, m, m, conv=conv)
    fields = {"D11": W.field(c0=a), "D22": W.field(c0=c), "v1": W.field(c0=v[0]),
              "v2": W.field(c0=v[1]), "f": W.field(c0=f)}
    S0 = ("cart", 0.0, ("poly", 0, 0, 0, 0), ("poly", 0, 0, 0, 0))
    return W.problem(g, fields, [(W.const(0.0), S0)], [], W.timing(1e-3, 1, 1))


def fields(oracle_mod, prob, seed):
    o = oracle_mod.Oracle(prob)
    U = np.random.default_rng(seed).normal(size=(o.ne, o.nx)) + o.initial()
    return o, o.lift(U), o.edge(U)


PROBLEMS = {
    "tanh": lambda: W.config2(n=6, m=7),
    "annulus": lambda: W.config3(n_r=5, n_theta=8, m=7),
    "sec412": lambda: W.paper_cdr(2, lam=0.1, n=5, m=9),
    "ragged_9x5": lambda: W.problem(W.grid("sine", 5, 6, 9, 5, gparam=0.2, conv="upwind"),
                                    W.config1()["fields"], W.config1()["bc"],
                                    W.config1()["src"], W.timing(1e-3, 1, 2)),
}


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_two_point_and_central_forms_are_the_plain_solver(oracle_mod, name):
    """points = 2 on an upwind grid and points = 4 with r = 0 on a central grid take the
    same arithmetic as the plain ADI solver (bit for bit)."""
    prob = PROBLEMS[name]()
    for conv, points in (("upwind", 2), ("central", 4)):
        prob["grid"]["conv"] = conv
        o, u0, e = fields(oracle_mod, prob, 3)
        dt = 20.0 * o.dt_micro_limit()
        tf = adi.time_factors(prob)
        ref = adi.adi_burst(prob["grid"], o.coef, u0, e, 0.011, dt, 2, tf)
        got = adi.adi_burst(prob["grid"], o.coef, u0, e, 0.011, dt, 2, tf, points, 0.0)
        assert np.array_equal(got, ref), (conv, np.max(np.abs(got - ref)))


@pytest.mark.parametrize("form", [(3, 0.0), (4, 0.5), (4, 1.0 / 3.0)],
                         ids=["p3", "p4r0.50", "p4r0.33"])
@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_operator_is_the_explicit_upwind_burst(oracle_mod, name, form):
    """Forward Euler with the split operator's two halves summed equals the explicit
    higher-order upwind burst (itself pinned by its cubic error terms)."""
    points, r = form
    prob = PROBLEMS[name]()
    o, u0, e = fields(oracle_mod, prob, 4)
    dt = 0.3 * o.dt_micro_limit()
    tf = adi.time_factors(prob)
    ref = upwind.burst(prob["grid"], o.coef, u0, e, 0.013, dt, 3, tf, points, r)
    got = adi.fe_burst(prob["grid"], o.coef, u0, e, 0.013, dt, 3, tf, points, r)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def d1_stencil(points, r, d, forward):
    """Offsets and weights of the first difference as printed in Sec. 4.1.2 (backward
    side); the forward side is its mirror image (offset -> -offset, weight -> -weight)."""
    if points == 3:
        w = {0: 3.0 / (2 * d), -1: -4.0 / (2 * d), -2: 1.0 / (2 * d)}
    else:
        w = {1: 1.0 / (2 * d) - r / (3 * d), -1: -1.0 / (2 * d) - 3 * r / (3 * d),
             0: 3 * r / (3 * d), -2: r / (3 * d)}
    if forward:
        w = {-k: -v for k, v in w.items()}
    return w


@pytest.mark.parametrize("nu", [0.9, -0.9])
@pytest.mark.parametrize("form", [(3, 0.0), (4, 0.5), (4, 0.2)], ids=["p3", "p4r0.5", "p4r0.2"])
def test_reduces_to_crank_nicolson_of_a_banded_matrix(oracle_mod, form, nu):
    """A field constant along eta with zero eta edge data: one Peaceman-Rachford step is
    the Crank-Nicolson step of the xi operator, built here as a matrix from the printed
    stencils with u_{-1} = u_1 - 2 d g-, u_{-2} = u_2 - 4 d g-, u_m = u_{m-2} + 2 d g+,
    u_{m+1} = u_{m-3} + 4 d g+ folded in by hand."""
    points, r = form
    a, c = 0.7, 1.3
    p = const_problem(a, c, v=(nu, 0.0))
    o = oracle_mod.Oracle(p)
    g = p["grid"]
    mx, me = g["m_xi"], g["m_eta"]
    dx = g["h_xi"] / (mx - 1)
    rng = np.random.default_rng(8)
    row = rng.normal(size=mx)
    u0 = np.tile(row, (o.P, me, 1))
    e = np.zeros((o.P, 4, o.M))
    gm, gp = rng.normal(), rng.normal()
    e[:, 0, :] = gm
    e[:, 1, :] = gp
    dt = 40.0 * o.dt_micro_limit()
    got = adi.adi_burst(g, o.coef, u0, e, 0.0, dt, 1, adi.time_factors(p), points, r)
    w = {k: -nu * v for k, v in d1_stencil(points, r, dx, nu < 0).items()}
    for k, v in {-1: a / dx ** 2, 0: -2 * a / dx ** 2, 1: a / dx ** 2}.items():
        w[k] = w.get(k, 0.0) + v
    A = np.zeros((mx, mx))
    b = np.zeros(mx)
    for i in range(mx):
        for k, wk in w.items():
            j = i + k
            if j < 0:  # ghost below the first point: u_j = u_{-j} + 2 j d g-
                A[i, -j] += wk
                b[i] += wk * 2 * j * dx * gm
            elif j > mx - 1:  # ghost above the last: u_j = u_{2(m-1)-j} + 2 (j-m+1) d g+
                A[i, 2 * (mx - 1) - j] += wk
                b[i] += wk * 2 * (j - mx + 1) * dx * gp
            else:
                A[i, j] += wk
    I = np.eye(mx)
    cn = np.linalg.solve(I - 0.5 * dt * A, (I + 0.5 * dt * A) @ row + dt * b)
    for l in range(me):
        np.testing.assert_allclose(got[0, l], cn, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("form", [(3, 0.0), (4, 0.5)], ids=["p3", "p4r0.5"])
def test_linear_fields_move_exactly(oracle_mod, form):
    """Constant coefficients, a linear field with its exact edge gradients: every form is
    exact on it, so the field moves by t (-nu q1 - omega q2) at any step size."""
    points, r = form
    nu, om = 0.8, -0.6
    p = const_problem(0.7, 1.3, v=(nu, om))
    o = oracle_mod.Oracle(p)
    xi, eta = o.node_coords()
    q = np.random.default_rng(9).normal(size=3)
    U = q[0] + q[1] * xi[None, :] + q[2] * eta[:, None]
    u0, e = o.lift(U), o.edge(U)
    dt = 50.0 * o.dt_micro_limit()
    got = adi.adi_burst(p["grid"], o.coef, u0, e, 0.0, dt, 3, adi.time_factors(p), points, r)
    np.testing.assert_allclose(got, u0 + 3 * dt * (-nu * q[1] - om * q[2]), rtol=1e-11,
                               atol=1e-11)


@pytest.mark.parametrize("form", [(3, 0.0), (4, 0.5)], ids=["p3", "p4r0.5"])
def test_second_order_in_time(oracle_mod, form):
    """Against a reference with 64x smaller steps, halving the step divides the error by
    about 4 (the Sec. 4.1.2 coefficients on patches of 0.05 of the domain, a burst over
    tau = 2e-4; on the paper's 1e-3 patches every step size here is deep in the stiff
    range, where the error sits at its floor)."""
    points, r = form
    p = W.paper_cdr(2, lam=0.1, n=5, m=9, h=0.05)
    o = oracle_mod.Oracle(p)
    U = o.initial()
    u0, e = o.lift(U)[:3], o.edge(U)[:3]
    tau = 2e-4
    tf = adi.time_factors(p)
    ref = adi.adi_burst(p["grid"], o.coef, u0, e, 0.0, tau / 256, 256, tf, points, r)
    errs = []
    for n in (4, 8, 16):
        v = adi.adi_burst(p["grid"], o.coef, u0, e, 0.0, tau / n, n, tf, points, r)
        errs.append(np.max(np.abs(v - ref)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(rates) > 1.8, (errs, rates)
