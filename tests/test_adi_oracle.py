"""The ADI micro solver's oracle (oracle/adi.py) pinned: its operator against the C
oracle's explicit burst, exact evolution of quadratics, the reduction to Crank-Nicolson
for fields that vary along one direction (against a 1-D matrix built here), L2 stability
far above the explicit bound, and second order in time."""
import math

import numpy as np
import pytest

from oracle import adi
from paper_2405_08764_amd import workloads as W


def make(oracle_mod, prob):
    return oracle_mod.Oracle(prob)


def const_problem(a=0.7, c=1.3, v=(0.0, 0.0), f=0.0, conv="central", n=6, m=9):
    g = W.grid("identity", n, n, m, m, conv=conv)
    fields = {"D11": W.field(c0=a), "D22": W.field(c0=c), "v1": W.field(c0=v[0]),
              "v2": W.field(c0=v[1]), "f": W.field(c0=f)}
    S0 = ("cart", 0.0, ("poly", 0, 0, 0, 0), ("poly", 0, 0, 0, 0))
    return W.problem(g, fields, [(W.const(0.0), S0)], [], W.timing(1e-3, 1, 1))


@pytest.mark.parametrize("name", ["config1", "tanh", "annulus"])
def test_operator_matches_the_explicit_burst(oracle_mod, name):
    prob = {"config1": lambda: W.config1(),
            "tanh": lambda: W.config2(n=7, m=7),
            "annulus": lambda: W.config3(n_r=6, n_theta=8, m=7)}[name]()
    o = make(oracle_mod, prob)
    U = np.random.default_rng(4).normal(size=(o.ne, o.nx)) + o.initial()
    u0, e = o.lift(U), o.edge(U)
    dt = 0.3 * o.dt_micro_limit()
    ref, rc = o.burst(u0, e, 0.013, dt, 3)
    got = adi.fe_burst(prob["grid"], o.coef, u0, e, 0.013, dt, 3, adi.time_factors(prob))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def test_quadratics_evolve_exactly(oracle_mod):
    """Constant alpha, gamma and nothing else: Q + (2 alpha q3 + 2 gamma q5) t solves the
    micro problem with the exact edge gradients, and both half steps reproduce it."""
    a, c = 0.7, 1.3
    p = const_problem(a, c)
    o = make(oracle_mod, p)
    xi, eta = o.node_coords()
    q = np.random.default_rng(5).normal(size=6)
    U = (q[0] + q[1] * xi[None, :] + q[2] * eta[:, None] + q[3] * xi[None, :] ** 2
         + q[4] * xi[None, :] * eta[:, None] + q[5] * eta[:, None] ** 2)
    u0, e = o.lift(U), o.edge(U)
    dt = 50.0 * o.dt_micro_limit()
    got = adi.adi_burst(p["grid"], o.coef, u0, e, 0.0, dt, 4, adi.time_factors(p))
    np.testing.assert_allclose(got, u0 + 4 * dt * (2 * a * q[3] + 2 * c * q[5]),
                               rtol=1e-11, atol=1e-11)


def test_reduces_to_crank_nicolson_along_one_direction(oracle_mod):
    """A field constant along eta with zero eta edge data: the eta operator vanishes on it,
    so a Peaceman-Rachford step is the Crank-Nicolson step of the xi operator, here built
    as a dense matrix from its stencil (ghost points folded by hand)."""
    a, c = 0.7, 1.3
    p = const_problem(a, c, v=(0.9, 0.0), conv="upwind")
    o = make(oracle_mod, p)
    g = p["grid"]
    mx, me = g["m_xi"], g["m_eta"]
    dx = g["h_xi"] / (mx - 1)
    rng = np.random.default_rng(6)
    row = rng.normal(size=mx)
    u0 = np.tile(row, (o.P, me, 1))
    e = np.zeros((o.P, 4, o.M))
    e[:, 0, :] = rng.normal()  # the xi- edge gradient, same on every row
    e[:, 1, :] = rng.normal()
    dt = 40.0 * o.dt_micro_limit()
    got = adi.adi_burst(g, o.coef, u0, e, 0.0, dt, 1, adi.time_factors(p))
    nu = 0.9
    A = np.zeros((mx, mx))
    b = np.zeros(mx)
    for k in range(mx):  # alpha (uE - 2u + uW)/dx^2 - nu (u - uW)/dx, upwind (nu > 0)
        wW = a / dx ** 2 + nu / dx
        wE = a / dx ** 2
        A[k, k] -= wW + wE
        if k > 0:
            A[k, k - 1] += wW
        else:  # uW = u_1 - 2 dx g-
            A[k, 1] += wW
            b[k] -= 2 * dx * e[0, 0, 0] * wW
        if k < mx - 1:
            A[k, k + 1] += wE
        else:  # uE = u_{m-2} + 2 dx g+
            A[k, mx - 2] += wE
            b[k] += 2 * dx * e[0, 1, 0] * wE
    I = np.eye(mx)
    cn = np.linalg.solve(I - 0.5 * dt * A, (I + 0.5 * dt * A) @ row + dt * b)
    for l in range(me):
        np.testing.assert_allclose(got[0, l], cn, rtol=1e-11, atol=1e-11)


def test_stable_far_above_the_explicit_bound(oracle_mod):
    """Constant diffusion, zero edge data: the L2 norm does not grow at 100x the
    explicit step."""
    p = const_problem(0.7, 1.3)
    o = make(oracle_mod, p)
    rng = np.random.default_rng(7)
    u0 = rng.normal(size=(o.P, o.me, o.mx))
    e = np.zeros((o.P, 4, o.M))
    dt = 100.0 * o.dt_micro_limit()
    v = u0
    norms = [np.linalg.norm(v)]
    for _ in range(5):
        v = adi.adi_burst(p["grid"], o.coef, v, e, 0.0, dt, 2, adi.time_factors(p))
        norms.append(np.linalg.norm(v))
    assert all(norms[k + 1] <= norms[k] * (1 + 1e-12) for k in range(5)), norms


def test_second_order_in_time(oracle_mod):
    """Against a reference with 64x smaller steps, halving the step divides the error by
    about 4 (config-1 coefficients, a burst over tau = 2e-4)."""
    p = W.config1()
    o = make(oracle_mod, p)
    U = o.initial()
    u0, e = o.lift(U), o.edge(U)
    tau = 2e-4
    tf = adi.time_factors(p)
    ref = adi.adi_burst(p["grid"], o.coef, u0[:4], e[:4], 0.0, tau / 256, 256, tf)
    errs = []
    for n in (4, 8, 16):
        v = adi.adi_burst(p["grid"], o.coef, u0[:4], e[:4], 0.0, tau / n, n, tf)
        errs.append(np.max(np.abs(v - ref)))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(rates) > 1.8, (errs, rates)
