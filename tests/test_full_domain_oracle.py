"""The oracle's full-domain explicit solver (the lattice scheme the patch bursts use,
applied to the whole computational box) pinned to exact solutions and invariants.

The paper compares patch dynamics with a full-domain method-of-lines solution on one
lattice (Sec. 4.1.2, Table PDvsFDS); here that comparator is forward Euler with the
bursts' differences.  Pins: second differences are exact on quadratics and first
differences (central: quadratics, 2-point upwind: linear functions), so with the
manufactured source -L[Q] the polynomial Q is a discrete steady state; a constant field
with a divergence-free velocity and no reaction is a steady state on any map; the error
against a smooth manufactured solution falls at the order of the differences.
"""
import math

import numpy as np
import pytest

from paper_2405_08764_amd import workloads as W


def make(oracle_mod, prob, threads=1):
    return oracle_mod.Oracle(prob, threads=threads)


def poly(a=0.0, b=0.0, c=0.0, d=0.0):
    return ("poly", float(a), float(b), float(c), float(d))


def _problem(geometry, fields, terms, src_terms, conv, gparam=0.0):
    g = W.grid(geometry, 5, 5, 5, 5, gparam=gparam, conv=conv)
    return W.problem(g, fields, terms, src_terms, W.timing(1e-3, 1, 1))


def _poly_terms(q):
    """Q(x, y) = q0 + q1 x + q2 y + q3 x^2 + q4 x y + q5 y^2 as three separable terms."""
    return [("cart", 1.0, poly(q[0], q[1], q[3]), poly(1.0)),
            ("cart", 1.0, poly(1.0), poly(0.0, q[2], q[5])),
            ("cart", q[4], poly(0.0, 1.0), poly(0.0, 1.0))]


def _lattice(n_x, n_y):
    return np.linspace(0.0, 1.0, n_x), np.linspace(0.0, 1.0, n_y)


@pytest.mark.parametrize("conv,quadratic", [("central", True), ("upwind", False)])
def test_polynomial_steady_state(oracle_mod, conv, quadratic):
    """With source -L[Q] and Dirichlet data Q, the lattice scheme keeps Q for any number
    of steps (identity map, constant D and v, ragged 23 x 17 lattice)."""
    rng = np.random.default_rng(11)
    q = rng.normal(size=6)
    if not quadratic:
        q[3:] = 0.0
    fields = {"D11": W.field(c0=0.7), "D22": W.field(c0=1.3), "v1": W.field(c0=0.8),
              "v2": W.field(c0=-0.6), "f": W.field()}
    terms = _poly_terms(q)
    p = _problem("identity", fields, [(W.const(1.0), S) for S in terms],
                 [(W.const(1.0), 0.0, S) for S in terms], conv)
    o = make(oracle_mod, p)
    n_x, n_y = 23, 17
    xs, ys = _lattice(n_x, n_y)
    Q = (q[0] + q[1] * xs[None, :] + q[2] * ys[:, None] + q[3] * xs[None, :] ** 2
         + q[4] * xs[None, :] * ys[:, None] + q[5] * ys[:, None] ** 2)
    dt = 0.4 * o.full_domain_limit(n_x, n_y)
    U = o.full_domain(n_x, n_y, Q.copy(), 0.0, dt, 40)
    np.testing.assert_allclose(U, Q, rtol=0, atol=1e-12)


@pytest.mark.parametrize("conv", ["upwind", "central"])
def test_constant_preserved_on_mapped_box(oracle_mod, conv):
    """A constant with zero reaction and source and a constant (divergence-free) velocity
    is a steady state of eq. (Physical_Problem); on the sine map the lattice scheme keeps
    it to round-off."""
    fields = {"D11": W.field(c0=0.05), "D22": W.field(c0=0.08), "v1": W.field(c0=0.8),
              "v2": W.field(c0=-0.6), "f": W.field()}
    S = ("cart", 1.0, poly(1.0), poly(1.0))
    p = _problem("sine", fields, [(W.const(2.5), S)], [], conv, gparam=0.3)
    o = make(oracle_mod, p)
    n_x, n_y = 29, 21
    dt = 0.4 * o.full_domain_limit(n_x, n_y)
    U = o.full_domain(n_x, n_y, np.full((n_y, n_x), 2.5), 0.0, dt, 60)
    assert np.max(np.abs(U - 2.5)) < 1e-13


def _manufactured(geometry, conv, with_v, gparam=0.0):
    p = W.config1()
    p["grid"] = W.grid(geometry, 5, 5, 5, 5, gparam=gparam, conv=conv)
    if not with_v:
        p["fields"]["v1"] = W.field()
        p["fields"]["v2"] = W.field()
    return p


def _err(oracle_mod, p, n, T=0.05):
    o = make(oracle_mod, p)
    steps = int(math.ceil(T / (0.4 * o.full_domain_limit(n, n))))
    dt = T / steps
    xi = np.linspace(0.0, 1.0, n)
    U0 = np.array([[o.boundary_value(x, y, 0.0) for x in xi] for y in xi])
    U = o.full_domain(n, n, U0, 0.0, dt, steps)
    xs = np.empty((n, n))
    ys = np.empty((n, n))
    for j in range(n):
        for i in range(n):
            m = o.metric(xi[i], xi[j])
            xs[j, i], ys[j, i] = m[0], m[1]
    ex = math.exp(-T) * np.sin(math.pi * xs) * np.sin(math.pi * ys)
    return np.max(np.abs(U - ex))


@pytest.mark.parametrize("geometry,conv,with_v,order", [
    ("identity", "central", False, 1.8), ("sine", "central", False, 1.8),
    ("identity", "upwind", True, 0.9), ("sine", "upwind", True, 0.9)])
def test_manufactured_convergence(oracle_mod, geometry, conv, with_v, order):
    """Error against the exact solution e^{-t} sin(pi x) sin(pi y) (variable D and v,
    reaction 1, the config-1 source) falls at about second order with central differences
    and at least first order with the 2-point upwind difference (dt ~ h^2)."""
    p = _manufactured(geometry, conv, with_v, gparam=0.3 if geometry == "sine" else 0.0)
    errs = [_err(oracle_mod, p, n) for n in (17, 33, 65)]
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[0] > errs[1] > errs[2], errs
    assert rates[-1] >= order, (errs, rates)


def test_point_step_equals_lattice_step(oracle_mod):
    """The one-node entry point reproduces the lattice sweep bit for bit (it is the spot
    check used on lattices too large for a sweep)."""
    p = W.config2(n=5, m=5)
    o = make(oracle_mod, p)
    n_x, n_y = 31, 27
    rng = np.random.default_rng(3)
    U = rng.uniform(-1.0, 1.0, (n_y, n_x))
    dt = 0.4 * o.full_domain_limit(n_x, n_y)
    t = 0.013
    V = o.full_domain(n_x, n_y, U.copy(), t, dt, 1)
    for j in range(n_y):
        for i in range(n_x):
            assert o.full_domain_point(n_x, n_y, U, t, dt, i, j) == V[j, i], (i, j)
