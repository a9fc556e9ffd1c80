"""The higher-order upwind burst's oracle (oracle/upwind.py) pinned: its 2-point form and its
4-point form at r = 0 against the C oracle's explicit bursts (upwind and central), exact
operator values on quadratics (ghost layers included) for both sides of the flow, the
leading error terms on cubics that fix each formula's coefficients (3-point: -dp^2 u'''/3;
4-point: dp^2 u''' (1/6 - r/3), so exact on cubics at r = 1/2), mirror symmetry, and a
steady quadratic held fixed by whole bursts."""
import numpy as np
import pytest

from oracle import adi, upwind
from paper_2405_08764_amd import workloads as W


def with_conv(prob, conv):
    prob["grid"]["conv"] = conv
    return prob


PROBS = {
    "config1": lambda: W.config1(),
    "tanh": lambda: W.config2(n=7, m=7),
    "annulus": lambda: W.config3(n_r=6, n_theta=8, m=7),
    "ragged_9x5": lambda: W.problem(W.grid("sine", 5, 6, 9, 5, gparam=0.2),
                                    W.config1()["fields"], W.config1()["bc"],
                                    W.config1()["src"], W.timing(1e-3, 1, 2)),
}


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("conv", ["upwind", "central"])
def test_reduces_to_the_c_oracle_burst(oracle_mod, name, conv):
    """points = 2 is the bursts' 2-point upwind difference; points = 4 with r = 0 is the
    central difference.  Both against the C oracle's own explicit burst."""
    prob = with_conv(PROBS[name](), conv)
    o = oracle_mod.Oracle(prob)
    U = np.random.default_rng(8).normal(size=(o.ne, o.nx)) + o.initial()
    u0, e = o.lift(U), o.edge(U)
    dt = 0.3 * o.dt_micro_limit()
    ref, rc = o.burst(u0, e, 0.021, dt, 3)
    assert rc == 0
    points, r = (2, 0.7) if conv == "upwind" else (4, 0.0)
    got = upwind.burst(prob["grid"], o.coef, u0, e, 0.021, dt, 3, adi.time_factors(prob),
                       points, r)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))


def patch(mx=9, me=7, dx=0.013, de=0.021, x0=0.31, y0=-0.17):
    x = x0 + dx * np.arange(mx)
    y = y0 + de * np.arange(me)
    return x[None, :], y[:, None], dx, de


def quad(q, x, y):
    u = q[0] + q[1] * x + q[2] * y + q[3] * x * x + q[4] * x * y + q[5] * y * y
    ux = q[1] + 2 * q[3] * x + q[4] * y
    uy = q[2] + q[4] * x + 2 * q[5] * y
    return u, ux, uy, 2 * q[3], 2 * q[5]


def exact_edges(q, x, y, M):
    """Gradient data at the patch's four edges, padded to length M."""
    _, ux, uy, _, _ = quad(q, x, y)
    me, mx = ux.shape
    e = np.zeros((4, M))
    e[0, :me] = ux[:, 0]
    e[1, :me] = ux[:, -1]
    e[2, :mx] = uy[0, :]
    e[3, :mx] = uy[-1, :]
    return e


@pytest.mark.parametrize("points,r", [(3, 0.0), (4, 0.0), (4, 1.0 / 3.0), (4, 0.5), (4, 1.0)])
def test_operator_exact_on_quadratics(points, r):
    """Every point, edges included, and velocity components of both signs: the second-order
    formulas with both ghost layers reproduce the operator of a quadratic exactly."""
    rng = np.random.default_rng(points * 10 + int(6 * r))
    x, y, dx, de = patch()
    me, mx = 7, 9
    q = rng.normal(size=6)
    u, ux, uy, uxx, uyy = quad(q, x, y)
    u = u + 0 * x * y
    al, ga = rng.uniform(0.5, 2, (me, mx)), rng.uniform(0.5, 2, (me, mx))
    nu, om = rng.normal(size=(me, mx)), rng.normal(size=(me, mx))
    ph = rng.normal(size=(me, mx))
    e = exact_edges(q, x, y, 9)
    got = upwind.operator(u, al, ga, nu, om, ph, 0.0, e, dx, de, points, r)
    ref = al * uxx + ga * uyy - nu * ux - om * uy + ph * u
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-9 * np.max(np.abs(ref)))


def test_two_point_is_not_exact_on_quadratics():
    """The control: the first-order formula misses by -+dp u''/2 on the same quadratic."""
    x, y, dx, de = patch()
    q = np.array([0.3, -0.2, 0.5, 1.7, 0.0, 0.0])
    u, ux, _, uxx, _ = quad(q, x, y)
    u = u + 0 * y
    ex = upwind.extend(u, ux[:, 0] + 0 * y[:, 0], ux[:, -1] + 0 * y[:, 0], dx)
    nu = np.where(np.arange(9)[None, :] % 2 == 0, 1.0, -1.0) * np.ones((7, 1))
    d1 = upwind.first_difference(ex, nu, dx, 2, 0.0)
    np.testing.assert_allclose(d1 - ux, -np.sign(nu) * dx * uxx / 2, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("points,r", [(3, 0.0), (4, 0.0), (4, 0.5), (4, 1.0), (4, 2.0)])
def test_cubic_error_terms(points, r):
    """On u = c3 x^3 + ... the interior error of each formula is a fixed multiple of
    dp^2 u''' = 6 c3 dp^2, the same on both sides of the flow."""
    x, y, dx, de = patch(mx=11)
    c = np.array([0.4, -1.1, 0.6, 2.3])
    u = (c[0] + c[1] * x + c[2] * x * x + c[3] * x ** 3) * np.ones((7, 1))
    ux = (c[1] + 2 * c[2] * x + 3 * c[3] * x * x) * np.ones((7, 1))
    ex = upwind.extend(u, np.zeros(7), np.zeros(7), dx)
    for sgn in (1.0, -1.0):
        d1 = upwind.first_difference(ex, sgn * np.ones((7, 11)), dx, points, r)
        lead = -1.0 / 3.0 if points == 3 else 1.0 / 6.0 - r / 3.0
        err = (d1 - ux)[:, 2:-2]
        np.testing.assert_allclose(err, lead * 6 * c[3] * dx * dx * np.ones_like(err),
                                   rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("points,r", [(2, 0.0), (3, 0.0), (4, 0.4)])
def test_mirror_symmetry(points, r):
    """Reflecting xi (k -> m-1-k) with nu -> -nu and the xi edge data swapped and negated
    reflects the operator."""
    rng = np.random.default_rng(21 + points)
    me, mx = 6, 8
    dx, de = 0.017, 0.011
    u = rng.normal(size=(me, mx))
    al, ga, ph = rng.uniform(0.5, 2, (me, mx)), rng.uniform(0.5, 2, (me, mx)), rng.normal(size=(me, mx))
    nu, om = rng.normal(size=(me, mx)), rng.normal(size=(me, mx))
    e = rng.normal(size=(4, 8))
    got = upwind.operator(u, al, ga, nu, om, ph, 0.0, e, dx, de, points, r)
    er = np.array([-e[1], -e[0], e[2][::-1], e[3][::-1]])
    f = lambda a: a[:, ::-1]
    mir = upwind.operator(f(u), f(al), f(ga), -f(nu), f(om), f(ph), 0.0, er, dx, de, points, r)
    np.testing.assert_allclose(f(mir), got, rtol=1e-12, atol=1e-12 * np.max(np.abs(got)))


@pytest.mark.parametrize("points,r", [(3, 0.0), (4, 0.5), (4, 1.0)])
def test_steady_quadratic_stays_fixed(points, r):
    """Constant-coefficient bursts whose source cancels the operator of a quadratic keep it
    to rounding over many nano steps (the time loop, source and ghost layers together)."""
    rng = np.random.default_rng(5)
    me, mx = 7, 9
    x, y, dx, de = patch(mx=mx, me=me)
    q = rng.normal(size=6)
    u, ux, uy, uxx, uyy = quad(q, x, y)
    u = u + 0 * x * y
    a, g, v, w, f = 0.8, 1.4, 9.0, -7.0, 0.3
    src = -(a * uxx + g * uyy - v * ux - w * uy + f * u)
    coef = np.stack([np.full((me, mx), a), np.full((me, mx), g), np.full((me, mx), v),
                     np.full((me, mx), w), np.full((me, mx), f), src])[:, None]
    grid = {"m_xi": mx, "m_eta": me, "h_xi": dx * (mx - 1), "h_eta": de * (me - 1)}
    e = exact_edges(q, x, y, mx)[None]
    dt = 0.1 * min(dx, de) ** 2
    out = upwind.burst(grid, coef, u[None], e, 0.0, dt, 40, lambda t: [1.0], points, r)
    np.testing.assert_allclose(out[0], u, rtol=1e-10, atol=1e-10 * np.max(np.abs(u)))


def test_rejects_unknown_formulas():
    with pytest.raises(ValueError):
        upwind.first_difference(np.zeros((2, 9)), np.zeros((2, 5)), 0.1, 5, 0.0)
