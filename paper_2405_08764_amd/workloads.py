"""Seeded synthetic workloads shaped like the paper's test problems.

This module only *describes* problems: geometry, macro/micro resolution, the physical
fields D, v, f as analytic expressions, the initial/Dirichlet data and the source terms,
and the time parameters.  It holds none of the method's arithmetic, so both the HIP path
and the CPU oracle take their inputs from here.

A problem is a plain dict::

    {"grid":   {geometry, gparam, xi0, xi1, eta0, eta1, n_xi, n_eta, periodic_xi,
                h_xi, h_eta, m_xi, m_eta, conv, c0},
     "fields": {"D11": field, "D22": field, "v1": field, "v2": field, "f": field},
     "bc":     [(tfun, sfun), ...],          # u_b = sum T(t) S(x, y)
     "src":    [(tfun, c, sfun), ...],       # g = sum T(t) (c S - L[S])
     "time":   {t0, dt_macro, n_steps, n_t, dt_micro}}

field = {"c0", "cx", "cy", "modes": [(amp, kx, ky, ph)], "polar": [(amp, p0, p1, p2, n, ph)]}
  F = c0 + cx x + cy y + sum amp cos(kx x + ky y + ph)
        + sum amp (p0 + p1 r + p2 r^2) cos(n theta + ph)     (polar terms: annulus only)
tfun = ("const", a) | ("exp", a, b) | ("sin", a, b, c)      a | a e^{bt} | a + b sin(ct)
sfun = ("cart" | "polar", amp, fn1, fn1)                    amp f(x) g(y) | amp f(r) g(theta)
fn1  = ("sin", a, b) | ("cos", a, b) | ("exp", a, b) | ("poly", c0, c1, c2, c3)

Sizes follow the workloads of the paper: the sine-stretched unit square of Sec. 4.1
(eq. Stretching_Transformation), the annulus of Sec. 4.2 (eq. Transformation_Annulus), and
the synthetic variants (tanh stretching, random Fourier-mode coefficients, non-axisymmetric
conductivity, batches of mixed instances) that stand in for them at GPU scale.
"""
from __future__ import annotations

import copy
import math

import numpy as np

MASTER_SEED = 240508764
TWO_PI = 2.0 * math.pi


def field(c0=0.0, cx=0.0, cy=0.0, modes=(), polar=()):
    return {"c0": float(c0), "cx": float(cx), "cy": float(cy),
            "modes": [tuple(float(v) for v in m) for m in modes],
            "polar": [tuple(float(v) for v in p) for p in polar]}


def const(a):
    return ("const", float(a))


def texp(a, b):
    return ("exp", float(a), float(b))


def tsin(a, b, c):
    return ("sin", float(a), float(b), float(c))


def grid(geometry, n_xi, n_eta, m_xi, m_eta, *, gparam=0.0, box=(0.0, 1.0, 0.0, 1.0),
         periodic_xi=False, ratio=0.2, conv="upwind", c0="trapezoid", h_xi=None, h_eta=None):
    """Macro grid with patch edges h = ratio * Delta unless h is given explicitly."""
    xi0, xi1, eta0, eta1 = (float(v) for v in box)
    d_xi = (xi1 - xi0) / (n_xi if periodic_xi else n_xi - 1)
    d_eta = (eta1 - eta0) / (n_eta - 1)
    return {"geometry": geometry, "gparam": float(gparam), "xi0": xi0, "xi1": xi1,
            "eta0": eta0, "eta1": eta1, "n_xi": int(n_xi), "n_eta": int(n_eta),
            "periodic_xi": bool(periodic_xi),
            "h_xi": float(h_xi if h_xi is not None else ratio * d_xi),
            "h_eta": float(h_eta if h_eta is not None else ratio * d_eta),
            "m_xi": int(m_xi), "m_eta": int(m_eta), "conv": conv, "c0": c0}


def timing(dt_macro, n_steps, n_t, *, ratio=20.0, t0=0.0):
    """tau = dt_macro / ratio, split into n_t forward-Euler nano steps."""
    tau = dt_macro / ratio
    return {"t0": float(t0), "dt_macro": float(dt_macro), "n_steps": int(n_steps),
            "n_t": int(n_t), "dt_micro": tau / n_t}


def problem(grid_, fields, bc, src, time_):
    return {"grid": grid_, "fields": fields, "bc": list(bc), "src": list(src),
            "time": time_}


def with_time(prob, dt_macro=None, n_steps=None, n_t=None, ratio=20.0):
    """Copy of prob with new time parameters (unspecified ones are kept)."""
    p = copy.deepcopy(prob)
    t = p["time"]
    dtm = t["dt_macro"] if dt_macro is None else dt_macro
    ns = t["n_steps"] if n_steps is None else n_steps
    nt = t["n_t"] if n_t is None else n_t
    p["time"] = timing(dtm, ns, nt, ratio=ratio, t0=t["t0"])
    return p


def sin_prod_x_y(c1=0.0, c2=0.0):
    """Modes of c1 sin(2 pi x) sin(2 pi y) + c2 cos(2 pi x) cos(2 pi y)."""
    k = TWO_PI
    return [(0.5 * (c1 + c2), k, -k, 0.0), (0.5 * (c2 - c1), k, k, 0.0)]


# ------------------------------------------------------------------ the paper's problems

def paper_cdr(variant=1, lam=0.1, n=11, m=11, n_steps=2000, T=1.0, n_t=2,
              h=1e-3, tau=1e-6, conv="upwind"):
    """Sec. 4.1.1 (variant 1: D = 1, v = (10x, 10y)) and Sec. 4.1.2 (variant 2:
    D = 1 + x, v = (1 + 10x, 10y)); f = 20, exact solution e^{x+y+t}, sine stretching."""
    g = grid("sine", n, n, m, m, gparam=lam, h_xi=h, h_eta=h, conv=conv)
    if variant == 1:
        D = field(c0=1.0)
        v1 = field(cx=10.0)
    else:
        D = field(c0=1.0, cx=1.0)
        v1 = field(c0=1.0, cx=10.0)
    fields = {"D11": D, "D22": copy.deepcopy(D), "v1": v1, "v2": field(cy=10.0),
              "f": field(c0=20.0)}
    S = ("cart", 1.0, ("exp", 1.0, 0.0), ("exp", 1.0, 0.0))
    dtm = T / n_steps
    return problem(g, fields, [(texp(1.0, 1.0), S)], [(texp(1.0, 1.0), 1.0, S)],
                   timing(dtm, n_steps, n_t, ratio=dtm / tau))


def paper_annulus(n_theta=16, n_r=11, m=21, n_steps=500, T=0.2, n_t=1500, h=1e-3,
                  tau=1e-6):
    """Sec. 4.2: u_t = Laplacian(u) on 1 <= r <= 2, theta periodic, initial data
    (r - 1)(2 - r) sin(theta), homogeneous Dirichlet data on both circles."""
    g = grid("annulus", n_theta, n_r, m, m, box=(0.0, TWO_PI, 1.0, 2.0), periodic_xi=True,
             h_xi=h, h_eta=h, conv="central")
    one = field(c0=1.0)
    fields = {"D11": one, "D22": copy.deepcopy(one), "v1": field(), "v2": field(),
              "f": field()}
    S = ("polar", 1.0, ("poly", -2.0, 3.0, -1.0, 0.0), ("sin", 1.0, 0.0))
    dtm = T / n_steps
    return problem(g, fields, [(const(1.0), S)], [], timing(dtm, n_steps, n_t, ratio=dtm / tau))


# ------------------------------------------------------- the synthetic GPU-scale configs

def config1(n_t=11):
    """Unit square, 11x11 macro nodes, 9x9 micro points per patch (h = 0.2 Delta),
    D = diag(0.01(1 + 0.5 sin2pix sin2piy), 0.01(1 + 0.5 cos2pix cos2piy)),
    v = (1 + 0.3 sin2piy, 0.5 + 0.3 cos2pix), reaction 1, source manufactured from
    u = e^{-t} sin(pi x) sin(pi y), 10 macro steps to t = 0.1."""
    g = grid("identity", 11, 11, 9, 9, conv="upwind")
    fields = {
        "D11": field(c0=0.01, modes=sin_prod_x_y(c1=0.005)),
        "D22": field(c0=0.01, modes=sin_prod_x_y(c2=0.005)),
        "v1": field(c0=1.0, modes=[(0.3, 0.0, TWO_PI, -0.5 * math.pi)]),
        "v2": field(c0=0.5, modes=[(0.3, TWO_PI, 0.0, 0.0)]),
        "f": field(c0=1.0),
    }
    S = ("cart", 1.0, ("sin", math.pi, 0.0), ("sin", math.pi, 0.0))
    return problem(g, fields, [(texp(1.0, -1.0), S)], [(texp(1.0, -1.0), -1.0, S)],
                   timing(0.01, 10, n_t))


def fourier_field(rng, base, scale, n_modes=8, kmax=3):
    """base + scale * s, s a sum of n_modes cos(2 pi (p x + q y) + theta) terms with
    p, q in 0..kmax not both zero, amplitudes U[-1,1] normalised so |s| <= 1."""
    modes = []
    a = rng.uniform(-1.0, 1.0, n_modes)
    a = a / np.sum(np.abs(a))
    for k in range(n_modes):
        while True:
            p, q = rng.integers(0, kmax + 1, 2)
            if p or q:
                break
        th = rng.uniform(0.0, TWO_PI)
        modes.append((scale * a[k], TWO_PI * p, TWO_PI * q, th))
    return field(c0=base, modes=modes)


def config2(seed=MASTER_SEED + 2000, n=65, m=17, beta=2.5, eps=1e-3, n_steps=1000,
            dt_macro=9.0e-5, n_t=225):
    """Stretched square: n x n macro nodes with tanh stretching clustered at x = 1 and
    y = 1, 17x17 micro points per patch, convection-dominated (eps = 1e-3), D and v from 8
    seeded random Fourier modes (amplitude 0.3), source (1 + sin 4 pi t) g(x, y) with
    g = -L[sin(pi x) sin(pi y)], Dirichlet data and initial state sin(pi x) sin(pi y)."""
    rng = np.random.default_rng(seed)
    g = grid("tanh", n, n, m, m, gparam=beta, conv="upwind")
    fields = {
        "D11": fourier_field(rng, eps, 0.3 * eps),
        "D22": fourier_field(rng, eps, 0.3 * eps),
        "v1": fourier_field(rng, 1.0, 0.3),
        "v2": fourier_field(rng, 0.5, 0.3),
        "f": field(),
    }
    w = ("cart", 1.0, ("sin", math.pi, 0.0), ("sin", math.pi, 0.0))
    return problem(g, fields, [(const(1.0), w)], [(tsin(1.0, 1.0, 4.0 * math.pi), 0.0, w)],
                   timing(dt_macro, n_steps, n_t))


def annulus_k_field():
    """k(r, theta) = 1 + 0.5 cos(3 theta) (r - 1)."""
    return field(c0=1.0, polar=[(0.5, -1.0, 1.0, 0.0, 3.0, 0.0)])


def config3(n_r=64, n_theta=256, m=21, n_steps=2000, dt_macro=3.0e-5, n_t=492):
    """Annulus 1 <= r <= 2, theta periodic: 64 radial x 256 angular macro nodes, 21x21
    micro points per patch, u_t = div(k grad u), k = 1 + 0.5 cos(3 theta)(r - 1),
    manufactured solution e^{-2t}(r-1)(2-r)cos(2 theta) + 0.1 sin(theta)."""
    g = grid("annulus", n_theta, n_r, m, m, box=(0.0, TWO_PI, 1.0, 2.0), periodic_xi=True,
             conv="central")
    k = annulus_k_field()
    fields = {"D11": k, "D22": copy.deepcopy(k), "v1": field(), "v2": field(), "f": field()}
    S1 = ("polar", 1.0, ("poly", -2.0, 3.0, -1.0, 0.0), ("cos", 2.0, 0.0))
    S2 = ("polar", 0.1, ("poly", 1.0, 0.0, 0.0, 0.0), ("sin", 1.0, 0.0))
    bc = [(texp(1.0, -2.0), S1), (const(1.0), S2)]
    src = [(texp(1.0, -2.0), -2.0, S1), (const(1.0), 0.0, S2)]
    return problem(g, fields, bc, src, timing(dt_macro, n_steps, n_t))


def fit_time(prob, dt_macro_limit, dt_micro_limit, n_steps, frac=0.4, ratio=20.0):
    """Time parameters from the explicit bounds: dt_macro at frac of the macro bound,
    tau = dt_macro / ratio, n_t nano steps at no more than frac of the micro bound."""
    dtm = frac * dt_macro_limit
    n_t = max(1, int(math.ceil((dtm / ratio) / (frac * dt_micro_limit))))
    return with_time(prob, dt_macro=dtm, n_steps=n_steps, n_t=n_t, ratio=ratio)


def config4_instance(i, seed=MASTER_SEED + 4000, n_range=(17, 129), m_range=(9, 33),
                     n_steps=1):
    """Instance i of the mixed batch: square (tanh stretching beta ~ U[0, 3]) or annulus
    (50/50), N x N macro nodes with N ~ U{n_range}, m x m micro points with m odd ~
    U{m_range}, eps ~ log-U[1e-3, 1e-2], D and v from seeded Fourier modes (scalar D on
    the annulus), reaction ~ U[0, 2], upwind convection, manufactured sources as the
    square (e^-t sin pi x sin pi y) and annulus (e^-2t (r-1)(2-r) cos 2 theta + 0.1 sin
    theta) configurations.  Time parameters are placeholders: fit them with fit_time
    from the explicit bounds."""
    rng = np.random.default_rng(seed + i)
    annulus = bool(rng.random() < 0.5)
    N = int(rng.integers(n_range[0], n_range[1] + 1))
    m = int(rng.choice(np.arange(m_range[0], m_range[1] + 1, 2)))
    beta = float(rng.uniform(0.0, 3.0))
    react = float(rng.uniform(0.0, 2.0))
    eps = float(10.0 ** rng.uniform(-3.0, -2.0))
    if annulus:
        k = fourier_field(rng, eps, 0.3 * eps)
        fields = {"D11": k, "D22": copy.deepcopy(k), "v1": fourier_field(rng, 1.0, 0.3),
                  "v2": fourier_field(rng, 0.5, 0.3), "f": field(c0=react)}
        g = grid("annulus", N, N, m, m, box=(0.0, TWO_PI, 1.0, 2.0), periodic_xi=True,
                 conv="upwind")
        S1 = ("polar", 1.0, ("poly", -2.0, 3.0, -1.0, 0.0), ("cos", 2.0, 0.0))
        S2 = ("polar", 0.1, ("poly", 1.0, 0.0, 0.0, 0.0), ("sin", 1.0, 0.0))
        bc = [(texp(1.0, -2.0), S1), (const(1.0), S2)]
        src = [(texp(1.0, -2.0), -2.0, S1), (const(1.0), 0.0, S2)]
    else:
        fields = {"D11": fourier_field(rng, eps, 0.3 * eps),
                  "D22": fourier_field(rng, eps, 0.3 * eps),
                  "v1": fourier_field(rng, 1.0, 0.3), "v2": fourier_field(rng, 0.5, 0.3),
                  "f": field(c0=react)}
        g = grid("tanh", N, N, m, m, gparam=beta, conv="upwind")
        S = ("cart", 1.0, ("sin", math.pi, 0.0), ("sin", math.pi, 0.0))
        bc = [(texp(1.0, -1.0), S)]
        src = [(texp(1.0, -1.0), -1.0, S)]
    return problem(g, fields, bc, src, timing(1.0, n_steps, 1))


def config4(n_instances=512, **kw):
    """The mixed batch: config4_instance(i) for i < n_instances."""
    return [config4_instance(i, **kw) for i in range(n_instances)]


def n_patches(g):
    nx = g["n_xi"] if g["periodic_xi"] else g["n_xi"] - 2
    return nx * (g["n_eta"] - 2)


def updates_per_step(prob):
    g = prob["grid"]
    return n_patches(g) * g["m_xi"] * g["m_eta"] * prob["time"]["n_t"]
