"""The Fourier-Bessel solution of the annulus problem, Sec. 4.2, eq. (Annulus_AS).

u_a(xi, eta, t) = (pi^2 / 2) sum_m I_m B_m Z1(mu_m eta) sin(xi) exp(-mu_m^2 t),
I_m = int_1^2 psi (psi - 1)(2 - psi) Z1(mu_m psi) dpsi,
B_m = mu_m^2 J1(2 mu_m)^2 / (J1(mu_m)^2 - J1(2 mu_m)^2),
Z1(mu eta) = J1(mu) Y1(mu eta) - Y1(mu) J1(mu eta),
mu_m the positive roots of J1(mu) Y1(2 mu) - Y1(mu) J1(2 mu) = 0.
Test-side only (SciPy Bessel functions).
"""
import functools
import math

import numpy as np
from scipy import integrate, optimize, special


def _cross(mu):
    return special.j1(mu) * special.y1(2 * mu) - special.y1(mu) * special.j1(2 * mu)


@functools.lru_cache(maxsize=None)
def roots(n):
    out = []
    x = 0.5
    step = 0.01
    f0 = _cross(x)
    while len(out) < n:
        x1 = x + step
        f1 = _cross(x1)
        if f0 == 0.0 or f0 * f1 < 0.0:
            out.append(optimize.brentq(_cross, x, x1, xtol=1e-15, rtol=1e-15))
        x, f0 = x1, f1
    return tuple(out)


def Z1(mu, eta):
    return special.j1(mu) * special.y1(mu * eta) - special.y1(mu) * special.j1(mu * eta)


@functools.lru_cache(maxsize=None)
def coefficients(n):
    out = []
    for mu in roots(n):
        I, _ = integrate.quad(lambda p: p * (p - 1) * (2 - p) * Z1(mu, p), 1.0, 2.0,
                              epsabs=1e-14, epsrel=1e-13, limit=200)
        B = mu * mu * special.j1(2 * mu) ** 2 / (special.j1(mu) ** 2 - special.j1(2 * mu) ** 2)
        out.append((mu, I * B))
    return tuple(out)


def u_exact(xi, eta, t, n_terms=60):
    xi = np.asarray(xi, dtype=float)
    eta = np.asarray(eta, dtype=float)
    s = np.zeros(np.broadcast(xi, eta).shape)
    for mu, c in coefficients(n_terms):
        s = s + c * Z1(mu, eta) * math.exp(-mu * mu * t)
    return (math.pi ** 2 / 2.0) * s * np.sin(xi)
