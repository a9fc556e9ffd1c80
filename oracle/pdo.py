"""ctypes binding of the FP64 CPU oracle (``libpdo.so``, built from ``pdo.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg of the
benchmark use it; the product path never imports it.  Shares no code with the HIP
library: its structures mirror ``pdo.h`` only.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdo.so")
LIB_LD_PATH = os.path.join(HERE, "libpdo_ld.so")
SRC = os.path.join(HERE, "pdo.c")

MAXMODE, MAXPOLAR, MAXTERM = 16, 4, 4
GEOM = {"identity": 0, "sine": 1, "tanh": 2, "annulus": 3}
CONV = {"upwind": 0, "central": 1}
C0 = {"trapezoid": 0, "printed": 1}
FN = {"sin": 0, "cos": 1, "exp": 2, "poly": 3}
TF = {"const": 0, "exp": 1, "sin": 2}


def build(force=False):
    """Compile the oracle with gcc (-O2 -ffp-contract=off, OpenMP over patches): the FP64
    build and the same source in x87 extended precision (long double)."""
    newest = max(os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "pdo.h")))
    for path, extra in ((LIB_PATH, []), (LIB_LD_PATH, ["-DPDO_REAL=long double"])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < newest:
            tmp = path + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                                   "-shared", *extra, SRC, "-o", tmp, "-lm"], cwd=HERE)
            os.replace(tmp, path)
    return LIB_PATH


class Grid(C.Structure):
    _fields_ = [("geometry", C.c_int), ("gparam", C.c_double), ("xi0", C.c_double),
                ("xi1", C.c_double), ("eta0", C.c_double), ("eta1", C.c_double),
                ("n_xi", C.c_int), ("n_eta", C.c_int), ("periodic_xi", C.c_int),
                ("h_xi", C.c_double), ("h_eta", C.c_double), ("m_xi", C.c_int),
                ("m_eta", C.c_int), ("conv", C.c_int), ("c0mode", C.c_int),
                ("core_points", C.c_int)]


class Field(C.Structure):
    _fields_ = [("c0", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("nmode", C.c_int), ("amp", C.c_double * MAXMODE),
                ("kx", C.c_double * MAXMODE), ("ky", C.c_double * MAXMODE),
                ("ph", C.c_double * MAXMODE), ("npolar", C.c_int),
                ("pamp", C.c_double * MAXPOLAR), ("pc0", C.c_double * MAXPOLAR),
                ("pc1", C.c_double * MAXPOLAR), ("pc2", C.c_double * MAXPOLAR),
                ("pn", C.c_double * MAXPOLAR), ("pph", C.c_double * MAXPOLAR)]


class Fn1(C.Structure):
    _fields_ = [("type", C.c_int), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("d", C.c_double)]


class Sfun(C.Structure):
    _fields_ = [("kind", C.c_int), ("amp", C.c_double), ("f", Fn1), ("g", Fn1)]


class Tfun(C.Structure):
    _fields_ = [("type", C.c_int), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("D11", Field), ("D22", Field), ("v1", Field), ("v2", Field), ("f", Field),
                ("n_bc", C.c_int), ("bc_t", Tfun * MAXTERM), ("bc_s", Sfun * MAXTERM),
                ("n_src", C.c_int), ("src_t", Tfun * MAXTERM), ("src_c", C.c_double * MAXTERM),
                ("src_s", Sfun * MAXTERM)]


_libs = {}
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int)


def lib(extended=False):
    """The FP64 oracle, or with extended=True its long-double build."""
    key = bool(extended)
    if key not in _libs:
        build()
        L = C.CDLL(LIB_LD_PATH if key else LIB_PATH)
        GP, PP = C.POINTER(Grid), C.POINTER(Problem)
        sig = {
            "pdo_check": (C.c_int, [GP, PP]),
            "pdo_num_patches": (C.c_int, [GP]),
            "pdo_patch_map": (None, [GP, _IP]),
            "pdo_tables": (None, [GP, _DP]),
            "pdo_tables_size": (C.c_int, [GP]),
            "pdo_metric": (None, [GP, C.c_double, C.c_double, _DP]),
            "pdo_coeffs_at": (None, [GP, PP, C.c_double, C.c_double, _DP]),
            "pdo_coefficients": (None, [GP, PP, _DP]),
            "pdo_coefficients_masked": (None, [GP, PP, C.POINTER(C.c_ubyte), _DP]),
            "pdo_boundary_value": (C.c_double, [GP, PP, C.c_double, C.c_double, C.c_double]),
            "pdo_initial": (None, [GP, PP, C.c_double, _DP]),
            "pdo_edge": (None, [GP, _DP, _DP]),
            "pdo_lift": (None, [GP, _DP, _DP]),
            "pdo_burst": (C.c_int, [GP, PP, _DP, _DP, _DP, C.c_double, C.c_double, C.c_int]),
            "pdo_restrict": (None, [GP, _DP, _DP]),
            "pdo_macro_update": (None, [GP, PP, _DP, _DP, _DP, C.c_double, C.c_double,
                                        C.c_double]),
            "pdo_step": (C.c_int, [GP, PP, _DP, _DP, _DP, C.c_double, C.c_double, C.c_double,
                                   C.c_int, C.POINTER(C.c_ubyte)]),
            "pdo_solve": (C.c_int, [GP, PP, _DP, _DP, C.c_double, C.c_double, C.c_int,
                                    C.c_double, C.c_int]),
            "pdo_dt_micro_limit": (C.c_double, [GP, _DP, C.c_int]),
            "pdo_dt_macro_limit": (C.c_double, [GP, PP]),
            "pdo_full_domain": (C.c_int, [GP, PP, C.c_int, C.c_int, _DP, C.c_double,
                                          C.c_double, C.c_int]),
            "pdo_full_domain_point": (C.c_double, [GP, PP, C.c_int, C.c_int, _DP, C.c_double,
                                                   C.c_double, C.c_int, C.c_int]),
            "pdo_set_threads": (None, [C.c_int]),
            "pdo_get_threads": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _libs[key] = L
    return _libs[key]


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _field(d):
    F = Field()
    F.c0, F.cx, F.cy = d["c0"], d["cx"], d["cy"]
    F.nmode = len(d["modes"])
    assert F.nmode <= MAXMODE
    for k, (a, kx, ky, ph) in enumerate(d["modes"]):
        F.amp[k], F.kx[k], F.ky[k], F.ph[k] = a, kx, ky, ph
    F.npolar = len(d["polar"])
    assert F.npolar <= MAXPOLAR
    for k, (a, p0, p1, p2, n, ph) in enumerate(d["polar"]):
        F.pamp[k], F.pc0[k], F.pc1[k], F.pc2[k], F.pn[k], F.pph[k] = a, p0, p1, p2, n, ph
    return F


def _fn1(t):
    f = Fn1()
    f.type = FN[t[0]]
    vals = list(t[1:]) + [0.0] * (4 - len(t[1:]))
    f.a, f.b, f.c, f.d = vals
    return f


def _sfun(s):
    S = Sfun()
    S.kind = 0 if s[0] == "cart" else 1
    S.amp = s[1]
    S.f = _fn1(s[2])
    S.g = _fn1(s[3])
    return S


def _tfun(t):
    T = Tfun()
    T.type = TF[t[0]]
    vals = list(t[1:]) + [0.0] * (3 - len(t[1:]))
    T.a, T.b, T.c = vals
    return T


def make_grid(g):
    G = Grid()
    G.geometry = GEOM[g["geometry"]]
    G.gparam = g["gparam"]
    G.xi0, G.xi1, G.eta0, G.eta1 = g["xi0"], g["xi1"], g["eta0"], g["eta1"]
    G.n_xi, G.n_eta = g["n_xi"], g["n_eta"]
    G.periodic_xi = int(g["periodic_xi"])
    G.h_xi, G.h_eta = g["h_xi"], g["h_eta"]
    G.m_xi, G.m_eta = g["m_xi"], g["m_eta"]
    G.conv = CONV[g["conv"]]
    G.c0mode = C0[g["c0"]]
    G.core_points = int(g.get("core", 0))
    return G


def make_problem(p):
    P = Problem()
    fl = p["fields"]
    P.D11, P.D22, P.v1, P.v2, P.f = (_field(fl[k]) for k in ("D11", "D22", "v1", "v2", "f"))
    P.n_bc = len(p["bc"])
    for m, (t, s) in enumerate(p["bc"]):
        P.bc_t[m] = _tfun(t)
        P.bc_s[m] = _sfun(s)
    P.n_src = len(p["src"])
    for k, (t, c, s) in enumerate(p["src"]):
        P.src_t[k] = _tfun(t)
        P.src_c[k] = c
        P.src_s[k] = _sfun(s)
    return P


class Oracle:
    """The oracle on one problem dict (see ``paper_2405_08764_amd.workloads``)."""

    def __init__(self, prob, threads=1, extended=False):
        self.prob = prob
        self.L = lib(extended)
        self.g = make_grid(prob["grid"])
        self.p = make_problem(prob)
        self.G = C.byref(self.g)
        self.Pp = C.byref(self.p)
        rc = self.L.pdo_check(self.G, self.Pp)
        if rc != 0:
            raise ValueError("oracle rejects the problem (status %d)" % rc)
        self.L.pdo_set_threads(threads)
        gd = prob["grid"]
        self.nx, self.ne = gd["n_xi"], gd["n_eta"]
        self.mx, self.me = gd["m_xi"], gd["m_eta"]
        self.P = self.L.pdo_num_patches(self.G)
        self.M = max(self.mx, self.me)
        self.ncoef = 5 + len(prob["src"])
        self._coef = None

    # -- tables and maps
    def patch_map(self):
        out = np.zeros((self.P, 11), dtype=np.int32)
        self.L.pdo_patch_map(self.G, out.ctypes.data_as(_IP))
        return out

    def tables(self):
        out = np.zeros(self.L.pdo_tables_size(self.G))
        self.L.pdo_tables(self.G, _dp(out))
        return out

    def metric(self, xi, eta):
        out = np.zeros(16)
        self.L.pdo_metric(self.G, float(xi), float(eta), _dp(out))
        return out

    def coeffs_at(self, xi, eta):
        out = np.zeros(self.ncoef)
        self.L.pdo_coeffs_at(self.G, self.Pp, float(xi), float(eta), _dp(out))
        return out

    @property
    def coef(self):
        if self._coef is None:
            c = np.zeros((self.ncoef, self.P, self.me, self.mx))
            self.L.pdo_coefficients(self.G, self.Pp, _dp(c))
            self._coef = c
        return self._coef

    def coefficients_for(self, mask):
        """Fill the coefficient planes of the patches with mask[p] set only (zeros
        elsewhere): enough for steps restricted to those patches on a large grid."""
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mk.shape == (self.P,)
        c = np.zeros((self.ncoef, self.P, self.me, self.mx))
        self.L.pdo_coefficients_masked(self.G, self.Pp, mk.ctypes.data_as(C.POINTER(C.c_ubyte)),
                                       _dp(c))
        self._coef = c
        return c

    def boundary_value(self, xi, eta, t):
        return self.L.pdo_boundary_value(self.G, self.Pp, float(xi), float(eta), float(t))

    def initial(self, t=None):
        t = self.prob["time"]["t0"] if t is None else t
        U = np.zeros((self.ne, self.nx))
        self.L.pdo_initial(self.G, self.Pp, float(t), _dp(U))
        return U

    # -- the steps of one macro step
    def edge(self, U):
        e = np.zeros((self.P, 4, self.M))
        self.L.pdo_edge(self.G, _dp(np.ascontiguousarray(U, dtype=np.float64)), _dp(e))
        return e

    def lift(self, U):
        u = np.zeros((self.P, self.me, self.mx))
        self.L.pdo_lift(self.G, _dp(np.ascontiguousarray(U, dtype=np.float64)), _dp(u))
        return u

    def burst(self, u, e, t_n, dt, n_t):
        u = np.array(u, dtype=np.float64, order="C")
        rc = self.L.pdo_burst(self.G, self.Pp, _dp(self.coef), _dp(u),
                              _dp(np.ascontiguousarray(e)), float(t_n), float(dt), int(n_t))
        return u, rc

    def restrict(self, u):
        Ub = np.zeros(self.P)
        self.L.pdo_restrict(self.G, _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(Ub))
        return Ub

    def macro_update(self, Un, Ubar, t_n, Dt, tau):
        V = np.zeros((self.ne, self.nx))
        self.L.pdo_macro_update(self.G, self.Pp, _dp(np.ascontiguousarray(Un)),
                                _dp(np.ascontiguousarray(Ubar)), _dp(V), float(t_n),
                                float(Dt), float(tau))
        return V

    def step(self, U, t_n, Dt=None, dt=None, n_t=None, mask=None):
        t = self.prob["time"]
        Dt = t["dt_macro"] if Dt is None else Dt
        dt = t["dt_micro"] if dt is None else dt
        n_t = t["n_t"] if n_t is None else n_t
        V = np.zeros((self.ne, self.nx))
        mp = None
        if mask is not None:
            mk = np.ascontiguousarray(mask, dtype=np.uint8)
            mp = mk.ctypes.data_as(C.POINTER(C.c_ubyte))
        rc = self.L.pdo_step(self.G, self.Pp, _dp(self.coef),
                             _dp(np.ascontiguousarray(U, dtype=np.float64)), _dp(V),
                             float(t_n), float(Dt), float(dt), int(n_t), mp)
        if rc != 0:
            raise FloatingPointError("oracle step status %d" % rc)
        return V

    def step_refresh(self, U, t_n, n_refresh, Dt=None, dt=None, n_t=None):
        """One macro step with the edge data refreshed during the burst.  The paper fixes
        the edge gradients for the whole burst (Sec. 3.3 step (ii)) and names refreshing
        them as the refinement; the reading taken here: the n_t nano steps run as
        n_refresh sub-bursts (sub-burst q: nano steps n_t q // Q .. n_t (q + 1) // Q - 1,
        from t_n + (n_t q // Q) dt); before each later sub-burst every patch is restricted
        (eq. Restriction), the macro field takes those averages at the patch nodes and
        the Dirichlet data at the sub-burst's start time on the boundary nodes, and the
        eq. (edge) gradients are taken from that field.  Then restriction and projective
        step as in step()."""
        t = self.prob["time"]
        Dt = t["dt_macro"] if Dt is None else Dt
        dt = t["dt_micro"] if dt is None else dt
        n_t = t["n_t"] if n_t is None else n_t
        U = np.array(U, dtype=np.float64, order="C")
        e = self.edge(U)
        u = self.lift(U)
        nodes = self.patch_map()[:, 6]
        bnd = np.ones(U.size, dtype=bool)
        bnd[nodes] = False
        xi, eta = self.node_coords()
        jj, ii = np.divmod(np.nonzero(bnd)[0], self.nx)
        for q in range(n_refresh):
            s0, s1 = n_t * q // n_refresh, n_t * (q + 1) // n_refresh
            u, rc = self.burst(u, e, t_n + s0 * dt, dt, s1 - s0)
            if rc != 0:
                raise FloatingPointError("oracle burst status %d" % rc)
            if q + 1 < n_refresh:
                W = np.empty(U.size)
                W[nodes] = self.restrict(u)
                for j, i in zip(jj, ii):
                    W[j * self.nx + i] = self.boundary_value(xi[i], eta[j], t_n + s1 * dt)
                e = self.edge(W.reshape(U.shape))
        return self.macro_update(U, self.restrict(u), t_n, Dt, n_t * dt)

    def solve(self, U=None, n_steps=None, t0=None):
        t = self.prob["time"]
        U = self.initial() if U is None else np.array(U, dtype=np.float64, order="C")
        n_steps = t["n_steps"] if n_steps is None else n_steps
        t0 = t["t0"] if t0 is None else t0
        rc = self.L.pdo_solve(self.G, self.Pp, _dp(self.coef), _dp(U), float(t0),
                              float(t["dt_macro"]), int(n_steps), float(t["dt_micro"]),
                              int(t["n_t"]))
        if rc != 0:
            raise FloatingPointError("oracle solve status %d" % rc)
        return U

    def dt_micro_limit(self):
        return self.L.pdo_dt_micro_limit(self.G, _dp(self.coef), self.ncoef)

    def dt_macro_limit(self):
        return self.L.pdo_dt_macro_limit(self.G, self.Pp)

    def full_domain(self, n_x, n_y, U, t0, dt, n_steps):
        U = np.array(U, dtype=np.float64, order="C")
        rc = self.L.pdo_full_domain(self.G, self.Pp, int(n_x), int(n_y), _dp(U), float(t0),
                                    float(dt), int(n_steps))
        if rc != 0:
            raise FloatingPointError("oracle full-domain status %d" % rc)
        return U

    def full_domain_point(self, n_x, n_y, U, t, dt, i, j):
        U = np.ascontiguousarray(U, dtype=np.float64)
        return self.L.pdo_full_domain_point(self.G, self.Pp, int(n_x), int(n_y), _dp(U),
                                            float(t), float(dt), int(i), int(j))

    def full_domain_limit(self, n_x, n_y):
        """Explicit forward-Euler bound over the lattice nodes (the same 5-point bound as
        the micro limit, at the lattice spacing)."""
        gd = self.prob["grid"]
        hx = (gd["xi1"] - gd["xi0"]) / (n_x if gd["periodic_xi"] else n_x - 1)
        hy = (gd["eta1"] - gd["eta0"]) / (n_y - 1)
        lim = math.inf
        for j in range(n_y):
            for i in range(n_x):
                c = self.coeffs_at(gd["xi0"] + i * hx, gd["eta0"] + j * hy)
                b = 1.0 / (2 * c[0] / hx ** 2 + 2 * c[1] / hy ** 2 + abs(c[2]) / hx
                           + abs(c[3]) / hy + abs(c[4]))
                lim = min(lim, b)
        return lim

    # -- helpers
    def node_coords(self):
        gd = self.prob["grid"]
        d_xi = (gd["xi1"] - gd["xi0"]) / (self.nx if gd["periodic_xi"] else self.nx - 1)
        d_eta = (gd["eta1"] - gd["eta0"]) / (self.ne - 1)
        xi = gd["xi0"] + np.arange(self.nx) * d_xi
        eta = gd["eta0"] + np.arange(self.ne) * d_eta
        return xi, eta

    def patch_mask(self):
        """Boolean [n_eta, n_xi] of the nodes that carry a patch."""
        m = np.zeros((self.ne, self.nx), dtype=bool)
        pm = self.patch_map()
        m[pm[:, 1], pm[:, 0]] = True
        return m


def timed_steps(orc, U, n_steps, t0=0.0):
    """Run n_steps oracle macro steps; return (U, seconds)."""
    t = orc.prob["time"]
    s = time.perf_counter()
    for k in range(n_steps):
        U = orc.step(U, t0 + k * t["dt_macro"])
    return U, time.perf_counter() - s
