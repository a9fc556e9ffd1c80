"""Thin ctypes binding of libpd.so (include/pd.h) with the same call names.

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch provides device memory and streams.  Loading fails loudly when the library has not
been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpd.so")

MAXMODE, MAXPOLAR, MAXTERM = 16, 4, 4
GEOM = {"identity": 0, "sine": 1, "tanh": 2, "annulus": 3}
CONV = {"upwind": 0, "central": 1}
C0MODE = {"trapezoid": 0, "printed": 1}
PREC = {"f64": 0, "f32": 1}
FN = {"sin": 0, "cos": 1, "exp": 2, "poly": 3}
TF = {"const": 0, "exp": 1, "sin": 2}
OPT_ALLOW_UNSTABLE, OPT_ROWS_PER_LANE, OPT_PATCHES_PER_BLOCK, OPT_BLOCK_THREADS = 1, 2, 3, 4
OPT_COLS_PER_LANE, OPT_EXCHANGE, OPT_RESIDENT_SOLVE = 5, 6, 7
TUNE_FORCE = 1

STATUS = {0: "PD_OK", -1: "PD_EINVAL", -2: "PD_ESTATE", -3: "PD_EUNSTABLE", -4: "PD_EDEVICE",
          -5: "PD_ENONFINITE", -6: "PD_ENOMEM"}


class PdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("gparam", C.c_double), ("xi0", C.c_double),
                ("xi1", C.c_double), ("eta0", C.c_double), ("eta1", C.c_double),
                ("n_xi", C.c_int32), ("n_eta", C.c_int32), ("periodic_xi", C.c_int32),
                ("h_xi", C.c_double), ("h_eta", C.c_double), ("m_xi", C.c_int32),
                ("m_eta", C.c_int32), ("conv", C.c_int32), ("c0mode", C.c_int32),
                ("precision", C.c_int32), ("device", C.c_int32), ("max_sources", C.c_int32),
                ("core_points", C.c_int32)]


class Field(C.Structure):
    _fields_ = [("c0", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("nmode", C.c_int32), ("amp", C.c_double * MAXMODE),
                ("kx", C.c_double * MAXMODE), ("ky", C.c_double * MAXMODE),
                ("ph", C.c_double * MAXMODE), ("npolar", C.c_int32),
                ("pamp", C.c_double * MAXPOLAR), ("pc0", C.c_double * MAXPOLAR),
                ("pc1", C.c_double * MAXPOLAR), ("pc2", C.c_double * MAXPOLAR),
                ("pn", C.c_double * MAXPOLAR), ("pph", C.c_double * MAXPOLAR)]


class Fn1(C.Structure):
    _fields_ = [("type", C.c_int32), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("d", C.c_double)]


class Sfun(C.Structure):
    _fields_ = [("kind", C.c_int32), ("amp", C.c_double), ("f", Fn1), ("g", Fn1)]


class Tfun(C.Structure):
    _fields_ = [("type", C.c_int32), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double)]


class CoeffDesc(C.Structure):
    _fields_ = [("D11", Field), ("D22", Field), ("v1", Field), ("v2", Field), ("f", Field),
                ("n_bc", C.c_int32), ("bc_t", Tfun * MAXTERM), ("bc_s", Sfun * MAXTERM),
                ("n_src", C.c_int32), ("src_t", Tfun * MAXTERM),
                ("src_c", C.c_double * MAXTERM), ("src_s", Sfun * MAXTERM)]


class Info(C.Structure):
    _fields_ = [("n_patches", C.c_int32), ("m_xi", C.c_int32), ("m_eta", C.c_int32),
                ("n_xi", C.c_int32), ("n_eta", C.c_int32), ("n_points", C.c_int64),
                ("workspace_bytes", C.c_size_t), ("dt_micro_limit", C.c_double),
                ("dt_macro_limit", C.c_double), ("coefficients_set", C.c_int32),
                ("n_time_sources", C.c_int32), ("rows_per_lane", C.c_int32),
                ("patches_per_block", C.c_int32), ("block_threads", C.c_int32),
                ("cols_per_lane", C.c_int32), ("exchange", C.c_int32),
                ("tuned", C.c_int32), ("tuned_ms", C.c_double),
                ("resident_solve", C.c_int32), ("resident_refresh", C.c_int32)]


class BatchMember(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("U", C.c_void_p), ("t0", C.c_double),
                ("dt_macro", C.c_double), ("dt_micro", C.c_double), ("n_t", C.c_int32)]


class BatchInfo(C.Structure):
    _fields_ = [("n_members", C.c_int32), ("n_items", C.c_int32), ("blocks", C.c_int32),
                ("time_sources", C.c_int32), ("workspace_bytes", C.c_size_t),
                ("lds_bytes", C.c_size_t), ("tuned", C.c_int32), ("tuned_ms", C.c_double),
                ("updates_per_step", C.c_int64)]


class FdInfo(C.Structure):
    _fields_ = [("n_x", C.c_int32), ("n_y", C.c_int32), ("workspace_bytes", C.c_size_t),
                ("dt_limit", C.c_double), ("dt", C.c_double), ("spacing_x", C.c_double),
                ("spacing_y", C.c_double)]


EXPORTS = {
    "pd_create_grid": (C.c_int32, [C.POINTER(GridDesc), C.POINTER(C.c_void_p)]),
    "pd_destroy_grid": (C.c_int32, [C.c_void_p]),
    "pd_query": (C.c_int32, [C.c_void_p, C.POINTER(Info)]),
    "pd_bind_workspace": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pd_set_coefficients": (C.c_int32, [C.c_void_p, C.POINTER(CoeffDesc), C.c_void_p]),
    "pd_initial": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "pd_lift_bc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pd_micro_burst": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                   C.c_int32, C.c_void_p]),
    "pd_micro_burst_adi": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                       C.c_double, C.c_int32, C.c_void_p]),
    "pd_micro_burst_upwind": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                          C.c_double, C.c_int32, C.c_int32, C.c_double,
                                          C.c_void_p]),
    "pd_micro_burst_adi_upwind": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                              C.c_double, C.c_int32, C.c_int32, C.c_double,
                                              C.c_void_p]),
    "pd_restrict": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pd_macro_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                  C.c_double, C.c_int32, C.c_void_p, C.c_void_p]),
    "pd_macro_step_refresh": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                          C.c_double, C.c_double, C.c_int32, C.c_int32,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p]),
    "pd_patch_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                  C.c_double, C.c_int32, C.c_void_p]),
    "pd_apply_boundary": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "pd_solve": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int32,
                             C.c_double, C.c_int32, C.c_void_p]),
    "pd_sync": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pd_get_patch_map": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pd_get_tables_size": (C.c_int32, [C.c_void_p]),
    "pd_get_tables": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pd_copy_coefficients": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pd_set_option": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int64]),
    "pd_autotune": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                                C.c_int32, C.c_int32, C.c_uint32, C.POINTER(C.c_double),
                                C.c_void_p]),
    "pd_batch_create": (C.c_int32, [C.POINTER(BatchMember), C.c_int32, C.POINTER(C.c_void_p)]),
    "pd_batch_destroy": (C.c_int32, [C.c_void_p]),
    "pd_batch_query": (C.c_int32, [C.c_void_p, C.POINTER(BatchInfo)]),
    "pd_batch_bind_workspace": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pd_batch_get_shape": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]),
    "pd_batch_set_shape": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32]),
    "pd_batch_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                      C.c_void_p]),
    "pd_batch_solve": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "pd_batch_sync": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pd_closure_create": (C.c_int32, [C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]),
    "pd_closure_destroy": (C.c_int32, [C.c_void_p]),
    "pd_closure_query": (C.c_int32, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_int32)]),
    "pd_closure_bind_workspace": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pd_closure_set_params": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pd_closure_get_params": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pd_closure_set_standardisation": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pd_closure_get_standardisation": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pd_closure_fit_standardisation": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p,
                                                   C.c_int64, C.c_void_p]),
    "pd_closure_set_target_scale": (C.c_int32, [C.c_void_p, C.c_float, C.c_float]),
    "pd_closure_get_target_scale": (C.c_int32, [C.c_void_p, C.POINTER(C.c_float),
                                                C.POINTER(C.c_float)]),
    "pd_closure_features": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p]),
    "pd_closure_targets": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                       C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pd_closure_gradients": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                         C.c_void_p, C.c_void_p, C.c_void_p]),
    "pd_closure_gradients_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p,
                                                 C.c_int32, C.c_void_p, C.c_void_p,
                                                 C.c_void_p]),
    "pd_noalloc_scratch_bytes": (C.c_size_t, []),
    "pd_closure_train": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                     C.c_int32, C.c_float, C.c_uint32, C.c_void_p,
                                     C.c_void_p]),
    "pd_closure_infer": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.c_void_p]),
    "pd_closure_patch_step": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "pd_batch_closure_bytes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "pd_batch_closure_attach": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                            C.c_void_p, C.c_size_t]),
    "pd_batch_closure_solve": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "pd_batch_closure_stats": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64),
                                           C.POINTER(C.c_int64), C.c_int32]),
    "pd_fd_create": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]),
    "pd_fd_destroy": (C.c_int32, [C.c_void_p]),
    "pd_fd_query": (C.c_int32, [C.c_void_p, C.POINTER(FdInfo)]),
    "pd_fd_bind_workspace": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pd_fd_prepare": (C.c_int32, [C.c_void_p, C.c_double, C.c_void_p]),
    "pd_fd_initial": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "pd_fd_solve": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p]),
    "pd_fd_sync": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "pd_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load libpd.so; raises if it was not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2405_08764_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise PdError(status, lib().pd_last_error().decode())


def _ptr(t, numel=0, dtype=torch.float64, device=None, name="tensor"):
    """Device address of t for the C ABI, after the checks the ABI cannot make itself: it
    takes raw pointers without lengths, so a host tensor, another dtype, a strided view,
    a buffer shorter than the call's layout or a tensor on another device would become an
    out-of-bounds device access.  Raises PdError (PD_EINVAL) before any library call.
    The checks run type, dtype, layout, length, then placement, so each is reachable
    with host tensors too."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise PdError(-1, f"{name}: expected a torch tensor, got {type(t).__name__}")
    if dtype is not None and t.dtype != dtype:
        raise PdError(-1, f"{name}: dtype {t.dtype}, the call needs {dtype}")
    if not t.is_contiguous():
        raise PdError(-1, f"{name}: must be contiguous")
    if t.numel() < numel:
        raise PdError(-1, f"{name}: {t.numel()} elements, the call's layout needs {numel}")
    if not t.is_cuda:
        raise PdError(-1, f"{name}: must be a device tensor, got one on {t.device}")
    if device is not None and t.device != device:
        raise PdError(-1, f"{name}: on {t.device}, the handle lives on {device}")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None and not torch.cuda.is_available():
        return C.c_void_p(0)
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _field(d):
    F = Field()
    F.c0, F.cx, F.cy = d["c0"], d["cx"], d["cy"]
    F.nmode = len(d["modes"])
    for k, (a, kx, ky, ph) in enumerate(d["modes"]):
        F.amp[k], F.kx[k], F.ky[k], F.ph[k] = a, kx, ky, ph
    F.npolar = len(d["polar"])
    for k, (a, p0, p1, p2, n, ph) in enumerate(d["polar"]):
        F.pamp[k], F.pc0[k], F.pc1[k], F.pc2[k], F.pn[k], F.pph[k] = a, p0, p1, p2, n, ph
    return F


def _fn1(t):
    f = Fn1()
    f.type = FN[t[0]]
    v = list(t[1:]) + [0.0] * (4 - len(t) + 1)
    f.a, f.b, f.c, f.d = v[:4]
    return f


def _sfun(s):
    S = Sfun()
    S.kind = 0 if s[0] == "cart" else 1
    S.amp = s[1]
    S.f, S.g = _fn1(s[2]), _fn1(s[3])
    return S


def _tfun(t):
    T = Tfun()
    T.type = TF[t[0]]
    v = list(t[1:]) + [0.0] * (3 - len(t) + 1)
    T.a, T.b, T.c = v[:3]
    return T


def grid_desc(g, precision="f64", device=0, max_sources=0):
    D = GridDesc()
    D.geometry = GEOM[g["geometry"]]
    D.gparam = g["gparam"]
    D.xi0, D.xi1, D.eta0, D.eta1 = g["xi0"], g["xi1"], g["eta0"], g["eta1"]
    D.n_xi, D.n_eta = g["n_xi"], g["n_eta"]
    D.periodic_xi = int(g["periodic_xi"])
    D.h_xi, D.h_eta = g["h_xi"], g["h_eta"]
    D.m_xi, D.m_eta = g["m_xi"], g["m_eta"]
    D.conv = CONV[g["conv"]]
    D.c0mode = C0MODE[g["c0"]]
    D.precision = PREC[precision]
    D.device = device
    D.max_sources = max_sources
    D.core_points = int(g.get("core", 0))
    return D


def coeff_desc(prob):
    Cd = CoeffDesc()
    fl = prob["fields"]
    Cd.D11, Cd.D22, Cd.v1, Cd.v2, Cd.f = (_field(fl[k]) for k in ("D11", "D22", "v1", "v2", "f"))
    Cd.n_bc = len(prob["bc"])
    for m, (t, s) in enumerate(prob["bc"]):
        Cd.bc_t[m], Cd.bc_s[m] = _tfun(t), _sfun(s)
    Cd.n_src = len(prob["src"])
    for k, (t, c, s) in enumerate(prob["src"]):
        Cd.src_t[k], Cd.src_c[k], Cd.src_s[k] = _tfun(t), c, _sfun(s)
    return Cd


class Grid:
    """One problem on one device: grid, workspace (a torch uint8 tensor) and coefficients.

    Method names follow the C ABI (pd_lift_bc -> lift_bc, ...).  Tensors are float64 on
    the grid's device; calls run on the current torch stream.
    """

    def __init__(self, prob, precision="f64", device=0, coefficients=True):
        self.prob = prob
        self.L = lib()
        self.device = torch.device("cuda", device) if torch.cuda.is_available() else None
        self.h = C.c_void_p()
        desc = grid_desc(prob["grid"], precision, device, max_sources=max(1, len(prob["src"])))
        _check(self.L.pd_create_grid(C.byref(desc),
                                     C.byref(self.h)))
        self.info = self.query()
        self.P = self.info.n_patches
        self.mx, self.me = self.info.m_xi, self.info.m_eta
        self.nx, self.ne = self.info.n_xi, self.info.n_eta
        self.M = max(self.mx, self.me)
        self.ws = None
        if coefficients:
            self.bind()
            self.set_coefficients()

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            self.L.pd_destroy_grid(self.h)
            self.h = C.c_void_p()

    def query(self):
        I = Info()
        _check(self.L.pd_query(self.h, C.byref(I)))
        return I

    def bind(self):
        n = self.info.workspace_bytes
        self.ws = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        _check(self.L.pd_bind_workspace(self.h, C.c_void_p(aligned), n))

    def set_coefficients(self, prob=None, stream=None):
        self._cd = coeff_desc(prob or self.prob)
        _check(self.L.pd_set_coefficients(self.h, C.byref(self._cd), _stream(stream)))
        self.info = self.query()

    # -- checked device pointers of the call layouts (include/pd.h)
    def _U(self, t, name="U"):
        return _ptr(t, self.ne * self.nx, torch.float64, self.device, name)

    def _state(self, t, name="patch_state"):
        return _ptr(t, self.P * self.me * self.mx, torch.float64, self.device, name)

    def _edge(self, t, name="edge"):
        return _ptr(t, self.P * 4 * self.M, torch.float64, self.device, name)

    def _perpatch(self, t, name="Ubar"):
        return _ptr(t, self.P, torch.float64, self.device, name)

    def set_option(self, option, value):
        _check(self.L.pd_set_option(self.h, option, int(value)))
        self.info = self.query()

    # -- host-side tables
    def patch_map(self):
        out = torch.zeros((self.P, 11), dtype=torch.int32)
        _check(self.L.pd_get_patch_map(self.h, C.c_void_p(out.data_ptr())))
        return out

    def tables(self):
        out = torch.zeros(self.L.pd_get_tables_size(self.h), dtype=torch.float64)
        _check(self.L.pd_get_tables(self.h, C.c_void_p(out.data_ptr())))
        return out

    def coefficients(self):
        nc = 5 + len(self.prob["src"])
        out = torch.empty((nc, self.P, self.me, self.mx), dtype=torch.float64, device=self.device)
        _check(self.L.pd_copy_coefficients(
            self.h, _ptr(out, nc * self.P * self.me * self.mx, torch.float64, self.device,
                         "coefficients"), _stream()))
        return out

    # -- the steps
    def new_U(self):
        return torch.zeros((self.ne, self.nx), dtype=torch.float64, device=self.device)

    def initial(self, t=None, U=None):
        U = self.new_U() if U is None else U
        t = self.prob["time"]["t0"] if t is None else t
        _check(self.L.pd_initial(self.h, self._U(U), float(t), _stream()))
        return U

    def lift_bc(self, U):
        state = torch.empty((self.P, self.me, self.mx), dtype=torch.float64, device=self.device)
        edge = torch.empty((self.P, 4, self.M), dtype=torch.float64, device=self.device)
        _check(self.L.pd_lift_bc(self.h, self._U(U), self._state(state), self._edge(edge),
                                 _stream()))
        return state, edge

    def micro_burst(self, state, edge, t_n, dt, n_t):
        _check(self.L.pd_micro_burst(self.h, self._state(state), self._edge(edge), float(t_n),
                                     float(dt),
                                     int(n_t), _stream()))
        return state

    def micro_burst_adi(self, state, edge, t_n, dt, n_t):
        _check(self.L.pd_micro_burst_adi(self.h, self._state(state), self._edge(edge), float(t_n),
                                         float(dt),
                                         int(n_t), _stream()))
        return state

    def micro_burst_upwind(self, state, edge, t_n, dt, n_t, points=3, r=0.5):
        _check(self.L.pd_micro_burst_upwind(self.h, self._state(state), self._edge(edge), float(t_n),
                                            float(dt), int(n_t), int(points), float(r),
                                            _stream()))
        return state

    def micro_burst_adi_upwind(self, state, edge, t_n, dt, n_t, points=3, r=0.5):
        _check(self.L.pd_micro_burst_adi_upwind(self.h, self._state(state), self._edge(edge),
                                                float(t_n), float(dt), int(n_t), int(points),
                                                float(r), _stream()))
        return state

    def restrict(self, state):
        Ub = torch.empty(self.P, dtype=torch.float64, device=self.device)
        _check(self.L.pd_restrict(self.h, self._state(state), self._perpatch(Ub), _stream()))
        return Ub

    def macro_step(self, U_n, t_n, dt_macro=None, dt_micro=None, n_t=None, Ubar=None,
                   out=None):
        t = self.prob["time"]
        dt_macro = t["dt_macro"] if dt_macro is None else dt_macro
        dt_micro = t["dt_micro"] if dt_micro is None else dt_micro
        n_t = t["n_t"] if n_t is None else n_t
        out = self.new_U() if out is None else out
        _check(self.L.pd_macro_step(self.h, self._U(U_n, "U_n"), self._U(out, "U_np1"), float(t_n),
                                    float(dt_macro), float(dt_micro), int(n_t),
                                    self._perpatch(Ubar), _stream()))
        return out

    def macro_step_refresh(self, U_n, t_n, n_refresh, dt_macro=None, dt_micro=None, n_t=None,
                           out=None):
        """pd_macro_step_refresh: the burst split into n_refresh sub-bursts with the edge
        data recomputed between them (work buffers are kept on the grid object)."""
        t = self.prob["time"]
        dt_macro = t["dt_macro"] if dt_macro is None else dt_macro
        dt_micro = t["dt_micro"] if dt_micro is None else dt_micro
        n_t = t["n_t"] if n_t is None else n_t
        out = self.new_U() if out is None else out
        if getattr(self, "_refresh_bufs", None) is None:
            f64 = dict(dtype=torch.float64, device=self.device)
            self._refresh_bufs = (torch.empty((self.P, self.me, self.mx), **f64),
                                  torch.empty((self.P, 4, self.M), **f64),
                                  torch.empty((self.P,), **f64), self.new_U())
        st, ed, ub, uw = self._refresh_bufs
        _check(self.L.pd_macro_step_refresh(self.h, self._U(U_n, "U_n"), self._U(out, "U_np1"),
                                            float(t_n), float(dt_macro), float(dt_micro),
                                            int(n_t), int(n_refresh), self._state(st),
                                            self._edge(ed), self._perpatch(ub),
                                            self._U(uw, "U_work"), _stream()))
        return out

    def patch_step(self, U_n, t_n, out, dt_macro=None, dt_micro=None, n_t=None):
        t = self.prob["time"]
        _check(self.L.pd_patch_step(
            self.h, self._U(U_n, "U_n"), self._U(out, "U_np1"), float(t_n),
            float(t["dt_macro"] if dt_macro is None else dt_macro),
            float(t["dt_micro"] if dt_micro is None else dt_micro),
            int(t["n_t"] if n_t is None else n_t), _stream()))
        return out

    def autotune(self, U=None, t_n=None, reps=5, force=False, dt_macro=None, dt_micro=None,
                 n_t=None):
        """Time every allowed launch shape of the fused step and keep the fastest; returns
        the measured ms per step."""
        t = self.prob["time"]
        U = self.initial() if U is None else U
        best = C.c_double(0.0)
        _check(self.L.pd_autotune(
            self.h, self._U(U), float(t["t0"] if t_n is None else t_n),
            float(t["dt_macro"] if dt_macro is None else dt_macro),
            float(t["dt_micro"] if dt_micro is None else dt_micro),
            int(t["n_t"] if n_t is None else n_t), int(reps), TUNE_FORCE if force else 0,
            C.byref(best), _stream()))
        return best.value

    def apply_boundary(self, U, t):
        _check(self.L.pd_apply_boundary(self.h, self._U(U), float(t), _stream()))
        return U

    def solve(self, U=None, n_steps=None, t0=None, dt_macro=None, dt_micro=None, n_t=None):
        t = self.prob["time"]
        U = self.initial() if U is None else U
        _check(self.L.pd_solve(self.h, self._U(U), float(t["t0"] if t0 is None else t0),
                               float(t["dt_macro"] if dt_macro is None else dt_macro),
                               int(t["n_steps"] if n_steps is None else n_steps),
                               float(t["dt_micro"] if dt_micro is None else dt_micro),
                               int(t["n_t"] if n_t is None else n_t), _stream()))
        return U

    def sync(self):
        _check(self.L.pd_sync(self.h, _stream()))


class Batch:
    """Independent grids advanced together by the persistent batch kernel (pd_batch_*).

    grids: Grid objects (FP64, coefficients set); Us: their macro fields (default: each
    grid's initial data).  Time parameters come from each grid's problem description.
    The Grid objects are kept alive with the batch (their workspaces are in use).
    """

    def __init__(self, grids, Us=None):
        self.L = lib()
        self.grids = list(grids)
        self.U = [g.initial() for g in self.grids] if Us is None else list(Us)
        n = len(self.grids)
        arr = (BatchMember * n)()
        for i, (g, U) in enumerate(zip(self.grids, self.U)):
            t = g.prob["time"]
            g._U(U, f"U of member {i}")
            arr[i] = BatchMember(g.h.value, U.data_ptr(), float(t["t0"]), float(t["dt_macro"]),
                                 float(t["dt_micro"]), int(t["n_t"]))
        self.h = C.c_void_p()
        _check(self.L.pd_batch_create(arr, n, C.byref(self.h)))
        need = self.query().workspace_bytes
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.grids[0].device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        _check(self.L.pd_batch_bind_workspace(self.h, C.c_void_p(base + off), need))

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            self.L.pd_batch_destroy(self.h)
            self.h = C.c_void_p()

    def query(self):
        info = BatchInfo()
        _check(self.L.pd_batch_query(self.h, C.byref(info)))
        return info

    def shape(self, i):
        s, p = C.c_int32(), C.c_int32()
        _check(self.L.pd_batch_get_shape(self.h, i, C.byref(s), C.byref(p)))
        return s.value, p.value

    def set_shape(self, i, shape):
        _check(self.L.pd_batch_set_shape(self.h, i, int(shape)))

    def autotune(self, reps=3):
        best = C.c_double(0.0)
        _check(self.L.pd_batch_autotune(self.h, int(reps), C.byref(best), _stream()))
        return best.value

    def solve(self, n_steps):
        _check(self.L.pd_batch_solve(self.h, int(n_steps), _stream()))
        return self.U

    def sync(self):
        _check(self.L.pd_batch_sync(self.h, _stream()))

    def attach_closure(self, closure, stride=100, threshold=1.0):
        """Use `closure` for closure_solve, checking one item in `stride` per member and
        step and falling back to the plain scheme above `threshold`."""
        nbytes = C.c_size_t()
        _check(self.L.pd_batch_closure_bytes(self.h, C.byref(nbytes)))
        self.cl_ws = torch.empty(nbytes.value + 256, dtype=torch.uint8,
                                 device=self.grids[0].device)
        base = self.cl_ws.data_ptr()
        _check(self.L.pd_batch_closure_attach(self.h, closure.h, int(stride), float(threshold),
                                              C.c_void_p(base + (-base) % 256), nbytes.value))
        self.closure = closure

    def closure_solve(self, n_steps):
        _check(self.L.pd_batch_closure_solve(self.h, int(n_steps), _stream()))
        return self.U

    def closure_stats(self, reset=False):
        a, b = C.c_int64(), C.c_int64()
        _check(self.L.pd_batch_closure_stats(self.h, C.byref(a), C.byref(b), int(reset)))
        return a.value, b.value


BATCH_MENU = [(2, 1, 3), (2, 1, 5), (2, 1, 6), (2, 1, 7), (2, 2, 3), (1, 1, 5), (1, 2, 3),
              (1, 3, 2), (1, 4, 2), (3, 2, 4), (3, 3, 2),
              (3, 2, 3)]  # (exchange, columns, rows) of the batch kernel's menu, by index


class FullDomain:
    """The full-domain lattice of a grid's problem (pd_fd_*): forward Euler with the
    bursts' differences on one n_x x n_y lattice over the whole box."""

    def __init__(self, grid, n_x, n_y, dt=None, frac=0.5):
        self.L = lib()
        self.grid = grid  # kept alive: the lattice uses its problem
        self.h = C.c_void_p()
        _check(self.L.pd_fd_create(grid.h, int(n_x), int(n_y), C.byref(self.h)))
        need = self.query().workspace_bytes
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=grid.device)
        base = self.ws.data_ptr()
        _check(self.L.pd_fd_bind_workspace(self.h, C.c_void_p(base + (-base) % 256), need))
        self.n_x, self.n_y = int(n_x), int(n_y)
        if dt is None:
            self.prepare(1e-300)  # any positive step: the call reports the bound
            dt = frac * self.query().dt_limit
        self.prepare(dt)

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            self.L.pd_fd_destroy(self.h)
            self.h = C.c_void_p()

    def query(self):
        info = FdInfo()
        _check(self.L.pd_fd_query(self.h, C.byref(info)))
        return info

    def prepare(self, dt, stream=None):
        _check(self.L.pd_fd_prepare(self.h, float(dt), _stream(stream)))

    @property
    def dt(self):
        return self.query().dt

    def new_U(self):
        return torch.empty((self.n_y, self.n_x), dtype=torch.float64, device=self.grid.device)

    def initial(self, t=0.0, U=None, stream=None):
        U = self.new_U() if U is None else U
        _check(self.L.pd_fd_initial(self.h, self._U(U), float(t), _stream(stream)))
        return U

    def solve(self, U, t0, n_steps, stream=None):
        _check(self.L.pd_fd_solve(self.h, self._U(U), float(t0), int(n_steps),
                                  _stream(stream)))
        return U

    def sync(self, stream=None):
        _check(self.L.pd_fd_sync(self.h, _stream(stream)))

    def _U(self, t, name="U"):
        return _ptr(t, self.n_y * self.n_x, torch.float64, self.grid.device, name)


N_FEAT, N_PARAMS = 33, 20993
NOALLOC_MAX_ROWS = 4096  # PD_NOALLOC_MAX_ROWS of include/pd.h


class Closure:
    """The learned closure's device state (pd_closure_*): parameters, optimiser moments,
    standardisation, packed bfloat16 weights and training scratch in one workspace."""

    def __init__(self, device=0, max_batch=8192):
        import numpy as np
        self.L = lib()
        self.device = torch.device("cuda", device)
        self.h = C.c_void_p()
        _check(self.L.pd_closure_create(device, max_batch, C.byref(self.h)))
        nbytes = C.c_size_t()
        _check(self.L.pd_closure_query(self.h, C.byref(nbytes), None))
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        _check(self.L.pd_closure_bind_workspace(self.h, C.c_void_p(base + (-base) % 256),
                                                nbytes.value))
        self.max_batch = max_batch
        self._np = np

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            self.L.pd_closure_destroy(self.h)
            self.h = C.c_void_p()

    def _X(self, t, n, name="X"):
        return _ptr(t, n * N_FEAT, torch.float32, self.device, name)

    def _y(self, t, n, name="y"):
        return _ptr(t, n, torch.float32, self.device, name)

    def set_params(self, flat):
        a = self._np.ascontiguousarray(flat, dtype=self._np.float32)
        assert a.size == N_PARAMS
        _check(self.L.pd_closure_set_params(self.h, a.ctypes.data_as(C.c_void_p)))

    def params(self):
        a = self._np.zeros(N_PARAMS, dtype=self._np.float32)
        _check(self.L.pd_closure_get_params(self.h, a.ctypes.data_as(C.c_void_p)))
        return a

    def set_standardisation(self, mu, sd):
        m = self._np.ascontiguousarray(mu, dtype=self._np.float32)
        d = self._np.ascontiguousarray(sd, dtype=self._np.float32)
        _check(self.L.pd_closure_set_standardisation(self.h, m.ctypes.data_as(C.c_void_p),
                                                     d.ctypes.data_as(C.c_void_p)))

    def standardisation(self):
        m = self._np.zeros(N_FEAT, dtype=self._np.float32)
        d = self._np.zeros(N_FEAT, dtype=self._np.float32)
        _check(self.L.pd_closure_get_standardisation(self.h, m.ctypes.data_as(C.c_void_p),
                                                     d.ctypes.data_as(C.c_void_p)))
        return m, d

    def fit_standardisation(self, X, y=None):
        n = X.shape[0]
        _check(self.L.pd_closure_fit_standardisation(self.h, self._X(X, n), self._y(y, n), n,
                                                     _stream()))

    def set_target_scale(self, mean, sd):
        _check(self.L.pd_closure_set_target_scale(self.h, float(mean), float(sd)))

    def target_scale(self):
        m, s = C.c_float(), C.c_float()
        _check(self.L.pd_closure_get_target_scale(self.h, C.byref(m), C.byref(s)))
        return m.value, s.value

    def gradients(self, X, y):
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        n = X.shape[0]
        _check(self.L.pd_closure_gradients(self.h, self._X(X, n), self._y(y, n), n,
                                           self._y(g, N_PARAMS, "grad"),
                                           self._y(loss, 1, "loss"), _stream()))
        return g, loss

    def gradients_noalloc(self, X, y, grad, loss):
        """pd_closure_gradients_noalloc into the caller's grad [N_PARAMS] and loss [1]
        (FP32 device tensors); at most NOALLOC_MAX_ROWS rows."""
        n = X.shape[0]
        _check(self.L.pd_closure_gradients_noalloc(self.h, self._X(X, n), self._y(y, n), n,
                                                   self._y(grad, N_PARAMS, "grad"),
                                                   self._y(loss, 1, "loss"), _stream()))
        return grad, loss

    def train(self, X, y, batch=4096, epochs=1, lr=1e-3, seed=0):
        losses = self._np.zeros(max(epochs, 1), dtype=self._np.float32)
        n = X.shape[0]
        _check(self.L.pd_closure_train(self.h, self._X(X, n), self._y(y, n), n, batch, epochs,
                                       float(lr), seed, losses.ctypes.data_as(C.c_void_p),
                                       _stream()))
        return losses[:epochs]

    def infer(self, X):
        out = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        n = X.shape[0]
        _check(self.L.pd_closure_infer(self.h, self._X(X, n), self._y(out, n, "out"), n,
                                       _stream()))
        return out

    @staticmethod
    def features(grid, U, t_n):
        X = torch.empty((grid.P, N_FEAT), dtype=torch.float32, device=grid.device)
        F0 = torch.empty(grid.P, dtype=torch.float64, device=grid.device)
        s = torch.empty(grid.P, dtype=torch.float64, device=grid.device)
        _check(grid.L.pd_closure_features(
            grid.h, grid._U(U), float(t_n),
            _ptr(X, grid.P * N_FEAT, torch.float32, grid.device, "X"),
            grid._perpatch(F0, "F0"), grid._perpatch(s, "s"), _stream()))
        return X, F0, s

    @staticmethod
    def targets(grid, U_n, U_np1, t_n, dt_macro, X=None, y=None):
        X = torch.empty((grid.P, N_FEAT), dtype=torch.float32, device=grid.device) if X is None else X
        y = torch.empty(grid.P, dtype=torch.float32, device=grid.device) if y is None else y
        _check(grid.L.pd_closure_targets(
            grid.h, grid._U(U_n, "U_n"), grid._U(U_np1, "U_np1"), float(t_n), float(dt_macro),
            _ptr(X, grid.P * N_FEAT, torch.float32, grid.device, "X"),
            _ptr(y, grid.P, torch.float32, grid.device, "y"), _stream()))
        return X, y

    def patch_step(self, grid, U_n, t_n, out=None, dt_macro=None, with_fhat=False):
        out = torch.empty_like(U_n) if out is None else out
        fh = torch.empty(grid.P, dtype=torch.float64, device=grid.device) if with_fhat else None
        dtm = grid.prob["time"]["dt_macro"] if dt_macro is None else dt_macro
        _check(self.L.pd_closure_patch_step(self.h, grid.h, grid._U(U_n, "U_n"),
                                            grid._U(out, "U_np1"), float(t_n), float(dtm),
                                            grid._perpatch(fh, "F_hat"), _stream()))
        return (out, fh) if with_fhat else out
