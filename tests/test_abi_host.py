"""The C ABI without a GPU: the library loads, exports every function that
include/pd.h declares, validates descriptors, and builds the patch index map and the
stencil tables bit-identically to the oracle's independent construction (Sec. 3,
eq. Lagrange_2D, eq. edge, trapezoid weights, eq. C_0 constants)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2405_08764_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pd.h")


@pytest.fixture(scope="module")
def pd():
    from paper_2405_08764_amd import pd as pdmod
    if not os.path.exists(pdmod.LIB_PATH):
        from paper_2405_08764_amd import build
        build.build()
    pdmod.lib()
    return pdmod


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("pd_create_grid", "pd_set_coefficients", "pd_lift_bc", "pd_micro_burst",
              "pd_restrict", "pd_macro_step", "pd_solve"):
        assert n in names


def test_library_exports_every_declared_symbol(pd):
    L = pd.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(pd.EXPORTS), "binding and header disagree"


def _grid(pd, prob, precision="f64"):
    return pd.Grid(prob, precision=precision, coefficients=False)


CASES = {
    "config1": lambda: W.config1(),
    "config2_small": lambda: W.config2(n=17, m=17),
    "config3_small": lambda: W.config3(n_r=11, n_theta=16, m=21),
    "config2_core9": lambda: dict(W.config2(n=17, m=17),
                                  grid=dict(W.config2(n=17, m=17)["grid"], core=9)),
    "config3_core7_printed_c0": lambda: dict(
        W.config3(n_r=11, n_theta=16, m=21),
        grid=dict(W.config3(n_r=11, n_theta=16, m=21)["grid"], core=7, c0="printed")),
    "paper_cdr": lambda: W.paper_cdr(2, lam=0.1),
    "paper_annulus": lambda: W.paper_annulus(),
    "ragged": lambda: W.problem(W.grid("identity", 9, 6, 7, 5, box=(0, 2.0, -1.0, 0.5)),
                                W.config1()["fields"], [], [], W.timing(1e-3, 1, 3)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_patch_map_and_tables_bit_exact(pd, oracle_mod, case):
    prob = CASES[case]()
    g = _grid(pd, prob)
    o = oracle_mod.Oracle(prob)
    assert g.P == o.P
    np.testing.assert_array_equal(g.patch_map().numpy(), o.patch_map())
    a, b = g.tables().numpy(), o.tables()
    assert a.shape == b.shape
    assert a.tobytes() == b.tobytes(), np.nonzero(a != b)


def test_info_and_workspace_size(pd):
    prob = W.config2(n=17, m=17)
    g = _grid(pd, prob)
    I = g.query()
    assert I.n_patches == 15 * 15 and I.n_points == 225 * 289
    # planes for alpha, gamma, nu, omega, phi and the problem's one source term
    assert I.workspace_bytes >= (5 + 1) * I.n_points * 8
    assert I.workspace_bytes < (5 + 2) * I.n_points * 8 + (1 << 21)  # + tables, time factors
    assert I.rows_per_lane > 0 and I.block_threads % 64 == 0 and I.block_threads <= 256
    d = pd.grid_desc(prob["grid"], max_sources=pd.MAXTERM + 1)
    h = C.c_void_p()
    assert pd.lib().pd_create_grid(C.byref(d), C.byref(h)) == -1


@pytest.mark.parametrize("field,value", [("h_xi", 1.0), ("m_xi", 2), ("m_eta", 65),
                                         ("n_xi", 2), ("conv", "none")])
def test_invalid_descriptors_rejected(pd, field, value):
    prob = W.config1()
    if field == "conv":
        d = pd.grid_desc(prob["grid"])
        d.conv = 7
    else:
        prob["grid"][field] = value
        d = pd.grid_desc(prob["grid"])
    h = C.c_void_p()
    st = pd.lib().pd_create_grid(C.byref(d), C.byref(h))
    assert st == -1 and not h.value
    assert pd.lib().pd_last_error()


def test_sine_needs_unit_box_and_lambda_below_one(pd):
    prob = W.paper_cdr(1, lam=1.0)
    d = pd.grid_desc(prob["grid"])
    h = C.c_void_p()
    assert pd.lib().pd_create_grid(C.byref(d), C.byref(h)) == -1


def test_calls_without_workspace_report_state_error(pd):
    g = _grid(pd, W.config1())
    with pytest.raises(pd.PdError) as e:
        g.set_coefficients()
    assert e.value.status == -2


def test_config4_generator_is_seeded_and_mixed():
    """The mixed batch: deterministic per instance, both geometries, the stated ranges."""
    from paper_2405_08764_amd import workloads as W
    a = W.config4(64)
    b = W.config4(64)
    assert a == b
    geos = {p["grid"]["geometry"] for p in a}
    assert geos == {"tanh", "annulus"}
    for p in a:
        g = p["grid"]
        assert 17 <= g["n_xi"] <= 129 and g["n_xi"] == g["n_eta"]
        assert 9 <= g["m_xi"] <= 33 and g["m_xi"] % 2 == 1
        assert abs(g["h_xi"] / ((g["xi1"] - g["xi0"]) / (g["n_xi"] - (0 if g["periodic_xi"] else 1))) - 0.2) < 1e-12
        assert 0.0 <= p["fields"]["f"]["c0"] <= 2.0
        eps = p["fields"]["D11"]["c0"]
        assert 1e-3 <= eps <= 1e-2
    assert W.config4_instance(3) != W.config4_instance(4)


def test_batch_create_rejects_members_without_coefficients(pd):
    """pd_batch_create validates its members on the host (no device needed)."""
    import ctypes as C
    from paper_2405_08764_amd import workloads as W
    g = pd.Grid(W.config1(), coefficients=False)
    arr = (pd.BatchMember * 1)()
    arr[0] = pd.BatchMember(g.h.value, 0x1000, 0.0, 0.01, 1e-5, 4)
    h = C.c_void_p()
    st = pd.lib().pd_batch_create(arr, 1, C.byref(h))
    assert st == -2  # PD_ESTATE: no workspace / coefficients
    assert pd.lib().pd_batch_create(arr, 0, C.byref(h)) == -1


def test_full_domain_lattice_host_checks(pd):
    """pd_fd_create validates the lattice on the host; the workspace covers eight weight
    planes and a second field buffer; calls before a workspace report a state error."""
    g = _grid(pd, W.config1())
    L = pd.lib()
    h = C.c_void_p()
    assert L.pd_fd_create(g.h, 2, 9, C.byref(h)) == -1
    assert L.pd_fd_create(None, 9, 9, C.byref(h)) == -1
    assert L.pd_fd_create(g.h, 33, 17, C.byref(h)) == 0
    info = pd.FdInfo()
    assert L.pd_fd_query(h, C.byref(info)) == 0
    assert (info.n_x, info.n_y) == (33, 17)
    assert info.workspace_bytes >= 9 * 33 * 17 * 8
    assert math.isclose(info.spacing_x, 1.0 / 32) and math.isclose(info.spacing_y, 1.0 / 16)
    assert info.dt_limit == 0.0 and info.dt == 0.0
    assert L.pd_fd_prepare(h, 1e-6, None) == -2
    assert L.pd_fd_solve(h, None, 0.0, 1, None) == -2
    assert L.pd_fd_bind_workspace(h, C.c_void_p(256), 16) == -6
    assert L.pd_fd_destroy(h) == 0
    # a periodic xi axis divides the box into n_x intervals
    ga = _grid(pd, W.config3(n_r=11, n_theta=16, m=9))
    assert L.pd_fd_create(ga.h, 64, 11, C.byref(h)) == 0
    assert L.pd_fd_query(h, C.byref(info)) == 0
    assert math.isclose(info.spacing_x, 2 * math.pi / 64)
    assert L.pd_fd_destroy(h) == 0


@pytest.mark.parametrize("core", [1, 4, 19])
def test_core_points_validated(pd, core):
    """core_points must be 0 or 2..m with the parity of m (m = 17 here)."""
    prob = W.config2(n=9, m=17)
    d = pd.grid_desc(dict(prob["grid"], core=core))
    h = C.c_void_p()
    assert pd.lib().pd_create_grid(C.byref(d), C.byref(h)) == -1


def test_binding_rejects_bad_tensors_before_the_library(pd, monkeypatch):
    """The C ABI takes raw device pointers without lengths; the binding checks dtype,
    layout, length and placement first and raises PD_EINVAL without calling the library
    (a bad pointer would otherwise become an out-of-bounds device access)."""
    import torch
    g = _grid(pd, W.config2(n=9, m=5))
    calls = []

    real = g.L

    class Spy:
        def __getattr__(self, name):
            def call(*a):
                calls.append(name)
                raise AssertionError(f"library reached: {name}")
            return call

    g.L = Spy()
    P, me, mx, M = g.P, g.me, g.mx, g.M
    state = torch.zeros((P, me, mx), dtype=torch.float64)
    edge = torch.zeros((P, 4, M), dtype=torch.float64)
    cases = [
        ("dtype", state.float(), edge, "dtype"),
        ("short", state[:-1], edge, "elements"),
        ("strided", state.transpose(1, 2), edge, "contiguous"),
        ("host", state, edge, "device tensor"),
        ("not a tensor", state.numpy(), edge, "torch tensor"),
    ]
    try:
        for label, st, ed, msg in cases:
            with pytest.raises(pd.PdError) as ei:
                g.micro_burst(st, ed, 0.0, 1e-6, 3)
            assert ei.value.status == -1 and msg in str(ei.value), (label, str(ei.value))
        U = torch.zeros((g.ne, g.nx), dtype=torch.float64)
        with pytest.raises(pd.PdError, match="elements"):
            g.solve(U[:-1])
        with pytest.raises(pd.PdError, match="dtype"):
            g.apply_boundary(U.float(), 0.0)
        with pytest.raises(pd.PdError, match="device tensor"):
            g.restrict(state)
    finally:
        g.L = real
    assert not calls
