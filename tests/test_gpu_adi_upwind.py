"""ADI micro burst with the higher-order upwind differences (pd_micro_burst_adi_upwind)
against the oracle's Peaceman-Rachford burst with the same forms, its 2-point and r = 0
forms against the library's plain ADI burst, and whole macro steps of the paper's
Sec. 4.1.2 setup (ADI micro solver, n_t = 2, 3- and 4-point upwind) against the oracle's
composition of the same steps."""
import math

import numpy as np
import pytest
import torch

from oracle import adi
from paper_2405_08764_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def pd():
    from paper_2405_08764_amd import pd as m
    m.lib()
    assert torch.cuda.is_available()
    return m


def say(*a):
    print("[adi-upwind]", *a, flush=True)


def ragged(conv, mx, me, geom="sine", gparam=0.2):
    c1 = W.config1()
    return W.problem(W.grid(geom, 5, 6, mx, me, gparam=gparam, conv=conv), c1["fields"],
                     c1["bc"], c1["src"], W.timing(1e-3, 1, 2))


# name: (problem, dt as a multiple of the explicit bound (None: the problem's own), n_t)
CASES = {
    "config1": (lambda: W.config1(), 20.0, 3),
    "tanh": (lambda: W.config2(n=7, m=9), 30.0, 2),
    "annulus": (lambda: W.config3(n_r=6, n_theta=8, m=9), 20.0, 2),
    "sec412": (lambda: W.paper_cdr(2, lam=0.1, n=6, m=11), None, 2),
    "m31": (lambda: W.config2(n=5, m=31), 20.0, 2),  # two lines of 31 fill a wave
    "m40": (lambda: W.config2(n=4, m=40), 20.0, 2),  # largest square patch in 64 KiB
    "ragged_13x7": (lambda: ragged("central", 13, 7), 20.0, 3),
    "ragged_5x12": (lambda: ragged("upwind", 5, 12, "tanh", 1.5), 20.0, 2),
    "m3": (lambda: W.paper_cdr(2, lam=0.1, n=6, m=3), None, 2),
}
FORMS = [(3, 0.0), (4, 0.5), (4, 1.0 / 3.0), (2, 0.0)]


def run_case(pd, oracle_mod, prob, factor, n_t, points, r, seed=3):
    g = pd.Grid(prob)
    o = oracle_mod.Oracle(prob)
    lim = g.query().dt_micro_limit
    dt = prob["time"]["dt_micro"] if factor is None else factor * lim
    U = g.initial() + 0.1 * torch.randn(g.new_U().shape, dtype=torch.float64,
                                        generator=torch.Generator().manual_seed(seed)).cuda()
    state, edge = g.lift_bc(U)
    u0 = state.cpu().numpy().copy()
    e = edge.cpu().numpy()
    g.micro_burst_adi_upwind(state, edge, 0.017, dt, n_t, points, r)
    g.sync()
    got = state.cpu().numpy()
    ref = adi.adi_burst(prob["grid"], o.coef, u0, e, 0.017, dt, n_t, adi.time_factors(prob),
                        points, r)
    return float(np.max(np.abs(got - ref))) / max(1.0, float(np.max(np.abs(ref)))), dt / lim


@pytest.mark.parametrize("form", FORMS, ids=lambda f: f"p{f[0]}r{f[1]:.2f}")
@pytest.mark.parametrize("name", sorted(CASES))
def test_adi_upwind_burst_matches_oracle(pd, oracle_mod, name, form):
    make, factor, n_t = CASES[name]
    points, r = form
    err, ratio = run_case(pd, oracle_mod, make(), factor, n_t, points, r)
    say(name, points, f"{r:.3f}", "dt / explicit bound", f"{ratio:.1f}", "max rel err", err)
    assert err <= TOL, err


@pytest.mark.parametrize("conv", ["upwind", "central"])
def test_reduces_to_the_plain_adi_burst(pd, conv):
    """points = 2 on an upwind grid and points = 4 with r = 0 on a central grid are the
    library's own ADI burst up to rounding order."""
    prob = W.paper_cdr(2, lam=0.1, n=9, m=11)
    prob["grid"]["conv"] = conv
    g = pd.Grid(prob)
    t = prob["time"]
    state, edge = g.lift_bc(g.initial())
    s2 = state.clone()
    g.micro_burst_adi(state, edge, 0.02, t["dt_micro"], t["n_t"])
    points, r = (2, 0.0) if conv == "upwind" else (4, 0.0)
    g.micro_burst_adi_upwind(s2, edge, 0.02, t["dt_micro"], t["n_t"], points, r)
    g.sync()
    err = float((state - s2).abs().max()) / max(1.0, float(state.abs().max()))
    say(conv, "vs plain ADI burst", err)
    assert err <= 1e-13, err


@pytest.mark.parametrize("points,r", [(3, 0.0), (4, 0.5)])
def test_sec412_macro_steps_match_oracle(pd, oracle_mod, points, r):
    """Sec. 4.1.2's setup (sine map lambda = 0.1, D = 1 + x, v = (1 + 10x, 10y), f = 20,
    h = 1e-3, tau = 1e-6, 10 micro intervals, n_t = 2 ADI steps) with the 3-point and
    4-point upwind forms: lift, burst, restriction and projective step, four macro steps,
    against the oracle's composition of its own steps."""
    prob = W.paper_cdr(2, lam=0.1, n=11, m=11, n_steps=4, T=4 * 5e-4)
    g = pd.Grid(prob)
    o = oracle_mod.Oracle(prob)
    t = prob["time"]
    tf = adi.time_factors(prob)
    U = g.initial()
    Uo = U.cpu().numpy().copy()
    for s in range(t["n_steps"]):
        tn = t["t0"] + s * t["dt_macro"]
        state, edge = g.lift_bc(U)
        g.micro_burst_adi_upwind(state, edge, tn, t["dt_micro"], t["n_t"], points, r)
        U = g.macro_step(U, tn, Ubar=g.restrict(state))
        uo = adi.adi_burst(prob["grid"], o.coef, o.lift(Uo), o.edge(Uo), tn, t["dt_micro"],
                           t["n_t"], tf, points, r)
        Uo = o.macro_update(Uo, o.restrict(uo), tn, t["dt_macro"], t["n_t"] * t["dt_micro"])
    g.sync()
    got = U.cpu().numpy()
    err = float(np.max(np.abs(got - Uo))) / max(1.0, float(np.max(np.abs(Uo))))
    say("sec412 macro", points, r, "max rel err", err)
    assert err <= TOL, err


def test_adi_upwind_rejects_bad_arguments(pd):
    g = pd.Grid(W.config1())
    state, edge = g.lift_bc(g.initial())
    bad = [(0.0, 2, 3, 0.5), (1e-6, 0, 3, 0.5), (1e-6, 2, 1, 0.5), (1e-6, 2, 5, 0.5),
           (1e-6, 2, 4, math.nan)]
    for dt, n, points, r in bad:
        with pytest.raises(pd.PdError) as e:
            g.micro_burst_adi_upwind(state, edge, 0.0, dt, n, points, r)
        assert e.value.status == -1
    big = pd.Grid(W.config2(n=4, m=41))  # 5 * 41^2 + 4 * 41 doubles exceed 64 KiB of LDS
    s2 = torch.zeros((big.P, 41, 41), dtype=torch.float64, device="cuda")
    e2 = torch.zeros((big.P, 4, 41), dtype=torch.float64, device="cuda")
    with pytest.raises(pd.PdError) as e:
        big.micro_burst_adi_upwind(s2, e2, 0.0, 1e-7, 2, 3, 0.5)
    assert e.value.status == -1 and "8192" in str(e.value)
