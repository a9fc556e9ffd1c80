"""Higher-order upwind burst (pd_micro_burst_upwind) against the oracle's burst with the same
differences, its 2-point and r = 0 forms against the library's own explicit burst, and
whole macro steps with the coefficients of the paper's Sec. 4.1.2 (where the 3- and 4-point
forms were tried) against the oracle's composition of the same steps."""
import math

import numpy as np
import pytest
import torch

from oracle import adi, upwind
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
    print("[upwind]", *a, flush=True)


def ragged(conv, mx=13, me=7):
    c1 = W.config1()
    return W.problem(W.grid("sine", 5, 6, mx, me, gparam=0.2, conv=conv), c1["fields"],
                     c1["bc"], c1["src"], W.timing(1e-3, 1, 2))


CASES = {
    "config1": lambda: W.config1(),
    "tanh": lambda: W.config2(n=7, m=9),
    "annulus": lambda: W.config3(n_r=6, n_theta=8, m=9),
    "sec412": lambda: W.paper_cdr(2, lam=0.1, n=6, m=11),
    "ragged_13x7": lambda: ragged("central"),
    "m3": lambda: W.config2(n=6, m=3),
    "m4": lambda: ragged("upwind", 4, 4),
    "ragged_5x6": lambda: ragged("upwind", 5, 6),
    "ragged_6x5": lambda: ragged("upwind", 6, 5),
    "m32": lambda: W.config2(n=5, m=32),
}
FORMS = [(2, 0.0), (3, 0.0), (4, 0.5), (4, 1.0 / 3.0)]


def burst_case(pd, oracle_mod, prob, points, r, n_t, factor, seed, lds=False):
    """lds: the LDS-tile kernel even where the patch fits the in-wave kernel."""
    g = pd.Grid(prob)
    if lds:
        g.set_option(pd.OPT_EXCHANGE, 1)
    o = oracle_mod.Oracle(prob)
    dt = factor * g.query().dt_micro_limit
    U = g.initial() + 0.1 * torch.randn(g.new_U().shape, dtype=torch.float64,
                                        generator=torch.Generator().manual_seed(seed)).cuda()
    state, edge = g.lift_bc(U)
    u0 = state.cpu().numpy().copy()
    e = edge.cpu().numpy()
    g.micro_burst_upwind(state, edge, 0.013, dt, n_t, points, r)
    g.sync()
    got = state.cpu().numpy()
    ref = upwind.burst(prob["grid"], o.coef, u0, e, 0.013, dt, n_t, adi.time_factors(prob),
                       points, r)
    return float(np.max(np.abs(got - ref))) / max(1.0, float(np.max(np.abs(ref))))


@pytest.mark.parametrize("lds", [False, True], ids=["auto", "lds"])
@pytest.mark.parametrize("form", FORMS, ids=lambda f: f"p{f[0]}r{f[1]:.2f}")
@pytest.mark.parametrize("name", sorted(CASES))
def test_upwind_burst_matches_oracle(pd, oracle_mod, name, form, lds):
    """Both kernels: the in-wave one wherever the patch fits a wave (all but m = 32 here)
    and the LDS-tile one."""
    points, r = form
    err = burst_case(pd, oracle_mod, CASES[name](), points, r, 5, 0.4, 7, lds)
    say(name, points, r, "lds" if lds else "auto", "max rel err", err)
    assert err <= TOL, err


@pytest.mark.parametrize("lds", [False, True], ids=["auto", "lds"])
def test_long_burst_matches_oracle(pd, oracle_mod, lds):
    """Many nano steps (the ping-pong state and ghost layers over a long run)."""
    err = burst_case(pd, oracle_mod, W.config2(n=6, m=17), 3, 0.0, 61, 0.3, 11, lds)
    say("long burst max rel err", err)
    assert err <= TOL, err


@pytest.mark.parametrize("lds", [False, True], ids=["auto", "lds"])
def test_burst_beyond_one_time_table_chunk(pd, oracle_mod, lds):
    """300 nano steps with a time-dependent source: the kernels' tables of source time
    factors are refilled every 256 steps."""
    err = burst_case(pd, oracle_mod, W.config2(n=5, m=9), 4, 0.5, 300, 0.2, 13, lds)
    say("300-step burst max rel err", err)
    assert err <= TOL, err


def test_in_wave_and_lds_kernels_agree_on_the_config2_patch(pd):
    """The two kernels on 17 x 17 patches (the benchmark's shape) over 40 nano steps agree
    to rounding."""
    prob = W.config2(n=9, m=17)
    outs = []
    for lds in (False, True):
        g = pd.Grid(prob)
        if lds:
            g.set_option(pd.OPT_EXCHANGE, 1)
        dt = 0.4 * g.query().dt_micro_limit
        state, edge = g.lift_bc(g.initial())
        g.micro_burst_upwind(state, edge, 0.02, dt, 40, 3, 0.0)
        g.sync()
        outs.append(state)
    err = float((outs[0] - outs[1]).abs().max()) / max(1.0, float(outs[1].abs().max()))
    say("in-wave vs LDS", err)
    assert err <= 1e-13, err


@pytest.mark.parametrize("conv", ["upwind", "central"])
def test_reduces_to_the_explicit_burst(pd, conv):
    """points = 2 on an upwind grid and points = 4 with r = 0 on a central grid are the
    library's own explicit burst up to rounding order."""
    prob = W.config2(n=9, m=17)
    prob["grid"]["conv"] = conv
    g = pd.Grid(prob)
    dt = 0.4 * g.query().dt_micro_limit
    state, edge = g.lift_bc(g.initial())
    s2 = state.clone()
    g.micro_burst(state, edge, 0.02, dt, 8)
    points, r = (2, 0.0) if conv == "upwind" else (4, 0.0)
    g.micro_burst_upwind(s2, edge, 0.02, dt, 8, points, r)
    g.sync()
    err = float((state - s2).abs().max()) / max(1.0, float(state.abs().max()))
    say(conv, "vs explicit burst", err)
    assert err <= 1e-13, err


@pytest.mark.parametrize("points,r", [(3, 0.0), (4, 0.5)])
def test_sec412_macro_steps_match_oracle(pd, oracle_mod, points, r):
    """Sec. 4.1.2's coefficients (sine map lambda = 0.1, D = 1 + x, v = (1 + 10x, 10y),
    f = 20), patches of 0.2 of the macro spacing and the time parameters at 0.4 of the
    explicit bounds (the paper's tau = 1e-6 over 10 micro intervals of 1e-4 is far beyond
    the explicit bound): lift, higher-order upwind burst, restriction and projective step,
    four macro steps, against the oracle's composition."""
    prob = W.paper_cdr(2, lam=0.1, n=9, m=11, h=0.025)
    o = oracle_mod.Oracle(prob)
    prob = W.fit_time(prob, o.dt_macro_limit(), o.dt_micro_limit(), 4)
    g = pd.Grid(prob)
    o = oracle_mod.Oracle(prob)
    t = prob["time"]
    say("sec412 n_t", t["n_t"], "dt_micro", t["dt_micro"])
    tf = adi.time_factors(prob)
    U = g.initial()
    Uo = U.cpu().numpy().copy()
    for s in range(t["n_steps"]):
        tn = t["t0"] + s * t["dt_macro"]
        state, edge = g.lift_bc(U)
        g.micro_burst_upwind(state, edge, tn, t["dt_micro"], t["n_t"], points, r)
        U = g.macro_step(U, tn, Ubar=g.restrict(state))
        uo = upwind.burst(prob["grid"], o.coef, o.lift(Uo), o.edge(Uo), tn, t["dt_micro"],
                          t["n_t"], tf, points, r)
        Uo = o.macro_update(Uo, o.restrict(uo), tn, t["dt_macro"], t["n_t"] * t["dt_micro"])
    g.sync()
    got = U.cpu().numpy()
    err = float(np.max(np.abs(got - Uo))) / max(1.0, float(np.max(np.abs(Uo))))
    say("sec412 macro", points, r, "max rel err", err)
    assert err <= TOL, err


def test_upwind_rejects_bad_arguments(pd):
    g = pd.Grid(W.config1())
    state, edge = g.lift_bc(g.initial())
    bad = [(0.0, 2, 3, 0.5), (1e-6, 0, 3, 0.5), (1e-6, 2, 1, 0.5), (1e-6, 2, 5, 0.5),
           (1e-6, 2, 4, math.nan)]
    for dt, n, points, r in bad:
        with pytest.raises(pd.PdError) as e:
            g.micro_burst_upwind(state, edge, 0.0, dt, n, points, r)
        assert e.value.status == -1
    big = pd.Grid(W.config2(n=5, m=33))  # 33 * 33 > 1024 micro points
    s2 = torch.zeros((big.P, 33, 33), dtype=torch.float64, device="cuda")
    e2 = torch.zeros((big.P, 4, 33), dtype=torch.float64, device="cuda")
    with pytest.raises(pd.PdError) as e:
        big.micro_burst_upwind(s2, e2, 0.0, 1e-7, 2, 3, 0.5)
    assert e.value.status == -1 and "1024" in str(e.value)
