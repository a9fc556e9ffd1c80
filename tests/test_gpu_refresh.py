"""Macro step with the edge data refreshed between sub-bursts (pd_macro_step_refresh)
against the oracle's composition of the same steps; n_refresh = 1 against the split
pd_macro_step; and the argument checks."""
import numpy as np
import pytest
import torch

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
    print("[refresh]", *a, flush=True)


CASES = {
    "config1_Q3": (lambda: W.config1(n_t=11), 3, 4),
    "tanh_Q2": (lambda: W.with_time(W.config2(n=13, m=9), dt_macro=2e-4, n_t=50), 2, 3),
    "annulus_Q5": (lambda: W.with_time(W.config3(n_r=9, n_theta=16, m=9), dt_macro=4e-4,
                                       n_t=23), 5, 3),
    "sine_cdr_Q4": (lambda: W.paper_cdr(2, lam=0.2, n=9, m=7, n_t=8, T=1e-3, n_steps=2), 4, 2),
    "config1_Q11": (lambda: W.config1(n_t=11), 11, 2),  # one nano step per sub-burst
}


@pytest.mark.parametrize("xch", [0, 1, 2, 3])
@pytest.mark.parametrize("name", sorted(CASES))
def test_refresh_matches_oracle(pd, oracle_mod, name, xch):
    """Every sub-burst on the automatic launch shape (xch 0) or on one exchange family."""
    make, Q, steps = CASES[name]
    prob = make()
    g = pd.Grid(prob)
    info = g.query()
    t = prob["time"]
    if t["dt_micro"] > 0.5 * info.dt_micro_limit or t["dt_macro"] > 0.5 * info.dt_macro_limit:
        prob = W.fit_time(prob, info.dt_macro_limit, info.dt_micro_limit, steps)
        g = pd.Grid(prob)
        t = prob["time"]
    if xch:
        try:
            g.set_option(pd.OPT_EXCHANGE, xch)
        except pd.PdError:
            pytest.skip(f"no launch shape with exchange {xch} for this patch size")
    say(name, "Q", Q, "n_t", t["n_t"], "steps", steps, "exchange", g.query().exchange)
    o = oracle_mod.Oracle(prob)
    U = g.initial()
    Uo = U.cpu().numpy().copy()
    V = g.new_U()
    for s in range(steps):
        tn = t["t0"] + s * t["dt_macro"]
        g.macro_step_refresh(U, tn, Q, out=V)
        U, V = V, U
        Uo = o.step_refresh(Uo, tn, Q)
    g.sync()
    got = U.cpu().numpy()
    err = float(np.max(np.abs(got - Uo))) / max(1.0, float(np.max(np.abs(Uo))))
    say(name, "max rel err", err)
    assert err <= TOL, err


def test_one_sub_burst_is_the_split_step(pd):
    prob = W.config2(n=17, m=9)
    g = pd.Grid(prob)
    t = prob["time"]
    U = g.initial()
    state, edge = g.lift_bc(U)
    g.micro_burst(state, edge, 0.02, t["dt_micro"], t["n_t"])
    Ubar = g.restrict(state)
    a = g.macro_step(U, 0.02, Ubar=Ubar)
    b = g.macro_step_refresh(U, 0.02, 1)
    g.sync()
    assert torch.equal(a, b)


def test_refresh_argument_checks(pd):
    prob = W.config1()
    g = pd.Grid(prob)
    U = g.initial()
    for Q in (0, prob["time"]["n_t"] + 1):
        with pytest.raises(pd.PdError) as e:
            g.macro_step_refresh(U, 0.0, Q)
        assert e.value.status == -1
    with pytest.raises(pd.PdError) as e:
        g.macro_step_refresh(U, 0.0, 2, out=U)
    assert e.value.status == -1



def patch_nodes(prob):
    """Flat macro-node index of each patch, in patch order (rows of interior nodes; every
    column when xi is periodic, the interior columns otherwise)."""
    gd = prob["grid"]
    nx, ne = gd["n_xi"], gd["n_eta"]
    cols = range(nx) if gd["periodic_xi"] else range(1, nx - 1)
    return torch.tensor([j * nx + i for j in range(1, ne - 1) for i in cols], device="cuda")


@pytest.mark.parametrize("name", sorted(CASES))
def test_refresh_equals_its_stages(pd, name):
    """The refresh step's combined kernels (the time factors of every sub-burst in one
    launch; restriction, patch-node values and Dirichlet data in one launch; restriction,
    projective step and Dirichlet data in one launch) against the same step built from the
    separate entry points (lift, burst, restriction, boundary, projective step): bit for
    bit, intermediate edge data included through the result."""
    make, Q, _ = CASES[name]
    prob = make()
    g = pd.Grid(prob)
    info = g.query()
    t = prob["time"]
    if t["dt_micro"] > 0.5 * info.dt_micro_limit or t["dt_macro"] > 0.5 * info.dt_macro_limit:
        prob = W.fit_time(prob, info.dt_macro_limit, info.dt_micro_limit, 2)
        g = pd.Grid(prob)
        t = prob["time"]
    g.set_option(pd.OPT_RESIDENT_SOLVE, 0)  # the separate-launch form
    dt, n_t = t["dt_micro"], t["n_t"]
    tn = t["t0"] + 0.37 * t["dt_macro"]
    U = g.initial(tn)
    got = g.macro_step_refresh(U, tn, Q)
    nodes = patch_nodes(prob)
    assert nodes.numel() == info.n_patches
    state, edge = g.lift_bc(U)
    Uw = U.clone()
    for q in range(Q):
        s0, s1 = n_t * q // Q, n_t * (q + 1) // Q
        g.micro_burst(state, edge, tn + s0 * dt, dt, s1 - s0)
        if q + 1 < Q:
            Uw.view(-1)[nodes] = g.restrict(state)
            g.apply_boundary(Uw, tn + s1 * dt)
            _, edge = g.lift_bc(Uw)
    ref = g.macro_step(U, tn, Ubar=g.restrict(state))
    g.sync()
    assert g.query().resident_refresh == 0
    say(name, "Q", Q, "max |diff| vs stages", float((got - ref).abs().max()))
    assert torch.equal(got, ref)


@pytest.mark.parametrize("Q", [2, 5, 16, 17])
@pytest.mark.parametrize("name", sorted(CASES))
def test_resident_refresh_equals_separate_launches(pd, name, Q):
    """The resident refreshed step (one launch for all sub-bursts, the edge data exchanged
    between waves) against the separate-launch form on the in-wave shape: the same up to
    rounding order (the forcing moves by the change of the ghost terms instead of being
    formed again from the state) over three steps; Q = 17 exceeds the resident form's
    Dirichlet table and takes the separate launches."""
    make, _, _ = CASES[name]
    prob = make()
    g0 = pd.Grid(prob)
    info = g0.query()
    t = prob["time"]
    if t["dt_micro"] > 0.5 * info.dt_micro_limit or t["dt_macro"] > 0.5 * info.dt_macro_limit:
        prob = W.fit_time(prob, info.dt_macro_limit, info.dt_micro_limit, 3)
        t = prob["time"]
    if Q > t["n_t"]:
        prob = W.with_time(prob, n_t=Q + 3)
        t = prob["time"]
    out = []
    for resident in (1, 0):
        g = pd.Grid(prob)
        try:
            g.set_option(pd.OPT_EXCHANGE, 2)
        except pd.PdError:
            pytest.skip("no in-wave launch shape for this patch size")
        if 9 * g.query().patches_per_block > 64:  # the resident form's limit: 7 per wave
            g.set_option(pd.OPT_PATCHES_PER_BLOCK, 7)
        g.set_option(pd.OPT_RESIDENT_SOLVE, resident)
        U = g.initial()
        V = g.new_U()
        for s_ in range(3):
            g.macro_step_refresh(U, t["t0"] + s_ * t["dt_macro"], Q, out=V)
            U, V = V, U
        g.sync()
        assert g.query().resident_refresh == (1 if resident and Q <= 16 else 0)
        out.append(U.cpu().numpy())
    err = float(np.max(np.abs(out[0] - out[1]))) / max(1.0, float(np.max(np.abs(out[1]))))
    say(name, "Q", Q, "resident vs separate", err)
    assert err <= 1e-12, err
