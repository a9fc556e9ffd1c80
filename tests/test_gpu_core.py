"""Restriction over a central core of each patch (pd_grid_desc.core_points): the fused
scheme, the split restriction and the batch against the oracle (and each other)."""
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
    print("[core]", *a, flush=True)


def with_core(prob, core, **g):
    q = dict(prob)
    q["grid"] = dict(prob["grid"], core=core, **g)
    return q


def fitted(pd, prob, n_steps):
    info = pd.Grid(prob).query()
    return W.fit_time(prob, info.dt_macro_limit, info.dt_micro_limit, n_steps)


CASES = {
    "config1_core5": lambda pd: with_core(W.config1(), 5),
    "tanh_core9": lambda pd: fitted(pd, with_core(W.config2(n=13, m=17), 9), 6),
    "annulus_core11": lambda pd: fitted(pd, with_core(W.config3(n_r=9, n_theta=16, m=21), 11), 5),
    "sine_core3_printed": lambda pd: fitted(pd, with_core(W.paper_cdr(2, lam=0.2, n=9, m=7), 3,
                                                          c0="printed"), 4),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_core_solve_matches_oracle(pd, oracle_mod, name):
    prob = CASES[name](pd)
    say(name, prob["grid"]["core"], prob["time"]["n_t"], prob["time"]["n_steps"])
    g = pd.Grid(prob)
    got = g.solve().cpu().numpy()
    ref = oracle_mod.Oracle(prob).solve()
    err = float(np.max(np.abs(got - ref))) / max(1.0, float(np.max(np.abs(ref))))
    say(name, "max rel err", err)
    assert err <= TOL, err


def test_core_split_restriction_matches_oracle(pd, oracle_mod):
    prob = with_core(W.config2(n=13, m=17), 9)
    g = pd.Grid(prob)
    o = oracle_mod.Oracle(prob)
    state = torch.randn((g.P, g.me, g.mx), dtype=torch.float64,
                        generator=torch.Generator().manual_seed(2)).cuda()
    got = g.restrict(state).cpu().numpy()
    ref = o.restrict(state.cpu().numpy())
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_core_shapes_and_batch_bitwise(pd):
    """Every launch shape and the batch kernel give the same bits with a core."""
    prob = fitted(pd, with_core(W.config2(n=11, m=17), 7), 5)
    g = pd.Grid(prob)
    ref = g.solve().cpu().numpy()
    seen = 0
    for xch in (1, 2, 3):
        gx = pd.Grid(prob)
        try:
            gx.set_option(pd.OPT_EXCHANGE, xch)
        except pd.PdError:
            continue
        assert gx.solve().cpu().numpy().tobytes() == ref.tobytes(), xch
        seen += 1
    assert seen >= 2
    U0 = pd.Grid(prob).initial()
    B = pd.Batch([pd.Grid(prob)], [U0.clone()])
    B.solve(prob["time"]["n_steps"])
    torch.cuda.synchronize()
    B.sync()
    assert B.U[0].cpu().numpy().tobytes() == ref.tobytes()
