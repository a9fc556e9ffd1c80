"""The resident fused solve (waves kept on the device across the macro steps of a replay,
neighbour flags instead of a launch per step) against one launch per step: bitwise the
same macro fields on square, stretched, periodic-annulus and ragged grids, for step counts
that use whole replays, a remainder, or both; every problem also stays within the oracle's
tolerance through the fused-solve parity tests, which run on this path by default."""
import numpy as np
import pytest
import torch

from paper_2405_08764_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pd():
    from paper_2405_08764_amd import pd as m
    m.lib()
    assert torch.cuda.is_available()
    return m


def say(*a):
    print("[resident]", *a, flush=True)


def ragged():
    c1 = W.config1()
    return W.problem(W.grid("sine", 9, 8, 13, 7, gparam=0.2, conv="upwind"), c1["fields"],
                     c1["bc"], c1["src"], W.timing(1e-3, 40, 3))


CASES = {
    "config1": lambda: W.config1(),
    "tanh_m17": lambda: W.config2(n=17, m=17),
    "annulus": lambda: W.config3(n_r=8, n_theta=24, m=9),
    "sine_m11": lambda: W.problem(W.grid("sine", 12, 10, 11, 11, gparam=0.3, conv="central"),
                                  W.config1()["fields"], W.config1()["bc"], W.config1()["src"],
                                  W.timing(1e-3, 40, 4)),
    "ragged_13x7": ragged,
}


def solve(pd, prob, resident, steps, shape=None):
    g = pd.Grid(prob)
    g.set_option(pd.OPT_EXCHANGE, 2)
    if shape:
        for k, v in zip((pd.OPT_COLS_PER_LANE, pd.OPT_ROWS_PER_LANE), shape):
            g.set_option(k, v)
    g.set_option(pd.OPT_RESIDENT_SOLVE, 1 if resident else 0)
    U = g.initial()
    g.solve(U, n_steps=steps)
    g.sync()
    assert g.query().resident_solve == (1 if resident else 0)  # the path asked for ran
    return U.cpu().numpy()


@pytest.mark.parametrize("steps", [16, 37], ids=["replay", "replays+rest"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_resident_solve_equals_one_launch_per_step(pd, name, steps):
    prob = CASES[name]()
    a = solve(pd, prob, True, steps)
    b = solve(pd, prob, False, steps)
    say(name, steps, "max |diff|", float(np.max(np.abs(a - b))))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", [(1, 7), (2, 3), (3, 2)], ids=["C1R7", "C2R3", "C3R2"])
def test_resident_solve_every_lane_block(pd, shape):
    """Other in-wave lane blocks (and so other patches per wave) on the config 2 problem."""
    prob = W.config2(n=13, m=17)
    a = solve(pd, prob, True, 20, shape)
    b = solve(pd, prob, False, 20, shape)
    assert np.array_equal(a, b)


def test_resident_solve_full_config2(pd):
    """The config 2 grid (65 x 65 macro nodes, 3969 patches of 17 x 17): every wave resident
    at once, 48 steps (three replays)."""
    prob = W.config2()
    a = solve(pd, prob, True, 48, (2, 6))
    b = solve(pd, prob, False, 48, (2, 6))
    say("config2 max |diff|", float(np.max(np.abs(a - b))))
    assert np.array_equal(a, b)


def test_resident_path_reported_on_graph_reuse(pd):
    """A second solve of whole replays reuses the captured graph; the grid still reports the
    resident path, and the two paths still agree."""
    prob = W.config2(n=11, m=17)
    out = []
    for resident in (1, 0):
        g = pd.Grid(prob)
        g.set_option(pd.OPT_EXCHANGE, 2)
        g.set_option(pd.OPT_RESIDENT_SOLVE, resident)
        U = g.initial()
        g.solve(U, n_steps=32)
        g.solve(U, n_steps=32, t0=prob["time"]["t0"] + 32 * prob["time"]["dt_macro"])
        g.sync()
        assert g.query().resident_solve == resident
        out.append(U.cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_two_time_sources_use_one_launch_per_step(pd):
    """With two time-dependent source terms pd_solve keeps one launch per step (the
    resident kernel is built for at most one) and reports it."""
    c2 = W.config2(n=11, m=17)
    src = list(c2["src"]) + [(("exp", 0.5, -1.0), -1.0, c2["src"][0][2])]
    prob = W.problem(c2["grid"], c2["fields"], c2["bc"], src, c2["time"])
    g = pd.Grid(prob)
    assert g.query().n_time_sources == 2
    g.set_option(pd.OPT_EXCHANGE, 2)
    U = g.initial()
    g.solve(U, n_steps=16)
    g.sync()
    assert g.query().resident_solve == 0
    assert torch.isfinite(U).all()
