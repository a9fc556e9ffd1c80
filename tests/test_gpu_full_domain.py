"""Full-domain lattice (pd_fd_*) against the oracle's lattice solver.

Small ragged lattices: every node after hundreds of steps (across table chunks, odd and
even step counts) for the square, the sine and tanh maps and the periodic annulus, with
constant and time-dependent sources.  The benchmark's lattice (config-2 problem on
4097 x 4097 nodes): sampled nodes of a step after three steps, against the oracle's
one-node step.  Plus the error paths.
"""
import math

import numpy as np
import pytest
import torch

from paper_2405_08764_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11  # relative to the field's magnitude (FP64, a few hundred steps)


@pytest.fixture(scope="module")
def pd():
    from paper_2405_08764_amd import pd as m
    m.lib()
    assert torch.cuda.is_available()
    return m


def say(*a):
    print("[fd]", *a, flush=True)


def two_time_sources_and_a_constant():
    p = W.config1()
    S2 = ("cart", 0.3, ("cos", 2.0, 0.1), ("sin", 1.0, 0.4))
    S3 = ("cart", 0.5, ("poly", 1.0, 0.5, 0.0, 0.0), ("poly", 1.0, 0.0, -0.3, 0.0))
    p["src"] = p["src"] + [(W.tsin(1.0, 0.5, 6.0), 0.0, S2), (W.const(0.7), 0.0, S3)]
    return p


CASES = {
    "config1_37x29": (lambda: W.config1(), 37, 29, 150),
    "sine_cdr_41x41": (lambda: W.paper_cdr(2, lam=0.1), 41, 41, 300),
    "tanh_config2_65x49": (lambda: W.config2(n=9, m=5), 65, 49, 257),
    "annulus_64x21": (lambda: W.config3(n_r=11, n_theta=16, m=9), 64, 21, 120),
    "three_sources_23x31": (two_time_sources_and_a_constant, 23, 31, 64),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_lattice_matches_oracle(pd, oracle_mod, name):
    make, n_x, n_y, steps = CASES[name]
    prob = make()
    say(name, n_x, n_y, steps)
    g = pd.Grid(prob)
    f = pd.FullDomain(g, n_x, n_y, frac=0.5)
    dt = f.dt
    o = oracle_mod.Oracle(prob)
    t0 = 0.0125
    U = f.initial(t0)
    U0 = U.cpu().numpy().copy()
    f.solve(U, t0, steps)
    f.sync()
    got = U.cpu().numpy()
    ref = o.full_domain(n_x, n_y, U0, t0, dt, steps)
    scale = max(1.0, float(np.max(np.abs(ref))))
    err = float(np.max(np.abs(got - ref))) / scale
    say(name, "max rel err", err)
    assert err <= TOL, err
    # the initial data are u_b(t0) at every node
    xs = [0, n_x // 3, n_x - 1]
    for j in (0, n_y // 2, n_y - 1):
        for i in xs:
            hx = f.query().spacing_x
            hy = f.query().spacing_y
            gd = prob["grid"]
            v = o.boundary_value(gd["xi0"] + i * hx, gd["eta0"] + j * hy, t0)
            assert abs(U0[j, i] - v) <= 1e-14 * max(1.0, abs(v))


def test_zero_one_and_split_step_counts(pd):
    """0 steps leave U alone; n steps equal k + (n - k) steps resumed at t0 + k dt (to
    round-off: the resumed run takes its step times as (t0 + k dt) + s dt, so the time
    factors and Dirichlet data differ in the last bits)."""
    prob = W.config2(n=9, m=5)
    g = pd.Grid(prob)
    f = pd.FullDomain(g, 45, 37)
    dt = f.dt
    U = f.initial(0.0)
    ref = U.clone()
    f.solve(U, 0.0, 0)
    assert torch.equal(U, ref)
    A = ref.clone()
    f.solve(A, 0.0, 301)
    B = ref.clone()
    f.solve(B, 0.0, 117)
    f.solve(B, 0.0 + 117 * dt, 184)
    f.sync()
    scale = max(1.0, float(A.abs().max()))
    assert float((A - B).abs().max()) / scale <= 1e-13
    C1 = ref.clone()
    f.solve(C1, 0.0, 1)
    C2 = ref.clone()
    f.solve(C2, 0.0, 2)
    f.sync()
    assert not torch.equal(C1, ref) and not torch.equal(C1, C2)


def test_bench_lattice_sampled_against_oracle(pd, oracle_mod):
    """The benchmark's lattice: config-2 problem on 4097 x 4097 nodes at half the
    explicit bound.  After three steps, one more step is checked at 4000 sampled nodes
    (interior, the four boundary lines, corners) against the oracle's one-node step."""
    prob = W.config2()
    n = 4097
    say("bench lattice", n, n)
    g = pd.Grid(prob)
    f = pd.FullDomain(g, n, n, frac=0.5)
    dt = f.dt
    t0 = 0.0
    U = f.initial(t0)
    f.solve(U, t0, 3)
    U3 = U.cpu().numpy().copy()
    f.solve(U, t0 + 3 * dt, 1)
    f.sync()
    U4 = U.cpu().numpy()
    o = oracle_mod.Oracle(prob)
    rng = np.random.default_rng(7)
    pts = [(int(i), int(j)) for i, j in rng.integers(1, n - 1, (3000, 2))]
    for k in rng.integers(0, n, 200):
        k = int(k)
        pts += [(k, 0), (k, n - 1), (0, k), (n - 1, k), (1, k), (k, 1), (n - 2, k)]
    pts += [(0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1)]
    scale = max(1.0, float(np.max(np.abs(U3))))
    worst = 0.0
    for i, j in pts:
        ref = o.full_domain_point(n, n, U3, t0 + 3 * dt, dt, i, j)
        worst = max(worst, abs(U4[j, i] - ref) / scale)
    say("sampled nodes", len(pts), "max rel err", worst)
    assert worst <= 1e-13, worst


def test_unstable_step_rejected_and_nonfinite_reported(pd):
    prob = W.config1()
    g = pd.Grid(prob)
    f = pd.FullDomain(g, 33, 33)
    lim = f.query().dt_limit
    with pytest.raises(pd.PdError) as e:
        f.prepare(1.5 * lim)
    assert e.value.status == -3
    with pytest.raises(pd.PdError) as e:  # the failed prepare leaves no usable weights
        f.solve(f.initial(0.0), 0.0, 1)
    assert e.value.status == -2
    g.set_option(pd.OPT_ALLOW_UNSTABLE, 1)
    f.prepare(40.0 * lim)
    U = f.initial(0.0)
    f.solve(U, 0.0, 400)
    with pytest.raises(pd.PdError) as e:
        f.sync()
    assert e.value.status == -5
    f.sync()  # the flag was cleared
