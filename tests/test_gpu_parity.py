"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every case feeds both sides the same seeded synthetic problem; where a stage is checked on
its own, its inputs come from the oracle.  Bars: index maps and stencil tables bit-exact
(CPU test), FP64 whole runs within 1e-11 relative L2, the FP32 burst within 5e-6.
"""
import math
import sys

import numpy as np
import pytest
import torch

from paper_2405_08764_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pd():
    from paper_2405_08764_amd import pd as m
    m.lib()
    assert torch.cuda.is_available()
    return m


def fit_n_t(orc_mod, prob, frac=0.4):
    """Keep tau = n_t dt_micro of the problem, pick n_t at frac of the explicit bound."""
    o = orc_mod.Oracle(prob)
    t = prob["time"]
    tau = t["n_t"] * t["dt_micro"]
    return W.with_time(prob, n_t=int(math.ceil(tau / (frac * o.dt_micro_limit()))),
                       ratio=t["dt_macro"] / tau)


def rel_l2(a, b, mask=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if mask is not None:
        a, b = a[mask], b[mask]
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cases():
    return {
        "config1": W.config1(),
        "config2_17x17": W.config2(n=17, m=17, n_steps=12),
        "config3_16x11": W.config3(n_r=11, n_theta=16, m=21, n_steps=8),
        "sec412_sine": W.paper_cdr(2, lam=0.1, n=11, m=11, n_steps=4, T=4 * 5e-4),
        "sec42_annulus": W.paper_annulus(n_theta=16, n_r=11, m=9, n_steps=4, T=4 * 4e-4),
        "ragged_13x7": W.problem(W.grid("identity", 9, 12, 13, 7, box=(0, 2.0, -1.0, 0.5)),
                                 W.config1()["fields"], W.config1()["bc"], W.config1()["src"],
                                 W.timing(2e-3, 5, 1)),
        # two constant-in-time and two time-dependent source terms (every branch of the
        # source handling in the burst prologue and the nano update)
        "four_sources": W.problem(
            W.grid("tanh", 9, 9, 9, 9, gparam=1.5, conv="upwind"),
            W.config1()["fields"], W.config1()["bc"],
            [(W.const(1.0), 0.5, ("cart", 1.0, ("sin", math.pi, 0.0), ("sin", math.pi, 0.0))),
             (W.const(-0.7), 0.0, ("cart", 0.3, ("cos", 2 * math.pi, 0.0),
                                   ("poly", 1.0, 0.5, 0.0, 0.0))),
             (W.texp(1.0, -1.0), -1.0, ("cart", 1.0, ("sin", math.pi, 0.0),
                                         ("sin", math.pi, 0.0))),
             (W.tsin(1.0, 0.5, 3.0), 0.0, ("cart", 0.8, ("poly", 0.0, 1.0, -1.0, 0.0),
                                           ("cos", math.pi, 0.25)))],
            W.timing(2e-3, 5, 1)),
        "printed_c0_central": W.problem(
            W.grid("sine", 10, 10, 11, 11, gparam=0.3, conv="central", c0="printed"),
            W.config1()["fields"], W.config1()["bc"], W.config1()["src"], W.timing(2e-3, 5, 1)),
    }


@pytest.fixture(scope="module")
def problems(oracle_mod):
    return {k: fit_n_t(oracle_mod, v) for k, v in cases().items()}


CASE_NAMES = sorted(cases())


@pytest.mark.parametrize("case", CASE_NAMES)
def test_coefficients_match_oracle(pd, oracle_mod, problems, case):
    prob = problems[case]
    say("coefficients", case)
    g = pd.Grid(prob)
    o = oracle_mod.Oracle(prob)
    a = g.coefficients().cpu().numpy()
    b = o.coef
    for c in range(b.shape[0]):
        scale = float(max(np.max(np.abs(b[c])), 1e-300))
        err = float(np.max(np.abs(a[c] - b[c])))
        assert err <= 1e-12 * scale, (case, c, err, scale)
    I = g.query()
    assert abs(I.dt_micro_limit / o.dt_micro_limit() - 1) < 1e-12
    assert abs(I.dt_macro_limit / o.dt_macro_limit() - 1) < 1e-12


@pytest.mark.parametrize("case", CASE_NAMES)
def test_lift_bc_and_restrict_match_oracle(pd, oracle_mod, problems, case):
    """Steps (i), (ii) and (iv) on their own."""
    prob = problems[case]
    say("lift_bc/restrict", case)
    g = pd.Grid(prob)
    o = oracle_mod.Oracle(prob)
    U0 = o.initial()
    Ug = g.initial()
    e_init = float(np.max(np.abs(Ug.cpu().numpy() - U0)))
    assert e_init <= 1e-14 * float(np.max(np.abs(U0))) + 1e-300, e_init
    U = torch.from_numpy(U0).cuda()
    state, edge = g.lift_bc(U)
    torch.cuda.synchronize()
    u_o, e_o = o.lift(U0), o.edge(U0)
    e_lift = float(np.max(np.abs(state.cpu().numpy() - u_o)))
    e_edge = float(np.max(np.abs(edge.cpu().numpy() - e_o)))
    assert e_lift <= 1e-13 * float(np.max(np.abs(U0))), e_lift
    assert e_edge <= 1e-11 * max(float(np.max(np.abs(e_o))), 1.0), e_edge
    # restriction of the oracle's lifted field
    Ub = g.restrict(torch.from_numpy(u_o).cuda()).cpu().numpy()
    np.testing.assert_allclose(Ub, o.restrict(u_o), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("xch", [0, 1, 2, 3])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", CASE_NAMES)
def test_burst_matches_oracle(pd, oracle_mod, problems, case, precision, xch):
    """Step (iii) on its own, from the oracle's lifted field and edge data, on the
    automatic launch shape (xch 0) and on each neighbour-exchange family (LDS, in-wave,
    hybrid) where the patch fits it: the change u(tau) - u(0) agrees."""
    prob = problems[case]
    say("burst", case, precision, "exchange", xch)
    g = pd.Grid(prob, precision=precision)
    if xch:
        try:
            g.set_option(pd.OPT_EXCHANGE, xch)
        except pd.PdError:
            pytest.skip(f"no launch shape with exchange {xch} for this patch size")
    o = oracle_mod.Oracle(prob, extended=True)
    U0 = o.initial()
    u0, e0 = o.lift(U0), o.edge(U0)
    t = prob["time"]
    u_o, rc = o.burst(u0, e0, 0.0, t["dt_micro"], t["n_t"])
    assert rc == 0
    st = torch.from_numpy(u0).cuda()
    g.micro_burst(st, torch.from_numpy(e0).cuda(), 0.0, t["dt_micro"], t["n_t"])
    g.sync()
    u_g = st.cpu().numpy()
    d_o, d_g = u_o - u0, u_g - u0
    # The oracle advances u itself, so its change carries round-off ~ eps |u| per nano
    # step (random walk); the device advances the increment and is more accurate.
    floor = 8.0 * np.finfo(np.float64).eps * np.max(np.abs(u0)) * math.sqrt(t["n_t"])
    tol = 1e-9 if precision == "f64" else 2e-4
    err = float(np.max(np.abs(d_g - d_o)))
    bar = float(tol * np.max(np.abs(d_o)) + floor)
    say(f"  max change {np.max(np.abs(d_o)):.3e}  diff {err:.3e}  bar {bar:.3e}")
    assert err <= bar, (err, bar)


@pytest.mark.parametrize("case", CASE_NAMES)
def test_split_macro_update_matches_oracle(pd, oracle_mod, problems, case):
    """Steps (v)-(vi) and the Dirichlet data from a given restriction."""
    prob = problems[case]
    say("macro update", case)
    g = pd.Grid(prob)
    o = oracle_mod.Oracle(prob)
    t = prob["time"]
    U0 = o.initial()
    Ub = o.restrict(o.burst(o.lift(U0), o.edge(U0), 0.0, t["dt_micro"], t["n_t"])[0])
    tau = t["n_t"] * t["dt_micro"]
    ref = o.macro_update(U0, Ub, 0.0, t["dt_macro"], tau)
    out = g.macro_step(torch.from_numpy(U0).cuda(), 0.0, Ubar=torch.from_numpy(Ub).cuda())
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", CASE_NAMES)
def test_solve_matches_oracle(pd, oracle_mod, problems, case, precision):
    """The whole scheme, Sec. 3.3 repeated to the final time, fused on the device and
    replayed from a HIP graph: FP64 within 1e-11 relative L2, FP32 within 5e-6."""
    prob = problems[case]
    say("solve", case, precision, prob["time"])
    g = pd.Grid(prob, precision=precision)
    # the extended-precision build of the oracle: same steps, round-off floor ~1e-18
    o = oracle_mod.Oracle(prob, threads=4, extended=True)
    ref = o.solve()
    U = g.solve()
    g.sync()
    err = rel_l2(U.cpu().numpy(), ref, o.patch_mask())
    say("  rel L2", err)
    assert err <= (1e-11 if precision == "f64" else 5e-6), err


@pytest.mark.parametrize("xch", [1, 2, 3])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fused_step_equals_split_path(pd, oracle_mod, problems, precision, xch):
    """The fused kernel (either neighbour exchange) and the stage-by-stage calls compute
    the same macro step."""
    prob = problems["config3_16x11"]
    g = pd.Grid(prob, precision=precision)
    g.set_option(pd.OPT_EXCHANGE, xch)
    t = prob["time"]
    U = g.initial()
    fused = g.macro_step(U, 0.0)
    st, ed = g.lift_bc(U)
    g.micro_burst(st, ed, 0.0, t["dt_micro"], t["n_t"])
    Ub = g.restrict(st)
    split = g.macro_step(U, 0.0, Ubar=Ub)
    torch.cuda.synchronize()
    d = (fused - split).abs().max().item() / (fused - U).abs().max().item()
    assert d < (1e-10 if precision == "f64" else 1e-4), d


def cone_reference(oracle_mod, prob, nodes, K):
    """U^K at the given nodes by the oracle, advancing only the patches within the
    dependency cone of each node (Chebyshev distance K-1-s at step s, periodic in xi)."""
    o = oracle_mod.Oracle(prob, threads=8, extended=True)
    pm = o.patch_map()
    t = prob["time"]
    out = {}
    for (i, j) in nodes:
        U = o.initial()
        for s in range(K):
            r = K - 1 - s
            di = np.abs(pm[:, 0] - i)
            if prob["grid"]["periodic_xi"]:
                di = np.minimum(di, o.nx - di)
            mask = (di <= r) & (np.abs(pm[:, 1] - j) <= r)
            U = o.step(U, t["t0"] + s * t["dt_macro"], mask=mask.astype(np.uint8))
        out[(i, j)] = U[j, i]
    return out


@pytest.mark.parametrize("which", ["config2", "config3"])
def test_full_size_sampled(pd, oracle_mod, which):
    """Full-size workloads in the launch configuration the benchmark times: K macro steps
    on the GPU against the oracle at sampled nodes, each computed over its dependency
    cone only."""
    prob = W.config2() if which == "config2" else W.config3()
    K = 3
    say("full size", which)
    g = pd.Grid(prob)
    U = g.solve(n_steps=K)
    g.sync()
    Ug = U.cpu().numpy()
    rng = np.random.default_rng(5)
    nx, ne = prob["grid"]["n_xi"], prob["grid"]["n_eta"]
    lo = 0 if prob["grid"]["periodic_xi"] else 1
    nodes = [(int(rng.integers(lo, nx - lo)), int(rng.integers(1, ne - 1))) for _ in range(4)]
    nodes += [(lo, 1), (nx - 1 - lo, ne - 2)]  # corners of the patch lattice
    ref = cone_reference(oracle_mod, prob, nodes, K)
    for (i, j), v in ref.items():
        assert abs(Ug[j, i] - v) <= 1e-11 * max(abs(v), 1e-3), ((i, j), Ug[j, i], v)


def test_bitwise_determinism_across_runs_and_launch_shapes(pd, problems):
    """Repeats and every supported launch shape give the same bits (the update of a
    point does not depend on the lane mapping; the restriction order is fixed).  This
    is also the race check of the LDS exchange."""
    prob = problems["config2_17x17"]
    g = pd.Grid(prob)
    ref = g.solve().cpu().numpy()
    again = g.solve().cpu().numpy()
    assert ref.tobytes() == again.tobytes()
    seen = set()
    for xch in (1, 2, 3):
        for C in (1, 2, 3):
            for R in (2, 3, 4, 5, 6, 7, 8, 9, 11):
                for ppb in (1, 2, 0):
                    try:
                        g.set_option(pd.OPT_EXCHANGE, xch)
                        g.set_option(pd.OPT_COLS_PER_LANE, C)
                        g.set_option(pd.OPT_ROWS_PER_LANE, R)
                        g.set_option(pd.OPT_PATCHES_PER_BLOCK, ppb)
                    except pd.PdError:
                        continue
                    I = g.query()
                    key = (I.exchange, I.cols_per_lane, I.rows_per_lane, I.patches_per_block)
                    if (I.exchange, I.cols_per_lane, I.rows_per_lane) != (xch, C, R) or key in seen:
                        continue
                    seen.add(key)
                    out = g.solve().cpu().numpy()
                    assert out.tobytes() == ref.tobytes(), key
    assert {k[0] for k in seen} == {1, 2, 3}, seen


def test_split_burst_bitwise_across_launch_shapes(pd, problems):
    """The split-mode burst (caller-owned patch states) gives the same bits on every
    supported launch shape of every exchange family, as the fused step does."""
    prob = problems["config2_17x17"]
    g = pd.Grid(prob)
    t = prob["time"]
    U = g.initial()
    st0, ed = g.lift_bc(U)
    st = st0.clone()
    g.micro_burst(st, ed, 0.0, t["dt_micro"], t["n_t"])
    ref = st.cpu().numpy()
    seen = set()
    for xch in (1, 2, 3):
        for C in (1, 2, 3, 4):
            for R in (2, 3, 4, 5, 6, 7, 8, 9, 11):
                for ppb in (1, 2, 0):
                    try:
                        g.set_option(pd.OPT_EXCHANGE, xch)
                        g.set_option(pd.OPT_COLS_PER_LANE, C)
                        g.set_option(pd.OPT_ROWS_PER_LANE, R)
                        g.set_option(pd.OPT_PATCHES_PER_BLOCK, ppb)
                    except pd.PdError:
                        continue
                    I = g.query()
                    key = (I.exchange, I.cols_per_lane, I.rows_per_lane, I.patches_per_block)
                    if (I.exchange, I.cols_per_lane, I.rows_per_lane) != (xch, C, R) or key in seen:
                        continue
                    seen.add(key)
                    st = st0.clone()
                    g.micro_burst(st, ed, 0.0, t["dt_micro"], t["n_t"])
                    assert st.cpu().numpy().tobytes() == ref.tobytes(), key
    say("split shapes", len(seen))
    assert {k[0] for k in seen} == {1, 2, 3}, seen


@pytest.mark.parametrize("name", ["config1", "sec412_sine", "ragged_13x7"])
def test_graph_solve_equals_single_steps_and_resume(pd, problems, name):
    """pd_solve (graph replay of one boundary/time-table node and one fused burst per
    step, device clock, a remainder outside the graph) equals repeated pd_macro_step, and
    a run split in two with the state as checkpoint resumes bit-exactly."""
    t = problems[name]["time"]
    prob = W.with_time(problems[name], n_steps=21,
                       ratio=t["dt_macro"] / (t["n_t"] * t["dt_micro"]))
    g = pd.Grid(prob)
    t = prob["time"]
    full = g.solve().cpu().numpy()
    U = g.initial()
    for s in range(t["n_steps"]):
        U = g.macro_step(U, t["t0"] + s * t["dt_macro"])
    assert U.cpu().numpy().tobytes() == full.tobytes()
    U = g.solve(n_steps=9)
    U = g.solve(U=U, n_steps=12, t0=t["t0"] + 9 * t["dt_macro"])
    # the clock computes t_n = t0 + n dt; a resumed run starts a new clock at t0 + 9 dt
    np.testing.assert_allclose(U.cpu().numpy(), full, rtol=1e-14, atol=1e-15)


def test_autotune_keeps_results_and_caches(pd, problems):
    """The autotuner times the allowed launch shapes, keeps the fastest (results are
    bitwise those of any other shape) and answers a second grid of the same kind from its
    cache."""
    prob = problems["config2_17x17"]
    g = pd.Grid(prob)
    ref = g.solve().cpu().numpy()
    ms = g.autotune(reps=2, force=True)
    I = g.query()
    assert I.tuned == 1 and ms > 0 and I.tuned_ms == ms
    assert g.solve().cpu().numpy().tobytes() == ref.tobytes()
    g2 = pd.Grid(prob)
    assert g2.autotune(reps=2) == ms
    J = g2.query()
    assert (J.exchange, J.cols_per_lane, J.rows_per_lane, J.patches_per_block,
            J.block_threads) == (I.exchange, I.cols_per_lane, I.rows_per_lane,
                                 I.patches_per_block, I.block_threads)
    g2.set_option(pd.OPT_EXCHANGE, 1)  # options drop the tuned shape
    assert g2.query().tuned == 0


def test_stability_guard_and_nonfinite_flag(pd, problems):
    prob = problems["config1"]
    g = pd.Grid(prob)
    lim = g.query().dt_micro_limit
    U = g.initial()
    st, ed = g.lift_bc(U)
    with pytest.raises(pd.PdError) as e:
        g.micro_burst(st, ed, 0.0, 2.0 * lim, 3)
    assert e.value.status == -3
    with pytest.raises(pd.PdError) as e:
        g.macro_step(U, 0.0, dt_macro=10 * g.query().dt_macro_limit)
    assert e.value.status == -3
    V = U.clone()
    V[5, 5] = float("nan")
    g.macro_step(V, 0.0)
    with pytest.raises(pd.PdError) as e:
        g.sync()
    assert e.value.status == -5
    g.macro_step(U, 0.0)
    g.sync()  # flag cleared


def test_constant_field_preserved_on_gpu(pd):
    """Constant state, zero reaction and source, divergence-free velocity: the fused
    step returns the constant (deviation form: exactly)."""
    g_ = W.grid("sine", 12, 12, 9, 9, gparam=0.2, conv="upwind")
    fields = {"D11": W.field(c0=0.3), "D22": W.field(c0=0.5), "v1": W.field(c0=1.0),
              "v2": W.field(c0=-0.5), "f": W.field()}
    S = ("cart", 1.0, ("poly", 1, 0, 0, 0), ("poly", 1, 0, 0, 0))
    prob = W.problem(g_, fields, [(W.const(2.5), S)], [], W.timing(1e-5, 30, 40))
    for prec in ("f64", "f32"):
        g = pd.Grid(prob, precision=prec)
        U = g.solve()
        g.sync()
        assert (U - 2.5).abs().max().item() == 0.0, prec
