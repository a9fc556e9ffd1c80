"""The largest patches of the mixed batch (m = 31 and 33 micro points per side) against the
oracle, Sec. 3.3 steps (i)-(vi).

At these sizes the launch shapes differ most from the small cases: multi-wave teams
(hybrid and LDS exchanges, up to 256 threads per patch with idle lanes) and the widest
in-wave bands.  Three checks:
- every launch shape the single-grid autotuner may pick at m = 31 and 33 (square and
  annulus, small macro grids) against the extended oracle (<= 1e-11 relative L2), all
  shapes bitwise equal;
- members with m = 31 and 33 in the persistent batch kernel, every menu shape that
  accepts them, bitwise equal to the single-grid solves;
- the full mixed batch of 512 instances in its autotuned launch configuration: after two
  macro steps, sampled nodes of six members (the 129 x 129 square with m = 33, the
  129 x 129 annulus, a 127 x 127 annulus with m = 33, m = 31 members, a small-m member)
  against the oracle stepped over each node's dependency cone, <= 1e-11 per node.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2405_08764_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[large]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pd():
    from paper_2405_08764_amd import pd as m
    m.lib()
    assert torch.cuda.is_available()
    return m


def member(m, geometry, n_range=(8, 8)):
    """The first mixed-batch instance drawn with patch size m and the given geometry on a
    small macro grid (the same seeded stream as the batch, other sizes)."""
    for i in range(400):
        p = W.config4_instance(i, n_range=n_range, m_range=(m, m))
        if p["grid"]["geometry"] == geometry:
            return p
    raise AssertionError((m, geometry))


def fitted(oracle_mod, prob, n_steps):
    o = oracle_mod.Oracle(prob)
    return W.fit_time(prob, o.dt_macro_limit(), o.dt_micro_limit(), n_steps)


def reset(pd, g):
    """All launch-shape options back to automatic (each value 0 is always accepted)."""
    for opt in (pd.OPT_PATCHES_PER_BLOCK, pd.OPT_BLOCK_THREADS, pd.OPT_ROWS_PER_LANE,
                pd.OPT_COLS_PER_LANE, pd.OPT_EXCHANGE):
        g.set_option(opt, 0)


def all_shapes(pd, g):
    """Every distinct launch shape the options reach (the autotuner's candidates)."""
    seen = []
    for xch in (1, 2, 3):
        for C in (1, 2, 3, 4):
            for R in (2, 3, 4, 5, 6, 7, 8, 9, 11):
                for thr in (64, 128, 192, 256):
                    try:
                        reset(pd, g)
                        g.set_option(pd.OPT_EXCHANGE, xch)
                        g.set_option(pd.OPT_COLS_PER_LANE, C)
                        g.set_option(pd.OPT_ROWS_PER_LANE, R)
                        g.set_option(pd.OPT_BLOCK_THREADS, thr)
                    except pd.PdError:
                        continue
                    I = g.query()
                    key = (I.exchange, I.cols_per_lane, I.rows_per_lane,
                           I.patches_per_block, I.block_threads)
                    if (I.exchange, I.cols_per_lane, I.rows_per_lane) != (xch, C, R):
                        continue
                    if key not in seen:
                        seen.append(key)
    return seen


# lane blocks (rows R, columns C) the burst kernels are built for
LANE_BLOCKS = ([(r, 1) for r in (3, 4, 5, 6, 7, 8, 9, 11)] + [(r, 2) for r in range(2, 7)]
               + [(r, 3) for r in (2, 3, 4)] + [(2, 4), (3, 4)])


def fits_one_wave(m):
    return any(-(-m // c) * -(-m // r) <= 64 for r, c in LANE_BLOCKS)


def set_shape(pd, g, key):
    xch, C, R, ppb, thr = key
    reset(pd, g)
    g.set_option(pd.OPT_EXCHANGE, xch)
    g.set_option(pd.OPT_COLS_PER_LANE, C)
    g.set_option(pd.OPT_ROWS_PER_LANE, R)
    g.set_option(pd.OPT_BLOCK_THREADS, thr)
    g.set_option(pd.OPT_PATCHES_PER_BLOCK, ppb)
    I = g.query()
    assert (I.exchange, I.cols_per_lane, I.rows_per_lane, I.patches_per_block,
            I.block_threads) == key


@pytest.mark.parametrize("m,geometry", [(33, "tanh"), (33, "annulus"), (31, "tanh"),
                                        (31, "annulus")])
def test_every_single_grid_shape_matches_oracle(pd, oracle_mod, m, geometry):
    n_steps = 3
    prob = fitted(oracle_mod, member(m, geometry), n_steps)
    say("single grid", m, geometry, prob["grid"]["n_xi"], "n_t", prob["time"]["n_t"])
    o = oracle_mod.Oracle(prob, threads=8, extended=True)
    ref = o.solve()
    mask = o.patch_mask()
    g = pd.Grid(prob)
    shapes = all_shapes(pd, g)
    say("  shapes", len(shapes), sorted({s[0] for s in shapes}))
    # the LDS and hybrid exchanges always apply; the in-wave one only where a whole patch
    # fits one wave's 64 lanes with some lane block (none does at m >= 31)
    assert {s[0] for s in shapes} == ({1, 2, 3} if fits_one_wave(m) else {1, 3}), shapes
    first = None
    for key in shapes:
        set_shape(pd, g, key)
        U = g.solve()
        g.sync()
        got = U.cpu().numpy()
        if first is None:
            first = got
            err = float(np.linalg.norm(got[mask] - ref[mask]) / np.linalg.norm(ref[mask]))
            say("  rel L2 vs extended oracle", err)
            assert err <= 1e-11, err
        assert got.tobytes() == first.tobytes(), key


def test_batch_largest_patches_bitwise_on_every_menu_shape(pd, oracle_mod):
    n_steps = 4
    probs = [fitted(oracle_mod, member(m, geo, n_range=(7, 9)), n_steps)
             for m in (31, 33) for geo in ("tanh", "annulus")]
    say("members", [(p["grid"]["geometry"], p["grid"]["n_xi"], p["grid"]["m_xi"],
                     p["time"]["n_t"]) for p in probs])
    grids = [pd.Grid(p) for p in probs]
    U0 = [g.initial() for g in grids]
    ref = [g.solve(U.clone(), n_steps=n_steps).cpu().numpy() for g, U in zip(grids, U0)]
    B = pd.Batch(grids, [U.clone() for U in U0])
    ran = []
    for s in range(len(pd.BATCH_MENU)):
        took = []
        for i in range(len(grids)):
            try:
                B.set_shape(i, s)
                took.append(i)
            except pd.PdError:
                pass
        if not took:
            continue
        for U, u0 in zip(B.U, U0):
            U.copy_(u0)
        B.solve(n_steps)
        torch.cuda.synchronize()
        B.sync()
        for i in took:
            assert B.U[i].cpu().numpy().tobytes() == ref[i].tobytes(), (s, i)
        ran.append((s, tuple(took)))
    say("menu shapes run", ran)
    # the shapes the batch autotuner picks for m = 31 and 33 (hybrid C2R4, C2R3, C3R2)
    assert {9, 10, 11} <= {s for s, _ in ran}, ran


def cone_nodes(prob, rng, n_random=3):
    g = prob["grid"]
    nx, ne = g["n_xi"], g["n_eta"]
    lo = 0 if g["periodic_xi"] else 1
    nodes = [(int(rng.integers(lo, nx - lo)), int(rng.integers(1, ne - 1)))
             for _ in range(n_random)]
    nodes.append((nx - 1 - lo, ne - 2))
    return nodes


def cone_check(oracle_mod, prob, nodes, K):
    """U^K at the nodes by the extended oracle, each step advancing only the patches in
    the node's dependency cone (Chebyshev distance K-1-s at step s, periodic in xi);
    coefficients are built for the union of the cones only."""
    o = oracle_mod.Oracle(prob, threads=8, extended=True)
    pm = o.patch_map()
    periodic = prob["grid"]["periodic_xi"]

    def cone(i, j, r):
        di = np.abs(pm[:, 0] - i)
        if periodic:
            di = np.minimum(di, o.nx - di)
        return (di <= r) & (np.abs(pm[:, 1] - j) <= r)

    union = np.zeros(o.P, dtype=bool)
    for (i, j) in nodes:
        union |= cone(i, j, K - 1)
    o.coefficients_for(union.astype(np.uint8))
    t = prob["time"]
    out = {}
    for (i, j) in nodes:
        U = o.initial()
        for s in range(K):
            U = o.step(U, t["t0"] + s * t["dt_macro"],
                       mask=cone(i, j, K - 1 - s).astype(np.uint8))
        out[(i, j)] = U[j, i]
    return out


CONE_MEMBERS = [213, 406, 25, 0, 32, 45]  # 129^2 m 33 square, 129^2 annulus, 127^2 m 33
#                                           annulus, m 31 annulus, m 31 square, m 15 square


def test_full_config4_batch_sampled_against_oracle(pd, oracle_mod):
    K = 2
    torch.cuda.empty_cache()
    probs = W.config4(512)
    grids = []
    for p in probs:
        g = pd.Grid(p)
        info = g.query()
        g.prob = W.fit_time(p, info.dt_macro_limit, info.dt_micro_limit, K)
        grids.append(g)
    assert grids[213].prob["grid"]["n_xi"] == 129 and grids[213].mx == 33
    assert grids[406].prob["grid"]["n_xi"] == 129 and grids[25].mx == 33
    B = pd.Batch(grids)
    ms = B.autotune(reps=2)
    info = B.query()
    say(f"batch of 512: {info.n_items} items, {info.blocks} blocks, tuned {ms:.1f} ms")
    for U, g in zip(B.U, grids):
        g.initial(U=U)
    B.solve(K)
    torch.cuda.synchronize()
    B.sync()
    rng = np.random.default_rng(11)
    for i in CONE_MEMBERS:
        g = grids[i]
        shape, ppb = B.shape(i)
        nodes = cone_nodes(g.prob, rng)
        say(f"member {i}: {g.prob['grid']['geometry']} N={g.nx} m={g.mx} "
            f"n_t={g.prob['time']['n_t']} shape {pd.BATCH_MENU[shape]}x{ppb} nodes {nodes}")
        got = B.U[i].cpu().numpy()
        ref = cone_check(oracle_mod, g.prob, nodes, K)
        for (ii, jj), v in ref.items():
            d = abs(got[jj, ii] - v)
            assert d <= 1e-11 * max(abs(v), 1e-3), (i, (ii, jj), got[jj, ii], v, d)
