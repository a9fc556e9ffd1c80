"""Batched persistent form: many mixed instances in one launch per macro step.

Each member's result must be bitwise that of pd_solve on its own grid (the batch kernel
runs the same team bodies), for every shape of the batch kernel's menu, after the
autotuner, across graph replays and remainders; and small members match the extended
FP64 oracle like any single grid.
"""
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
    print("[batch]", *a, flush=True)


def fitted(pd, prob, n_steps):
    """The instance with time parameters at 0.4 of the GPU-computed explicit bounds."""
    info = pd.Grid(prob).query()
    return W.fit_time(prob, info.dt_macro_limit, info.dt_micro_limit, n_steps)


def instances(pd, n, n_steps, n_range=(7, 12), m_range=(5, 29)):
    return [fitted(pd, W.config4_instance(i, n_range=n_range, m_range=m_range), n_steps)
            for i in range(n)]


def run_single(pd, probs, U0, n_steps):
    out = []
    for p, U in zip(probs, U0):
        g = pd.Grid(p)
        out.append(g.solve(U.clone(), n_steps=n_steps).cpu().numpy())
    return out


@pytest.mark.parametrize("n_steps", [5, 21])
def test_batch_equals_single_grids_bitwise_on_every_menu_shape(pd, n_steps):
    probs = instances(pd, 14, n_steps)
    say("members", [(p["grid"]["geometry"], p["grid"]["n_xi"], p["grid"]["m_xi"],
                     p["time"]["n_t"]) for p in probs])
    grids = [pd.Grid(p) for p in probs]
    U0 = [g.initial() for g in grids]
    ref = run_single(pd, probs, U0, n_steps)
    B = pd.Batch(grids, [U.clone() for U in U0])
    covered = set()
    M = len(pd.BATCH_MENU)
    for i in range(len(grids)):
        order = [s for s in range(M) if s not in covered] + sorted(covered)
        for s in order:
            try:
                B.set_shape(i, s)
            except pd.PdError:
                continue
            covered.add(s)
            break
    assert covered == set(range(len(pd.BATCH_MENU))), covered
    B.solve(n_steps)
    torch.cuda.synchronize()
    B.sync()
    for i, U in enumerate(B.U):
        assert U.cpu().numpy().tobytes() == ref[i].tobytes(), (i, B.shape(i))


def test_batch_autotune_keeps_results(pd):
    n_steps = 6
    probs = instances(pd, 6, n_steps, m_range=(5, 21))
    grids = [pd.Grid(p) for p in probs]
    U0 = [g.initial() for g in grids]
    ref = run_single(pd, probs, U0, n_steps)
    B = pd.Batch(grids, [U.clone() for U in U0])
    ms = B.autotune(reps=2)
    info = B.query()
    assert info.tuned == 1 and ms > 0 and info.tuned_ms == ms
    assert info.n_items > 0 and info.blocks > 0
    B.solve(n_steps)
    torch.cuda.synchronize()
    for i, U in enumerate(B.U):
        assert U.cpu().numpy().tobytes() == ref[i].tobytes(), (i, B.shape(i))
    # a second solve from the same start gives the same bits (the queue rewinds itself)
    for U, U_init in zip(B.U, U0):
        U.copy_(U_init)
    B.solve(n_steps)
    torch.cuda.synchronize()
    for i, U in enumerate(B.U):
        assert U.cpu().numpy().tobytes() == ref[i].tobytes(), i


def test_batch_members_match_extended_oracle(pd, oracle_mod):
    """Two small members (one square, one annulus) against the extended-precision oracle,
    with time parameters from the oracle's own bounds."""
    n_steps = 4
    probs = []
    i = 0
    kinds = set()
    while len(probs) < 2:
        p = W.config4_instance(i, n_range=(7, 10), m_range=(5, 9))
        i += 1
        if p["grid"]["geometry"] in kinds:
            continue
        kinds.add(p["grid"]["geometry"])
        o = oracle_mod.Oracle(p)
        probs.append(W.fit_time(p, o.dt_macro_limit(), o.dt_micro_limit(), n_steps))
    grids = [pd.Grid(p) for p in probs]
    B = pd.Batch(grids)
    B.solve(n_steps)
    torch.cuda.synchronize()
    for p, U in zip(probs, B.U):
        ref = oracle_mod.Oracle(p, extended=True).solve()
        got = U.cpu().numpy()
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say(p["grid"]["geometry"], "rel L2", rel)
        assert rel <= 1e-11, rel
