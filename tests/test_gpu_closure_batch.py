"""Batched closure steps: spot checks, the per-member fallback, and what the trained
network gains over the baseline operator alone, against the plain batched scheme."""
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


@pytest.fixture(scope="module")
def T():
    from paper_2405_08764_amd import closure_train
    return closure_train


def say(*a):
    print("[closure-batch]", *a, flush=True)


def members(T, n, n_steps, seed=W.MASTER_SEED + 4000, nr=(9, 24), mr=(5, 13)):
    return T.instance_grids(n, seed, n_steps, nr, mr)


def plain(pd, grids, U0, n_steps):
    B = pd.Batch(grids, [u.clone() for u in U0])
    B.solve(n_steps)
    torch.cuda.synchronize()
    return [u.clone() for u in B.U]


def random_closure(pd, T, seed=3):
    C = pd.Closure(max_batch=256)
    C.set_params(T.init_params(seed))
    C.set_standardisation(np.zeros(pd.N_FEAT), np.ones(pd.N_FEAT))
    return C


@pytest.mark.parametrize("n_steps", [3, 18])
def test_zero_threshold_falls_back_everywhere_and_equals_plain(pd, T, n_steps):
    grids = members(T, 8, n_steps)
    U0 = [g.initial() for g in grids]
    ref = plain(pd, grids, U0, n_steps)
    C = random_closure(pd, T)
    B = pd.Batch(grids, [u.clone() for u in U0])
    B.attach_closure(C, stride=7, threshold=0.0)
    B.closure_solve(n_steps)
    torch.cuda.synchronize()
    checked, fb = B.closure_stats()
    say("checked", checked, "fallbacks", fb)
    assert fb == len(grids) * n_steps and checked > 0
    for a, b in zip(B.U, ref):
        assert a.cpu().numpy().tobytes() == b.cpu().numpy().tobytes()


def test_bad_network_is_caught_by_the_spot_checks(pd, T):
    """A network with wild outputs never reaches the result: the spot residuals exceed a
    moderate threshold and every member falls back to the plain scheme."""
    n_steps = 5
    grids = members(T, 6, n_steps)
    U0 = [g.initial() for g in grids]
    ref = plain(pd, grids, U0, n_steps)
    C = random_closure(pd, T, seed=9)
    C.set_target_scale(0.0, 1e3)
    B = pd.Batch(grids, [u.clone() for u in U0])
    B.attach_closure(C, stride=50, threshold=0.05)
    B.closure_solve(n_steps)
    torch.cuda.synchronize()
    _, fb = B.closure_stats()
    assert fb == len(grids) * n_steps
    for a, b in zip(B.U, ref):
        assert a.cpu().numpy().tobytes() == b.cpu().numpy().tobytes()


def test_trained_closure_within_1e3_of_plain_and_better_than_the_baseline(pd, T):
    """Trained on plain-scheme pairs of instances disjoint from the evaluated ones; over 20
    macro steps of a held-out mixed batch the closure stays within 1e-3 relative L2 of the
    plain batch for every member, and beats the baseline operator alone (zero network)."""
    n_steps = 20
    tg = T.instance_grids(64, T.TRAIN_SEED, 40, (17, 48), (5, 13))
    X, y = T.generate(tg, steps=12, every=2)
    C, losses = T.train(X, y, epochs=25, batch=4096, lr=2e-3)
    say("pairs", X.shape[0], "loss first/last", losses[0], losses[-1])
    grids = members(T, 12, n_steps, nr=(17, 48), mr=(5, 13))
    U0 = [g.initial() for g in grids]
    ref = plain(pd, grids, U0, n_steps)
    errs = {}
    for name, net in (("trained", C), ("baseline", T.zero_closure(C))):
        B = pd.Batch(grids, [u.clone() for u in U0])
        B.attach_closure(net, stride=100, threshold=1e30)
        B.closure_solve(n_steps)
        torch.cuda.synchronize()
        errs[name] = np.array([T.rel_l2(a, b) for a, b in zip(B.U, ref)])
        say(name, "rel L2 max %.3g mean %.3g" % (errs[name].max(), errs[name].mean()),
            "checked", B.closure_stats()[0])
    assert errs["trained"].max() <= 1e-3
    assert errs["trained"].mean() <= 0.5 * errs["baseline"].mean()
