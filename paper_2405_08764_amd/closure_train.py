"""Training data, training and evaluation of the learned closure (pd_closure_*).

The plain patch scheme generates the training pairs: config-4-style instances with seeds
disjoint from the evaluation batch are stepped with the fused plain macro step, and
pd_closure_targets turns each step U_n -> U_np1 into (inputs, (F - F0)/s) pairs for every
patch.  Training, inference and the closure steps all run in the library's kernels; this
module only sequences the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import pd
from . import workloads as W

TRAIN_SEED = W.MASTER_SEED + 5000  # training instances (evaluation uses MASTER_SEED + 4000)


def fitted_grid(prob, n_steps):
    """A grid whose time parameters sit at 0.4 of its explicit bounds."""
    g = pd.Grid(prob)
    info = g.query()
    g.prob = W.fit_time(prob, info.dt_macro_limit, info.dt_micro_limit, n_steps)
    return g


def instance_grids(n, seed, n_steps, n_range=(17, 129), m_range=(9, 33)):
    return [fitted_grid(W.config4_instance(i, seed=seed, n_range=n_range, m_range=m_range),
                        n_steps) for i in range(n)]


def generate(grids, steps, every=1, max_pairs=None):
    """Training pairs from `steps` plain macro steps of each grid (every `every`-th step
    recorded).  Returns X [N][33] and y [N] on the device."""
    Xs, ys, total = [], [], 0
    for g in grids:
        t = g.prob["time"]
        U = g.initial()
        for k in range(steps):
            tn = t["t0"] + k * t["dt_macro"]
            V = g.macro_step(U, tn)
            if k % every == 0:
                X, y = pd.Closure.targets(g, U, V, tn, t["dt_macro"])
                Xs.append(X)
                ys.append(y)
                total += g.P
            U = V
            if max_pairs and total >= max_pairs:
                break
        if max_pairs and total >= max_pairs:
            break
    X = torch.cat(Xs)
    y = torch.cat(ys)
    if max_pairs:
        X, y = X[:max_pairs].contiguous(), y[:max_pairs].contiguous()
    return X, y


def init_params(seed):
    """Seeded initial parameters in the library's flat layout: weights U[-1, 1] /
    sqrt(fan_in), zero biases, the output layer scaled down."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (pd.N_FEAT, 128)) / np.sqrt(pd.N_FEAT)
    W2 = rng.uniform(-1, 1, (128, 128)) / np.sqrt(128)
    w3 = 0.5 * rng.uniform(-1, 1, 128) / np.sqrt(128)
    return np.concatenate([W1.ravel(), np.zeros(128), W2.ravel(), np.zeros(128), w3,
                           np.zeros(1)]).astype(np.float32)


def train(X, y, epochs=30, batch=4096, lr=1e-3, seed=0, max_batch=None, decay=0.9):
    """A closure fitted to (X, y): standardisation from X, then Adam epochs with the
    learning rate decayed per epoch.  Returns (closure, per-epoch losses)."""
    C = pd.Closure(max_batch=max_batch or batch)
    C.set_params(init_params(seed))
    C.fit_standardisation(X, y)
    losses = []
    for ep in range(epochs):
        losses.extend(C.train(X, y, batch=batch, epochs=1, lr=lr * decay ** ep,
                              seed=seed * 1000 + ep))
    return C, np.array(losses)


def zero_closure(like):
    """The same standardisation with a zero network: F_hat = F0 (the baseline alone)."""
    Z = pd.Closure(max_batch=256)
    Z.set_params(np.zeros(pd.N_PARAMS, dtype=np.float32))
    mu, sd = like.standardisation()
    Z.set_standardisation(mu, sd)
    Z.set_target_scale(0.0, 1.0)
    return Z


def rollout(C, g, n_steps, U0=None):
    """n_steps closure macro steps (every patch node by the network, Dirichlet nodes from
    the boundary data)."""
    t = g.prob["time"]
    U = (g.initial() if U0 is None else U0).clone()
    V = torch.empty_like(U)
    for k in range(n_steps):
        tn = t["t0"] + k * t["dt_macro"]
        C.patch_step(g, U, tn, out=V)
        g.apply_boundary(V, tn + t["dt_macro"])
        U, V = V, U
    return U


def rel_l2(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
