"""Learned closure on the GPU against its FP64 oracle: inputs, gradients, Adam, the
bfloat16 MFMA inference and the fused closure macro step."""
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
def cl():
    from oracle import closure
    return closure


def say(*a):
    print("[closure]", *a, flush=True)


def small(kind, n=11, m=7):
    for i in range(40):
        p = W.config4_instance(i, n_range=(n, n), m_range=(m, m))
        if p["grid"]["geometry"] == kind:
            return p
    raise AssertionError(kind)


def perturbed_initial(o, seed):
    U = o.initial()
    rng = np.random.default_rng(seed)
    return U + 0.05 * rng.standard_normal(U.shape) * (np.max(np.abs(U)) + 1e-3)


@pytest.mark.parametrize("kind", ["tanh", "annulus"])
def test_features_match_oracle(pd, cl, oracle_mod, kind):
    p = small(kind)
    o = oracle_mod.Oracle(p)
    U = perturbed_initial(o, 3)
    t = 0.37
    X0, F00, s0 = cl.features(o, U, t)
    g = pd.Grid(p)
    X, F0, s = pd.Closure.features(g, torch.from_numpy(U).cuda(), t)
    X, F0, s = X.cpu().numpy(), F0.cpu().numpy(), s.cpu().numpy()
    np.testing.assert_allclose(X, X0, rtol=2e-6, atol=2e-7)
    np.testing.assert_allclose(F0, F00, rtol=1e-10, atol=1e-12 * np.max(np.abs(F00)))
    np.testing.assert_allclose(s, s0, rtol=1e-10, atol=0)


def random_set(cl, n, seed):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((n, cl.N_FEAT)) * rng.uniform(0.5, 3.0, cl.N_FEAT)
         + rng.uniform(-2, 2, cl.N_FEAT)).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    return X, y


def f32params(cl, seed):
    flat = cl.flatten(cl.init_params(seed)).astype(np.float32)
    return flat, cl.unflatten(flat.astype(np.float64))


def test_gradients_and_loss_match_oracle(pd, cl):
    X, y = random_set(cl, 300, 1)
    flat, params = f32params(cl, 4)
    C = pd.Closure(max_batch=512)
    C.set_params(flat)
    C.fit_standardisation(torch.from_numpy(X).cuda())
    mu, sd = C.standardisation()
    mu_o, sd_o = cl.standardisation(X.astype(np.float64))
    np.testing.assert_allclose(mu, mu_o, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(sd, sd_o, rtol=1e-6)
    g, loss = C.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda())
    Xn = (X.astype(np.float64) - mu.astype(np.float64)) / sd.astype(np.float64)
    loss_o, g_o = cl.loss_and_grads(params, Xn, y.astype(np.float64))
    assert abs(loss.item() - loss_o) <= 1e-5 * loss_o
    got = cl.unflatten(g.cpu().numpy().astype(np.float64))
    for k in cl.PARAM_ORDER:
        err = np.max(np.abs(got[k] - g_o[k]))
        say("grad", k, err, np.max(np.abs(g_o[k])))
        assert err <= 2e-4 * np.max(np.abs(g_o[k])) + 1e-7, k


def test_adam_step_matches_oracle(pd, cl):
    X, y = random_set(cl, 256, 2)
    flat, params = f32params(cl, 5)
    C = pd.Closure(max_batch=256)
    C.set_params(flat)
    C.fit_standardisation(torch.from_numpy(X).cuda())
    mu, sd = C.standardisation()
    lr = 1e-3
    C.train(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), batch=256, epochs=1, lr=lr)
    new = cl.unflatten(C.params().astype(np.float64))
    Xn = (X.astype(np.float64) - mu.astype(np.float64)) / sd.astype(np.float64)
    _, g_o = cl.loss_and_grads(params, Xn, y.astype(np.float64))
    zeros = {k: np.zeros(np.shape(v)) for k, v in params.items()}
    ref, _, _ = cl.adam(params, g_o, zeros, zeros, 1, lr)
    for k in cl.PARAM_ORDER:
        d = np.abs(new[k] - ref[k])
        # a step is lr g / (|g| + eps); entries with |g| near eps may differ in size
        big = np.abs(g_o[k]) > 1e-5
        assert np.max(d[big], initial=0.0) <= 2e-3 * lr, k
        assert np.max(d) <= 1.1 * lr, k


def test_bf16_mfma_inference_matches_oracle(pd, cl):
    X, _ = random_set(cl, 1000, 3)
    flat, params = f32params(cl, 6)
    C = pd.Closure(max_batch=512)
    C.set_params(flat)
    C.fit_standardisation(torch.from_numpy(X).cuda())
    mu, sd = C.standardisation()
    out = C.infer(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    Xn = ((X - mu) / sd).astype(np.float32).astype(np.float64)
    ref = cl.forward_bf16(params, Xn)
    exact, _ = cl.forward(params, Xn)
    err = np.abs(out - ref)
    say("infer vs bf16 oracle: max", err.max(), "median", np.median(err), "ref scale",
        np.std(ref), "vs FP64 forward", np.max(np.abs(out - exact)))
    assert np.median(err) <= 1e-5 * np.std(ref)
    assert err.max() <= 5e-3 * np.std(ref)
    assert np.max(np.abs(out - exact)) <= 5e-2 * np.std(ref)


@pytest.mark.parametrize("kind", ["tanh", "annulus"])
def test_closure_patch_step_matches_oracle(pd, cl, oracle_mod, kind):
    p = small(kind, n=13, m=5)
    o = oracle_mod.Oracle(p)
    U = perturbed_initial(o, 7)
    t, dtm = 0.11, 1e-4
    X0, F00, s0 = cl.features(o, U, t)
    flat, params = f32params(cl, 8)
    flat[cl.N_FEAT * cl.HIDDEN:] *= 0.05  # a small correction
    params = cl.unflatten(flat.astype(np.float64))
    C = pd.Closure(max_batch=512)
    C.set_params(flat)
    mu, sd = cl.standardisation(X0)
    C.set_standardisation(mu, sd)
    mu32, sd32 = C.standardisation()
    g = pd.Grid(p)
    Ug = torch.from_numpy(U).cuda()
    out, fh = C.patch_step(g, Ug, t, out=Ug.clone(), dt_macro=dtm, with_fhat=True)
    fh = fh.cpu().numpy()
    Xn = ((X0.astype(np.float32) - mu32) / sd32).astype(np.float32).astype(np.float64)
    y = cl.forward_bf16(params, Xn)
    Fh_ref = F00 + s0 * y
    err = np.abs(fh - Fh_ref)
    say(kind, "F_hat err max", err.max(), "scale", np.max(s0))
    assert err.max() <= 5e-3 * np.max(s0) * np.std(y) + 1e-9 * np.max(np.abs(Fh_ref))
    pm = o.patch_map()
    Un = out.cpu().numpy()
    nodes = pm[:, 6]
    np.testing.assert_allclose(Un.ravel()[nodes], U.ravel()[nodes] + dtm * fh, rtol=0,
                               atol=1e-14 * np.max(np.abs(U)))
    mask = np.ones(U.size, bool)
    mask[nodes] = False
    assert np.array_equal(Un.ravel()[mask], U.ravel()[mask])


def test_training_reduces_the_loss(pd, cl):
    """A learnable target (a smooth function of a few inputs) is fitted."""
    rng = np.random.default_rng(9)
    X = rng.standard_normal((16384, cl.N_FEAT)).astype(np.float32)
    y = (np.tanh(X[:, 0]) * X[:, 3] + 0.5 * X[:, 7] ** 2).astype(np.float32)
    flat, _ = f32params(cl, 10)
    C = pd.Closure(max_batch=1024)
    C.set_params(flat)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    C.fit_standardisation(Xd)
    losses = C.train(Xd, yd, batch=1024, epochs=8, lr=2e-3, seed=1)
    say("losses", losses)
    assert losses[-1] < 0.1 * losses[0]
