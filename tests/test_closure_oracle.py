"""Pins of the closure oracle (CPU): each checks it against something other than itself."""
import math

import numpy as np
import pytest

from paper_2405_08764_amd import workloads as W


@pytest.fixture(scope="module")
def cl():
    from oracle import closure
    return closure


def square_problem(n=9, m=5):
    p = W.config4_instance(2, n_range=(n, n), m_range=(m, m))
    if p["grid"]["geometry"] != "tanh":
        p = W.config4_instance(0, n_range=(n, n), m_range=(m, m))
    assert p["grid"]["geometry"] == "tanh"
    return p


def annulus_problem(n=9, m=5):
    for i in range(20):
        p = W.config4_instance(i, n_range=(n, n), m_range=(m, m))
        if p["grid"]["geometry"] == "annulus":
            return p
    raise AssertionError


def node_field(o, f):
    gd = o.prob["grid"]
    nx, ne = gd["n_xi"], gd["n_eta"]
    Dxi = (gd["xi1"] - gd["xi0"]) / (nx if gd["periodic_xi"] else nx - 1)
    Deta = (gd["eta1"] - gd["eta0"]) / (ne - 1)
    xi = gd["xi0"] + Dxi * np.arange(nx)
    eta = gd["eta0"] + Deta * np.arange(ne)
    return f(xi[None, :], eta[:, None]) + 0.0 * xi[None, :] * eta[:, None], Dxi, Deta


def test_baseline_of_linear_and_quadratic_fields_is_the_continuous_operator(oracle_mod, cl):
    """Central differences are exact on quadratics: F0 equals alpha U_xixi + gamma U_etaeta
    - nu U_xi - omega U_eta + phi U + g at the node, with the centre coefficients."""
    p = square_problem()
    o = oracle_mod.Oracle(p)
    st = cl.static_part(o)
    A, B, Cc, D, E = 0.3, -1.2, 0.7, 2.0, -0.5
    U, Dxi, Deta = node_field(o, lambda x, y: A + B * x + Cc * y + D * x * x + E * y * y)
    t = 0.013
    X, F0, s = cl.features(o, U, t, st)
    T = cl.tfactor(p["src"][0][0], t)
    for k, e in enumerate(st):
        x, y = e["i"] * Dxi, e["j"] * Deta
        al, ga = e["a"] * Dxi ** 2, e["b"] * Deta ** 2
        nu, om = e["c"] * Dxi, e["d"] * Deta
        u = A + B * x + Cc * y + D * x * x + E * y * y
        exact = (al * 2 * D + ga * 2 * E - nu * (B + 2 * D * x) - om * (Cc + 2 * E * y)
                 + e["phi"] * u + T * e["src"][0])
        assert abs(F0[k] - exact) <= 1e-9 * (abs(exact) + 1.0), (k, F0[k], exact)


def test_stencil_indexing_wraps_and_clamps(oracle_mod, cl):
    """Brute force: the 5x5 stencil of a node-numbering field on the periodic annulus and
    on the clamped square."""
    for prob, periodic in ((annulus_problem(), True), (square_problem(), False)):
        o = oracle_mod.Oracle(prob)
        gd = prob["grid"]
        nx, ne = gd["n_xi"], gd["n_eta"]
        U = np.arange(nx * ne, dtype=float).reshape(ne, nx)
        for (i, j) in ((0, 1), (nx - 1, ne - 2), (1, 1), (nx // 2, ne // 2)):
            S = cl.stencil(U, i, j, periodic)
            for b in range(5):
                for a in range(5):
                    jj = j + b - 2
                    jj = 0 if jj < 0 else (ne - 1 if jj > ne - 1 else jj)
                    if periodic:
                        ii = (i + a - 2 + nx) % nx
                    else:
                        ii = 0 if i + a - 2 < 0 else (nx - 1 if i + a - 2 > nx - 1 else i + a - 2)
                    assert S[b, a] == jj * nx + ii


def test_stencil_features_are_scale_and_shift_invariant(oracle_mod, cl):
    """The stencil inputs see the shape of U, not its size: U -> 3U + 7 changes the
    differences by 3 and sigma by 3."""
    p = square_problem()
    o = oracle_mod.Oracle(p)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((p["grid"]["n_eta"], p["grid"]["n_xi"]))
    X1, _, _ = cl.features(o, U, 0.0)
    X2, _, _ = cl.features(o, 3.0 * U + 7.0, 0.0)
    np.testing.assert_allclose(X1[:, :24], X2[:, :24], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(X1[:, 25:30], X2[:, 25:30], rtol=0, atol=0)
    assert np.all(np.abs(X1[:, 24]) < 1) and np.all(np.abs(X1[:, 30]) < 1)
    sig = np.sqrt(np.mean(X1[:, :24] ** 2, axis=1))
    np.testing.assert_allclose(sig, 1.0, rtol=1e-12)


def test_gelu_matches_math_erf(cl):
    xs = np.linspace(-6, 6, 97)
    ref = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    np.testing.assert_allclose(cl.gelu(xs), ref, rtol=1e-14, atol=1e-16)
    h = 1e-6
    fd = (cl.gelu(xs + h) - cl.gelu(xs - h)) / (2 * h)
    np.testing.assert_allclose(cl.gelu_grad(xs), fd, rtol=1e-7, atol=1e-9)


def test_gradients_match_finite_differences(cl):
    rng = np.random.default_rng(11)
    params = cl.init_params(3)
    X = rng.standard_normal((7, cl.N_FEAT))
    y = rng.standard_normal(7)
    loss, g = cl.loss_and_grads(params, X, y)
    v = cl.flatten(params)
    gv = cl.flatten(g)
    idx = rng.choice(len(v), 60, replace=False)
    for k in idx:
        h = 1e-6
        vp, vm = v.copy(), v.copy()
        vp[k] += h
        vm[k] -= h
        lp, _ = cl.loss_and_grads(cl.unflatten(vp), X, y)
        lm, _ = cl.loss_and_grads(cl.unflatten(vm), X, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gv[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, gv[k])
    assert len(v) == cl.N_PARAMS == 20993


def test_first_adam_step_is_a_signed_learning_rate_step(cl):
    """With zero moments, the first bias-corrected Adam step moves every parameter by
    -lr g / (|g| + eps)."""
    params = cl.init_params(1)
    rng = np.random.default_rng(2)
    grads = {k: rng.standard_normal(np.shape(v)) for k, v in params.items()}
    zeros = {k: np.zeros(np.shape(v)) for k, v in params.items()}
    lr = 1e-3
    new, m, v = cl.adam(params, grads, zeros, zeros, 1, lr)
    for k in cl.PARAM_ORDER:
        expect = params[k] - lr * grads[k] / (np.abs(grads[k]) + 1e-8)
        np.testing.assert_allclose(new[k], expect, rtol=1e-12, atol=1e-15)


def test_bf16_rounding_bit_patterns(cl):
    one = 1.0
    ulp = 2.0 ** -7  # bfloat16 spacing at 1
    cases = [(one, one), (one + ulp / 2, one), (one + 3 * ulp / 2, one + 2 * ulp),
             (one + ulp / 2 + 2 ** -20, one + ulp), (-(one + ulp), -(one + ulp)), (0.0, 0.0)]
    for x, want in cases:
        assert cl.bf16(np.array([x]))[0] == want, (x, cl.bf16(np.array([x]))[0], want)


def test_micro_peclet_inputs_of_constant_coefficients(oracle_mod, cl):
    """Constant D and v on the untransformed square (beta = 0): the last two inputs are
    P/(1+P) with P = |v| dxi / (2 D) in each direction."""
    p = W.config4_instance(2, n_range=(9, 9), m_range=(7, 7))
    assert p["grid"]["geometry"] == "tanh"
    p["grid"]["gparam"] = 0.0
    eps, v1, v2 = 2e-3, 0.8, -0.3
    p["fields"] = {"D11": W.field(c0=eps), "D22": W.field(c0=eps), "v1": W.field(c0=v1),
                   "v2": W.field(c0=v2), "f": W.field(c0=0.5)}
    o = oracle_mod.Oracle(p)
    U = np.ones((9, 9))
    X, _, _ = cl.features(o, U, 0.0)
    dx = p["grid"]["h_xi"] / (7 - 1)
    for k, v in ((31, v1), (32, v2)):
        P = abs(v) * dx / (2 * eps)
        np.testing.assert_allclose(X[:, k], P / (1 + P), rtol=1e-12)


def test_targets_recover_the_correction(cl):
    F0 = np.array([1.0, -2.0, 0.5, 3.0])
    s = np.array([0.1, 0.2, 0.0, 1e-3])
    F = np.array([1.05, -2.1, 7.0, 4.0])
    np.testing.assert_allclose(cl.targets(F, F0, s), [0.5, -0.5, 0.0, 10.0])
