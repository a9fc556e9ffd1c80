"""Plain FP64 reference of the learned closure.  TEST INFRASTRUCTURE ONLY: used by the
test-suite, the smoke check and the CPU-baseline leg of the benchmark, never by the
product path.  Written independently of the HIP library (it shares no code with it).

The closure replaces the micro-burst of a patch by a small network that predicts the
patch's restricted time derivative F = (R(u(tau)) - U) / tau (eq. Time_Derivative) from
the local macro stencil, coefficient samples and scale factors; the plain patch scheme
produces its training targets and stays its fallback.  The network predicts a
correction to the macro finite-difference operator at the node,

    F0 = a (U_E - 2U + U_W) + b (U_N - 2U + U_S) - c (U_E - U_W)/2 - d (U_N - U_S)/2
         + phi U + g,

with a = alpha/Dxi^2, b = gamma/Deta^2, c = nu/Dxi, d = omega/Deta and alpha .. phi, g the
coefficients of eq. (Computational_Problem) at the patch centre at time t_n:

    F_hat = F0 + s * y_hat,   s = kappa sigma + 1e-3 (|g| + |phi U|),
    kappa = a + b + |c| + |d| + |phi|,  sigma = RMS of the 24 stencil differences.

The 33 inputs (before standardisation): the 24 differences U(i+a, j+b) - U(i, j) of the
5x5 stencil (a, b in -2..2, row-major in (b, a), centre skipped) divided by sigma; U/(|U| +
sigma); a, b, c, d, phi divided by kappa; q/(1 + |q|) with q = g/(kappa (|U| + sigma)); and
the micro cell Peclet numbers P/(1 + P) in each direction, P_xi = |nu| dxi / (2 alpha) with
the micro spacing dxi = h_xi/(m_xi - 1) (alpha = D11/h1^2 and nu carry the scale factors;
the micro spacing sets the size of the micro-upwind error the network corrects).  Stencil
indices wrap on a periodic axis and are clamped to the grid otherwise.  Network: 33 -> 128
-> 128 -> 1 with GELU(x) = x Phi(x) after the two hidden layers, trained with Adam on the
mean squared error of standardised targets (y - y_mean) / y_sd, so that y_hat = y_mean +
y_sd out.  Training targets of a plain step: y = clip((F - F0) / s, -10, 10).

Pins (tests/test_closure_oracle.py): F0 of linear and quadratic fields against closed
forms, the stencil indexing against a brute-force construction, scale invariance of the
stencil features, GELU against math.erf, the gradients against central finite
differences, the first Adam step against its closed form, bfloat16 rounding against
hand-worked bit patterns.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_FEAT = 33
HIDDEN = 128
N_PARAMS = N_FEAT * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1


def tfactor(tf, t):
    """Time factor of a source term: ("const", a) | ("exp", a, b) | ("sin", a, b, c)."""
    if tf[0] == "exp":
        return tf[1] * math.exp(tf[2] * t)
    if tf[0] == "sin":
        return tf[1] + tf[2] * math.sin(tf[3] * t)
    return tf[1]


def static_part(o):
    """Per patch: node (i, j), centre coefficients, the rates a, b, c, d, the micro-to-
    macro spacing ratios, and the source's spatial parts at the centre."""
    prob = o.prob
    gd = prob["grid"]
    pmap = o.patch_map()
    coef = o.coef
    mx, me = gd["m_xi"], gd["m_eta"]
    kc, lc = mx // 2, me // 2
    Dxi = (gd["xi1"] - gd["xi0"]) / (gd["n_xi"] if gd["periodic_xi"] else gd["n_xi"] - 1)
    Deta = (gd["eta1"] - gd["eta0"]) / (gd["n_eta"] - 1)
    out = []
    for p in range(o.P):
        i, j = int(pmap[p, 0]), int(pmap[p, 1])
        al, ga, nu, om, ph = (coef[f, p, lc, kc] for f in range(5))
        src = [coef[5 + q, p, lc, kc] for q in range(len(prob["src"]))]
        out.append({"i": i, "j": j, "a": al / (Dxi * Dxi), "b": ga / (Deta * Deta),
                    "c": nu / Dxi, "d": om / Deta, "phi": ph, "src": src,
                    "rx": gd["h_xi"] / (mx - 1) / Dxi, "re": gd["h_eta"] / (me - 1) / Deta})
    return out


def stencil(U, i, j, periodic):
    """5x5 macro values around node (i, j): rows b = -2..2 (eta), columns a = -2..2 (xi)."""
    ne, nx = U.shape
    S = np.zeros((5, 5))
    for b in range(-2, 3):
        jj = min(max(j + b, 0), ne - 1)
        for a in range(-2, 3):
            ii = (i + a) % nx if periodic else min(max(i + a, 0), nx - 1)
            S[b + 2, a + 2] = U[jj, ii]
    return S


def features(o, U, t_n, static=None):
    """Raw features X [P][33], baseline F0 [P] and scale s [P] of every patch."""
    prob = o.prob
    periodic = bool(prob["grid"]["periodic_xi"])
    st = static_part(o) if static is None else static
    P = len(st)
    X = np.zeros((P, N_FEAT))
    F0 = np.zeros(P)
    s = np.zeros(P)
    T = [tfactor(tf, t_n) for (tf, _, _) in prob["src"]]
    for p, e in enumerate(st):
        S = stencil(U, e["i"], e["j"], periodic)
        u = S[2, 2]
        dS = S - u
        diffs = [dS[b, a] for b in range(5) for a in range(5) if (a, b) != (2, 2)]
        sigma = math.sqrt(sum(x * x for x in diffs) / 24.0)
        g = sum(Tq * sq for Tq, sq in zip(T, e["src"]))
        a_, b_, c_, d_, ph = e["a"], e["b"], e["c"], e["d"], e["phi"]
        kappa = a_ + b_ + abs(c_) + abs(d_) + abs(ph)
        F0[p] = (a_ * (dS[2, 3] + dS[2, 1]) + b_ * (dS[3, 2] + dS[1, 2])
                 - c_ * (dS[2, 3] - dS[2, 1]) / 2.0 - d_ * (dS[3, 2] - dS[1, 2]) / 2.0
                 + ph * u + g)
        s[p] = kappa * sigma + 1e-3 * (abs(g) + abs(ph * u))
        inv = 1.0 / sigma if sigma > 0.0 else 0.0
        X[p, :24] = [x * inv for x in diffs]
        X[p, 24] = u / (abs(u) + sigma) if (abs(u) + sigma) > 0.0 else 0.0
        ik = 1.0 / kappa if kappa > 0.0 else 0.0
        X[p, 25:30] = [a_ * ik, b_ * ik, c_ * ik, d_ * ik, ph * ik]
        den = kappa * (abs(u) + sigma)
        q = g / den if den > 0.0 else 0.0
        X[p, 30] = q / (1.0 + abs(q))
        pex = abs(c_) * e["rx"] / (2.0 * a_) if a_ > 0.0 else 0.0
        pee = abs(d_) * e["re"] / (2.0 * b_) if b_ > 0.0 else 0.0
        X[p, 31] = pex / (1.0 + pex)
        X[p, 32] = pee / (1.0 + pee)
    return X, F0, s


def targets(F, F0, s):
    """Training targets of plain-scheme time derivatives F (see the module docstring)."""
    y = np.where(s > 0.0, (F - F0) / np.where(s > 0.0, s, 1.0), 0.0)
    return np.clip(y, -10.0, 10.0)


# ------------------------------------------------------------------------------ network

def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def init_params(seed):
    """Seeded initialisation: weights U[-1, 1] / sqrt(fan_in), zero biases."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.uniform(-1.0, 1.0, (N_FEAT, HIDDEN)) / math.sqrt(N_FEAT),
        "b1": np.zeros(HIDDEN),
        "W2": rng.uniform(-1.0, 1.0, (HIDDEN, HIDDEN)) / math.sqrt(HIDDEN),
        "b2": np.zeros(HIDDEN),
        "w3": rng.uniform(-1.0, 1.0, HIDDEN) / math.sqrt(HIDDEN),
        "b3": np.zeros(1),
    }


PARAM_ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def flatten(params):
    return np.concatenate([np.asarray(params[k], dtype=np.float64).ravel() for k in PARAM_ORDER])


def unflatten(vec):
    shapes = {"W1": (N_FEAT, HIDDEN), "b1": (HIDDEN,), "W2": (HIDDEN, HIDDEN),
              "b2": (HIDDEN,), "w3": (HIDDEN,), "b3": (1,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.array(vec[o:o + n], dtype=np.float64).reshape(shapes[k])
        o += n
    return out


def forward(params, X):
    """Network output for standardised inputs X [n][33]; also the pre-activations."""
    H1 = X @ params["W1"] + params["b1"]
    A1 = gelu(H1)
    H2 = A1 @ params["W2"] + params["b2"]
    A2 = gelu(H2)
    out = A2 @ params["w3"] + params["b3"][0]
    return out, (X, H1, A1, H2, A2)


def loss_and_grads(params, X, y):
    """Mean squared error over the batch and its gradients (backpropagation)."""
    out, (X, H1, A1, H2, A2) = forward(params, X)
    n = X.shape[0]
    r = out - y
    loss = float(np.mean(r * r))
    dout = 2.0 * r / n
    g = {}
    g["w3"] = A2.T @ dout
    g["b3"] = np.array([dout.sum()])
    dH2 = np.outer(dout, params["w3"]) * gelu_grad(H2)
    g["W2"] = A1.T @ dH2
    g["b2"] = dH2.sum(axis=0)
    dH1 = (dH2 @ params["W2"].T) * gelu_grad(H1)
    g["W1"] = X.T @ dH1
    g["b1"] = dH1.sum(axis=0)
    return loss, g


def adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new params, m, v."""
    new_p, new_m, new_v = {}, {}, {}
    for k in PARAM_ORDER:
        new_m[k] = beta1 * m[k] + (1.0 - beta1) * grads[k]
        new_v[k] = beta2 * v[k] + (1.0 - beta2) * grads[k] * grads[k]
        mh = new_m[k] / (1.0 - beta1 ** step)
        vh = new_v[k] / (1.0 - beta2 ** step)
        new_p[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return new_p, new_m, new_v


def standardisation(X):
    """Per-feature mean and standard deviation (a floor keeps constant features finite)."""
    mu = X.mean(axis=0)
    sd = np.sqrt(np.maximum(X.var(axis=0), 1e-12))
    return mu, sd


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def forward_bf16(params, Xn):
    """The inference arithmetic in FP64 with bfloat16 inputs, weights and first-layer
    activations (as the MFMA kernel rounds them), for comparison with FP32 accumulation."""
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    H1 = bf16(Xn) @ bf16(params["W1"]) + f32(params["b1"])
    A1 = bf16(gelu(H1))
    H2 = A1 @ bf16(params["W2"]) + f32(params["b2"])
    A2 = gelu(H2)
    return A2 @ bf16(params["w3"]) + f32(params["b3"])[0]
