"""Learned stopping rule and regularisation parameter: the small MLP, in FP64.

Test infrastructure only (see the package docstring).

The paper leaves the stopping index of DC-LSQR (Algorithm 6) and the
regularisation parameter to the user or to GCV (Sec. 3.1, Sec. 4).  The
learned part predicts both from the first steps of the bidiagonalisation; GCV
stays the fallback and the judge.  Everything below is the plain definition:

  features (16): for j = 1..8,  log(alpha_j / beta_j)  and
                                 log(|phibar_{j+1}| / beta_1)
                 (alpha, beta of Algorithm 4; phibar of Algorithm 6, so that
                 |phibar_{j+1}| = ||C - M(X_j)|| and phibar_1 = beta_1)
  network      : 16 -> 64 -> 64 -> 2, GELU (exact, with erf) after the two
                 hidden layers, outputs (t_lambda, t_k), normalised targets
                 t_lambda = (log lambda - mu) / sigma,  t_k = k / k_scale
  parameters   : one flat vector [W1 (64x16), b1, W2 (64x64), b2, W3 (2x64), b3],
                 weights row-major (output, input).  The stored network uses
                 them rounded to bfloat16 (round to nearest even).
  loss         : (1 / 2B) sum_b sum_o w_o (out_bo - t_bo)^2
  optimiser    : Adam (Kingma & Ba), bias-corrected.

No part of this module is shared with the HIP library.
"""
import math

import numpy as np

N_IN, N_H, N_OUT = 16, 64, 2
N_FEAT_STEPS = 8
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(P):
    """Views of the flat parameter vector as W1, b1, W2, b2, W3, b3."""
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(P[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    r = np.where(nan, u, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def gelu(x):
    """x Phi(x) with Phi the standard normal distribution function."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    x = np.asarray(x, dtype=np.float64)
    Phi = 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return Phi + x * phi


def features(alpha, beta, phibar):
    """The 16 inputs from alpha_1..8, beta_1..8 (beta[0] = beta_1 = ||C||) and
    phibar_2..9 (phibar[j] = phibar_{j+1}, phibar[0] = beta_1)."""
    f = np.empty(N_IN)
    for j in range(N_FEAT_STEPS):
        f[j] = math.log(alpha[j] / beta[j])
        f[N_FEAT_STEPS + j] = math.log(abs(phibar[j + 1]) / beta[0])
    return f


def forward(P, X):
    """Network outputs (B, 2) and the cached pre-activations for backward."""
    p = unpack(P)
    X = np.asarray(X, dtype=np.float64)
    h1 = X @ p["W1"].T + p["b1"]
    a1 = gelu(h1)
    h2 = a1 @ p["W2"].T + p["b2"]
    a2 = gelu(h2)
    out = a2 @ p["W3"].T + p["b3"]
    return out, {"X": X, "h1": h1, "a1": a1, "h2": h2, "a2": a2}


def backward(P, cache, dout):
    """Gradient of sum_b <dout_b, out_b> with respect to the flat parameters."""
    p = unpack(P)
    d3 = np.asarray(dout, dtype=np.float64)
    g = {"W3": d3.T @ cache["a2"], "b3": d3.sum(axis=0)}
    d2 = (d3 @ p["W3"]) * gelu_grad(cache["h2"])
    g["W2"] = d2.T @ cache["a1"]
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * gelu_grad(cache["h1"])
    g["W1"] = d1.T @ cache["X"]
    g["b1"] = d1.sum(axis=0)
    return np.concatenate([g[name].ravel() for name, _ in SIZES])


def loss_and_dout(out, T, w):
    """Weighted half mean squared error and its gradient with respect to out."""
    B = out.shape[0]
    r = out - T
    loss = 0.5 * float(np.sum(w * r * r)) / B
    return loss, (w * r) / B


def adam(P, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t is the 1-based step count); returns new P, m, v."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v
