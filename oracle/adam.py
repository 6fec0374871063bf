"""FP64 oracle of the radiation intensity response and of the fused
optimiser step (TEST INFRASTRUCTURE ONLY).

Radiation intensity response (Eq. 3): each Gaussian carries a feature
vector f in R^{N_f}; its intensity is the sigmoid of the inner product of
f with a vector of constant weights lambda (the paper adopts N_f = 16).
``rirf`` and ``rirf_grad`` are that function and its adjoint.

The paper trains the Gaussians with Adam (beta1 = 0.9, beta2 = 0.999,
eps = 1e-15) for 2x10^4 iterations; learning rates: positions 1.9e-4
decaying exponentially to 1.9e-6, features 2e-3, opacity 8e-3, scaling
5e-3, rotation 1e-3 (Sec. 4.1, implementation details).  The renderer
consumes activated parameters: scales = exp(log-scales), opacity =
sigmoid(logit), intensity = rirf(features, lambda), quaternions raw
(normalised by the renderer), means as is.

adam_step() maps the gradients of the activated parameters to the raw ones
(chain rule through the activations at the pre-step values), applies Adam
as Kingma & Ba's Algorithm 1 (bias-corrected moments), and returns the new
raw parameters, moments and activated copies.  All float64.
"""
from __future__ import annotations

import numpy as np

RAW = ("means", "log_scales", "quats", "opacity_logit", "features")
ACT = ("means", "scales", "quats", "opacity", "intensity")

PAPER = {"lr_means_start": 1.9e-4, "lr_means_end": 1.9e-6, "iters": 20000, "lr_feature": 2e-3,
         "lr_opacity": 8e-3, "lr_scales": 5e-3, "lr_quats": 1e-3, "beta1": 0.9, "beta2": 0.999,
         "eps": 1e-15, "n_features": 16}


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def rirf(features, weights):
    """Eq. 3: intensity = sigmoid(sum_k lambda_k f_k); features (n, N_f)."""
    w = np.atleast_1d(np.asarray(weights, np.float64))
    f = np.asarray(features, np.float64).reshape(len(features), w.size)
    return sigmoid(f @ w)


def rirf_grad(features, weights, dl_dintensity):
    """Adjoint of rirf: dL/df_k = dL/di * s (1 - s) * lambda_k."""
    s = rirf(features, weights)
    w = np.asarray(weights, np.float64)
    return (np.asarray(dl_dintensity, np.float64) * s * (1 - s))[:, None] * w[None, :]


def paper_lrs(t: int) -> dict:
    """Learning rates at step t (1-based): positions decay exponentially from
    start to end over the paper's iteration count (log-linear interpolation,
    held at the end value afterwards)."""
    P = PAPER
    frac = min(max(t - 1, 0), P["iters"]) / P["iters"]
    lr_m = float(np.exp((1 - frac) * np.log(P["lr_means_start"]) + frac * np.log(P["lr_means_end"])))
    return {"means": lr_m, "log_scales": P["lr_scales"], "quats": P["lr_quats"],
            "opacity_logit": P["lr_opacity"], "features": P["lr_feature"]}


def activate(raw: dict, weights) -> dict:
    return {"means": raw["means"].astype(np.float64),
            "scales": np.exp(raw["log_scales"].astype(np.float64)),
            "quats": raw["quats"].astype(np.float64),
            "opacity": sigmoid(raw["opacity_logit"].astype(np.float64)),
            "intensity": rirf(raw["features"], weights)}


def raw_grads(raw: dict, g_act: dict, weights) -> dict:
    """Chain rule from activated to raw parameters at the current raw values."""
    a = activate(raw, weights)
    return {"means": np.asarray(g_act["means"], np.float64),
            "log_scales": np.asarray(g_act["scales"], np.float64) * a["scales"],
            "quats": np.asarray(g_act["quats"], np.float64),
            "opacity_logit": np.asarray(g_act["opacity"], np.float64) * a["opacity"] * (1 - a["opacity"]),
            "features": rirf_grad(raw["features"], weights, g_act["intensity"])}


def adam_step(raw: dict, g_act: dict, m: dict, v: dict, t: int, lrs: dict, weights,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15):
    """One Adam step (Kingma & Ba, Algorithm 1) on the raw parameters.
    Returns (raw_new, m_new, v_new, activated_new), all float64."""
    g = raw_grads(raw, g_act, weights)
    raw_new, m_new, v_new = {}, {}, {}
    for k in RAW:
        p = raw[k].astype(np.float64)
        mk = beta1 * m[k].astype(np.float64) + (1 - beta1) * g[k]
        vk = beta2 * v[k].astype(np.float64) + (1 - beta2) * g[k] * g[k]
        mhat = mk / (1 - beta1 ** t)
        vhat = vk / (1 - beta2 ** t)
        raw_new[k] = p - lrs[k] * mhat / (np.sqrt(vhat) + eps)
        m_new[k], v_new[k] = mk, vk
    return raw_new, m_new, v_new, activate(raw_new, weights)
