"""Pins of the optimiser and intensity-response oracle: torch.optim.Adam on
the chain-ruled raw gradients (a library routine, float64 CPU), the
first-step closed form, torch autograd and finite differences of the
activations, special cases of Eq. 3, and the learning-rate schedule."""
import numpy as np
import pytest
import torch

from oracle import adam as A


def _state(n, seed, nf=16):
    rng = np.random.default_rng(seed)
    raw = {"means": rng.uniform(-1, 1, (n, 3)), "log_scales": rng.normal(np.log(0.02), 0.3, (n, 3)),
           "quats": rng.normal(size=(n, 4)), "opacity_logit": rng.normal(size=n),
           "features": rng.normal(size=(n, nf)) * 0.3}
    g = {"means": rng.normal(size=(n, 3)), "scales": rng.normal(size=(n, 3)) * 10,
         "quats": rng.normal(size=(n, 4)) * 0.1, "opacity": rng.normal(size=n),
         "intensity": rng.normal(size=n)}
    return raw, g


def _weights(nf, seed=9):
    return np.random.default_rng(seed).uniform(0.2, 1.5, nf)


def test_rirf_special_cases():
    f = np.random.default_rng(1).normal(size=(20, 1))
    # one feature: sigmoid(lambda f)
    np.testing.assert_allclose(A.rirf(f, [1.7]), 1 / (1 + np.exp(-1.7 * f[:, 0])), rtol=1e-15)
    # zero weights: intensity 1/2 and no gradient
    f16 = np.random.default_rng(2).normal(size=(20, 16))
    np.testing.assert_array_equal(A.rirf(f16, np.zeros(16)), 0.5)
    np.testing.assert_array_equal(A.rirf_grad(f16, np.zeros(16), np.ones(20)), 0.0)
    # features orthogonal to the weights leave the intensity at 1/2
    w = _weights(16)
    f_orth = f16 - np.outer(f16 @ w / (w @ w), w)
    np.testing.assert_allclose(A.rirf(f_orth, w), 0.5, atol=1e-14)


def test_rirf_gradient_against_torch_autograd():
    f = np.random.default_rng(3).normal(size=(30, 16))
    w = _weights(16)
    gi = np.random.default_rng(4).normal(size=30)
    ft = torch.tensor(f, requires_grad=True)
    (torch.sigmoid(ft @ torch.tensor(w)) * torch.tensor(gi)).sum().backward()
    np.testing.assert_allclose(A.rirf_grad(f, w, gi), ft.grad.numpy(), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("nf", [1, 16])
def test_matches_torch_adam_over_several_steps(nf):
    raw, _ = _state(50, 1, nf)
    w = _weights(nf)
    m = {k: np.zeros_like(v) for k, v in raw.items()}
    v = {k: np.zeros_like(x) for k, x in raw.items()}
    tp = {k: torch.tensor(x, dtype=torch.float64, requires_grad=True) for k, x in raw.items()}
    lrs0 = A.paper_lrs(1)
    opt = torch.optim.Adam([{"params": [tp[k]], "lr": lrs0[k]} for k in A.RAW],
                           betas=(0.9, 0.999), eps=1e-15)
    cur = {k: x.copy() for k, x in raw.items()}
    for t in range(1, 6):
        _, g = _state(50, 100 + t, nf)
        lrs = A.paper_lrs(t)
        new, m, v, act = A.adam_step(cur, g, m, v, t, lrs, w)
        # torch: set raw-parameter gradients by the same chain rule, then step
        rg = A.raw_grads({k: tp[k].detach().numpy() for k in A.RAW}, g, w)
        for gi, k in enumerate(A.RAW):
            tp[k].grad = torch.tensor(rg[k])
            opt.param_groups[gi]["lr"] = lrs[k]
        opt.step()
        for k in A.RAW:
            np.testing.assert_allclose(new[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)
        cur = new
    np.testing.assert_allclose(act["scales"], np.exp(cur["log_scales"]), rtol=1e-15)


def test_first_step_is_sign_of_gradient():
    raw, g = _state(40, 2)
    w = _weights(16)
    z = {k: np.zeros_like(x) for k, x in raw.items()}
    lrs = {k: 0.01 for k in A.RAW}
    new, m, v, _ = A.adam_step(raw, g, z, z, 1, lrs, w)
    rg = A.raw_grads(raw, g, w)
    for k in A.RAW:
        # m_hat = g and v_hat = g^2 at t = 1, so the step is -lr * g / (|g| + eps)
        np.testing.assert_allclose(raw[k] - new[k], 0.01 * np.sign(rg[k]), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(m[k], 0.1 * rg[k], rtol=1e-14)
        np.testing.assert_allclose(v[k], 0.001 * rg[k] ** 2, rtol=1e-14)


@pytest.mark.parametrize("nf", [1, 4])
def test_activation_chain_rule_by_finite_differences(nf):
    raw, g = _state(8, 4, nf)
    w = _weights(nf)
    rg = A.raw_grads(raw, g, w)
    def L(r):
        a = A.activate(r, w)
        return sum(float(np.sum(a[k] * g[k])) for k in A.ACT)
    for k in A.RAW:
        flat = raw[k].reshape(-1)
        for j in range(0, flat.size, 3):
            h = 1e-6
            x0 = flat[j]
            flat[j] = x0 + h; lp = L(raw)
            flat[j] = x0 - h; lm = L(raw)
            flat[j] = x0
            assert abs((lp - lm) / (2 * h) - rg[k].reshape(-1)[j]) <= 1e-6 * max(1.0, abs(rg[k].reshape(-1)[j]))


def test_position_learning_rate_schedule():
    assert A.paper_lrs(1)["means"] == pytest.approx(1.9e-4, rel=1e-12)
    assert A.paper_lrs(20001)["means"] == pytest.approx(1.9e-6, rel=1e-12)
    assert A.paper_lrs(10001)["means"] == pytest.approx(1.9e-5, rel=1e-12)   # geometric midpoint
    assert A.paper_lrs(50000)["means"] == pytest.approx(1.9e-6, rel=1e-12)
    lr = A.paper_lrs(7)
    assert (lr["features"], lr["opacity_logit"], lr["log_scales"], lr["quats"]) == (2e-3, 8e-3, 5e-3, 1e-3)
