"""Pins of the optimiser oracle: torch.optim.Adam on the chain-ruled raw
gradients (a library routine, float64 CPU), the first-step closed form,
finite differences of the activations, and the learning-rate schedule."""
import numpy as np
import pytest
import torch

from oracle import adam as A


def _state(n, seed):
    rng = np.random.default_rng(seed)
    raw = {"means": rng.uniform(-1, 1, (n, 3)), "log_scales": rng.normal(np.log(0.02), 0.3, (n, 3)),
           "quats": rng.normal(size=(n, 4)), "opacity_logit": rng.normal(size=n),
           "feature": rng.normal(size=n)}
    g = {"means": rng.normal(size=(n, 3)), "scales": rng.normal(size=(n, 3)) * 10,
         "quats": rng.normal(size=(n, 4)) * 0.1, "opacity": rng.normal(size=n),
         "intensity": rng.normal(size=n)}
    return raw, g


def test_matches_torch_adam_over_several_steps():
    raw, _ = _state(50, 1)
    lam = 1.7
    m = {k: np.zeros_like(v) for k, v in raw.items()}
    v = {k: np.zeros_like(x) for k, x in raw.items()}
    tp = {k: torch.tensor(x, dtype=torch.float64, requires_grad=True) for k, x in raw.items()}
    lrs0 = A.paper_lrs(1)
    opt = torch.optim.Adam([{"params": [tp[k]], "lr": lrs0[k]} for k in A.RAW],
                           betas=(0.9, 0.999), eps=1e-15)
    cur = {k: x.copy() for k, x in raw.items()}
    rng = np.random.default_rng(3)
    for t in range(1, 6):
        _, g = _state(50, 100 + t)
        lrs = A.paper_lrs(t)
        new, m, v, act = A.adam_step(cur, g, m, v, t, lrs, feature_weight=lam)
        # torch: set raw-parameter gradients by the same chain rule, then step
        rg = A.raw_grads({k: tp[k].detach().numpy() for k in A.RAW}, g, lam)
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
    z = {k: np.zeros_like(x) for k, x in raw.items()}
    lrs = {k: 0.01 for k in A.RAW}
    new, m, v, _ = A.adam_step(raw, g, z, z, 1, lrs)
    rg = A.raw_grads(raw, g)
    for k in A.RAW:
        # m_hat = g and v_hat = g^2 at t = 1, so the step is -lr * g / (|g| + eps)
        np.testing.assert_allclose(raw[k] - new[k], 0.01 * np.sign(rg[k]), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(m[k], 0.1 * rg[k], rtol=1e-14)
        np.testing.assert_allclose(v[k], 0.001 * rg[k] ** 2, rtol=1e-14)


@pytest.mark.parametrize("lam", [1.0, 0.5])
def test_activation_chain_rule_by_finite_differences(lam):
    raw, g = _state(8, 4)
    rg = A.raw_grads(raw, g, lam)
    def L(r):
        a = A.activate(r, lam)
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
    assert (lr["feature"], lr["opacity_logit"], lr["log_scales"], lr["quats"]) == (2e-3, 8e-3, 5e-3, 1e-3)
