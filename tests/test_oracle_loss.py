"""Pins of the Eq. 11 loss oracle: closed forms of SSIM (equal images,
constant images away from the border), torch autograd of the same
definition written with conv2d (float64), and finite differences."""
import numpy as np
import pytest
import torch

from oracle import loss as Lo


def test_window_is_normalised_gaussian():
    w = Lo.window_1d()
    assert w.shape == (11,) and abs(w.sum() - 1) < 1e-15
    assert w[5] == w.max() and np.allclose(w, w[::-1])
    np.testing.assert_allclose(w[6] / w[5], np.exp(-1 / (2 * 1.5 ** 2)), rtol=1e-14)


def test_equal_images_have_unit_ssim_and_zero_ssim_gradient():
    x = np.random.default_rng(1).uniform(size=(23, 17))
    np.testing.assert_allclose(Lo.ssim_map(x, x), 1.0, rtol=1e-12)
    np.testing.assert_allclose(Lo.ssim_map_grad(x, x), 0.0, atol=1e-12)


def test_constant_images_interior_closed_form():
    a, b = 0.3, 0.7
    x = np.full((30, 30), a)
    y = np.full((30, 30), b)
    s = Lo.ssim_map(x, y)
    # at least 5 pixels from the border the window sees only the constants
    ref = (2 * a * b + Lo.C1) * Lo.C2 / ((a * a + b * b + Lo.C1) * Lo.C2)
    np.testing.assert_allclose(s[5:-5, 5:-5], ref, rtol=1e-12)


def _torch_ssim_sum(x, y):
    w1 = torch.tensor(Lo.window_1d())
    w2 = (w1[:, None] * w1[None, :])[None, None]
    f = lambda t: torch.nn.functional.conv2d(t[None, None], w2, padding=5)[0, 0]
    mx, my = f(x), f(y)
    sxx, syy, sxy = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    s = ((2 * mx * my + Lo.C1) * (2 * sxy + Lo.C2)) / ((mx * mx + my * my + Lo.C1) * (sxx + syy + Lo.C2))
    return s.sum()


def test_ssim_and_gradient_against_torch_autograd():
    rng = np.random.default_rng(2)
    x = rng.uniform(size=(19, 26))
    y = np.clip(x + rng.normal(scale=0.1, size=x.shape), 0, 1)
    xt = torch.tensor(x, requires_grad=True)
    s = _torch_ssim_sum(xt, torch.tensor(y))
    s.backward()
    np.testing.assert_allclose(Lo.ssim_map(x, y).sum(), float(s.detach()), rtol=1e-13)
    np.testing.assert_allclose(Lo.ssim_map_grad(x, y), xt.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_loss_gradient_by_finite_differences():
    rng = np.random.default_rng(3)
    sizes = [(9, 7), (6, 11)]
    n = sum(w * h for w, h in sizes)
    x = rng.uniform(size=n)
    y = rng.uniform(size=n)
    L, g = Lo.loss_and_grad(x, y, sizes, 0.2)
    for j in range(0, n, 7):
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (Lo.loss_and_grad(xp, y, sizes)[0] - Lo.loss_and_grad(xm, y, sizes)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 + 1e-6 * abs(g[j]), (j, fd, g[j])


def test_gamma_zero_is_l1():
    rng = np.random.default_rng(4)
    x, y = rng.uniform(size=50), rng.uniform(size=50)
    L, g = Lo.loss_and_grad(x, y, [(10, 5)], 0.0)
    assert L == pytest.approx(np.abs(x - y).mean(), rel=1e-14)
    np.testing.assert_allclose(g, np.sign(x - y) / 50, rtol=1e-14)
