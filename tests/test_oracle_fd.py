"""Pin of the oracle's adjoint: central finite differences of its own
float64 forward (brute force), per parameter, on tiny scenes.

Smooth regime: alpha_min = 0 (so every rectangle is the whole detector),
t_min = 0 and o <= 0.9 (no clamp): the forward is then a smooth function of
every parameter and the adjoint must match the differences to ~1e-6.
A second test takes a random direction through all parameters with the
usual thresholds, where the forward is piecewise smooth.
"""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S

D = S.DETECTOR_SIDE
KEYS = ("means", "scales", "quats", "opacity", "intensity")


def _tiny(seed, n=5, W=16, views=2):
    rng = np.random.default_rng(seed)
    g = {
        "means": rng.uniform(-0.6, 0.6, (n, 3)),
        "scales": np.exp(rng.normal(math.log(0.25), 0.3, (n, 3))),
        "quats": rng.normal(size=(n, 4)),
        "opacity": rng.uniform(0.2, 0.9, n),
        "intensity": rng.uniform(0.1, 1.0, n),
    }
    cams = [O.camera(float(rng.uniform(0, 2 * math.pi)), S.L_SO, S.L_SD, W, W + 3 * v, D, D)
            for v in range(views)]
    npx = sum(c.width * c.height for c in cams)
    up = rng.normal(size=npx).astype(np.float32)
    return g, cams, up


def _loss(g, cams, st, up):
    img = np.concatenate([O.render_brute(g, c, st)["image"] for c in cams])
    return float(np.dot(img, up.astype(np.float64)))


@pytest.mark.parametrize("seed,lowpass", [(1, 0.3), (2, 0.0), (3, 0.3)])
def test_adjoint_matches_central_differences_smooth(seed, lowpass):
    st = O.Settings(alpha_min=0.0, t_min=0.0, lowpass=lowpass, tile=8)
    g, cams, up = _tiny(seed)
    grad = O.backward(g, cams, st, up)
    for key in KEYS:
        fd = np.zeros_like(g[key])
        flat = g[key].reshape(-1)
        for k in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[k]))
            x0 = flat[k]
            flat[k] = x0 + h
            lp = _loss(g, cams, st, up)
            flat[k] = x0 - h
            lm = _loss(g, cams, st, up)
            flat[k] = x0
            fd.reshape(-1)[k] = (lp - lm) / (2 * h)
        err = np.linalg.norm(grad[key] - fd) / max(np.linalg.norm(fd), 1e-30)
        assert err < 1e-6, (key, err)


def test_adjoint_directional_derivative_with_thresholds():
    st = O.Settings(tile=8)
    rng = np.random.default_rng(12)
    n, W = 40, 32
    g = {k: v.astype(np.float64) for k, v in S.gaussians(n, math.log(0.08), 0.3, 77).items()}
    cams = [O.camera(float(rng.uniform(0, 6.28)), S.L_SO, S.L_SD, W, W, D, D) for _ in range(2)]
    up = rng.normal(size=2 * W * W).astype(np.float32)
    grad = O.backward(g, cams, st, up)
    d = {k: rng.normal(size=v.shape) for k, v in g.items()}
    h = 1e-7
    gp = {k: g[k] + h * d[k] for k in g}
    gm = {k: g[k] - h * d[k] for k in g}
    fd = (_loss(gp, cams, st, up) - _loss(gm, cams, st, up)) / (2 * h)
    an = sum(float(np.sum(grad[k] * d[k])) for k in g)
    assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)


def test_adjoint_binned_equals_brute():
    st = O.Settings(tile=8)
    g = S.gaussians(300, math.log(0.05), 0.3, 5)
    cams = [O.camera(a, S.L_SO, S.L_SD, 48, 40, D, D) for a in (0.4, 2.9)]
    up = np.random.default_rng(1).normal(size=2 * 48 * 40).astype(np.float32)
    pr = O.pairs(g, cams, st)
    a = O.backward(g, cams, st, up)
    b = O.backward(g, cams, st, up, binned=(pr["values"], pr["ranges"]))
    # the two traversals visit the same contributors; only the float64
    # summation order of the per-pixel terms differs
    for k in KEYS:
        np.testing.assert_allclose(a[k], b[k], rtol=0, atol=1e-12 * np.abs(a[k]).max())


def test_adjoint_selection_is_exact_for_selected():
    st = O.Settings(tile=16)
    g = S.gaussians(500, math.log(0.05), 0.3, 6)
    cams = [O.camera(a, S.L_SO, S.L_SD, 64, 64, D, D) for a in (1.0, 4.0)]
    up = np.random.default_rng(2).normal(size=2 * 64 * 64).astype(np.float32)
    full = O.backward(g, cams, st, up)
    sel = np.zeros(500, bool)
    sel[::37] = True
    part = O.backward(g, cams, st, up, sel=sel)
    for k in KEYS:
        np.testing.assert_allclose(part[k][sel], full[k][sel], rtol=0,
                                   atol=1e-12 * np.abs(full[k]).max())
