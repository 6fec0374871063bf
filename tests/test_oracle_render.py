"""Pins of the oracle's blending (Eq. 10) and tile lists (Sec. 3.2).

Closed forms worked out by hand for one and two Gaussians, the exact
integral of a 2-D Gaussian (mass), telescoping and monotonicity
invariants, permutation invariance, the small-opacity (linear
superposition) limit, and brute force == binned traversal.
"""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S

D = S.DETECTOR_SIDE


def _cam(phi, W, H=None):
    return O.camera(phi, S.L_SO, S.L_SD, W, W if H is None else H, D, D)


def _gs(rows):
    """rows: list of (mean, scale, quat, opacity, intensity)."""
    return {"means": np.array([r[0] for r in rows], np.float32),
            "scales": np.array([r[1] for r in rows], np.float32),
            "quats": np.array([r[2] for r in rows], np.float32),
            "opacity": np.array([r[3] for r in rows], np.float32),
            "intensity": np.array([r[4] for r in rows], np.float32)}


def _f32(x):
    return float(np.float32(x))


@pytest.mark.parametrize("lowpass", [0.0, 0.3])
def test_single_gaussian_closed_form_footprint(lowpass):
    """One Gaussian at the origin, q = identity, phi = 0: its image is
    i * min(alpha_max, o exp(-x^2/(2 Sxx) - y^2/(2 Syy))) inside its
    rectangle where that is >= alpha_min, with Sxx = (f s_y/L_SO)^2 + k and
    Syy = (f s_z/L_SO)^2 + k worked out from Eq. 8-9, u = (W/2, H/2)."""
    W = 64
    st = O.Settings(lowpass=lowpass)
    s = (0.05, 0.04, 0.07)
    o, inten = 0.9, 0.6
    g = _gs([((0, 0, 0), s, (1, 0, 0, 0), o, inten)])
    c = _cam(0.0, W)
    r = O.render_brute(g, c, st)
    f = _f32(S.L_SD * W / D)
    k = _f32(lowpass)
    sxx = (f * _f32(s[1]) / S.L_SO) ** 2 + k
    syy = (f * _f32(s[2]) / S.L_SO) ** 2 + k
    kap = -2.0 * math.log(_f32(1 / 255))
    y, x = np.mgrid[0:W, 0:W]
    dx, dy = x + 0.5 - W / 2, y + 0.5 - W / 2
    a = _f32(o) * np.exp(-0.5 * (dx * dx / sxx + dy * dy / syy))
    alpha = np.minimum(_f32(0.99), a)
    rx, ry = math.sqrt(kap * sxx), math.sqrt(kap * syy)
    inrect = (np.abs(dx) <= rx) & (np.abs(dy) <= ry)
    want = np.where(inrect & (alpha >= _f32(1 / 255)), _f32(inten) * alpha, 0.0).ravel()
    # pixels whose decision sits within 1e-9 of a threshold are compared loosely
    np.testing.assert_allclose(r["image"], want, atol=1e-12)
    np.testing.assert_allclose(r["final_t"], 1.0 - want / _f32(inten), atol=1e-12)


def test_single_gaussian_mass():
    """Sum over pixels ~ i * integral of o exp(-m^2/2) over {o exp(-m^2/2) >= alpha_min}
    = i * 2 pi sqrt(det Sigma'') (o - alpha_min)."""
    W = 128
    st = O.Settings(lowpass=0.3)
    rng = np.random.default_rng(3)
    for _ in range(5):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        s = tuple(np.exp(rng.normal(math.log(0.05), 0.2, 3)))
        o = float(rng.uniform(0.2, 0.95))
        g = _gs([((0.1, -0.2, 0.05), s, tuple(q), o, 1.0)])
        c = _cam(float(rng.uniform(0, 6.28)), W)
        r = O.render_brute(g, c, st)
        p = O.project(g, c, st)
        sxx, sxy, syy = p["sig"][0]
        det = sxx * syy - sxy * sxy
        mass = 2 * math.pi * math.sqrt(det) * (_f32(o) - _f32(1 / 255))
        assert abs(r["image"].sum() - mass) <= 0.01 * mass


def test_two_gaussians_closed_form():
    """Two Gaussians on the principal ray at depths 3.5 and 4.5 (phi = 0, so
    t_z = L_SO - x): I = i1 a1 + i2 a2 (1 - a1), nearer first."""
    W = 32
    st = O.Settings(lowpass=0.3)
    s1, s2 = (0.05, 0.06, 0.05), (0.05, 0.09, 0.08)
    g = _gs([((-0.5, 0, 0), s2, (1, 0, 0, 0), 0.7, 0.3),   # far (t_z = 4.5), index 0
             ((0.5, 0, 0), s1, (1, 0, 0, 0), 0.6, 0.9)])   # near (t_z = 3.5), index 1
    c = _cam(0.0, W)
    r = O.render_brute(g, c, st)
    f = _f32(S.L_SD * W / D)
    k = _f32(0.3)
    y, x = np.mgrid[0:W, 0:W]
    dx, dy = x + 0.5 - W / 2, y + 0.5 - W / 2

    kap = -2.0 * math.log(_f32(1 / 255))

    def alpha(s, tz, o):
        sxx = (f * _f32(s[1]) / tz) ** 2 + k
        syy = (f * _f32(s[2]) / tz) ** 2 + k
        a = np.minimum(_f32(0.99), _f32(o) * np.exp(-0.5 * (dx * dx / sxx + dy * dy / syy)))
        inrect = (np.abs(dx) <= math.sqrt(kap * sxx)) & (np.abs(dy) <= math.sqrt(kap * syy))
        return np.where(inrect & (a >= _f32(1 / 255)), a, 0.0)

    a1, a2 = alpha(s1, 3.5, 0.6), alpha(s2, 4.5, 0.7)
    want = _f32(0.9) * a1 + _f32(0.3) * a2 * (1 - a1)
    np.testing.assert_allclose(r["image"], want.ravel(), atol=1e-12)
    # the near one (index 1) is blended first, so it is never the last contributor alone
    assert np.all(r["last"][(a2.ravel() > 0)] == 0)


def _scene(n, W, seed, s0=0.05, views=1):
    g = S.gaussians(n, math.log(s0), 0.3, seed)
    rng = np.random.default_rng(seed + 1)
    cams = [_cam(float(rng.uniform(0, 2 * math.pi)), W) for _ in range(views)]
    return g, cams


def test_compositing_invariants():
    st = O.Settings()
    g, cams = _scene(600, 48, 11)
    r = O.render_brute(g, cams[0], st)
    T = r["final_t"]
    assert np.all(T <= 1.0) and np.all(T >= st.t_min * (1 - 1e-6))
    assert np.all(r["image"] <= (1 - T) * g["intensity"].max() + 1e-12)
    assert np.all(r["image"] >= 0)
    # telescoping: with every intensity 1, I = 1 - T_final exactly (up to rounding)
    g1 = dict(g)
    g1["intensity"] = np.ones_like(g["intensity"])
    r1 = O.render_brute(g1, cams[0], st)
    np.testing.assert_allclose(r1["image"], 1.0 - r1["final_t"], atol=1e-12)


def test_alpha_clamp():
    """An o = 1 Gaussian centred on a pixel centre gives alpha = alpha_max there."""
    W = 32
    st = O.Settings()
    # u = (W/2, H/2) falls on a pixel corner; shift by half a pixel along world y
    f = _f32(S.L_SD * W / D)
    shift = 0.5 * S.L_SO / f
    g = _gs([((0, shift, -shift), (0.05, 0.05, 0.05), (1, 0, 0, 0), 1.0, 0.8)])
    c = _cam(0.0, W)
    p = O.project(g, c, st)
    assert np.abs(p["u"][0] - (W / 2 + 0.5)).max() < 1e-5
    r = O.render_brute(g, c, st, pix=np.array([(W // 2) * W + W // 2], np.int32))
    # the pixel centre is within 1e-5 px of u, so a = exp(-tiny) > alpha_max
    assert r["image"][0] == pytest.approx(_f32(0.99) * _f32(0.8), abs=1e-12)


def test_permutation_invariance():
    st = O.Settings()
    g, cams = _scene(400, 40, 21)
    perm = np.random.default_rng(5).permutation(400)
    gp = {k: v[perm] for k, v in g.items()}
    r = O.render_brute(g, cams[0], st)
    rp = O.render_brute(gp, cams[0], st)
    np.testing.assert_array_equal(r["image"], rp["image"])
    np.testing.assert_array_equal(r["final_t"], rp["final_t"])
    np.testing.assert_array_equal(perm[rp["last"][rp["last"] >= 0]], r["last"][r["last"] >= 0])


def test_disjoint_rects_order_free():
    """Gaussians whose rectangles are pairwise disjoint: depth order does not matter."""
    st = O.Settings()
    W = 64
    rows = []
    for gx in range(4):
        for gy in range(4):
            y = -0.75 + 0.5 * gx
            z = -0.75 + 0.5 * gy
            rows.append(((0.0, y, z), (0.02, 0.03, 0.02), (1, 0, 0, 0), 0.8, 0.1 + 0.05 * (gx + gy)))
    g = _gs(rows)
    c = _cam(0.0, W)
    p = O.project(g, c, st)
    rects = p["rect"]
    for a in range(len(rows)):
        for b in range(a + 1, len(rows)):
            ra, rb = rects[a], rects[b]
            assert ra[1] < rb[0] or rb[1] < ra[0] or ra[3] < rb[2] or rb[3] < ra[2]
    r0 = O.render_brute(g, c, st)
    g2 = dict(g)
    m = g["means"].copy()
    m[:, 0] = np.random.default_rng(1).uniform(-0.9, 0.9, len(rows))   # new depths
    g2["means"] = m
    # moving along the principal axis changes depth and scale; compare against the
    # sum of individually rendered Gaussians instead
    r2 = O.render_brute(g2, c, st)
    parts = sum(O.render_brute({k: v[j:j + 1] for k, v in g2.items()}, c, st)["image"]
                for j in range(len(rows)))
    np.testing.assert_allclose(r2["image"], parts, atol=1e-15)
    parts0 = sum(O.render_brute({k: v[j:j + 1] for k, v in g.items()}, c, st)["image"]
                 for j in range(len(rows)))
    np.testing.assert_allclose(r0["image"], parts0, atol=1e-15)


def test_small_opacity_linear_superposition():
    """alpha_min = 0, t_min = 0, o -> 0: I -> sum_j i_j o_j G_j(p) (Eq. 10 linearised)."""
    st = O.Settings(alpha_min=0.0, t_min=0.0)
    g, cams = _scene(50, 32, 31)
    g["opacity"] = np.full(50, 1e-4, np.float32)
    c = cams[0]
    r = O.render_brute(g, c, st)
    p = O.project(g, c, st)
    y, x = np.mgrid[0:32, 0:32]
    lin = np.zeros(32 * 32)
    for j in range(50):
        if not p["kept"][j]:
            continue
        A, B, Cc = p["conic"][j]
        dx = (x + 0.5 - p["u"][j][0]).ravel()
        dy = (y + 0.5 - p["u"][j][1]).ravel()
        G = np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy))
        lin += float(g["intensity"][j]) * float(g["opacity"][j]) * G
    # second-order terms are O(N * o) relative
    np.testing.assert_allclose(r["image"], lin, rtol=50 * 1e-4, atol=1e-12)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_brute_equals_binned(tile):
    st = O.Settings(tile=tile)
    g, cams = _scene(1500, 72, 41, views=2)
    cams.append(_cam(1.0, 40, 24))   # ragged, non-square view
    pr = O.pairs(g, cams, st)
    rb = O.render_binned(g, cams, st, pr["values"], pr["ranges"])
    brute = O.render_views(g, cams, st)
    np.testing.assert_array_equal(rb["image"], brute["image"])
    np.testing.assert_array_equal(rb["final_t"], brute["final_t"])
    np.testing.assert_array_equal(rb["evals"], brute["evals"])
    # n_contrib (list position) names the same last Gaussian as brute force
    off = 0
    toff = 0
    for c in cams:
        W, H = c.width, c.height
        txn = (W + tile - 1) // tile
        for py in range(H):
            for px in range(W):
                k = off + py * W + px
                nc = rb["n_contrib"][k]
                if nc == 0:
                    assert brute["last"][k] == -1
                else:
                    gt = toff + (py // tile) * txn + px // tile
                    assert pr["values"][pr["ranges"][gt][0] + nc - 1] == brute["last"][k]
        off += W * H
        toff += txn * ((H + tile - 1) // tile)


def test_tile_size_does_not_change_images():
    g, cams = _scene(800, 64, 51)
    imgs = []
    for tile in (8, 16, 32):
        st = O.Settings(tile=tile)
        pr = O.pairs(g, cams, st)
        imgs.append(O.render_binned(g, cams, st, pr["values"], pr["ranges"])["image"])
    np.testing.assert_array_equal(imgs[0], imgs[1])
    np.testing.assert_array_equal(imgs[0], imgs[2])


def test_rect_contains_every_contributing_pixel():
    """The float32 key-path rectangle contains every pixel where the float64
    alpha reaches alpha_min (checked without the rectangle, by brute force)."""
    st = O.Settings()
    W = 96
    g = S.gaussians(300, math.log(0.05), 0.6, 61)
    g["opacity"] = np.clip(g["opacity"] * 1.05, 0, 0.999).astype(np.float32)
    c = _cam(2.0, W)
    p = O.project(g, c, st)
    y, x = np.mgrid[0:W, 0:W]
    for j in range(300):
        if not p["kept"][j]:
            continue
        A, B, Cc = p["conic"][j]
        dx = x + 0.5 - p["u"][j][0]
        dy = y + 0.5 - p["u"][j][1]
        a = float(g["opacity"][j]) * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + Cc * dy * dy))
        ys, xs = np.nonzero(a >= st.alpha_min * (1 + 1e-9))
        xl, xh, yl, yh = p["rect"][j]
        assert np.all((xs >= xl) & (xs <= xh) & (ys >= yl) & (ys <= yh)), j
        # and the rectangle is the ellipse's bounding box: its extreme pixels
        # are within one pixel of the float64 bound
        kap = O.kappa(st.alpha_min)
        rx = math.sqrt(kap * p["sig"][j][0])
        ux = p["u"][j][0]
        if 0 < math.ceil(ux - rx - 0.5) and math.floor(ux + rx - 0.5) < W - 1:
            assert abs(xl - math.ceil(ux - rx - 0.5)) <= 1 and abs(xh - math.floor(ux + rx - 0.5)) <= 1
