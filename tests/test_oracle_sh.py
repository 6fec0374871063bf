"""Pins of the spherical-harmonics colour oracle: the basis against
scipy's complex spherical harmonics (Condon-Shortley phase) turned real,
orthonormality by quadrature over the sphere, the source position of the
Eq. 12 camera, and colours in closed form for degree 0 and an axis-aligned
degree-1 case."""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle as O
from oracle import sh as H


def _real_from_scipy(dirs, degree):
    x, y, z = dirs.T
    theta = np.arccos(np.clip(z, -1, 1))          # polar
    phi = np.arctan2(y, x)                         # azimuth
    cols = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            if hasattr(sp, "sph_harm_y"):
                c = sp.sph_harm_y(l, abs(m), theta, phi)
            else:
                c = sp.sph_harm(abs(m), l, phi, theta)
            if m < 0:
                cols.append(math.sqrt(2) * c.imag)
            elif m == 0:
                cols.append(c.real)
            else:
                cols.append(math.sqrt(2) * c.real)
    return np.stack(cols, axis=1)


def _dirs(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_basis_matches_scipy(degree):
    d = _dirs(500, degree)
    np.testing.assert_allclose(H.basis(d, degree), _real_from_scipy(d, degree), atol=1e-12)


def test_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform in phi: exact for these polynomials
    nt, nphi = 16, 32
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    C, P = np.meshgrid(ct, ph, indexing="ij")
    st = np.sqrt(1 - C * C)
    d = np.stack([st * np.cos(P), st * np.sin(P), C], axis=-1).reshape(-1, 3)
    w = (wt[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    Y = H.basis(d, 3)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_source_position_of_eq12_camera():
    for phi in (0.0, 0.7, math.pi / 2, 4.0):
        cam = O.camera(phi, 4.0, 6.0, 64, 64, 5.7646, 5.7646)
        np.testing.assert_allclose(H.source_position(cam),
                                   [4 * math.cos(phi), 4 * math.sin(phi), 0.0], atol=1e-5)


def test_colour_closed_forms():
    cam = O.camera(0.0, 4.0, 6.0, 64, 64, 5.7646, 5.7646)      # source at (4, 0, 0)
    means = np.array([[0.0, 0.0, 0.0], [4.0, 0.0, 2.0]], np.float32)
    k0 = np.array([[[0.3, -0.2, 5.0]], [[-9.0, 0.1, 0.0]]], np.float32)
    c = H.colors(means, k0, [cam], 0)[0]
    y0 = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(c[0], [0.3 * y0 + 0.5, -0.2 * y0 + 0.5, 5.0 * y0 + 0.5], rtol=1e-6)
    np.testing.assert_allclose(c[1], [0.0, 0.1 * y0 + 0.5, 0.5], rtol=1e-6)   # clamped red
    # degree 1: the direction from the source to the origin is -x, so only
    # the m = 1 term (-c1 x) contributes: +c1 per unit coefficient
    k1 = np.zeros((1, 4, 3), np.float32)
    k1[0, 3] = [1.0, 0.0, -1.0]
    k1[0, 1] = [7.0, 7.0, 7.0]        # m = -1 (y) and m = 0 (z) vanish on this ray
    k1[0, 2] = [7.0, 7.0, 7.0]
    c1 = math.sqrt(3 / (4 * math.pi))
    c = H.colors(means[:1], k1, [cam], 1)[0, 0]
    np.testing.assert_allclose(c, [0.5 + c1, 0.5, 0.5 - c1], rtol=1e-6, atol=1e-7)


def test_rgb_render_unit_colour_telescopes():
    """Every channel at colour 1 (degree-0 coefficient (1 - 1/2) / Y_0) gives
    I = 1 - T per pixel (the blending weights telescope), on two views."""
    import scenes as S
    g = S.gaussians(300, math.log(0.05), 0.3, 5)
    cams = [O.camera(a, S.L_SO, S.L_SD, 48, 40, S.DETECTOR_SIDE, S.DETECTOR_SIDE) for a in (0.3, 2.0)]
    k = np.zeros((300, 1, 3), np.float32)
    k[:, 0, :] = 0.5 * 2.0 * math.sqrt(math.pi)
    r = H.render_rgb(g, k, cams, O.Settings(tile=16), 0)
    assert r["image"].shape == (3, 2 * 48 * 40)
    for c in range(3):
        np.testing.assert_allclose(r["image"][c], 1.0 - r["final_t"], atol=1e-12)
    assert r["final_t"].min() < 0.9     # the scene covers the detector


def test_rgb_render_channels_are_linear_in_colour():
    """A channel equals the radiative render with that channel's colours as
    the intensity (the view's own lists, all views' pairs built at once)."""
    import scenes as S
    g = S.gaussians(200, math.log(0.05), 0.3, 9)
    cams = [O.camera(1.1, S.L_SO, S.L_SD, 40, 40, S.DETECTOR_SIDE, S.DETECTOR_SIDE)]
    k = np.random.default_rng(2).normal(0, 0.3, size=(200, 4, 3)).astype(np.float32)
    st = O.Settings(tile=16)
    r = H.render_rgb(g, k, cams, st, 1)
    gg = dict(g)
    gg["intensity"] = r["colors"][0, :, 1]
    pr = O.pairs(g, cams, st)
    ref = O.render_binned(gg, cams, st, pr["values"], pr["ranges"])
    np.testing.assert_allclose(r["image"][1], ref["image"], atol=1e-14)
