"""FP64 oracle of the spherical-harmonics colour model (TEST INFRASTRUCTURE ONLY).

The comparison model of Sec. 3.1 / Tab. 3a: the RGB Gaussian of 3D Gaussian
splatting, whose colour at view direction d is Eq. 2,
c(d, k) = sum_{l <= L} sum_{|m| <= l} k_l^m Y_l^m(d), one coefficient
triple (RGB) per basis function, blended like the radiative intensity
(Eq. 10) channel by channel.

Readings (the paper defers Y to its supplement): Y_l^m are the real
spherical harmonics with the Condon-Shortley phase, m < 0 from the sine and
m > 0 from the cosine part, evaluated on the unit direction from the X-ray
source to the Gaussian centre; basis index l^2 + l + m.  As in the cited
3D Gaussian splatting the colour is max(c + 1/2, 0).  Coefficients are laid
out [Gaussian][basis][channel].  The source position is -R^T t of the
float32 camera (Eq. 12: L_SO (cos phi, sin phi, 0)).
"""
from __future__ import annotations

import math

import numpy as np


def n_basis(degree: int) -> int:
    return (degree + 1) ** 2


def basis(dirs: np.ndarray, degree: int) -> np.ndarray:
    """Real SH Y_{l,m}(d) of unit directions dirs [m, 3] -> [m, (L+1)^2], float64.

    Cartesian forms of the real harmonics, each normalised so that its
    square integrates to 1 over the sphere; constants written from their
    closed forms."""
    d = np.asarray(dirs, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [np.full_like(x, 0.5 / math.sqrt(pi))]                      # l = 0
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [-c1 * y, c1 * z, -c1 * x]                              # m = -1, 0, 1
    if degree >= 2:
        a = 0.5 * math.sqrt(15.0 / pi)
        b = 0.25 * math.sqrt(5.0 / pi)
        c = 0.25 * math.sqrt(15.0 / pi)
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z,
                c * (x * x - y * y)]
    if degree >= 3:
        c33 = 0.25 * math.sqrt(35.0 / (2.0 * pi))
        c32 = 0.5 * math.sqrt(105.0 / pi)
        c31 = 0.25 * math.sqrt(21.0 / (2.0 * pi))
        c30 = 0.25 * math.sqrt(7.0 / pi)
        c32b = 0.25 * math.sqrt(105.0 / pi)
        r2 = x * x + y * y
        out += [-c33 * y * (3 * x * x - y * y), c32 * x * y * z, -c31 * y * (4 * z * z - r2),
                c30 * z * (2 * z * z - 3 * r2), -c31 * x * (4 * z * z - r2),
                c32b * z * (x * x - y * y), -c33 * x * (x * x - 3 * y * y)]
    if degree > 3:
        raise ValueError("degree <= 3")
    return np.stack(out, axis=1)


def source_position(cam) -> np.ndarray:
    """World position of the source, -R^T t, from the float32 camera."""
    r = np.array(cam.rot[:], np.float64).reshape(3, 3)
    t = np.array(cam.trans[:], np.float64)
    return -r.T @ t


def colors(means, sh, cams, degree: int) -> np.ndarray:
    """Per view and Gaussian RGB colour [V, n, 3] (Eq. 2, clamped as read)."""
    mu = np.asarray(means, np.float64)
    k = np.asarray(sh, np.float64).reshape(mu.shape[0], -1, 3)[:, :n_basis(degree), :]
    out = []
    for cam in cams:
        v = mu - source_position(cam)[None, :]
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        y = basis(v, degree)
        out.append(np.maximum(np.einsum("nb,nbc->nc", y, k) + 0.5, 0.0))
    return np.stack(out)


def render_rgb(g: dict, sh, cams, st, degree: int) -> dict:
    """Eq. 10 for each colour channel, the channel of the view's SH colour
    taking the place of the intensity; views one at a time over their own
    tile lists.  image is [3, total pixels] (planar), the others per pixel."""
    from . import pairs, render_binned
    col = colors(g["means"], sh, cams, degree)
    planes = [[], [], []]
    final_t, n_contrib, flags = [], [], []
    for v, cam in enumerate(cams):
        pr = pairs(g, [cam], st)
        for c in range(3):
            gc = dict(g)
            gc["intensity"] = col[v, :, c]
            r = render_binned(gc, [cam], st, pr["values"], pr["ranges"])
            planes[c].append(r["image"])
        final_t.append(r["final_t"])
        n_contrib.append(r["n_contrib"])
        flags.append(r["flags"])
    return {"image": np.stack([np.concatenate(p) for p in planes]),
            "final_t": np.concatenate(final_t), "n_contrib": np.concatenate(n_contrib),
            "flags": np.concatenate(flags), "colors": col}
