"""Pins of the oracle's camera and projection (Eq. 7-9, Eq. 12) to closed forms.

None of these retype the oracle's formulas: they check it against values
worked out by hand from the paper's matrices, against geometric facts of
the scanner (source position, principal ray) and against the exact line
integral of a 3-D Gaussian along the X-ray through a pixel.
"""
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eq12_camera.txt")


def _rows(c):
    return np.array(c.rot, dtype=np.float64).reshape(3, 3), np.array(c.trans, dtype=np.float64)


def test_eq12_golden_matrices():
    """M_ext at phi = 0, pi/2, pi, 3pi/2 equals the hand-evaluated Eq. 12 entries."""
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 4
    for r in rows:
        phi = float(r[0]) * math.pi
        want = np.array([float(x) for x in r[1:]]).reshape(3, 4)
        c = O.camera(phi, 4.0, 6.0, 64, 64, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
        R, t = _rows(c)
        got = np.concatenate([R, t[:, None]], axis=1)
        np.testing.assert_allclose(got, want, atol=1e-7)


@pytest.mark.parametrize("phi", [0.0, 0.3, 1.9, 3.5, 5.9])
def test_rotation_proper_and_source_at_origin_of_camera(phi):
    c = O.camera(phi, S.L_SO, S.L_SD, 128, 96, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    R, t = _rows(c)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-7)
    assert abs(np.linalg.det(R) - 1.0) < 1e-6
    # the X-ray source sits on the scanner circle at L_SO (cos phi, sin phi, 0)
    src = S.L_SO * np.array([math.cos(phi), math.sin(phi), 0.0])
    np.testing.assert_allclose(R @ src + t, 0.0, atol=1e-6)
    # the principal ray (camera +z) points from the source to the rotation axis
    np.testing.assert_allclose(R[2], -src / S.L_SO, atol=1e-7)
    # elevation fixed at zero: camera y is the world -z axis (Sec. 3.3)
    np.testing.assert_allclose(R[1], [0, 0, -1], atol=0)


def test_intrinsics_focal_and_principal_point():
    for W, H in [(64, 64), (256, 256), (512, 512), (100, 60)]:
        c = O.camera(0.7, S.L_SO, S.L_SD, W, H, S.DETECTOR_SIDE, 0.5 * S.DETECTOR_SIDE)
        assert c.cx == W / 2 and c.cy == H / 2
        assert c.fx == np.float32(S.L_SD * W / S.DETECTOR_SIDE)
        assert c.fy == np.float32(S.L_SD * H / (0.5 * S.DETECTOR_SIDE))


def _one(mean, scale=(0.05, 0.05, 0.05), quat=(1, 0, 0, 0), o=0.8, i=0.7):
    return {"means": np.array([mean], np.float32), "scales": np.array([scale], np.float32),
            "quats": np.array([quat], np.float32), "opacity": np.array([o], np.float32),
            "intensity": np.array([i], np.float32)}


def test_origin_maps_to_principal_point_and_offaxis_point():
    st = O.Settings()
    for phi in [0.0, 1.1, 4.0]:
        c = O.camera(phi, S.L_SO, S.L_SD, 64, 64, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
        p = O.project(_one((0, 0, 0)), c, st)
        assert p["kept"][0]
        np.testing.assert_allclose(p["t"][0], [0, 0, S.L_SO], atol=1e-6)
        np.testing.assert_allclose(p["u"][0], [32.0, 32.0], atol=1e-5)
    # mu = (0, 1, 0) at phi = 0: camera x = world y, depth L_SO -> u_x = f/L_SO + W/2
    c = O.camera(0.0, S.L_SO, S.L_SD, 64, 64, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    p = O.project(_one((0, 1, 0)), c, st)
    f = float(np.float32(S.L_SD * 64 / S.DETECTOR_SIDE))
    np.testing.assert_allclose(p["u"][0], [f / S.L_SO + 32.0, 32.0], atol=1e-5)
    # mu = (0, 0, 1): world +z is image up, so u_y = H/2 - f/L_SO
    p = O.project(_one((0, 0, 1)), c, st)
    np.testing.assert_allclose(p["u"][0], [32.0, 32.0 - f / S.L_SO], atol=1e-5)


@pytest.mark.parametrize("lowpass", [0.0, 0.3])
def test_sigma2d_closed_form_on_axis(lowpass):
    """q = identity, phi = 0, mu = 0: Sigma'' = diag((f s_y/L)^2 + k, (f s_z/L)^2 + k)."""
    st = O.Settings(lowpass=lowpass)
    c = O.camera(0.0, S.L_SO, S.L_SD, 64, 64, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    s = (0.03, 0.05, 0.02)
    p = O.project(_one((0, 0, 0), scale=s), c, st)
    f = float(np.float32(S.L_SD * 64 / S.DETECTOR_SIDE))
    L = S.L_SO
    sy, sz = float(np.float32(s[1])), float(np.float32(s[2]))
    k = float(np.float32(lowpass))
    want = [(f * sy / L) ** 2 + k, 0.0, (f * sz / L) ** 2 + k]
    np.testing.assert_allclose(p["sig"][0], want, rtol=1e-12, atol=1e-12)
    sxx, sxy, syy = want
    np.testing.assert_allclose(p["conic"][0], [1 / sxx, 0.0, 1 / syy], rtol=1e-12)


def test_sigma2d_closed_form_off_axis():
    """mu = (0, m, 0) at phi = 0: Sxx = (f/L)^2 s_y^2 + (f m / L^2)^2 s_x^2 + k, Sxy = 0.

    The second term comes from the third column of J (Eq. 9)."""
    st = O.Settings(lowpass=0.3)
    c = O.camera(0.0, S.L_SO, S.L_SD, 64, 64, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    m = float(np.float32(0.75))
    s = np.array((0.04, 0.03, 0.02), np.float32).astype(np.float64)
    p = O.project(_one((0, m, 0), scale=tuple(s)), c, st)
    f = float(np.float32(S.L_SD * 64 / S.DETECTOR_SIDE))
    L = S.L_SO
    k = float(np.float32(0.3))
    sxx = (f / L) ** 2 * s[1] ** 2 + (f * m / L ** 2) ** 2 * s[0] ** 2 + k
    syy = (f / L) ** 2 * s[2] ** 2 + k
    np.testing.assert_allclose(p["sig"][0], [sxx, 0.0, syy], rtol=1e-12, atol=1e-14)


def _ray_integral_exponent(mu, Sigma, src, direction):
    """Exact line integral of exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)) along the ray
    src + s * direction is c * exp(-E/2); returns E (the ray's Mahalanobis
    distance from mu) and the normalisation c."""
    P = np.linalg.inv(Sigma)
    r = direction / np.linalg.norm(direction)
    a = src - mu
    rPr = r @ P @ r
    E = a @ P @ a - (a @ P @ r) ** 2 / rPr
    return E, math.sqrt(2 * math.pi / rPr)


def test_ewa_footprint_matches_exact_ray_integral():
    """The projected 2-D Gaussian (Eq. 8-9) approximates the exact X-ray line
    integral of the 3-D Gaussian through each pixel centre; for a small
    Gaussian the Mahalanobis exponents agree to O(sigma / depth)."""
    rng = np.random.default_rng(7)
    st = O.Settings(lowpass=0.0)
    W = H = 256
    for trial in range(6):
        phi = float(rng.uniform(0, 2 * math.pi))
        c = O.camera(phi, S.L_SO, S.L_SD, W, H, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
        R, t = _rows(c)
        mu = rng.uniform(-0.8, 0.8, 3).astype(np.float32)
        q = rng.normal(size=4).astype(np.float32)
        q /= np.linalg.norm(q)
        s = np.exp(rng.normal(math.log(0.01), 0.3, 3)).astype(np.float32)
        g = _one(tuple(mu), scale=tuple(s), quat=tuple(q))
        p = O.project(g, c, st)
        # 3-D covariance Sigma = R S S^T R^T, with R from scipy's quaternion
        # routine (scalar-last convention there)
        q64 = q.astype(np.float64)
        Rq = Rotation.from_quat([q64[1], q64[2], q64[3], q64[0]]).as_matrix()
        Sig3 = Rq @ np.diag(s.astype(np.float64) ** 2) @ Rq.T
        src = S.L_SO * np.array([math.cos(phi), math.sin(phi), 0.0])
        u = p["u"][0]
        Q = np.array([[p["conic"][0][0], p["conic"][0][1]], [p["conic"][0][1], p["conic"][0][2]]])
        sig_px = math.sqrt(max(p["sig"][0][0], p["sig"][0][2]))
        for dxp, dyp in [(0, 0), (1, 0), (0, 1), (1.5, -1), (-2, 0.5)]:
            pix = u + sig_px * np.array([dxp, dyp])
            # the detector pixel's ray in camera space, then world space
            dcam = np.array([(pix[0] - c.cx) / c.fx, (pix[1] - c.cy) / c.fy, 1.0])
            dworld = R.T @ dcam
            E, _ = _ray_integral_exponent(mu.astype(np.float64), Sig3, src, dworld)
            d = pix - u
            E2 = d @ Q @ d
            assert abs(E - E2) <= 0.02 * max(1.0, E), (trial, dxp, dyp, E, E2)


def test_culling_rules():
    st = O.Settings()
    c = O.camera(0.0, S.L_SO, S.L_SD, 64, 64, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    # behind the near plane: t_z = 4 - x at phi = 0, so x = 3.9 gives t_z = 0.1
    assert not O.project(_one((3.9, 0, 0)), c, st)["kept"][0]
    # zero quaternion
    assert not O.project(_one((0, 0, 0), quat=(0, 0, 0, 0)), c, st)["kept"][0]
    # opacity below alpha_min can never contribute
    assert not O.project(_one((0, 0, 0), o=0.003), c, st)["kept"][0]
    assert O.project(_one((0, 0, 0), o=0.004), c, st)["kept"][0]
    # wholly outside the detector
    assert not O.project(_one((0, 3.0, 0)), c, st)["kept"][0]
    # non-finite input
    assert not O.project(_one((np.nan, 0, 0)), c, st)["kept"][0]
