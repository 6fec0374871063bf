"""Pins of the oracle's threshold rules of Eq. 10 (readings of the paper,
which gives no thresholds): termination before a Gaussian that would take
the transmittance below t_min, the alpha clamp and its zero derivative,
the index order of Gaussians at exactly equal depth, and the second
admissible result of a pixel with one decision within a rounding margin of
a threshold.

Every expected value is worked out by hand from the definition (stacks of
identical Gaussians centred on a pixel centre, where the Gaussian factor is
1 up to ~1e-15), or is a central finite difference of the oracle's own
float64 forward.  Inputs are float64 here (the oracle's float64 path uses
them as given; only the key path rounds them to float32).
"""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S

D = S.DETECTOR_SIDE
W = 32
KEYS = ("means", "scales", "quats", "opacity", "intensity")


def _cam(W=W, H=None):
    return O.camera(0.0, S.L_SO, S.L_SD, W, W if H is None else H, D, D)


def _f32(x):
    return float(np.float32(x))


def _centred(depth, W=W, dx=0.0, dy=0.0):
    """World position whose projection at phi = 0 lands on the centre of
    pixel (W/2 + dx, W/2 + dy) at camera depth t_z = depth (camera x = world
    y, camera y = -world z, t_z = L_SO - world x)."""
    f = _f32(S.L_SD * W / D)
    return (S.L_SO - depth, (0.5 + dx) * depth / f, -(0.5 + dy) * depth / f)


def _gs(rows):
    return {"means": np.array([r[0] for r in rows], np.float64),
            "scales": np.array([r[1] for r in rows], np.float64),
            "quats": np.array([r[2] for r in rows], np.float64),
            "opacity": np.array([r[3] for r in rows], np.float64),
            "intensity": np.array([r[4] for r in rows], np.float64)}


def _pix(W=W, dx=0, dy=0):
    return np.array([(W // 2 + dy) * W + W // 2 + dx], np.int32)


# ---- termination (T' < t_min stops blending; that Gaussian is excluded) ----

def _stack(k, o, inten, behind=None):
    rows = [(_centred(3.6), (0.05, 0.05, 0.05), (1, 0, 0, 0), o, inten) for _ in range(k)]
    if behind is not None:   # (opacity, intensity) of one more Gaussian further away
        rows.append((_centred(4.4), (0.05, 0.05, 0.05), (1, 0, 0, 0), behind[0], behind[1]))
    return _gs(rows)


def test_termination_stack_hand_worked():
    """14 identical Gaussians with alpha = 1/2 at the pixel: T after j
    contributors is 2^-j; the 14th would give 2^-14 < 1e-4 <= 2^-13, so
    exactly 13 contribute, I = i (1 - 2^-13), T = 2^-13, and 14 rectangle
    evaluations are made (the 14th is evaluated, then blending stops)."""
    st = O.Settings(alpha_min=1 / 255, t_min=1e-4)
    g = _stack(14, 0.5, 0.8)
    r = O.render_brute(g, _cam(), st, _pix())
    i = 0.8
    assert abs(r["image"][0] - i * (1 - 2.0 ** -13)) < 1e-12
    assert abs(r["final_t"][0] - 2.0 ** -13) < 1e-15
    assert r["last"][0] == 12           # Gaussian index of the 13th (ties: index order)
    assert r["evals"][0] == 14
    assert r["flags"][0] == 0


def test_zero_t_min_stops_at_the_smallest_normal_float():
    """t_min = 0 acts as 2^-126 (the smallest normal float32): 130 Gaussians
    with alpha = 1/2 give T = 2^-j after j contributors; the 127th would
    take T to 2^-127 < 2^-126, so exactly 126 contribute, T = 2^-126 and
    I = i (1 - 2^-126).  (The 126th lands on 2^-126 itself: not below, so it
    is blended, and that decision is flagged as sitting on the threshold.)"""
    st = O.Settings(alpha_min=1 / 255, t_min=0.0)
    g = _stack(130, 0.5, 0.8)
    r = O.render_brute(g, _cam(), st, _pix())
    assert r["final_t"][0] == 2.0 ** -126
    assert abs(r["image"][0] - 0.8 * (1 - 2.0 ** -126)) < 1e-12
    assert r["last"][0] == 125
    assert r["evals"][0] == 127


def test_termination_ends_blending():
    """A Gaussian behind the stack that alone would not take T below t_min
    (alpha = 0.1: 2^-13 * 0.9 > 1e-4) must not change the pixel: blending
    ended at the 14th Gaussian.  (Skipping that one and going on would add
    i' * 0.1 * 2^-13 here.)"""
    st = O.Settings(alpha_min=1 / 255, t_min=1e-4)
    a = O.render_brute(_stack(14, 0.5, 0.8), _cam(), st, _pix())
    b = O.render_brute(_stack(14, 0.5, 0.8, behind=(0.1, 0.9)), _cam(), st, _pix())
    assert b["image"][0] == a["image"][0]
    assert b["final_t"][0] == a["final_t"][0]
    assert b["last"][0] == 12 and b["evals"][0] == 14
    # with no termination the Gaussian behind is blended: I grows by i' a T
    st0 = O.Settings(alpha_min=1 / 255, t_min=0.0)
    c = O.render_brute(_stack(14, 0.5, 0.8, behind=(0.1, 0.9)), _cam(), st0, _pix())
    want = 0.8 * (1 - 2.0 ** -14) + 0.9 * 0.1 * 2.0 ** -14
    assert abs(c["image"][0] - want) < 1e-12 and c["last"][0] == 14


def test_termination_binned_list_position():
    """The binned traversal reports the 1-based list position of the last
    contributor (13) and the same pixel value."""
    st = O.Settings(alpha_min=1 / 255, t_min=1e-4, tile=16)
    g = _stack(14, 0.5, 0.8, behind=(0.1, 0.9))
    c = _cam()
    pr = O.pairs(g, [c], st)
    r = O.render_binned(g, [c], st, pr["values"], pr["ranges"])
    p = _pix()[0]
    assert r["n_contrib"][p] == 13 and r["evals"][p] == 14
    assert abs(r["image"][p] - 0.8 * (1 - 2.0 ** -13)) < 1e-12


def test_terminating_gaussian_gets_no_gradient():
    """Upstream at the stack's pixel only: the 14th (terminating) Gaussian
    and the one behind are not contributors, so their gradients are zero;
    intensity gradients of the 13 contributors are alpha T_j = 2^-(j+1)."""
    st = O.Settings(alpha_min=1 / 255, t_min=1e-4, tile=16)
    g = _stack(14, 0.5, 0.8, behind=(0.1, 0.9))
    c = _cam()
    up = np.zeros(W * W, np.float32)
    up[_pix()[0]] = 1.0
    gr = O.backward(g, [c], st, up)
    for k in KEYS:
        assert np.all(gr[k][13:] == 0), k
    np.testing.assert_allclose(gr["intensity"][:13], [2.0 ** -(j + 1) for j in range(13)],
                               rtol=1e-12)


# ---- the alpha clamp and its zero derivative ----------------------------

WW = 64


def _wide(o):
    """One wide Gaussian (about 8 pixels of standard deviation on a 64 x 64
    detector) centred on a pixel centre."""
    return _gs([(_centred(4.0, W=WW), (0.3, 0.5, 0.45), (1, 0, 0, 0), o, 0.7)])


def _loss(g, c, st, up):
    return float(np.dot(O.render_brute(g, c, st)["image"], up.astype(np.float64)))


def _fd(g, c, st, up, h=1e-6):
    out = {}
    for k in KEYS:
        fd = np.zeros_like(g[k])
        flat = g[k].reshape(-1)
        for j in range(flat.size):
            x0 = flat[j]
            flat[j] = x0 + h
            lp = _loss(g, c, st, up)
            flat[j] = x0 - h
            lm = _loss(g, c, st, up)
            flat[j] = x0
            fd.reshape(-1)[j] = (lp - lm) / (2 * h)
        out[k] = fd
    return out


def test_clamp_value_and_zero_derivative():
    """o = 1 at the pixel centre: alpha = alpha_max exactly there
    (I = 0.99 i).  On every pixel where o G exceeds alpha_max by a clear
    margin, alpha is the constant alpha_max, so the loss summed over those
    pixels has zero derivative in every parameter except the intensity
    (0.99 per pixel); the adjoint and central differences both say so."""
    st = O.Settings()
    c = _cam(WW)
    g = _wide(1.0)
    r = O.render_brute(g, c, st)
    p = _pix(WW)[0]
    assert abs(r["image"][p] - _f32(0.99) * 0.7) < 1e-9
    pr = O.project(g, c, st)
    u, q = pr["u"][0], pr["conic"][0]
    y, x = np.mgrid[0:WW, 0:WW]
    dx, dy = (x + 0.5 - u[0]).ravel(), (y + 0.5 - u[1]).ravel()
    a = np.exp(-0.5 * (q[0] * dx * dx + 2 * q[1] * dx * dy + q[2] * dy * dy))
    clamped = a > _f32(0.99) * (1 + 2e-3)
    assert 3 <= clamped.sum() <= 20
    up = clamped.astype(np.float32)
    gr = O.backward(g, [c], st, up)
    fd = _fd(g, c, st, up)
    for k in ("means", "scales", "quats", "opacity"):
        assert np.all(gr[k] == 0), (k, gr[k])
        assert np.abs(fd[k]).max() < 1e-9, (k, fd[k])
    assert abs(gr["intensity"][0] - _f32(0.99) * clamped.sum()) < 1e-9
    assert abs(fd["intensity"][0] - _f32(0.99) * clamped.sum()) < 1e-6


def test_below_clamp_derivative_matches_differences():
    """The other side of the kink: o = 0.95 (no pixel clamped), the same
    pixels: the adjoint's opacity, position and shape derivatives are
    nonzero and equal central differences of the forward."""
    st = O.Settings()
    c = _cam(WW)
    g = _wide(0.95)
    pr = O.project(g, c, st)
    u, q = pr["u"][0], pr["conic"][0]
    y, x = np.mgrid[0:WW, 0:WW]
    dx, dy = (x + 0.5 - u[0]).ravel(), (y + 0.5 - u[1]).ravel()
    a = np.exp(-0.5 * (q[0] * dx * dx + 2 * q[1] * dx * dy + q[2] * dy * dy))
    up = (a > 0.97).astype(np.float32) + 0.25 * (np.arange(WW * WW) % 3 == 0)
    gr = O.backward(g, [c], st, up.astype(np.float32))
    fd = _fd(g, c, st, up.astype(np.float32))
    assert abs(gr["opacity"][0]) > 1.0
    for k in KEYS:
        err = np.linalg.norm(gr[k] - fd[k]) / max(np.linalg.norm(fd[k]), 1e-30)
        assert err < 1e-6, (k, err)


# ---- equal depths: ascending Gaussian index first ------------------------

def _tie_pair(swap=False):
    rows = [(_centred(3.7, dx=-0.6), (0.05, 0.06, 0.05), (1, 0, 0, 0), 0.6, 0.9),
            (_centred(3.7, dx=0.6), (0.05, 0.05, 0.07), (1, 0, 0, 0), 0.7, 0.2)]
    return _gs(rows[::-1] if swap else rows)


def test_equal_depth_index_order():
    """Two Gaussians at exactly the same camera depth (same depth bits)
    overlapping a pixel: the lower index is blended first,
    I = i0 a0 + i1 a1 (1 - a0), with a_k read from each Gaussian rendered
    alone with unit intensity.  The other order would give
    i1 a1 + i0 a0 (1 - a1), which differs by a0 a1 (i0 - i1)."""
    st = O.Settings()
    c = _cam()
    pix = np.arange(W * W, dtype=np.int32)
    g = _tie_pair()
    pr = O.project(g, c, st)
    assert pr["depth_bits"][0] == pr["depth_bits"][1]
    alone = []
    for k in (0, 1):
        gk = {key: v[k:k + 1].copy() for key, v in g.items()}
        gk["intensity"][:] = 1.0
        alone.append(O.render_brute(gk, c, st, pix)["image"])
    a0, a1 = alone
    i0, i1 = 0.9, 0.2
    both = (a0 > 0) & (a1 > 0)
    assert both.sum() > 10
    r = O.render_brute(g, c, st, pix)
    np.testing.assert_allclose(r["image"], i0 * a0 + i1 * a1 * (1 - a0), rtol=0, atol=1e-14)
    other = i1 * a1 + i0 * a0 * (1 - a1)
    assert np.abs(r["image"] - other)[both].max() > 1e-3
    assert np.all(r["last"][both] == 1)
    # swapping the indices swaps the order: the blend follows the index, not the input slot
    rs = O.render_brute(_tie_pair(swap=True), c, st, pix)
    np.testing.assert_allclose(rs["image"], i1 * a1 + i0 * a0 * (1 - a1), rtol=0, atol=1e-14)
    # the sorted tile lists give the same order
    pb = O.pairs(g, [c], st)
    rb = O.render_binned(g, [c], st, pb["values"], pb["ranges"])
    np.testing.assert_array_equal(rb["image"], r["image"])


# ---- flagged decisions: the other admissible branch -----------------------

def test_flip_alpha_min_branch():
    """alpha within 1e-5 (relative) of alpha_min at the pixel is a flagged
    decision; the flipped branch skips (or keeps) the Gaussian."""
    amin = _f32(1 / 255)
    st = O.Settings(alpha_min=amin)
    c = _cam()
    o = amin * (1 + 3e-6)
    g = _gs([(_centred(3.9), (0.05, 0.05, 0.05), (1, 0, 0, 0), o, 0.5)])
    p = _pix()
    r = O.render_brute(g, c, st, p)
    rf = O.render_brute(g, c, st, p, flip=np.ones(1))
    assert O.n_flags(r["flags"])[0] == 1 and r["flags"][0] & O.FLAG_ALPHA_MIN
    kept = 0.5 * o
    assert {round(r["image"][0], 15), round(rf["image"][0], 15)} == {round(kept, 15), 0.0}


def test_flip_termination_branch():
    """Three identical Gaussians with (1 - alpha)^3 within 1e-5 of t_min:
    one flagged decision; one branch has 3 contributors, the other 2."""
    tmin = _f32(1e-4)
    st = O.Settings(t_min=tmin)
    o = 1 - tmin ** (1 / 3)
    g = _stack(3, o, 0.6)
    c = _cam()
    p = _pix()
    r = O.render_brute(g, c, st, p)
    rf = O.render_brute(g, c, st, p, flip=np.ones(1))
    assert O.n_flags(r["flags"])[0] == 1 and r["flags"][0] & O.FLAG_T_MIN
    a = o
    i = 0.6
    three, two = i * (1 - (1 - a) ** 3), i * (1 - (1 - a) ** 2)
    got = sorted([r["image"][0], rf["image"][0]])
    np.testing.assert_allclose(got, sorted([three, two]), rtol=0, atol=1e-9)
    assert sorted([r["last"][0], rf["last"][0]]) == [1, 2]


def test_flip_clamp_branch_and_gradient():
    """o G within 1e-5 of alpha_max: the flipped branch leaves alpha
    unclamped, and its opacity derivative is G instead of 0."""
    st = O.Settings()
    c = _cam()
    g = _gs([(_centred(4.0), (0.05, 0.05, 0.05), (1, 0, 0, 0), _f32(0.99) * (1 + 2e-6), 0.5)])
    p = _pix()
    r = O.render_brute(g, c, st, p)
    rf = O.render_brute(g, c, st, p, flip=np.ones(1))
    assert O.n_flags(r["flags"])[0] == 1 and r["flags"][0] & O.FLAG_CLAMP
    assert abs(r["image"][0] - rf["image"][0]) < 1e-5
    up = np.zeros(W * W, np.float32)
    up[p[0]] = 1.0
    flip = np.zeros(W * W, np.uint8)
    flip[p[0]] = 1
    g0 = O.backward(g, [c], st, up)
    g1 = O.backward(g, [c], st, up, flip=flip)
    assert sorted([abs(g0["opacity"][0]), abs(g1["opacity"][0])])[0] == 0.0
    assert max(abs(g0["opacity"][0]), abs(g1["opacity"][0])) > 0.4


def test_flip_only_subset_binned():
    """render_binned with ``only`` renders just the chosen pixels, and a
    flip on a pixel without a flagged decision changes nothing."""
    st = O.Settings(tile=8)
    g = S.gaussians(200, math.log(0.05), 0.3, 3)
    c = _cam(40, 24)
    pr = O.pairs(g, [c], st)
    full = O.render_binned(g, [c], st, pr["values"], pr["ranges"])
    only = np.zeros(40 * 24, np.uint8)
    only[::5] = 1
    flip = (O.n_flags(full["flags"]) == 0).astype(np.uint8)
    part = O.render_binned(g, [c], st, pr["values"], pr["ranges"], flip=flip, only=only)
    sel = only.astype(bool)
    np.testing.assert_array_equal(part["image"][sel], full["image"][sel])
    np.testing.assert_array_equal(part["n_contrib"][sel], full["n_contrib"][sel])
    assert np.all(part["image"][~sel] == 0)


def test_block_contributors_brute_force():
    """Per 8 x 8 block: distinct contributors counted by brute force, on
    two ragged views with tile sizes 8 and 32.  With t_min = 0 (no
    termination), Gaussian k is a contributor of pixel p exactly when
    removing it changes p's final transmittance."""
    g = S.gaussians(300, math.log(0.06), 0.3, 9)
    cams = [_cam(44, 30), O.camera(2.0, S.L_SO, S.L_SD, 24, 40, D, D)]
    st0 = O.Settings(t_min=0.0)
    sets_of = []
    for c in cams:
        base = O.render_brute(g, c, st0)["final_t"]
        sets = [set() for _ in range(c.width * c.height)]
        for k in range(g["means"].shape[0]):
            gk = {key: v.copy() for key, v in g.items()}
            gk["opacity"][k] = 0.0          # culled: below alpha_min
            tk = O.render_brute(gk, c, st0)["final_t"]
            for p in np.nonzero(tk != base)[0]:
                sets[p].add(k)
        sets_of.append(sets)
    for tile in (8, 32):
        st = O.Settings(tile=tile, t_min=0.0)
        pr = O.pairs(g, cams, st)
        got = O.block_contributors(g, cams, st, pr["values"], pr["ranges"])
        off = 0
        for c, sets in zip(cams, sets_of):
            Wc, Hc = c.width, c.height
            for by in range(0, Hc, 8):
                for bx in range(0, Wc, 8):
                    s = set()
                    for y in range(by, min(by + 8, Hc)):
                        for x in range(bx, min(bx + 8, Wc)):
                            s |= sets[y * Wc + x]
                    assert got[off + by * Wc + bx] == len(s), (tile, bx, by)
            mask = np.zeros((Hc, Wc), bool)
            mask[::8, ::8] = True
            assert np.all(got[off:off + Wc * Hc][~mask.ravel()] == 0)
            off += Wc * Hc
