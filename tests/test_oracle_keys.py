"""Pins of the oracle's tile lists (Sec. 3.2): keys, values and ranges.

- The key path is re-evaluated here with numpy float32 scalars (IEEE
  binary32, one rounding per operation, no fused multiply-add), which
  catches any contraction or reordering the C compiler might introduce.
- Pairs are re-derived by brute force: every tile of every view is tested
  against every rectangle, with no tile-span arithmetic.
- Sorting is re-done with numpy's lexsort.
"""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S

D = S.DETECTOR_SIDE
f32 = np.float32


def _key_path_np(mean, scale, quat, opac, c, st):
    """Float32 scalar re-evaluation of the key path; returns (depth_bits, rect) or None."""
    r = [f32(v) for v in c.rot]
    tr = [f32(v) for v in c.trans]
    mx, my, mz = (f32(v) for v in mean)
    tx = ((r[0] * mx + r[1] * my) + r[2] * mz) + tr[0]
    ty = ((r[3] * mx + r[4] * my) + r[5] * mz) + tr[1]
    tz = ((r[6] * mx + r[7] * my) + r[8] * mz) + tr[2]
    if not (np.isfinite(tx) and np.isfinite(ty) and np.isfinite(tz)):
        return None
    if not tz > f32(st.near_z):
        return None
    qw, qx, qy, qz = (f32(v) for v in quat)
    n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz
    if not n2 > 0:
        return None
    nn = np.sqrt(n2)
    w, x, y, z = qw / nn, qx / nn, qy / nn, qz / nn
    one, two = f32(1), f32(2)
    R = [one - two * (y * y + z * z), two * (x * y - w * z), two * (x * z + w * y),
         two * (x * y + w * z), one - two * (x * x + z * z), two * (y * z - w * x),
         two * (x * z - w * y), two * (y * z + w * x), one - two * (x * x + y * y)]
    s = [f32(v) for v in scale]
    M = [R[3 * a + b] * s[b] for a in range(3) for b in range(3)]
    fx, fy = f32(c.fx), f32(c.fy)
    tz2 = tz * tz
    J00, J11 = fx / tz, fy / tz
    J02, J12 = -((fx * tx) / tz2), -((fy * ty) / tz2)
    A = [J00 * r[k] + J02 * r[6 + k] for k in range(3)] + \
        [J11 * r[3 + k] + J12 * r[6 + k] for k in range(3)]
    B = [(A[3 * i] * M[k] + A[3 * i + 1] * M[3 + k]) + A[3 * i + 2] * M[6 + k]
         for i in range(2) for k in range(3)]
    k_ = f32(st.lowpass)
    sxx = ((B[0] * B[0] + B[1] * B[1]) + B[2] * B[2]) + k_
    syy = ((B[3] * B[3] + B[4] * B[4]) + B[5] * B[5]) + k_
    sxy = (B[0] * B[3] + B[1] * B[4]) + B[2] * B[5]
    det = sxx * syy - sxy * sxy
    if not det > 0:
        return None
    if not f32(opac) >= f32(st.alpha_min):
        return None
    ux = fx * (tx / tz) + f32(c.cx)
    uy = fy * (ty / tz) + f32(c.cy)
    kap = f32(-2.0 * math.log(float(f32(st.alpha_min))))
    rx, ry = np.sqrt(kap * sxx), np.sqrt(kap * syy)
    half = f32(0.5)
    xl, xh = np.ceil((ux - rx) - half), np.floor((ux + rx) - half)
    yl, yh = np.ceil((uy - ry) - half), np.floor((uy + ry) - half)
    wmax, hmax = f32(c.width - 1), f32(c.height - 1)
    if not (xl <= xh and xl <= wmax and xh >= 0 and yl <= yh and yl <= hmax and yh >= 0):
        return None
    rect = (int(max(xl, f32(0))), int(min(xh, wmax)), int(max(yl, f32(0))), int(min(yh, hmax)))
    return int(np.array(tz, dtype=np.float32).view(np.uint32)), rect


def _scene(n, s0, ss, seed):
    return S.gaussians(n, math.log(s0), ss, seed)


@pytest.mark.parametrize("seed,W,s0,ss", [(1, 64, 0.05, 0.3), (2, 100, 0.02, 0.6), (3, 37, 0.1, 0.5)])
def test_key_path_float32_double_implementation(seed, W, s0, ss):
    g = _scene(300, s0, ss, seed)
    g["opacity"][:10] = 0.002    # below alpha_min
    g["quats"][10] = 0           # degenerate quaternion
    st = O.Settings()
    c = O.camera(0.37 * seed, S.L_SO, S.L_SD, W, W - 5, D, D)
    p = O.project(g, c, st)
    for j in range(300):
        ref = _key_path_np(g["means"][j], g["scales"][j], g["quats"][j], g["opacity"][j], c, st)
        assert bool(p["kept"][j]) == (ref is not None), j
        if ref is not None:
            assert int(p["depth_bits"][j]) == ref[0], j
            assert tuple(int(v) for v in p["rect"][j]) == ref[1], j


def _brute_pairs(g, cams, st):
    keys, vals = [], []
    T = st.tile
    toff = 0
    for c in cams:
        p = O.project(g, c, st)
        txn, tyn = -(-c.width // T), -(-c.height // T)
        for i in range(g["means"].shape[0]):
            if not p["kept"][i]:
                continue
            xl, xh, yl, yh = p["rect"][i]
            for ty in range(tyn):
                for tx in range(txn):
                    # tile (tx, ty) covers pixels [tx*T, tx*T+T-1] x [ty*T, ty*T+T-1]
                    if xh < tx * T or xl > tx * T + T - 1 or yh < ty * T or yl > ty * T + T - 1:
                        continue
                    keys.append(((toff + ty * txn + tx) << 32) | int(p["depth_bits"][i]))
                    vals.append(i)
        toff += txn * tyn
    return np.array(keys, np.uint64), np.array(vals, np.uint32), toff


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_pairs_brute_force_and_sort(tile):
    st = O.Settings(tile=tile)
    g = _scene(250, 0.06, 0.4, 7)
    rng = np.random.default_rng(8)
    cams = [O.camera(float(rng.uniform(0, 6.3)), S.L_SO, S.L_SD, w, h, D, D)
            for w, h in [(64, 64), (50, 33), (96, 96)]]
    bk, bv, nt = _brute_pairs(g, cams, st)
    pr = O.pairs(g, cams, st)
    assert pr["n_pairs"] == len(bk) and pr["n_tiles"] == nt
    order = np.lexsort((bv, bk))
    np.testing.assert_array_equal(pr["keys"], bk[order])
    np.testing.assert_array_equal(pr["values"], bv[order])
    # ranges: each tile's run of keys
    tiles = (pr["keys"] >> np.uint64(32)).astype(np.int64)
    for gt in range(nt):
        idx = np.nonzero(tiles == gt)[0]
        if len(idx) == 0:
            assert tuple(pr["ranges"][gt]) == (0, 0)
        else:
            assert tuple(pr["ranges"][gt]) == (idx[0], idx[-1] + 1)
            assert np.all(np.diff(idx) == 1)


def test_sorted_order_is_depth_then_index():
    st = O.Settings(tile=16)
    g = _scene(400, 0.05, 0.3, 9)
    # duplicate some Gaussians so equal keys occur; ties must keep index order
    for k in range(20):
        for a in g:
            g[a][200 + k] = g[a][k]
    c = O.camera(1.3, S.L_SO, S.L_SD, 64, 64, D, D)
    pr = O.pairs(g, [c], st)
    k, v = pr["keys"], pr["values"]
    same = k[1:] == k[:-1]
    assert same.any()
    assert np.all(v[1:][same] > v[:-1][same])
    assert np.all(k[1:] >= k[:-1])
