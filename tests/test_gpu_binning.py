"""The per-tile lists (Sec. 3.2) on both of their GPU paths, bit-exact against
the oracle's sorted (tile << 32 | depth, index) pairs and tile ranges:

- counting (every view has at most 4096 tiles): 8 x 8 tiles on 512 x 512
  views (4096 tiles, the widest counter rows), partitions whose pairs span
  many LDS windows (large footprints, some wider than 32 tiles so their
  rectangle is read from the record), views of uneven size;
- emission + radix sort of the pairs by tile (a view with more tiles).

The item offsets the workspace exposes (the scan of the tile counts in
depth order, written by the list scatter on the counting path and by the
count scan on the other) are checked against a scan over the oracle's
depth order.  Sampled pixels of each run are also checked against the
brute-force renderer."""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S
from _gpu import compare_pixels, gpu_run, note, oracle_cams

pytestmark = pytest.mark.gpu


def _expected_offsets(g, cams, st):
    """Item offsets: per view, the items in (depth bits, index) order, the
    exclusive scan of their tile counts, from the pairs of the views before.
    A culled item sorts as the largest kept depth of the frame (its key is
    clamped there), by index among equal keys; its count is 0."""
    proj = [O.project(g, c, st) for c in cams]
    dmax = max(int(p["depth_bits"][p["kept"]].max()) for p in proj if p["kept"].any())
    out, start = [], 0
    for p in proj:
        T = st.tile
        r = p["rect"].astype(np.int64)
        cnt = np.where(p["kept"], (r[:, 1] // T - r[:, 0] // T + 1) * (r[:, 3] // T - r[:, 2] // T + 1), 0)
        key = np.where(p["kept"], p["depth_bits"].astype(np.int64), dmax)
        order = np.argsort(key, kind="stable")
        c_sorted = cnt[order]
        out.append(start + np.concatenate([[0], np.cumsum(c_sorted)[:-1]]))
        start += int(c_sorted.sum())
    return np.concatenate(out).astype(np.int64), start


def _check_tile_order(fr, ranges):
    """The blend launches' tile order (written by the list builder): workgroup
    b runs on XCD b % 8, which takes the b-th block of a split of the tiles
    into 8 contiguous blocks (sizes differing by at most one); within its
    block the order is a permutation of the block, longest list first in
    buckets of an eighth of an octave (a float32 log2 on the GPU, so a
    length may cross into the neighbouring bucket)."""
    import torch
    import paper_2403_04116_amd as P
    n = int(fr.total_tiles)
    v = P.xg_ws_inspect(fr.frame)
    order = fr.ws_tensor(v.tile_order - fr.ws.data_ptr(), torch.int32, n).cpu().numpy().astype(np.int64)
    r = np.asarray(ranges, dtype=np.int64).reshape(-1, 2)
    q, rem = divmod(n, 8)
    for x in range(8):
        t0 = x * q + min(x, rem)
        t1 = t0 + q + (1 if x < rem else 0)
        blk = order[t0:t1]
        np.testing.assert_array_equal(np.sort(blk), np.arange(t0, t1))
        f = 8.0 * np.log2((r[blk, 1] - r[blk, 0]).astype(np.float64) + 1.0)
        assert np.all(np.diff(f) < 1.0 + 1e-3), f"XCD block {x}: tiles not longest first"


def _check(g, angles, sizes, tile, label, sample=16):
    note(f"binning {label}: GPU")
    gpu = gpu_run(g, angles, sizes, tile=tile, backward=False)
    assert gpu["status"] == 0
    st = O.Settings(tile=tile)
    cams = oracle_cams(angles, sizes)
    note(f"binning {label}: oracle pairs")
    pr = O.pairs(g, cams, st)
    assert pr["keys"].size > 0
    np.testing.assert_array_equal(gpu["keys"], pr["keys"])
    np.testing.assert_array_equal(gpu["values"], pr["values"])
    np.testing.assert_array_equal(gpu["ranges"], pr["ranges"])
    # the item offsets the workspace exposes (scan of the tile counts in
    # depth order), whichever path wrote them
    import torch
    fr = gpu["frame"]
    n_items = int(g["means"].shape[0]) * len(cams)
    offs = fr.ws_tensor(fr.layout.offsets, torch.int32, n_items).cpu().numpy().view(np.uint32)
    exp, total = _expected_offsets(g, cams, st)
    assert total == pr["keys"].size == fr.n_pairs()
    np.testing.assert_array_equal(offs.astype(np.int64), exp)
    _check_tile_order(fr, pr["ranges"])
    rng = np.random.default_rng(17)
    off = 0
    for v, c in enumerate(cams):
        npx = c.width * c.height
        pix = rng.choice(npx, min(sample, npx), replace=False).astype(np.int32)
        compare_pixels(gpu["image"][off + pix], gpu["final_t"][off + pix], g, c, st, pix,
                       label=f"{label} view {v}")
        off += npx
    return gpu, pr


def test_counting_lists_widest_rows():
    # 8 x 8 tiles on 512 x 512: 4096 tiles per view
    g = S.gaussians(30000, math.log(0.02), 0.3, 501)
    gpu, pr = _check(g, [0.2, 2.4], [(512, 512), (512, 512)], 8, "tile 8, 4096 tiles/view")
    assert int(gpu["frame"].total_tiles) == 8192


def test_counting_lists_many_windows_and_wide_rectangles():
    # large footprints: partitions of 2048 items emit far more than one
    # window of pairs, and some rectangles are wider than 32 tiles
    g = S.gaussians(6000, math.log(0.08), 0.5, 502)
    g["scales"][:40] *= 8.0
    sizes = [(400, 320), (200, 136), (96, 64)]
    gpu, pr = _check(g, [0.7, 1.1, 3.0], sizes, 8, "large footprints")
    assert pr["keys"].size > 3 * 4096
    # widest rectangle of view 0 in tiles: more than the 32 a packed
    # rectangle holds, so the record supplies it
    tiles_x = (sizes[0][0] + 7) // 8
    t = (pr["keys"] >> 32).astype(np.int64)
    v0 = t < tiles_x * ((sizes[0][1] + 7) // 8)
    tx = t[v0] % tiles_x
    vals = pr["values"][v0].astype(np.int64)
    lo = np.full(vals.max() + 1, 1 << 30)
    hi = np.full(vals.max() + 1, -1)
    np.minimum.at(lo, vals, tx)
    np.maximum.at(hi, vals, tx)
    assert (hi - lo + 1).max() > 32


def test_counting_lists_uneven_views_tile16():
    g = S.gaussians(20000, math.log(0.02), 0.3, 503)
    _check(g, [0.1, 1.3, 2.9, 4.4], [(512, 512), (128, 128), (256, 256), (37, 300)], 16,
           "uneven views")


def test_radix_pair_sort_for_large_views():
    # 1100 x 1100 with 8 x 8 tiles = 138^2 = 19 044 tiles: above the counting
    # limit, so the pairs are emitted and radix sorted by tile
    g = S.gaussians(8000, math.log(0.01), 0.3, 504)
    gpu, _ = _check(g, [0.4, 2.0], [(1100, 1100), (64, 64)], 8, "large view, radix path")
    assert int(gpu["frame"].total_tiles) == 138 * 138 + 64



def test_tile_order_when_the_lists_are_empty():
    """The blend launches read the tile order whatever the lists hold: after
    a list build that exceeds the pair capacity (XG_ECAPACITY, every range
    empty) and for a scene without Gaussians, each XCD block is still a
    permutation of its tiles."""
    import torch
    import paper_2403_04116_amd as P
    note("tile order with empty lists")
    g = S.gaussians(3000, math.log(0.05), 0.3, 505)
    sizes = [(200, 120), (64, 64), (37, 300)]
    cams = P.cameras([0.2, 1.9, 3.3], sizes, S.L_SO, S.L_SD, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    frame = P.Frame(3000, cams, P.settings(tile=8), pair_capacity=16, device="cuda")
    gt = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda() for k in
          ("means", "scales", "quats", "opacity", "intensity")}
    frame.preprocess_sort(gt)
    torch.cuda.synchronize()
    assert frame.status() == P._lib.XG_ECAPACITY
    _check_tile_order(frame, np.zeros((int(frame.total_tiles), 2), np.uint32))
    g0 = {k: np.zeros((0,) + v.shape[1:], np.float32) for k, v in g.items()}
    r = gpu_run(g0, [0.2, 1.9, 3.3], sizes, tile=8, backward=False)
    assert r["status"] == 0 and r["keys"].size == 0
    _check_tile_order(r["frame"], r["ranges"])
