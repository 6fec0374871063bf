"""The comparison model on the GPU (RGB Gaussians with spherical-harmonics
colour, Eq. 2; forward only) against the FP64 oracle: per-(view, Gaussian)
colours for every degree, a ragged reduced scene (keys bit-exact, all three
channels, final T and last contributor), and the 200 000-Gaussian
8 x 512 x 512 launch on sampled pixels by brute force."""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S
from oracle import sh as H
from _gpu import KEYS, add_branches, compare_forward, compare_pixels, note, oracle_cams

pytestmark = pytest.mark.gpu

D = S.DETECTOR_SIDE


def _gpu_rgb(g, sh, degree, angles, sizes):
    import torch
    import paper_2403_04116_amd as P
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, D, D)
    frame = P.Frame(g["means"].shape[0], cams, P.settings(tile=16))
    gt = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda() for k in KEYS}
    frame.fit_capacity(gt)
    sht = torch.from_numpy(sh).cuda()
    image, final_t, n_contrib = frame.forward_rgb(gt, sht, degree)
    torch.cuda.synchronize()
    assert frame.status() == 0
    n = g["means"].shape[0]
    rec = frame.ws_tensor(frame.layout.records, torch.float32, 16 * n * len(sizes))
    colors = rec.view(len(sizes), n, 16)[:, :, 12:15].cpu().numpy()
    keys, vals, ranges = frame.sorted_pairs()
    return {"image": image.cpu().numpy(), "final_t": final_t.cpu().numpy(),
            "n_contrib": n_contrib.cpu().numpy(), "colors": colors,
            "keys": keys.cpu().numpy().view(np.uint64), "frame": frame}


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_colours_every_degree(degree):
    note(f"rgb colours degree {degree}")
    g = S.scene(1)
    sh = S.sh_coefficients(g["means"].shape[0], degree, 40 + degree, std=0.6)
    sizes, angles = [(64, 64), (48, 40)], [0.4, 2.9]
    gpu = _gpu_rgb(g, sh, degree, angles, sizes)
    ref = H.colors(g["means"], sh, oracle_cams(angles, sizes), degree)
    # float32 colours feed the image linearly (blending weights sum to <= 1)
    np.testing.assert_allclose(gpu["colors"], ref, rtol=0, atol=5e-6)
    assert (ref == 0).any() or degree == 0      # the clamp is exercised at std 0.6


def test_reduced_scene_all_channels():
    """Every channel of every view against the oracle's Eq. 10 with that
    channel's colours in place of the intensity (the blending decisions do
    not depend on the colour), under the forward parity rule (either branch
    of a single flagged decision)."""
    note("rgb reduced scene: 3 ragged views, degree 3")
    g = S.gaussians(1500, math.log(0.05), 0.3, 77)
    sh = S.sh_coefficients(1500, 3, 78)
    sizes, angles = [(64, 64), (80, 48), (37, 53)], [0.1, 1.9, 4.4]
    gpu = _gpu_rgb(g, sh, 3, angles, sizes)
    cams = oracle_cams(angles, sizes)
    st = O.Settings(tile=16)
    ref = H.render_rgb(g, sh, cams, st, 3)
    pr = O.pairs(g, cams, st)
    np.testing.assert_array_equal(gpu["keys"], pr["keys"])
    assert (O.n_flags(ref["flags"]) == 0).mean() > 0.99
    col = H.colors(g["means"], sh, cams, 3)
    off = 0
    for v, c in enumerate(cams):
        npx = c.width * c.height
        sl = slice(off, off + npx)
        pv = O.pairs(g, [c], st)
        for ch in range(3):
            gc = dict(g)
            gc["intensity"] = col[v, :, ch]
            r = O.render_binned(gc, [c], st, pv["values"], pv["ranges"])
            add_branches(r, gc, [c], st, pv["values"], pv["ranges"])
            compare_forward({"image": gpu["image"][ch][sl], "final_t": gpu["final_t"][sl],
                             "n_contrib": gpu["n_contrib"][sl]}, r, check_keys=False,
                            label=f"rgb view {v} channel {ch}")
        off += npx


def test_headline_launch_sampled_pixels():
    w = S.workload(3)
    g = S.scene(3)
    sh = S.sh_coefficients(w.n, 3, w.seeds["scene"] + 7)
    note("rgb 200k x 8 x 512^2, degree 3")
    gpu = _gpu_rgb(g, sh, 3, w.angles, w.sizes)
    cams = oracle_cams(w.angles, w.sizes)
    col = H.colors(g["means"], sh, cams, 3)
    st = O.Settings(tile=16)
    rng = np.random.default_rng(31)
    off = 0
    for v, c in enumerate(cams):
        npx = c.width * c.height
        pix = rng.choice(npx, 24, replace=False).astype(np.int32)
        for ch in range(3):
            gc = dict(g)
            gc["intensity"] = col[v, :, ch]
            compare_pixels(gpu["image"][ch][off + pix], gpu["final_t"][off + pix], gc, c, st, pix,
                           label=f"rgb view {v} channel {ch}")
        off += npx
