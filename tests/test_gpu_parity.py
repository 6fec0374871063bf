"""Parity of the HIP path (called through the C ABI) with the FP64 oracle.

Bar: sort keys, values and tile ranges bit-exact; images and final
transmittance within 1e-5 max abs and n_contrib equal on pixels where no
decision sits within a relative margin of a threshold; a pixel with one
such decision may match either branch (the oracle renders both); pixels
with two or more are excluded (at most 0.5% of pixels) and counted.
Gradients within 1e-4 relative L2 per parameter group, with the same
float32 upstream gradient fed to both and the oracle differentiating the
branch the GPU took.
"""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S
from _gpu import (KEYS, check_counts, compare_forward, compare_grads, gpu_run, grad_upstream, note,
                  oracle_run)

pytestmark = pytest.mark.gpu

SETTINGS = [(t, b) for t in (8, 16, 32) for b in (64, 128, 256)]


def test_workload1():
    """1000 Gaussians, one 64x64 view at angle 0, upstream ~ N(0, 1)."""
    w = S.workload(1)
    g = S.scene(1)
    note("workload1: forward")
    ref = oracle_run(g, w.angles, w.sizes)
    up = S.upstream_normal(w.n_pixels, w.seeds["upstream"])
    upm = grad_upstream(up, ref)
    gpu = gpu_run(g, w.angles, w.sizes, upstream=upm)
    m = compare_forward(gpu, ref, label="workload1")
    rg = O.backward(g, ref["cams"], ref["st"], upm, flip=m.flip)
    errs = compare_grads(gpu["grads"], rg)
    note(f"workload1: image err {m.err:.2e}, grad rel L2 {max(errs.values()):.2e}")
    counts = gpu["frame"].render_counts().cpu().numpy()
    check_counts(counts, ref, g, m, label="workload1")
    assert np.all(counts[1] <= counts[2]) and np.all(counts[2] <= counts[0])
    assert np.all((counts[1] > 0) == (gpu["n_contrib"] > 0))


def _multiview_scene(seed=5, n=2500):
    g = S.gaussians(n, math.log(0.05), 0.4, seed)
    sizes = [(96, 80), (50, 33), (128, 128), (8, 8)]
    rng = np.random.default_rng(seed + 1)
    angles = rng.uniform(0, 2 * math.pi, len(sizes)).tolist()
    return g, angles, sizes


@pytest.mark.parametrize("tile,lds", SETTINGS)
def test_ragged_multiview_all_settings(tile, lds):
    g, angles, sizes = _multiview_scene()
    note(f"ragged multiview tile={tile} lds={lds}")
    ref = oracle_run(g, angles, sizes, tile=tile)
    npx = sum(w * h for w, h in sizes)
    up = np.random.default_rng(9).normal(size=npx).astype(np.float32)
    upm = grad_upstream(up, ref)
    gpu = gpu_run(g, angles, sizes, tile=tile, lds=lds, upstream=upm)
    m = compare_forward(gpu, ref, label=f"ragged tile={tile} lds={lds}")
    rg = O.backward(g, ref["cams"], ref["st"], upm, binned=(ref["pairs"]["values"],
                                                            ref["pairs"]["ranges"]), flip=m.flip)
    compare_grads(gpu["grads"], rg)
    check_counts(gpu["frame"].render_counts().cpu().numpy(), ref, g, m,
                 label=f"ragged tile={tile} lds={lds}")


@pytest.mark.parametrize("tile,lds", [(8, 128), (16, 256), (32, 64)])
def test_persistent_queue(tile, lds):
    """Persistent launch over the heavy-first tile queue: same images as one
    workgroup per tile, gradients at parity, and repeated launches on the
    same workspace (the queue rewinds itself)."""
    g, angles, sizes = _multiview_scene(seed=41, n=3000)
    npx = sum(w * h for w, h in sizes)
    up = np.random.default_rng(7).normal(size=npx).astype(np.float32)
    note(f"persistent tile={tile} lds={lds}")
    ref = oracle_run(g, angles, sizes, tile=tile)
    upm = grad_upstream(up, ref)
    a = gpu_run(g, angles, sizes, tile=tile, lds=lds, upstream=upm, persistent=True)
    b = gpu_run(g, angles, sizes, tile=tile, lds=lds, upstream=upm, persistent=False)
    np.testing.assert_array_equal(a["image"], b["image"])
    np.testing.assert_array_equal(a["n_contrib"], b["n_contrib"])
    m = compare_forward(a, ref, label="persistent")
    rg = O.backward(g, ref["cams"], ref["st"], upm, binned=(ref["pairs"]["values"],
                                                            ref["pairs"]["ranges"]), flip=m.flip)
    compare_grads(a["grads"], rg)
    # three more launches on the same frame: identical images every time
    import torch
    frame = a["frame"]
    gt = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda() for k in KEYS}
    for _ in range(3):
        im, _, _ = frame.render_fwd(gt)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(im.cpu().numpy(), a["image"])


def test_images_bitwise_identical_across_tile_and_batch():
    g, angles, sizes = _multiview_scene(seed=11, n=4000)
    base = None
    for tile, lds in SETTINGS:
        note(f"invariance tile={tile} lds={lds}")
        r = gpu_run(g, angles, sizes, tile=tile, lds=lds, backward=False)
        if base is None:
            base = r
        else:
            np.testing.assert_array_equal(r["image"], base["image"])
            np.testing.assert_array_equal(r["final_t"], base["final_t"])


def test_batched_equals_per_view():
    g, angles, sizes = _multiview_scene(seed=21, n=3000)
    npx = sum(w * h for w, h in sizes)
    up = np.random.default_rng(3).normal(size=npx).astype(np.float32)
    note("batched vs per-view")
    b = gpu_run(g, angles, sizes, upstream=up)
    off = 0
    acc = {k: np.zeros_like(g[k], dtype=np.float64) for k in KEYS}
    for a, (w, h) in zip(angles, sizes):
        r = gpu_run(g, [a], [(w, h)], upstream=up[off:off + w * h])
        np.testing.assert_array_equal(r["image"], b["image"][off:off + w * h])
        np.testing.assert_array_equal(r["n_contrib"], b["n_contrib"][off:off + w * h])
        for k in KEYS:
            acc[k] += r["grads"][k]
        off += w * h
    for k in KEYS:
        d = np.linalg.norm(acc[k] - b["grads"][k]) / max(np.linalg.norm(acc[k]), 1e-30)
        assert d < 1e-5, (k, d)


def test_workload2_l1():
    """50 000 Gaussians, one 256x256 view, L1 upstream against a perturbed scene."""
    w = S.workload(2)
    g = S.scene(2)
    tgt = S.perturb(g, w.seeds["perturb"])
    note("workload2: oracle renders")
    ref = oracle_run(g, w.angles, w.sizes)
    reft = oracle_run(tgt, w.angles, w.sizes)
    up = np.sign(ref["image"] - reft["image"]).astype(np.float32)   # unnormalised L1
    upm = grad_upstream(up, ref)
    note("workload2: gpu")
    gpu = gpu_run(g, w.angles, w.sizes, upstream=upm)
    m = compare_forward(gpu, ref, label="workload2")
    rg = O.backward(g, ref["cams"], ref["st"], upm, binned=(ref["pairs"]["values"],
                                                            ref["pairs"]["ranges"]), flip=m.flip)
    errs = compare_grads(gpu["grads"], rg)
    note(f"workload2: grad rel L2 {errs}")


def test_empty_and_all_culled():
    sizes = [(40, 24), (16, 16)]
    angles = [0.3, 2.0]
    note("empty scene")
    g0 = {k: np.zeros((0,) + S.scene(1)[k].shape[1:], np.float32) for k in KEYS}
    r = gpu_run(g0, angles, sizes, upstream=np.ones(40 * 24 + 256, np.float32))
    assert np.all(r["image"] == 0) and np.all(r["final_t"] == 1) and np.all(r["n_contrib"] == 0)
    assert r["keys"].size == 0 and np.all(r["ranges"] == 0)
    note("all culled")
    g = S.gaussians(300, math.log(0.05), 0.3, 2)
    g["opacity"][:] = 0.001                       # below alpha_min
    g["quats"][:100] = 0                          # degenerate
    g["means"][100:200, 0] = 50.0                 # far outside every view
    r = gpu_run(g, angles, sizes, upstream=np.ones(40 * 24 + 256, np.float32))
    assert np.all(r["image"] == 0) and r["keys"].size == 0
    for k in KEYS:
        assert np.all(r["grads"][k] == 0)


def test_capacity_overflow_reports_and_recovers():
    import torch
    import paper_2403_04116_amd as P
    g, angles, sizes = _multiview_scene(seed=31, n=1500)
    dev = torch.device("cuda:0")
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    frame = P.Frame(1500, cams, P.settings(), pair_capacity=64, device=dev)
    gt = {k: torch.from_numpy(g[k]).to(dev) for k in KEYS}
    note("capacity overflow")
    frame.preprocess_sort(gt)
    img, ft, nc = frame.render_fwd(gt)
    torch.cuda.synchronize()
    assert frame.status() == P._lib.XG_ECAPACITY
    assert frame.n_pairs() > 64
    p = frame.fit_capacity(gt)
    assert frame.status() == P._lib.XG_OK and frame.capacity >= p
    img, ft, nc = frame.render_fwd(gt)
    ref = oracle_run(g, angles, sizes)
    compare_forward({"image": img.cpu().numpy(), "final_t": ft.cpu().numpy(),
                     "n_contrib": nc.cpu().numpy()}, ref, check_keys=False, label="regrown")


def _gs(rows):
    return {"means": np.array([r[0] for r in rows], np.float32),
            "scales": np.array([r[1] for r in rows], np.float32),
            "quats": np.array([r[2] for r in rows], np.float32),
            "opacity": np.array([r[3] for r in rows], np.float32),
            "intensity": np.array([r[4] for r in rows], np.float32)}


def test_special_scenes():
    """A Gaussian covering the whole detector, an o = 1 clamp at a pixel
    centre, a pile-up that drives the transmittance to t_min, and exactly
    equal depths (ties broken by index)."""
    W = 64
    f = float(np.float32(S.L_SD * W / S.DETECTOR_SIDE))
    sh = 0.5 * S.L_SO / f
    rows = [((0.0, 0.0, 0.0), (0.3, 0.9, 0.8), (1, 0, 0, 0), 0.5, 0.4),          # huge
            ((0.0, sh, -sh), (0.05, 0.05, 0.05), (1, 0, 0, 0), 1.0, 0.8)]       # clamp
    rng = np.random.default_rng(4)
    for k in range(400):                                                      # pile-up
        rows.append(((float(rng.uniform(-0.5, 0.5)), float(rng.normal(0, 0.05)),
                      float(rng.normal(0, 0.05))), (0.06, 0.06, 0.06), (1, 0, 0, 0), 0.6,
                     float(rng.uniform(0, 1))))
    for k in range(10):                                                       # equal depths
        rows.append(((0.2, -0.4 + 0.01 * k, 0.3), (0.04, 0.05, 0.03), (0.9, 0.1, 0.2, 0.3), 0.7, 0.5))
    g = _gs(rows)
    angles, sizes = [0.0, 1.0], [(W, W), (W, 40)]
    npx = W * W + W * 40
    up = np.random.default_rng(6).normal(size=npx).astype(np.float32)
    for tile in (8, 16, 32):
        note(f"special scenes tile={tile}")
        ref = oracle_run(g, angles, sizes, tile=tile)
        assert (ref["final_t"] < 2e-4).sum() > 50        # termination is exercised
        upm = grad_upstream(up, ref)
        gpu = gpu_run(g, angles, sizes, tile=tile, upstream=upm)
        m = compare_forward(gpu, ref, label=f"special tile={tile}")
        rg = O.backward(g, ref["cams"], ref["st"], upm, flip=m.flip)
        compare_grads(gpu["grads"], rg)
        check_counts(gpu["frame"].render_counts().cpu().numpy(), ref, g, m,
                     label=f"special tile={tile}")


def test_smooth_regime_and_paper_literal_lowpass():
    """alpha_min = 0 and t_min = 0 (every rectangle = whole detector), and
    the low-pass term switched off."""
    g = S.gaussians(60, math.log(0.12), 0.3, 8)
    g["opacity"] = np.minimum(g["opacity"], 0.9).astype(np.float32)
    angles, sizes = [0.4, 3.0], [(40, 40), (24, 36)]
    npx = 40 * 40 + 24 * 36
    up = np.random.default_rng(2).normal(size=npx).astype(np.float32)
    for kw in ({"alpha_min": 0.0, "t_min": 0.0}, {"lowpass": 0.0}):
        note(f"settings {kw}")
        ref = oracle_run(g, angles, sizes, tile=8, **kw)
        upm = grad_upstream(up, ref)
        gpu = gpu_run(g, angles, sizes, tile=8, upstream=upm, **kw)
        m = compare_forward(gpu, ref, label=f"settings {kw}")
        rg = O.backward(g, ref["cams"], ref["st"], upm, flip=m.flip)
        compare_grads(gpu["grads"], rg)


def test_l1_grad_kernel():
    import torch
    import paper_2403_04116_amd as P
    rng = np.random.default_rng(0)
    a = rng.normal(size=10007).astype(np.float32)
    b = rng.normal(size=10007).astype(np.float32)
    b[::7] = a[::7]
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    out = P.l1_grad(ta, tb, 0.25)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), (0.25 * np.sign(a - b)).astype(np.float32))
