"""Parity at the other full-size workloads, in the launch configuration the
benchmark uses (tile 16, LDS batch 256, every view in one batched launch):

- 1 000 000 Gaussians (anisotropic log-scales N(log 0.01, 0.6)), 16 views of
  512 x 512 at random azimuths;
- 300 000 Gaussians, 32 views of 128^2 / 256^2 / 512^2 at random azimuths.

The oracle handles a sample of the views: for those, the GPU's sorted
(tile, Gaussian) pairs of that view must equal the oracle's bit for bit
(tile ids offset by the view's first tile) and its image must meet the
image bar.  Gradients are checked on a frame of the sampled views, for a
random sample of Gaussians whose gradients the oracle computes exactly (it
processes every pixel inside their rectangles).
"""
import numpy as np
import pytest

import oracle as O
import scenes as S
from _gpu import (GRAD_TOL, KEYS, add_branches, compare_forward, gpu_run, grad_upstream, note,
                  oracle_cams)

pytestmark = pytest.mark.gpu


def _view_slices(sizes):
    px = np.cumsum([0] + [w * h for w, h in sizes])
    return [slice(int(px[k]), int(px[k + 1])) for k in range(len(sizes))]


def _check_views(c, views, grad_gaussians):
    w = S.workload(c)
    g = S.scene(c)
    note(f"workload{c}: gpu batched forward, {w.n_views} views")
    gpu = gpu_run(g, w.angles, w.sizes, tile=16, lds=256, backward=False)
    assert gpu["status"] == 0
    frame = gpu["frame"]
    tiles = (gpu["keys"] >> np.uint64(32)).astype(np.int64)
    sl = _view_slices(w.sizes)
    st = O.Settings(tile=16)
    for v in views:
        wv, hv = w.sizes[v]
        note(f"workload{c}: oracle view {v} ({wv}x{hv})")
        cam = oracle_cams([w.angles[v]], [(wv, hv)])
        pr = O.pairs(g, cam, st)
        t0 = frame.cams[v].tile_offset
        nt = ((wv + 15) // 16) * ((hv + 15) // 16)
        m = (tiles >= t0) & (tiles < t0 + nt)
        okeys = pr["keys"] + (np.uint64(t0) << np.uint64(32))
        np.testing.assert_array_equal(gpu["keys"][m], okeys)
        np.testing.assert_array_equal(gpu["values"][m], pr["values"])
        r = O.render_binned(g, cam, st, pr["values"], pr["ranges"])
        add_branches(r, g, cam, st, pr["values"], pr["ranges"])
        mt = compare_forward({k: gpu[k][sl[v]] for k in ("image", "final_t", "n_contrib")}, r,
                             check_keys=False, label=f"workload{c} view {v}")
        note(f"workload{c}: view {v}: {int(m.sum())} pairs bit-exact, image max err {mt.err:.2e}")
    del gpu, frame
    # gradients on a frame of the sampled views
    angles = [w.angles[v] for v in views]
    sizes = [w.sizes[v] for v in views]
    ref = {"cams": oracle_cams(angles, sizes)}
    note(f"workload{c}: oracle forward of the sampled views")
    pr = O.pairs(g, ref["cams"], st)
    r = O.render_binned(g, ref["cams"], st, pr["values"], pr["ranges"])
    add_branches(r, g, ref["cams"], st, pr["values"], pr["ranges"])
    npx = sum(a * b for a, b in sizes)
    up = np.random.default_rng(1000 * c + 3).normal(size=npx).astype(np.float32)
    up = (grad_upstream(up, r) / npx).astype(np.float32)
    note(f"workload{c}: gpu forward + backward of the sampled views")
    run = gpu_run(g, angles, sizes, tile=16, lds=256, upstream=up)
    gg = run["grads"]
    mt = compare_forward(run, {**r, "pairs": pr}, check_keys=False, label=f"workload{c} sampled views")
    sel = np.zeros(w.n, bool)
    sel[np.random.default_rng(1000 * c + 4).choice(w.n, grad_gaussians, replace=False)] = True
    note(f"workload{c}: oracle adjoint of {grad_gaussians} sampled Gaussians")
    rg = O.backward(g, ref["cams"], st, up, binned=(pr["values"], pr["ranges"]), sel=sel,
                    flip=mt.flip)
    for k in KEYS:
        a = gg[k][sel].astype(np.float64).reshape(-1)
        b = rg[k][sel].reshape(-1)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        assert rel <= GRAD_TOL, (k, rel)
    note(f"workload{c}: sampled gradients within {GRAD_TOL}")


def test_workload5_sampled_views():
    _check_views(5, views=[0, 9], grad_gaussians=4000)


def test_workload4_sampled_views():
    w = S.workload(4)
    # one view of each detector size
    views = []
    for side in sorted(set(w.sizes)):
        views.append(w.sizes.index(side))
    _check_views(4, views=views, grad_gaussians=3000)
