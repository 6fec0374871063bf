"""Stored-transmittance variant (xg_render_fwd_store / xg_render_bwd_store)
against the FP64 oracle's adjoint (which keeps every T_j of Eq. 10) and
against the division-based backward.  The forward's outputs are bitwise
those of xg_render_fwd; gradients meet the 1e-4 relative L2 bar, also when
pixels have more contributors than stored slots (the rest are divided
back)."""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S
from _gpu import KEYS, compare_forward, compare_grads, grad_upstream, note, oracle_run

pytestmark = pytest.mark.gpu


def _both(g, angles, sizes, slots, up, tile=16, lds=256):
    """Division path and stored path on one frame: (outputs, grads) of each."""
    import torch
    import paper_2403_04116_amd as P
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    frame = P.Frame(g["means"].shape[0], cams, P.settings(tile=tile, lds_batch=lds), device="cuda")
    gt = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda() for k in KEYS}
    upt = torch.from_numpy(np.ascontiguousarray(up, dtype=np.float32)).cuda()
    frame.fit_capacity(gt)
    a = frame.render_fwd(gt)
    ga = frame.backward(gt, upt, a[1], a[2])
    store = frame.new_store(slots)
    frame.preprocess_sort(gt)          # clears the 2-D accumulators
    b = frame.render_fwd_store(gt, store)
    gb = frame.backward_store(gt, upt, b[1], b[2], store)
    torch.cuda.synchronize()
    out = lambda o: [t.cpu().numpy() for t in o]
    grads = lambda gg: {k: gg[k].cpu().numpy() for k in KEYS}
    return out(a), grads(ga), out(b), grads(gb), store, frame


def _check(g, angles, sizes, slots, tile=16, lds=256, seed=3):
    ref = oracle_run(g, angles, sizes, tile=tile)
    npx = sum(w * h for w, h in sizes)
    up = np.random.default_rng(seed).normal(size=npx).astype(np.float32)
    up = grad_upstream(up, ref)
    fa, ga, fb, gb, store, frame = _both(g, angles, sizes, slots, up, tile, lds)
    for x, y in zip(fa, fb):
        np.testing.assert_array_equal(x, y)
    m = compare_forward({"image": fb[0], "final_t": fb[1], "n_contrib": fb[2]}, ref,
                        check_keys=False, label=f"stored slots={slots}")
    rg = O.backward(g, ref["cams"], ref["st"], up, binned=(ref["pairs"]["values"],
                                                          ref["pairs"]["ranges"]), flip=m.flip)
    errs = compare_grads(gb, rg)
    # stored and divided transmittances agree to float32 rounding
    for k in KEYS:
        d = np.linalg.norm(ga[k].astype(np.float64) - gb[k]) / max(np.linalg.norm(gb[k]), 1e-30)
        assert d < 2e-5, (k, d)
    return errs, store, frame, fb


def test_workload1_stored():
    w = S.workload(1)
    note("workload1 stored T")
    errs, store, frame, fb = _check(S.scene(1), w.angles, w.sizes, slots=256)
    # the per-pixel contributor counts the forward kept equal the counts pass
    counts = frame.render_counts().cpu().numpy()
    kept = store.contributors(frame).cpu().numpy()
    assert kept.sum() == counts[1].sum() and kept.max() == counts[1].max()
    np.testing.assert_array_equal(np.bincount(kept), np.bincount(counts[1], minlength=kept.max() + 1))


@pytest.mark.parametrize("slots", [1, 5, 40, 4096])
@pytest.mark.parametrize("tile,lds", [(8, 64), (16, 128), (32, 256)])
def test_ragged_multiview_stored(slots, tile, lds):
    """Slot counts below, near and above the per-pixel contributor counts."""
    g = S.gaussians(2500, math.log(0.05), 0.4, 5)
    sizes = [(96, 80), (50, 33), (128, 128), (8, 8)]
    angles = np.random.default_rng(6).uniform(0, 2 * math.pi, len(sizes)).tolist()
    note(f"stored T slots={slots} tile={tile} lds={lds}")
    _check(g, angles, sizes, slots, tile, lds)

