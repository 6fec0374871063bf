"""The training step captured as one HIP graph: replays match the eager
step (images bitwise, gradients to float32 atomic-order noise), with eager
work and synchronisations between replays, and the capacity check grows the
workspace and re-captures."""
import math

import numpy as np
import pytest

import scenes as S
from _gpu import KEYS, note

pytestmark = pytest.mark.gpu


def _setup(cap=None, n=3000, seed=61):
    import torch
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd.step import TrainStep
    g = S.gaussians(n, math.log(0.05), 0.4, seed)
    sizes = [(96, 80), (64, 64), (128, 96)]
    angles = np.random.default_rng(seed + 1).uniform(0, 2 * math.pi, len(sizes)).tolist()
    dev = torch.device("cuda:0")
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    frame = P.Frame(n, cams, P.settings(), pair_capacity=cap, device=dev)
    gt = {k: torch.from_numpy(g[k]).to(dev) for k in KEYS}
    npx = sum(w * h for w, h in sizes)
    target = torch.from_numpy(np.random.default_rng(seed + 2).uniform(0, 0.5, npx)
                              .astype(np.float32)).to(dev)
    return frame, gt, TrainStep(frame, gt, target, 1.0 / npx)


def _snapshot(step):
    import torch
    torch.cuda.synchronize()
    return (step.image.cpu().numpy().copy(), step.n_contrib.cpu().numpy().copy(),
            {k: step.grads[k].cpu().numpy().astype(np.float64) for k in KEYS})


def _same(a, b):
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    for k in KEYS:
        d = np.linalg.norm(a[2][k] - b[2][k]) / max(np.linalg.norm(a[2][k]), 1e-30)
        assert d < 1e-5, (k, d)


def test_graph_replays_match_eager():
    import torch
    frame, gt, step = _setup()
    frame.fit_capacity(gt)
    note("eager step")
    step.run()
    eager = _snapshot(step)
    note("capture")
    step.capture()
    for r in range(3):
        junk = torch.randn(4096, device="cuda") * 3.0 + 1.0       # eager work between replays
        torch.cuda.synchronize()
        assert float(junk.abs().sum()) > 0
        step.replay()
        note(f"replay {r}")
        _same(eager, _snapshot(step))
    assert step.check()


def test_graph_capacity_growth_recaptures():
    frame, gt, step = _setup(cap=256)
    note("eager step at small capacity")
    step.run()
    assert not step.check()            # overflowed: grown, stages re-run
    step.run()
    assert step.check()
    eager = _snapshot(step)
    big = frame.capacity
    frame.set_capacity(512)            # shrink again, capture, overflow inside the graph
    step.capture()
    step.replay()
    assert not step.check()            # grown and re-captured
    assert frame.capacity >= big - 2048
    step.replay()
    assert step.check()
    _same(eager, _snapshot(step))


def test_autotuner_picks_a_valid_setting_and_caches(tmp_path, monkeypatch):
    import torch
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd.autotune import autotune
    monkeypatch.setenv("XG_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    frame, gt, step = _setup(n=2000, seed=71)
    cams = list(frame.cams)
    note("autotune sweep")
    r = autotune(gt, cams, step.target, step.scale, steps=2, warmup=1)
    assert not r["cached"] and len(r["ms"]) == 9
    best = r["settings"]
    assert (best.tile, best.lds_batch) == min(r["ms"], key=r["ms"].get)
    r2 = autotune(gt, cams, step.target, step.scale, steps=2, warmup=1)
    assert r2["cached"] and (r2["settings"].tile, r2["settings"].lds_batch) == (best.tile, best.lds_batch)
    # the tuned setting renders the same image as the default one
    f2 = P.Frame(2000, cams, best, device="cuda")
    f2.fit_capacity(gt)
    im2, _, _ = f2.render_fwd(gt)
    frame.fit_capacity(gt)
    im1, _, _ = frame.render_fwd(gt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(im1.cpu().numpy(), im2.cpu().numpy())
