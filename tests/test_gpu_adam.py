"""Fused Adam (xg_adam_step) against the FP64 optimiser oracle: raw
parameters (16-feature intensity response), moments and activated copies
over several steps, inside a captured graph, and after a complete render +
backward + update step."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import adam as A
import scenes as S
from _gpu import KEYS, note, oracle_cams

pytestmark = pytest.mark.gpu

RAWK = A.RAW


def _raw(n, seed, nf):
    rng = np.random.default_rng(seed)
    return {"means": rng.uniform(-1, 1, (n, 3)).astype(np.float32),
            "log_scales": rng.normal(math.log(0.02), 0.3, (n, 3)).astype(np.float32),
            "quats": rng.normal(size=(n, 4)).astype(np.float32),
            "opacity_logit": rng.normal(size=n).astype(np.float32),
            "features": (rng.normal(size=(n, nf)) * 0.3).astype(np.float32)}


def _grads(n, seed):
    rng = np.random.default_rng(seed)
    return {"means": rng.normal(size=(n, 3)).astype(np.float32),
            "scales": (rng.normal(size=(n, 3)) * 5).astype(np.float32),
            "quats": (rng.normal(size=(n, 4)) * 0.1).astype(np.float32),
            "opacity": rng.normal(size=n).astype(np.float32),
            "intensity": rng.normal(size=n).astype(np.float32)}


def _weights(nf):
    return np.random.default_rng(nf).uniform(0.2, 1.5, nf).astype(np.float32)


def _gpu_opt(raw_np, w_np):
    import torch
    from paper_2403_04116_amd.optim import FusedAdam
    raw = {k: torch.from_numpy(v.copy()).cuda() for k, v in raw_np.items()}
    act = {"means": raw["means"], "quats": raw["quats"],
           "scales": torch.empty_like(raw["log_scales"]),
           "opacity": torch.empty_like(raw["opacity_logit"]),
           "intensity": torch.empty(raw["means"].shape[0], device="cuda")}
    return FusedAdam(raw, act, torch.from_numpy(w_np).cuda())


def _check(opt, raw_o, act_o, m_o, v_o, lrs):
    import torch
    torch.cuda.synchronize()
    lr = max(lrs.values())
    for k in RAWK:
        got = opt.raw[k].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, raw_o[k], rtol=2e-6, atol=1e-4 * lr)
    n = opt.n
    sizes = {"means": 3 * n, "log_scales": 3 * n, "quats": 4 * n, "opacity_logit": n,
             "features": opt.n_features * n}
    off = 0
    mm, vv = opt.m.cpu().numpy(), opt.v.cpu().numpy()
    for k in RAWK:
        sz = sizes[k]
        # float32 moments: cancellation in beta1 * m + (1 - beta1) * g leaves
        # absolute noise relative to the group's largest moment
        np.testing.assert_allclose(mm[off:off + sz], m_o[k].reshape(-1), rtol=1e-5,
                                   atol=1e-6 * np.abs(m_o[k]).max())
        np.testing.assert_allclose(vv[off:off + sz], v_o[k].reshape(-1), rtol=1e-5,
                                   atol=1e-6 * np.abs(v_o[k]).max())
        off += sz
    for k in ("scales", "opacity", "intensity"):
        np.testing.assert_allclose(opt.act[k].cpu().numpy(), act_o[k], rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("nf", [16, 1, 37])
def test_adam_steps_match_oracle(nf):
    import torch
    n = 5003
    raw_np = _raw(n, 1, nf)
    w = _weights(nf)
    opt = _gpu_opt(raw_np, w)
    cur = {k: v.astype(np.float64) for k, v in raw_np.items()}
    m = {k: np.zeros_like(v) for k, v in cur.items()}
    v = {k: np.zeros_like(x) for k, x in cur.items()}
    prev = cur
    for t in range(1, 5):
        g = _grads(n, 10 + t)
        note(f"adam step {t}, {nf} features")
        opt.step({k: torch.from_numpy(x).cuda() for k, x in g.items()})
        lrs = A.paper_lrs(t)
        # the oracle steps from the GPU's float32 parameters of the previous step
        cur, m, v, act = A.adam_step(prev, g, m, v, t, lrs, w.astype(np.float64))
        _check(opt, cur, act, m, v, lrs)
        prev = {k: opt.raw[k].cpu().numpy().astype(np.float64) for k in RAWK}
    assert int(opt.step_count.item()) == 4


def test_adam_in_captured_graph_advances_the_step():
    import torch
    n, nf = 2048, 16
    raw_np = _raw(n, 2, nf)
    w = _weights(nf)
    g = _grads(n, 3)
    gt = {k: torch.from_numpy(x).cuda() for k, x in g.items()}
    eager = _gpu_opt(raw_np, w)
    for _ in range(4):
        eager.step(gt)
    cap = _gpu_opt(raw_np, w)
    cap.step(gt)                      # step 1 eager (warm-up)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cap.step(gt)
    for r in range(3):                # steps 2..4 by replay
        junk = torch.ones(1000, device="cuda").sum()
        torch.cuda.synchronize()
        graph.replay()
    torch.cuda.synchronize()
    assert int(cap.step_count.item()) == 4
    for k in RAWK:
        np.testing.assert_allclose(cap.raw[k].cpu().numpy(), eager.raw[k].cpu().numpy(), rtol=0, atol=0)


def test_render_backward_adam_step_matches_oracle():
    """Complete step on a small scene: render, L1 upstream, backward, Adam."""
    import torch
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd.optim import FusedAdam
    g_np = S.gaussians(1500, math.log(0.05), 0.3, 5)
    sizes = [(64, 64), (48, 40)]
    angles = [0.5, 2.5]
    st_o = O.Settings(tile=16)
    cams_o = oracle_cams(angles, sizes)
    ref = O.render_views(g_np, cams_o, st_o)
    tgt = O.render_views(S.perturb(g_np, 7), cams_o, st_o)["image"]
    npx = sum(w * h for w, h in sizes)
    ok = ref["flags"] == 0
    # upstream fixed by the oracle's images (zero on flagged pixels)
    up = np.where(ok, np.sign(ref["image"] - tgt) / npx, 0).astype(np.float32)
    gt = {k: torch.from_numpy(x).cuda() for k, x in g_np.items()}
    opt = FusedAdam.from_activated(gt)
    frame = P.Frame(1500, P.cameras(angles, sizes, S.L_SO, S.L_SD, S.DETECTOR_SIDE, S.DETECTOR_SIDE),
                    P.settings(), device="cuda")
    frame.fit_capacity(opt.act)
    img, ft, nc = frame.render_fwd(opt.act)
    grads = frame.backward(opt.act, torch.from_numpy(up).cuda(), ft, nc)
    raw0 = {k: t.cpu().numpy().astype(np.float64) for k, t in opt.raw.items()}
    w = opt.weights.cpu().numpy().astype(np.float64)
    opt.step(grads)
    torch.cuda.synchronize()
    gref = O.backward(g_np, cams_o, st_o, up)
    z = {k: np.zeros_like(x) for k, x in raw0.items()}
    new, m, v, act = A.adam_step(raw0, {"means": gref["means"], "scales": gref["scales"],
                                        "quats": gref["quats"], "opacity": gref["opacity"],
                                        "intensity": gref["intensity"]}, z, z, 1, A.paper_lrs(1), w)
    # the first step moves each parameter by lr * sign(raw gradient): compare
    # where the oracle's gradient is well above the renderer's atomic-order noise
    rg = A.raw_grads(raw0, gref, w)
    for k in RAWK:
        got = opt.raw[k].cpu().numpy().astype(np.float64)
        big = np.abs(rg[k]) > 1e-2 * np.abs(rg[k]).max()
        np.testing.assert_allclose(got[big], new[k][big], rtol=1e-6,
                                   atol=1e-3 * A.paper_lrs(1)[k])
        assert big.mean() > 0.05, k


def _train_setup(cap=None, n=2500, seed=81):
    import torch
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd.optim import FusedAdam
    from paper_2403_04116_amd.step import TrainStep
    g = S.gaussians(n, math.log(0.05), 0.4, seed)
    sizes = [(96, 80), (64, 64)]
    angles = [0.3, 1.9]
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    frame = P.Frame(n, cams, P.settings(), pair_capacity=cap, device="cuda")
    opt = FusedAdam.from_activated({k: torch.from_numpy(g[k]).cuda() for k in KEYS})
    npx = sum(w * h for w, h in sizes)
    target = torch.from_numpy(np.random.default_rng(seed + 1).uniform(0, 0.5, npx)
                              .astype(np.float32)).cuda()
    return frame, opt, TrainStep(frame, opt.act, target, 1.0 / npx, optimizer=opt)


def test_overflowed_step_leaves_the_parameters_alone():
    import torch
    frame, opt, step = _train_setup(cap=128)
    before = {k: t.clone() for k, t in opt.raw.items()}
    note("overflowing step")
    step.run()
    assert not step.check()                     # overflow: workspace grown
    assert int(opt.step_count.item()) == 0
    for k in RAWK:
        assert torch.equal(before[k], opt.raw[k]), k
    assert float(opt.m.abs().max()) == 0.0
    step.run()
    assert step.check()
    assert int(opt.step_count.item()) == 1
    assert not torch.equal(before["means"], opt.raw["means"])


def test_captured_training_steps_follow_the_eager_ones():
    """Eager and replayed training steps from the same start: the parameter
    trajectories agree up to the renderer's atomic-order noise (a tiny
    gradient whose sign flips moves a parameter by 2 lr on the first step)."""
    import torch
    fe, oe, se = _train_setup()
    fe.fit_capacity(oe.act)
    fg, og, sg = _train_setup()
    fg.fit_capacity(og.act)
    sg.capture()
    assert int(og.step_count.item()) == 0        # the warm-up left the optimiser out
    for r in range(4):
        se.run()
        junk = torch.ones(513, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        sg.replay()
        note(f"train step {r}")
        assert se.check() and sg.check()
    assert int(oe.step_count.item()) == 4 and int(og.step_count.item()) == 4
    for k in RAWK:
        a, b = oe.raw[k].cpu().numpy(), og.raw[k].cpu().numpy()
        assert np.isfinite(b).all()
        lr = A.paper_lrs(1)[k]
        close = np.abs(a - b) <= 1e-2 * lr
        assert close.mean() > 0.98, (k, close.mean())
