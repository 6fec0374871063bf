"""The allocation-free loss gradient (xg_loss_grad_static, called through
the C ABI) against the workspace form xg_loss_grad on the same inputs: two
calls in a row on one device, the second with fewer and smaller views, so
the static array keeps the first call's contents when the second runs.
Both forms launch the same kernels on the same data, so the gradients and
the loss value must agree bit for bit (stronger than the 1e-4 rel L2
tolerance of the loss gradient against the oracle)."""
import numpy as np
import pytest

import scenes as S
from _gpu import note

pytestmark = pytest.mark.gpu


def _inputs(sizes, seed):
    rng = np.random.default_rng(seed)
    n = sum(w * h for w, h in sizes)
    x = rng.uniform(0, 1, n).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.1, n), 0, 1).astype(np.float32)
    eq = rng.uniform(size=n) < 0.05
    y[eq] = x[eq]
    return x, y


def _both(sizes, seed, gamma):
    import torch
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd import _lib as X
    angles = np.linspace(0, np.pi, len(sizes), endpoint=False)
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    frame = P.Frame(16, cams)
    x, y = _inputs(sizes, seed)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    g_ws = torch.full_like(xt, 7.0)
    g_st = torch.full_like(xt, -7.0)
    l_ws = torch.full((1,), 123.0, device="cuda")
    l_st = torch.full((1,), -123.0, device="cuda")
    X.xg_loss_grad(frame.frame, xt.data_ptr(), yt.data_ptr(), gamma, g_ws.data_ptr(),
                   l_ws.data_ptr(), stream)
    # the static form reads neither the workspace pointer nor its size
    f = X.XgFrame(frame.frame.n, frame.frame.n_views, frame.frame.cams, frame.frame.cams_dev,
                  frame.frame.settings, None, 0, frame.frame.pair_capacity)
    X.xg_loss_grad_static(f, xt.data_ptr(), yt.data_ptr(), gamma, g_st.data_ptr(),
                          l_st.data_ptr(), stream)
    torch.cuda.synchronize()
    return g_ws.cpu().numpy(), g_st.cpu().numpy(), float(l_ws.item()), float(l_st.item())


def test_static_loss_grad_matches_workspace_form_twice():
    # 8 views of 512 x 512 (the headline image set, 25.2 MB of maps), then
    # three ragged views: the second call leaves most of the array untouched
    for sizes, seed, gamma in (([(512, 512)] * 8, 11, 0.2),
                               ([(130, 70), (37, 29), (5, 3)], 12, 0.55)):
        note(f"loss_grad_static {len(sizes)} views {sizes[0]} gamma={gamma}")
        g_ws, g_st, l_ws, l_st = _both(sizes, seed, gamma)
        assert np.array_equal(g_ws, g_st), float(np.abs(g_ws - g_st).max())
        assert l_ws == l_st, (l_ws, l_st)
        assert np.isfinite(g_st).all() and l_st != -123.0


def test_static_loss_grad_rejects_oversize_frames():
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd import _lib as X
    cams = P.cameras([0.0], [(2048, 2048)], S.L_SO, S.L_SD, S.DETECTOR_SIDE, S.DETECTOR_SIDE)
    frame = P.Frame(16, cams)
    with pytest.raises(X.XgError) as e:
        X.xg_loss_grad_static(frame.frame, 256, 256, 0.2, 256)
    assert e.value.status == X.XG_ECAPACITY
