"""The fused entry points against the separate ones, bit for bit:
xg_render_fwd_l1 (forward blend with the L1 gradient in its epilogue)
against xg_render_fwd + xg_l1_grad, and xg_preprocess_bwd_write against
clearing + xg_preprocess_bwd, including Gaussians that no view touches
(written as zeros over stale values)."""
import math

import numpy as np
import pytest

import scenes as S
from _gpu import KEYS, note

pytestmark = pytest.mark.gpu

D = S.DETECTOR_SIDE


def _setup(n, sizes, angles, seed):
    import torch
    import paper_2403_04116_amd as P
    g = S.gaussians(n, math.log(0.05), 0.3, seed)
    # a few Gaussians far outside every view: culled, no gradient
    g["means"][:5] = np.float32([40.0, 40.0, 40.0])
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, D, D)
    frame = P.Frame(n, cams, P.settings(tile=16))
    gt = {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda() for k in KEYS}
    frame.fit_capacity(gt)
    return P, frame, gt


@pytest.mark.parametrize("n,sizes", [(2000, [(64, 64), (80, 48), (37, 53)]), (30000, [(256, 256)] * 2)])
def test_fused_forward_l1_and_written_gradients(n, sizes):
    import torch
    from paper_2403_04116_amd import _lib as X
    note(f"fused entry points n={n} views={len(sizes)}")
    angles = [0.3 + 1.7 * k for k in range(len(sizes))]
    P, frame, gt = _setup(n, sizes, angles, 90 + n)
    npx = frame.total_pixels
    target = torch.rand(npx, device="cuda")
    # a target equal to the image in places (sign 0)
    img0, _, _ = frame.render_fwd(gt)
    target[::7] = img0[::7]
    scale = 1.0 / npx
    gs = P.drr.gaussians_struct(gt)

    image, final_t, n_contrib = frame.new_outputs()
    dl = torch.empty(npx, device="cuda")
    X.xg_render_fwd(frame.frame, gs, image.data_ptr(), final_t.data_ptr(), n_contrib.data_ptr(), 0)
    X.xg_l1_grad(image.data_ptr(), target.data_ptr(), dl.data_ptr(), npx, scale, 0)

    image2, final_t2, n_contrib2 = frame.new_outputs()
    dl2 = torch.full((npx,), float("nan"), device="cuda")
    X.xg_render_fwd_l1(frame.frame, gs, image2.data_ptr(), final_t2.data_ptr(), n_contrib2.data_ptr(),
                       target.data_ptr(), scale, dl2.data_ptr(), 0)
    torch.cuda.synchronize()
    for a, b in ((image, image2), (final_t, final_t2), (n_contrib, n_contrib2), (dl, dl2)):
        assert torch.equal(a, b)
    assert (dl2 == 0).any()

    g1 = frame.new_grads(gt)
    g1.zero_()
    frame.backward(gt, dl, final_t, n_contrib, grads=g1)
    # the written gradients from the same 2-D accumulators (the reverse
    # blend's float atomics add in no fixed order, so it runs once)
    g2 = frame.new_grads(gt)
    g2.flat.fill_(float("nan"))   # stale contents must be overwritten
    X.xg_preprocess_bwd_write(frame.frame, gs, X.XgGrads(*(g2[k].data_ptr() for k in P.drr.PARAMS)), 0)
    torch.cuda.synchronize()
    for k in P.drr.PARAMS:
        assert torch.equal(g1[k], g2[k]), k
    assert torch.all(g2["means"][:5] == 0)


def test_fused_forward_validation():
    import torch
    from paper_2403_04116_amd import _lib as X
    P, frame, gt = _setup(100, [(32, 32)], [0.0], 3)
    gs = P.drr.gaussians_struct(gt)
    image, final_t, n_contrib = frame.new_outputs()
    with pytest.raises(X.XgError):
        X.xg_render_fwd_l1(frame.frame, gs, image.data_ptr(), final_t.data_ptr(), n_contrib.data_ptr(),
                           0, 1.0, image.data_ptr(), 0)
    with pytest.raises(X.XgError):
        X.xg_render_fwd_l1(frame.frame, gs, image.data_ptr(), final_t.data_ptr(), n_contrib.data_ptr(),
                           image.data_ptr(), float("inf"), final_t.data_ptr(), 0)
