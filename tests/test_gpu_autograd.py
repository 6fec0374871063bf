"""The differentiable wrapper (DRRFunction / render(), Eq. 5 with the
hand-written backward of Sec. 3.2) driven by torch.autograd on the GPU.

- An L1 loss against an oracle-rendered target of a perturbed scene, then
  loss.backward(): the parameters' .grad against the FP64 oracle adjoint for
  the same float32 upstream gradient (captured from autograd), 1e-4
  relative L2, on workload 1 and on a ragged multi-view scene.
- A tiny smooth-regime scene (alpha_min = 0, t_min = 0, o <= 0.9): .grad
  against FP64 central differences of the oracle's forward.
- Misuse: a second forward before the backward raises; a second backward
  of the same graph (retain_graph) adds the same gradients again; a pair
  overflow in the forward grows the workspace and renders again.
"""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S
from _gpu import KEYS, GRAD_TOL, compare_forward, compare_grads, note, oracle_run

pytestmark = pytest.mark.gpu

D = S.DETECTOR_SIDE


def _leaves(g):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(g[k])).cuda().requires_grad_(True) for k in KEYS}


def _frame(g, angles, sizes, **kw):
    import paper_2403_04116_amd as P
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, D, D)
    return P.Frame(g["means"].shape[0], cams, P.settings(**kw), device="cuda")


def _l1_autograd(g, angles, sizes, seed, label):
    """render() -> masked mean |I - I*| -> backward; returns (.grad, the
    upstream autograd handed to the renderer, the forward outputs)."""
    import torch
    import paper_2403_04116_amd as P
    ref = oracle_run(g, angles, sizes)
    tgt = oracle_run(S.perturb(g, seed), angles, sizes)["image"]
    leaves = _leaves(g)
    frame = _frame(g, angles, sizes)
    image, final_t, n_contrib = P.DRRFunction.apply(*(leaves[k] for k in KEYS), frame)
    assert not final_t.requires_grad and not n_contrib.requires_grad
    captured = []
    image.register_hook(lambda t: captured.append(t.detach().clone()))
    # pixels excluded from gradient comparisons carry zero weight in the loss
    w = torch.from_numpy(ref["grad_ok"].astype(np.float32)).cuda()
    target = torch.from_numpy(tgt.astype(np.float32)).cuda()
    loss = ((image - target).abs() * w).mean()
    loss.backward()
    torch.cuda.synchronize()
    up = captured[0].cpu().numpy()
    out = {"image": image.detach().cpu().numpy(), "final_t": final_t.cpu().numpy(),
           "n_contrib": n_contrib.cpu().numpy()}
    note(f"{label}: loss {loss.item():.4e}, nonzero upstream {(up != 0).mean():.3f}")
    return {k: leaves[k].grad.cpu().numpy() for k in KEYS}, up, out, ref


@pytest.mark.parametrize("case", ["workload1", "ragged"])
def test_l1_backward_matches_oracle_adjoint(case):
    if case == "workload1":
        w = S.workload(1)
        g, angles, sizes, seed = S.scene(1), w.angles, w.sizes, w.seeds["perturb"]
    else:
        g = S.gaussians(2500, math.log(0.05), 0.4, 55)
        sizes = [(96, 80), (50, 33), (128, 128), (8, 8)]
        angles = np.random.default_rng(56).uniform(0, 2 * math.pi, len(sizes)).tolist()
        seed = 57
    grads, up, out, ref = _l1_autograd(g, angles, sizes, seed, case)
    m = compare_forward(out, ref, check_keys=False, label=case)
    assert np.all(up[~ref["grad_ok"]] == 0)
    rg = O.backward(g, ref["cams"], ref["st"], up, binned=(ref["pairs"]["values"],
                                                         ref["pairs"]["ranges"]), flip=m.flip)
    errs = compare_grads(grads, rg)
    note(f"{case}: autograd gradients rel L2 {max(errs.values()):.2e}")


def test_smooth_regime_against_finite_differences():
    """loss = sum_p u_p I(p) on 4 Gaussians and two 16 x 16 views, no
    thresholds: .grad from autograd against central differences (h = 1e-6)
    of the oracle's float64 forward."""
    import torch
    import paper_2403_04116_amd as P
    rng = np.random.default_rng(91)
    n = 4
    g = {"means": rng.uniform(-0.5, 0.5, (n, 3)).astype(np.float32),
         "scales": np.exp(rng.normal(math.log(0.25), 0.3, (n, 3))).astype(np.float32),
         "quats": rng.normal(size=(n, 4)).astype(np.float32),
         "opacity": rng.uniform(0.2, 0.9, n).astype(np.float32),
         "intensity": rng.uniform(0.1, 1.0, n).astype(np.float32)}
    angles, sizes = [0.3, 2.2], [(16, 16), (16, 19)]
    npx = 16 * 16 + 16 * 19
    u = rng.normal(size=npx).astype(np.float32)
    leaves = _leaves(g)
    frame = _frame(g, angles, sizes, tile=8, alpha_min=0.0, t_min=0.0)
    image = P.render(leaves, frame)
    (image * torch.from_numpy(u).cuda()).sum().backward()
    torch.cuda.synchronize()
    st = O.Settings(tile=8, alpha_min=0.0, t_min=0.0)
    cams = [O.camera(a, S.L_SO, S.L_SD, w, h, D, D) for a, (w, h) in zip(angles, sizes)]
    g64 = {k: v.astype(np.float64) for k, v in g.items()}

    def loss(gg):
        im = np.concatenate([O.render_brute(gg, c, st)["image"] for c in cams])
        return float(np.dot(im, u.astype(np.float64)))

    for k in KEYS:
        fd = np.zeros_like(g64[k])
        flat = g64[k].reshape(-1)
        for j in range(flat.size):
            x0 = flat[j]
            h = 1e-6 * max(1.0, abs(x0))
            flat[j] = x0 + h
            lp = loss(g64)
            flat[j] = x0 - h
            lm = loss(g64)
            flat[j] = x0
            fd.reshape(-1)[j] = (lp - lm) / (2 * h)
        got = leaves[k].grad.cpu().numpy().astype(np.float64)
        rel = np.linalg.norm(got - fd) / np.linalg.norm(fd)
        note(f"finite differences {k}: rel L2 {rel:.2e}")
        assert rel <= GRAD_TOL, (k, rel)


def test_second_forward_before_backward_raises():
    import paper_2403_04116_amd as P
    g = S.gaussians(300, math.log(0.05), 0.3, 4)
    frame = _frame(g, [0.5], [(32, 32)])
    leaves = _leaves(g)
    a = P.render(leaves, frame)
    b = P.render(leaves, frame)            # the frame now holds b's lists
    with pytest.raises(RuntimeError, match="rendered again"):
        a.sum().backward()
    b.sum().backward()                     # b's own backward works


def test_retained_graph_second_backward_adds_the_same_gradients():
    import torch
    import paper_2403_04116_amd as P
    g = S.gaussians(800, math.log(0.05), 0.3, 6)
    frame = _frame(g, [0.5, 2.0], [(48, 40), (32, 32)])
    leaves = _leaves(g)
    image = P.render(leaves, frame)
    u = torch.from_numpy(np.random.default_rng(1).normal(size=image.numel()).astype(np.float32)).cuda()
    loss = (image * u).sum()
    loss.backward(retain_graph=True)
    first = {k: leaves[k].grad.clone() for k in KEYS}
    loss.backward()
    torch.cuda.synchronize()
    for k in KEYS:
        d = (leaves[k].grad - 2 * first[k]).norm() / first[k].norm().clamp_min(1e-30)
        assert d.item() < 1e-5, (k, d.item())


def test_overflow_in_forward_grows_and_renders_again():
    import torch
    import paper_2403_04116_amd as P
    g = S.gaussians(1500, math.log(0.05), 0.4, 31)
    angles, sizes = [0.3, 1.7], [(64, 64), (40, 24)]
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, D, D)
    frame = P.Frame(1500, cams, P.settings(), pair_capacity=64, device="cuda")
    leaves = _leaves(g)
    image = P.render(leaves, frame)
    torch.cuda.synchronize()
    assert frame.capacity > 64 and frame.status() == 0
    ref = oracle_run(g, angles, sizes)
    ft = frame.render_fwd({k: v.detach() for k, v in leaves.items()})
    compare_forward({"image": image.detach().cpu().numpy(), "final_t": ft[1].cpu().numpy(),
                     "n_contrib": ft[2].cpu().numpy()}, ref, check_keys=False, label="regrown")
