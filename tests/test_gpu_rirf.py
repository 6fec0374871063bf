"""Radiation intensity response (Eq. 3) on the GPU (xg_rirf_fwd /
xg_rirf_bwd) against the FP64 oracle, and through torch autograd."""
import numpy as np
import pytest

from oracle import adam as A
from _gpu import note

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nf", [(1, 1), (257, 16), (10007, 16), (3000, 64), (0, 16)])
def test_rirf_forward_backward(n, nf):
    import torch
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd import _lib as X
    rng = np.random.default_rng(n + nf)
    f = (rng.normal(size=(n, nf)) * 0.5).astype(np.float32)
    w = rng.uniform(-1.5, 1.5, nf).astype(np.float32)
    gi = rng.normal(size=n).astype(np.float32)
    note(f"rirf n={n} nf={nf}")
    ft, wt, git = (torch.from_numpy(x).cuda() for x in (f, w, gi))
    inten = P.rirf(ft, wt)
    gf = torch.full((n, nf), 0.25, device="cuda")        # accumulates onto existing values
    X.xg_rirf_bwd(ft.data_ptr(), wt.data_ptr(), n, nf, git.data_ptr(), gf.data_ptr(), 0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(inten.cpu().numpy(), A.rirf(f, w), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(gf.cpu().numpy(), 0.25 + A.rirf_grad(f, w, gi), rtol=1e-5, atol=1e-6)


def test_rirf_autograd_function():
    import torch
    import paper_2403_04116_amd as P
    rng = np.random.default_rng(5)
    f = torch.from_numpy((rng.normal(size=(500, 16)) * 0.5).astype(np.float32)).cuda().requires_grad_()
    w = torch.from_numpy(rng.uniform(0.2, 1.5, 16).astype(np.float32)).cuda()
    up = torch.from_numpy(rng.normal(size=500).astype(np.float32)).cuda()
    (P.RIRFFunction.apply(f, w) * up).sum().backward()
    torch.cuda.synchronize()
    ref = A.rirf_grad(f.detach().cpu().numpy(), w.cpu().numpy(), up.cpu().numpy())
    np.testing.assert_allclose(f.grad.cpu().numpy(), ref, rtol=1e-5, atol=1e-6)
