"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
the FP64 oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle as O
import scenes as S

D = S.DETECTOR_SIDE
KEYS = ("means", "scales", "quats", "opacity", "intensity")
IMG_TOL = 1e-5      # max abs image error on unflagged pixels
GRAD_TOL = 1e-4     # relative L2 gradient error per parameter group
FLAG_FRAC = 0.005   # at most this fraction of pixels may sit within a threshold margin


def note(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_cams(angles, sizes):
    return [O.camera(float(a), S.L_SO, S.L_SD, w, h, D, D) for a, (w, h) in zip(angles, sizes)]


def gpu_run(g: dict, angles, sizes, tile=16, lds=256, upstream=None, cap=None, lowpass=0.3,
            alpha_min=1.0 / 255.0, t_min=1e-4, backward=True, persistent=False):
    """Forward (and optionally backward) on cuda:0 through the C ABI."""
    import torch
    import paper_2403_04116_amd as P
    dev = torch.device("cuda:0")
    cams = P.cameras(angles, sizes, S.L_SO, S.L_SD, D, D)
    st = P.settings(tile=tile, lds_batch=lds, lowpass=lowpass, alpha_min=alpha_min, t_min=t_min,
                    persistent=persistent)
    n = g["means"].shape[0]
    frame = P.Frame(n, cams, st, pair_capacity=cap, device=dev)
    gt = {k: torch.from_numpy(np.ascontiguousarray(g[k])).to(dev) for k in KEYS}
    frame.fit_capacity(gt)
    image, final_t, n_contrib = frame.render_fwd(gt)
    keys, vals, ranges = frame.sorted_pairs()
    out = {"frame": frame, "image": image.cpu().numpy(), "final_t": final_t.cpu().numpy(),
           "n_contrib": n_contrib.cpu().numpy(),
           "keys": keys.cpu().numpy().view(np.uint64), "values": vals.cpu().numpy().view(np.uint32),
           "ranges": ranges.cpu().numpy().view(np.uint32), "status": frame.status()}
    if backward and upstream is not None:
        up = torch.from_numpy(np.ascontiguousarray(upstream, dtype=np.float32)).to(dev)
        grads = frame.backward(gt, up, final_t, n_contrib)
        torch.cuda.synchronize()
        out["grads"] = {k: grads[k].cpu().numpy() for k in KEYS}
    torch.cuda.synchronize()
    return out


def oracle_run(g: dict, angles, sizes, tile=16, lowpass=0.3, alpha_min=1.0 / 255.0, t_min=1e-4):
    st = O.Settings(tile=tile, lowpass=lowpass, alpha_min=alpha_min, t_min=t_min)
    cams = oracle_cams(angles, sizes)
    pr = O.pairs(g, cams, st)
    r = O.render_binned(g, cams, st, pr["values"], pr["ranges"])
    return {"st": st, "cams": cams, "pairs": pr, **r}


def compare_forward(gpu, ref, check_keys=True):
    if check_keys:
        assert gpu["keys"].shape == ref["pairs"]["keys"].shape, (gpu["keys"].shape,
                                                                 ref["pairs"]["keys"].shape)
        np.testing.assert_array_equal(gpu["keys"], ref["pairs"]["keys"])
        np.testing.assert_array_equal(gpu["values"], ref["pairs"]["values"])
        np.testing.assert_array_equal(gpu["ranges"], ref["pairs"]["ranges"])
    ok = ref["flags"] == 0
    assert (~ok).mean() <= FLAG_FRAC, f"flagged fraction {(~ok).mean()}"
    err = np.abs(gpu["image"].astype(np.float64) - ref["image"])[ok]
    terr = np.abs(gpu["final_t"].astype(np.float64) - ref["final_t"])[ok]
    assert err.max(initial=0) <= IMG_TOL, f"image max abs error {err.max()}"
    assert terr.max(initial=0) <= IMG_TOL, f"final_t max abs error {terr.max()}"
    np.testing.assert_array_equal(gpu["n_contrib"][ok], ref["n_contrib"][ok])
    return ok, float(err.max(initial=0))


def compare_grads(gpu_grads, ref_grads):
    errs = {}
    for k in KEYS:
        a = gpu_grads[k].astype(np.float64).reshape(-1)
        b = ref_grads[k].reshape(-1)
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)
        errs[k] = rel
        assert rel <= GRAD_TOL, f"{k}: rel L2 {rel}"
    return errs
