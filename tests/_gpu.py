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


def add_branches(r: dict, g: dict, cams, st, values, ranges) -> dict:
    """Adds to a binned oracle render ``r`` what the parity rule needs for
    pixels whose decisions sit within a rounding margin of a threshold:
    - "single": exactly one flagged decision.  "alt" holds the render with
      that decision taken the other way (both branches are admissible);
    - "multi": two or more flagged decisions (excluded, counted);
    - "grad_ok": pixels whose upstream gradient is kept in gradient
      comparisons: not "multi", and not a "single" pixel whose two branches
      give the same outputs within the tolerance (there the branch the GPU
      took, which decides the pixel's gradient, cannot be read from its
      outputs)."""
    nf = O.n_flags(r["flags"])
    single, multi = nf == 1, nf >= 2
    r["single"], r["multi"] = single, multi
    if single.any():
        a = O.render_binned(g, cams, st, values, ranges, flip=single, only=single)
        r["alt"] = {k: a[k] for k in ("image", "final_t", "n_contrib", "evals")}
        same = single & (np.abs(r["image"] - a["image"]) <= 2 * IMG_TOL) \
            & (np.abs(r["final_t"] - a["final_t"]) <= 2 * IMG_TOL) & (r["n_contrib"] == a["n_contrib"])
    else:
        r["alt"] = None
        same = np.zeros_like(single)
    r["grad_ok"] = ~(multi | same)
    return r


def oracle_run(g: dict, angles, sizes, tile=16, lowpass=0.3, alpha_min=1.0 / 255.0, t_min=1e-4):
    st = O.Settings(tile=tile, lowpass=lowpass, alpha_min=alpha_min, t_min=t_min)
    cams = oracle_cams(angles, sizes)
    pr = O.pairs(g, cams, st)
    r = O.render_binned(g, cams, st, pr["values"], pr["ranges"])
    add_branches(r, g, cams, st, pr["values"], pr["ranges"])
    return {"st": st, "cams": cams, "pairs": pr, **r}


def grad_upstream(up, ref) -> np.ndarray:
    """The upstream gradient fed to both backward passes: zero on pixels
    excluded from gradient comparisons (see add_branches)."""
    return np.where(ref["grad_ok"], up, 0.0).astype(np.float32)


class Match:
    """Outcome of a forward comparison: ``flip`` marks pixels where the GPU
    took the other branch of a single flagged decision (pass it to
    oracle.backward), ``ok`` the pixels that were compared."""

    def __init__(self, ok, flip, err, frac_single, frac_multi):
        self.ok, self.flip, self.err = ok, flip, err
        self.frac_single, self.frac_multi = frac_single, frac_multi

    def __iter__(self):   # ok, err = compare_forward(...)
        return iter((self.ok, self.err))


def _agree(gpu, ref, sel):
    """Per pixel of ``sel``: image and final T within IMG_TOL, equal n_contrib."""
    e = np.abs(gpu["image"][sel].astype(np.float64) - ref["image"][sel])
    t = np.abs(gpu["final_t"][sel].astype(np.float64) - ref["final_t"][sel])
    return (e <= IMG_TOL) & (t <= IMG_TOL) & (gpu["n_contrib"][sel] == ref["n_contrib"][sel]), e


def compare_forward(gpu, ref, check_keys=True, label="") -> Match:
    """The forward parity rule: keys, values and ranges bit-exact; on pixels
    with no flagged decision image and final T within IMG_TOL and n_contrib
    equal; a pixel with one flagged decision may match either branch; pixels
    with more are excluded (at most FLAG_FRAC of them).  Reports the flagged
    fractions."""
    if check_keys:
        assert gpu["keys"].shape == ref["pairs"]["keys"].shape, (gpu["keys"].shape,
                                                                 ref["pairs"]["keys"].shape)
        np.testing.assert_array_equal(gpu["keys"], ref["pairs"]["keys"])
        np.testing.assert_array_equal(gpu["values"], ref["pairs"]["values"])
        np.testing.assert_array_equal(gpu["ranges"], ref["pairs"]["ranges"])
    single, multi = ref["single"], ref["multi"]
    assert multi.mean() <= FLAG_FRAC, f"flagged (2+ decisions) fraction {multi.mean()}"
    zero = ~(single | multi)
    good, e0 = _agree(gpu, ref, zero)
    if not good.all():
        bad = np.nonzero(zero)[0][~good][:5]
        raise AssertionError(f"{label}: {int((~good).sum())} unflagged pixels differ, e.g. {bad}: "
                             f"gpu {gpu['image'][bad]} {gpu['n_contrib'][bad]} oracle "
                             f"{ref['image'][bad]} {ref['n_contrib'][bad]}; max err {e0.max()}")
    flip = np.zeros(single.shape, np.uint8)
    if single.any():
        m0, _ = _agree(gpu, ref, single)
        m1, _ = _agree(gpu, ref["alt"], single)
        assert (m0 | m1).all(), f"{label}: {int((~(m0 | m1)).sum())} single-flag pixels match neither branch"
        flip[np.nonzero(single)[0][~m0 & m1]] = 1
    note(f"{label} flagged pixels: {single.mean():.2e} one decision ({int(flip.sum())} on the other "
         f"branch), {multi.mean():.2e} two or more (excluded)")
    return Match(~multi, flip, float(e0.max(initial=0)), float(single.mean()), float(multi.mean()))


def compare_pixels(gpu_image, gpu_t, g, cam, st, pix, label=""):
    """Brute-force check of sampled pixels ``pix`` of one view (flat y*W+x)
    under the same rule (either branch of a single flagged decision)."""
    r = O.render_brute(g, cam, st, pix)
    nf = O.n_flags(r["flags"])
    single, multi = nf == 1, nf >= 2
    e = np.abs(gpu_image.astype(np.float64) - r["image"])
    t = np.abs(gpu_t.astype(np.float64) - r["final_t"])
    ok = (e <= IMG_TOL) & (t <= IMG_TOL)
    if single.any():
        a = O.render_brute(g, cam, st, pix, flip=single)
        ok |= single & (np.abs(gpu_image - a["image"]) <= IMG_TOL) & (np.abs(gpu_t - a["final_t"]) <= IMG_TOL)
    assert ok[~multi].all(), (label, e[~multi & ~ok], t[~multi & ~ok])
    return float(e[~multi].max(initial=0)), int(single.sum()), int(multi.sum())


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


def block_first(cams) -> np.ndarray:
    """For every pixel of the concatenated views, the index of the first
    pixel of its 8 x 8 block (blocks 8-aligned in each view)."""
    out, off = [], 0
    for c in cams:
        W, H = c.width, c.height
        y, x = np.mgrid[0:H, 0:W]
        out.append((off + (y // 8 * 8) * W + x // 8 * 8).ravel())
        off += W * H
    return np.concatenate(out)


def check_counts(counts, ref, g, m: Match, label=""):
    """The GPU's work counts (xg_render_counts rows) against the oracle.
    Row 0 (evaluations) and row 1 (contributors) per pixel on every pixel
    the forward rule compared, taking the branch the GPU took; row 3 (the
    backward's wavefront reductions: Gaussians contributing to a block) per
    8 x 8 block without a flagged pixel.  Rows 4-7 count how the kernels walk
    the lists; they are checked for consistency with rows 0-3."""
    ok = m.ok
    ev = ref["evals"].copy()
    if ref["alt"] is not None:
        f = m.flip.astype(bool)
        ev[f] = ref["alt"]["evals"][f]
    np.testing.assert_array_equal(counts[0][ok], ev[ok])
    pr = ref["pairs"]
    blocks = O.block_contributors(g, ref["cams"], ref["st"], pr["values"], pr["ranges"])
    first = block_first(ref["cams"])
    flagged = np.zeros(first.shape, bool)
    np.logical_or.at(flagged, first, ref["single"] | ref["multi"])
    heads = np.unique(first)
    clean = heads[~flagged[heads]]
    np.testing.assert_array_equal(counts[3][clean], blocks[clean])
    # structure: per block, reductions <= backward visits <= forward visits;
    # per pixel, contributors <= backward evaluations <= revisited evaluations
    # and forward evaluations <= evaluations of the definition
    assert np.all(counts[3][heads] <= counts[4][heads]) and np.all(counts[4][heads] <= counts[5][heads])
    assert np.all(counts[1] <= counts[7]) and np.all(counts[7] <= counts[2])
    assert np.all(counts[6] <= counts[0])
    nonhead = np.ones(first.shape, bool)
    nonhead[heads] = False
    assert np.all(counts[3:6][:, nonhead] == 0)
    note(f"{label} counts: evaluations {int(counts[0].sum())}, reductions {int(counts[3].sum())} "
         f"({int(clean.size)} of {int(heads.size)} blocks compared), backward visits "
         f"{int(counts[4].sum())}, forward visits {int(counts[5].sum())}")
