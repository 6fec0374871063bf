"""Autotuner for the rendering settings that do not change results.

Tile size and LDS batch only change how the same per-pixel sequence of
Gaussians is scheduled: images are bitwise identical across all of them
(pixel offsets are taken from the enclosing 32 x 32 block, whatever the
tile), so the tuner may pick freely.  It times the complete fwd+bwd step
(TrainStep) for every candidate on the caller's scene and views and caches
the fastest per workload signature in a JSON file
(``$XG_AUTOTUNE_CACHE``, default ``~/.cache/xgauss_autotune.json``).
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import _lib as X
from .drr import Frame, settings
from .step import TrainStep

TILES = (8, 16, 32)
BATCHES = (64, 128, 256)


def _cache_path() -> str:
    return os.environ.get("XG_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "xgauss_autotune.json"))


def signature(n: int, cams, base: X.XgSettings) -> str:
    """Workload signature: Gaussian count (log2 bucket), view-size histogram,
    and the result-affecting constants."""
    sizes = {}
    for c in cams:
        k = f"{c.width}x{c.height}"
        sizes[k] = sizes.get(k, 0) + 1
    sz = ",".join(f"{k}:{sizes[k]}" for k in sorted(sizes))
    return (f"n~2^{int(round(math.log2(max(n, 1))))}|views[{sz}]|lp{base.lowpass:g}"
            f"|am{base.alpha_min:g}|aM{base.alpha_max:g}|tm{base.t_min:g}")


def autotune(g: dict, cams, target: torch.Tensor, scale: float, base: X.XgSettings | None = None,
             tiles=TILES, batches=BATCHES, steps: int = 5, warmup: int = 2, use_cache: bool = True,
             device="cuda") -> dict:
    """Returns {"settings": best XgSettings, "ms": {(tile, batch): ms}, "cached": bool}."""
    base = base if base is not None else settings()
    n = g["means"].shape[0]
    sig = signature(n, cams, base)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and sig in cache:
        t, b = cache[sig]["tile"], cache[sig]["lds_batch"]
        return {"settings": settings(tile=t, lds_batch=b, lowpass=base.lowpass,
                                     alpha_min=base.alpha_min, alpha_max=base.alpha_max,
                                     t_min=base.t_min, near_z=base.near_z),
                "ms": {tuple(map(int, k.split("x"))): v for k, v in cache[sig]["ms"].items()},
                "cached": True}
    times = {}
    capacity = None
    stream = torch.cuda.current_stream()
    for t in tiles:
        for b in batches:
            st = settings(tile=t, lds_batch=b, lowpass=base.lowpass, alpha_min=base.alpha_min,
                          alpha_max=base.alpha_max, t_min=base.t_min, near_z=base.near_z)
            frame = Frame(n, cams, st, pair_capacity=capacity, device=device)
            frame.fit_capacity(g)
            step = TrainStep(frame, g, target, scale)
            for _ in range(warmup):
                step.run()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                step.run()
            e1.record(stream)
            torch.cuda.synchronize()
            if not step.check():
                raise RuntimeError("pair capacity exceeded while tuning")
            times[(t, b)] = e0.elapsed_time(e1) / steps
            del step, frame
    best = min(times, key=times.get)
    if use_cache:
        cache[sig] = {"tile": best[0], "lds_batch": best[1],
                      "ms": {f"{k[0]}x{k[1]}": v for k, v in times.items()},
                      "when": time.strftime("%Y-%m-%d %H:%M:%S")}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, path)
    t, b = best
    return {"settings": settings(tile=t, lds_batch=b, lowpass=base.lowpass, alpha_min=base.alpha_min,
                                 alpha_max=base.alpha_max, t_min=base.t_min, near_z=base.near_z),
            "ms": times, "cached": False}
