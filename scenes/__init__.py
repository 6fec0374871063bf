"""Seeded synthetic scenes for the radiative Gaussian splatting hot path.

This module only draws random inputs: Gaussian parameter arrays, scanner
angles and detector sizes, perturbations and upstream gradients.  It holds
none of the rendering arithmetic, so both the FP64 oracle and the GPU path
can take their inputs from here without sharing any of the method's code.

The paper's CT scenes (two public CT collections projected with a tomography
toolbox) are not available, so these seeded draws stand in for them.  The
geometry is a circular cone-beam scanner (Sec. 3.3, Eq. 12): the source
circles the origin at distance ``L_SO`` in the z = 0 plane and the flat
detector sits at ``L_SD`` from the source.

Distributions, per Gaussian, drawn in this order from
``numpy.random.default_rng(seed)`` in float64 and cast once to float32:

1. means       ~ U[-1, 1]^3 (the scanned cuboid)
2. log-scales  ~ N(log s0, sigma_s) per axis; scales = exp(log-scales)
3. quaternions ~ N(0, I_4), normalised (w, x, y, z; scalar first)
4. opacity     = logistic(N(0, 1))
5. intensity   ~ U[0, 1]  (the activated view-independent intensity, Eq. 3)

Workload 6 is the forward-only scan of the initialised model: centres on
the ACUI grid (Sec. 3.3, Eq. 13; the grid itself is the method's, computed
by the library or the oracle, so only its parameters live here) and the
other attributes drawn as in 2-5 ("randomly initialised").  Its 100 views
are evenly spaced over 0-180 degrees, like the paper's 100 projections per
scene.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Scanner geometry shared by every workload (source-object and
# source-detector distances, scene units).
L_SO = 4.0
L_SD = 6.0
# Physical detector side.  The detector must cover the projection of the
# cuboid [-1, 1]^3 from every source angle; its bounding sphere (radius
# sqrt(3)) seen from distance L_SO spans a half-angle with tangent
# sqrt(3) / sqrt(L_SO^2 - 3), which the detector at L_SD must contain.
DETECTOR_SIDE = 2.0 * L_SD * math.sqrt(3.0) / math.sqrt(L_SO * L_SO - 3.0)


@dataclass
class Workload:
    """One synthetic workload: Gaussian count, views and distributions."""

    number: int
    n: int
    sizes: list            # [(width, height)] per view
    angles: list           # source azimuth per view, radians
    log_scale_mean: float
    log_scale_std: float
    upstream: str          # "normal" | "l1_sum" | "l1_mean"
    adam: bool = False
    notes: str = ""
    seeds: dict = field(default_factory=dict)

    @property
    def n_views(self) -> int:
        return len(self.sizes)

    @property
    def n_pixels(self) -> int:
        return int(sum(w * h for w, h in self.sizes))

    def describe(self) -> str:
        uniq = sorted(set(self.sizes))
        sz = ",".join(f"{w}x{h}" for w, h in uniq)
        return (f"N={self.n} Gaussians, {self.n_views} view(s) of {sz}, "
                f"log-scale N(log {math.exp(self.log_scale_mean):.3g}, {self.log_scale_std})")


# ACUI grid of workload 6: cuboid side 2 (the scanned cube [-1, 1]^3),
# 256^3 voxels, sampling interval 8 voxels.
ACUI_SIZE = (2.0, 2.0, 2.0)
ACUI_GRID = (256, 256, 256)
ACUI_D = 8.0


def _seeds(c: int) -> dict:
    return {"scene": 1000 * c, "camera": 1000 * c + 1,
            "perturb": 1000 * c + 2, "upstream": 1000 * c + 3}


def workload(c: int) -> Workload:
    """The five synthetic workloads (1: tiny single view ... 5: training scale)."""
    s = _seeds(c)
    if c == 1:
        return Workload(1, 1000, [(64, 64)], [0.0], math.log(0.05), 0.3, "normal", seeds=s)
    if c == 2:
        rng = np.random.default_rng(s["camera"])
        return Workload(2, 50_000, [(256, 256)], [float(rng.uniform(0.0, 2 * math.pi))],
                        math.log(0.05), 0.3, "l1_sum", seeds=s)
    if c == 3:
        return Workload(3, 200_000, [(512, 512)] * 8,
                        [2.0 * math.pi * k / 8 for k in range(8)],
                        math.log(0.02), 0.3, "l1_mean", seeds=s)
    if c == 4:
        rng = np.random.default_rng(s["camera"])
        angles = rng.uniform(0.0, 2 * math.pi, size=32).tolist()
        side = rng.choice(np.array([128, 256, 512]), size=32).tolist()
        return Workload(4, 300_000, [(int(x), int(x)) for x in side], angles,
                        math.log(0.02), 0.3, "l1_mean", seeds=s)
    if c == 5:
        rng = np.random.default_rng(s["camera"])
        angles = rng.uniform(0.0, 2 * math.pi, size=16).tolist()
        return Workload(5, 1_000_000, [(512, 512)] * 16, angles,
                        math.log(0.01), 0.6, "l1_mean", adam=True, seeds=s)
    if c == 6:
        # n is the grid's point count, filled in by whoever builds the grid;
        # scales around half the grid spacing 2 * 8 / 256
        return Workload(6, 0, [(512, 512)] * 100, [math.pi * k / 100 for k in range(100)],
                        math.log(0.03125), 0.3, "none", seeds=s,
                        notes="ACUI grid (Eq. 13), forward only")
    raise ValueError(f"unknown workload {c}")


def gaussians(n: int, log_scale_mean: float, log_scale_std: float, seed: int) -> dict:
    """Draw ``n`` Gaussians; returns float32 C-contiguous SoA arrays."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    logit = rng.normal(0.0, 1.0, size=n)
    inten = rng.uniform(0.0, 1.0, size=n)
    return {
        "means": np.ascontiguousarray(means, dtype=np.float32),
        "scales": np.ascontiguousarray(np.exp(log_scales), dtype=np.float32),
        "quats": np.ascontiguousarray(quats, dtype=np.float32),
        "opacity": np.ascontiguousarray(1.0 / (1.0 + np.exp(-logit)), dtype=np.float32),
        "intensity": np.ascontiguousarray(inten, dtype=np.float32),
    }


def attributes(n: int, log_scale_mean: float, log_scale_std: float, seed: int) -> dict:
    """Scales, quaternions, opacity and intensity of ``n`` Gaussians whose
    centres come from elsewhere (the ACUI grid): draws 2-5 above, in order."""
    rng = np.random.default_rng(seed)
    log_scales = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    logit = rng.normal(0.0, 1.0, size=n)
    inten = rng.uniform(0.0, 1.0, size=n)
    return {
        "scales": np.ascontiguousarray(np.exp(log_scales), dtype=np.float32),
        "quats": np.ascontiguousarray(quats, dtype=np.float32),
        "opacity": np.ascontiguousarray(1.0 / (1.0 + np.exp(-logit)), dtype=np.float32),
        "intensity": np.ascontiguousarray(inten, dtype=np.float32),
    }


def sh_coefficients(n: int, degree: int, seed: int, std: float = 0.3) -> np.ndarray:
    """Spherical-harmonics colour coefficients of the comparison model,
    float32 [n, (degree + 1)^2, 3] ~ N(0, std^2)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.normal(0.0, std, size=(n, (degree + 1) ** 2, 3)), dtype=np.float32)


def perturb(g: dict, seed: int) -> dict:
    """A perturbed copy of a scene (the target scene for the L1 workloads)."""
    rng = np.random.default_rng(seed)
    n = g["means"].shape[0]
    means = g["means"].astype(np.float64) + rng.normal(0.0, 0.02, size=(n, 3))
    ls = np.log(g["scales"].astype(np.float64)) + rng.normal(0.0, 0.1, size=(n, 3))
    q = g["quats"].astype(np.float64) + rng.normal(0.0, 0.05, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    o = g["opacity"].astype(np.float64)
    logit = np.log(o / (1.0 - o)) + rng.normal(0.0, 0.25, size=n)
    inten = np.clip(g["intensity"].astype(np.float64) + rng.normal(0.0, 0.05, size=n), 0.0, 1.0)
    return {
        "means": np.ascontiguousarray(means, dtype=np.float32),
        "scales": np.ascontiguousarray(np.exp(ls), dtype=np.float32),
        "quats": np.ascontiguousarray(q, dtype=np.float32),
        "opacity": np.ascontiguousarray(1.0 / (1.0 + np.exp(-logit)), dtype=np.float32),
        "intensity": np.ascontiguousarray(inten, dtype=np.float32),
    }


def scene(c: int, n: int | None = None) -> dict:
    """Gaussians of workload ``c`` (optionally only the first ``n`` draws' worth)."""
    w = workload(c)
    return gaussians(w.n if n is None else n, w.log_scale_mean, w.log_scale_std, w.seeds["scene"])


def upstream_normal(n_pixels: int, seed: int) -> np.ndarray:
    """Per-pixel upstream gradient ~ N(0, 1), float32."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.normal(0.0, 1.0, size=n_pixels), dtype=np.float32)


def detector_side(width: int, height: int) -> tuple:
    """Physical detector extent (same for every pixel count)."""
    return DETECTOR_SIDE, DETECTOR_SIDE


def small_views(sizes, seed: int) -> tuple:
    """Random azimuths for a list of detector sizes (test helper)."""
    rng = np.random.default_rng(seed)
    return list(sizes), rng.uniform(0.0, 2 * math.pi, size=len(sizes)).tolist()
