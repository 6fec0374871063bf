"""Randomised parity: random scenes (50-40 000 Gaussians, log-normal scales),
1-9 views of random size (8-300 pixels a side, one case in five up to 700,
so some views take the radix-sorted list path with 8 x 8 tiles), every tile
size and LDS batch, alpha_min in {0, 0.02, 1/255} and t_min in {0, 1e-4,
1e-2}: keys, values and ranges bit-exact, images under the forward rule,
gradients within the relative L2 bound, against the oracle.  Scenes with
alpha_min = 0 (every rectangle the whole detector) are kept small: with
thousands of contributors per pixel the float32 transmittance drifts past
the relative margin that flags a t_min decision.  The generator is seeded,
so every run draws the same cases."""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S
from _gpu import compare_forward, compare_grads, gpu_run, grad_upstream, note, oracle_run

pytestmark = pytest.mark.gpu


def _cases(k, seed):
    rng = np.random.default_rng(seed)
    for i in range(k):
        n = int(rng.integers(50, 40000))
        nv = int(rng.integers(1, 10))
        big = rng.random() < 0.2
        hi = 701 if big else 301
        sizes = [(int(rng.integers(8, hi)), int(rng.integers(8, hi))) for _ in range(nv)]
        amin = float(rng.choice([1.0 / 255.0, 0.02, 0.0]))
        tmin = float(rng.choice([1e-4, 1e-2, 0.0]))
        if amin == 0.0:
            n = min(n, 400)
            sizes = [(min(w, 64), min(h, 64)) for w, h in sizes]
        angles = rng.uniform(0, 2 * math.pi, nv).tolist()
        tile = int(rng.choice([8, 16, 32]))
        lds = int(rng.choice([64, 128, 256]))
        lm = float(rng.uniform(math.log(0.01), math.log(0.1)))
        ls = float(rng.uniform(0.2, 0.6))
        s = int(rng.integers(0, 1 << 30))
        yield i, n, sizes, angles, tile, lds, lm, ls, amin, tmin, s


@pytest.mark.parametrize("case", list(_cases(24, 777)), ids=lambda c: f"case{c[0]}")
def test_random_scene(case):
    i, n, sizes, angles, tile, lds, lm, ls, amin, tmin, seed = case
    label = (f"case {i}: n={n} views={sizes} tile={tile} lds={lds} alpha_min={amin:.4f} "
             f"t_min={tmin} seed={seed}")
    note(label)
    g = S.gaussians(n, lm, ls, seed)
    ref = oracle_run(g, angles, sizes, tile=tile, alpha_min=amin, t_min=tmin)
    up = np.random.default_rng(seed + 1).normal(size=sum(w * h for w, h in sizes)).astype(np.float32)
    upm = grad_upstream(up, ref)
    gpu = gpu_run(g, angles, sizes, tile=tile, lds=lds, upstream=upm, alpha_min=amin, t_min=tmin)
    assert gpu["status"] == 0
    m = compare_forward(gpu, ref, label=label)
    rg = O.backward(g, ref["cams"], ref["st"], upm, binned=(ref["pairs"]["values"], ref["pairs"]["ranges"]),
                    flip=m.flip)
    compare_grads(gpu["grads"], rg)


def _cases_pst(k, seed):
    rng = np.random.default_rng(seed)
    for i in range(k):
        n = int(rng.integers(50, 30000))
        nv = int(rng.integers(1, 8))
        sizes = [(int(rng.integers(8, 301)), int(rng.integers(8, 301))) for _ in range(nv)]
        angles = rng.uniform(0, 2 * math.pi, nv).tolist()
        tile = int(rng.choice([8, 16, 32]))
        lds = int(rng.choice([64, 128, 256]))
        lm = float(rng.uniform(math.log(0.01), math.log(0.1)))
        ls = float(rng.uniform(0.2, 0.6))
        mode = str(rng.choice(["persistent", "stored"]))
        slots = int(rng.choice([1, 5, 40, 4096]))
        s = int(rng.integers(0, 1 << 30))
        yield i, n, sizes, angles, tile, lds, lm, ls, mode, slots, s


@pytest.mark.parametrize("case", list(_cases_pst(12, 555)), ids=lambda c: f"case{c[0]}-{c[8]}")
def test_random_scene_persistent_or_stored(case):
    """The persistent tile queue (XG_F_PERSISTENT) and the stored-transmittance
    variant (random slot counts, from 1 to more than any pixel needs) on
    random scenes at the default thresholds."""
    import test_gpu_store as TS
    i, n, sizes, angles, tile, lds, lm, ls, mode, slots, seed = case
    note(f"case {i}: {mode} slots={slots} n={n} views={sizes} tile={tile} lds={lds} seed={seed}")
    g = S.gaussians(n, lm, ls, seed)
    if mode == "stored":
        TS._check(g, angles, sizes, slots, tile=tile, lds=lds, seed=seed)
        return
    ref = oracle_run(g, angles, sizes, tile=tile)
    up = np.random.default_rng(seed + 1).normal(size=sum(w * h for w, h in sizes)).astype(np.float32)
    upm = grad_upstream(up, ref)
    gpu = gpu_run(g, angles, sizes, tile=tile, lds=lds, upstream=upm, persistent=True)
    assert gpu["status"] == 0
    m = compare_forward(gpu, ref, label=f"case {i} persistent")
    rg = O.backward(g, ref["cams"], ref["st"], upm, binned=(ref["pairs"]["values"], ref["pairs"]["ranges"]),
                    flip=m.flip)
    compare_grads(gpu["grads"], rg)
