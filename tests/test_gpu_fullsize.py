"""Parity at full size: 200 000 Gaussians, 8 views of 512 x 512 at evenly
spaced angles, tile 16, LDS batch 256 (the benchmarked configuration).

The oracle emits and sorts every pair (bit-exact comparison of all ~8M
keys), renders every pixel over its own sorted lists (pinned equal to brute
force on small scenes), spot-checks sampled pixels by brute force, checks
the GPU's per-pixel evaluation counts and per-block reduction counts (the
denominators of the reported throughput), and computes the adjoint of all
Gaussians for an L1 upstream gradient whose target image is rendered by
the oracle from a perturbed scene.
"""
import numpy as np
import pytest

import oracle as O
import scenes as S
from _gpu import (check_counts, compare_forward, compare_grads, compare_pixels, gpu_run,
                  grad_upstream, note, oracle_run)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def workload3():
    w = S.workload(3)
    g = S.scene(3)
    note("workload3: oracle pairs + render (full size)")
    ref = oracle_run(g, w.angles, w.sizes)
    tgt = S.perturb(g, w.seeds["perturb"])
    note("workload3: oracle target render")
    reft = oracle_run(tgt, w.angles, w.sizes)
    up = (np.sign(ref["image"] - reft["image"]) / w.n_pixels).astype(np.float32)
    upm = grad_upstream(up, ref)
    note("workload3: gpu forward + backward")
    gpu = gpu_run(g, w.angles, w.sizes, tile=16, lds=256, upstream=upm)
    m = compare_forward(gpu, ref, label="workload3")
    return w, g, ref, gpu, upm, m


def test_workload3_keys_and_images(workload3):
    w, g, ref, gpu, _, m = workload3
    assert gpu["status"] == 0
    note(f"workload3: {ref['pairs']['n_pairs']} pairs bit-exact, image max err {m.err:.2e}, "
         f"flagged: one decision {m.frac_single:.2e}, two or more {m.frac_multi:.2e}")


def test_workload3_work_counts(workload3):
    """Evaluation counts per pixel equal the oracle's (the evals/s
    denominator), and per-block reduction counts too."""
    w, g, ref, gpu, _, m = workload3
    counts = gpu["frame"].render_counts().cpu().numpy()
    check_counts(counts, ref, g, m, label="workload3")


def test_workload3_sampled_pixels_brute_force(workload3):
    w, g, ref, gpu, _, _ = workload3
    rng = np.random.default_rng(17)
    off = 0
    for v, c in enumerate(ref["cams"]):
        npx = c.width * c.height
        pix = rng.choice(npx, 64, replace=False).astype(np.int32)
        compare_pixels(gpu["image"][off + pix], gpu["final_t"][off + pix], g, c, ref["st"], pix,
                       label=f"view {v}")
        off += npx


def test_workload3_gradients(workload3):
    w, g, ref, gpu, upm, m = workload3
    note("workload3: oracle adjoint")
    rg = O.backward(g, ref["cams"], ref["st"], upm, binned=(ref["pairs"]["values"],
                                                            ref["pairs"]["ranges"]), flip=m.flip)
    errs = compare_grads(gpu["grads"], rg)
    note(f"workload3: grad rel L2 {errs}")
