"""ACUI initialisation (Eq. 13) on the GPU and the forward scan of the
initialised model: the point grid bit-exact against the oracle, then a
reduced scan (ragged views, keys bit-exact, images to 1e-5) and the full
100-view 512 x 512 scan of the benchmark (all keys bit-exact, sampled
pixels against the brute-force oracle)."""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S
from oracle import acui
from _gpu import compare_forward, compare_pixels, gpu_run, note, oracle_cams, oracle_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("size,grid,d", [((2, 2, 2), (256, 256, 256), 8.0),
                                         ((3.0, 1.5, 0.75), (100, 60, 30), 3.5),
                                         ((1, 1, 1), (4, 4, 4), 3.0),
                                         ((2.0, 1.0, 0.5), (7, 9, 11), 1.0),
                                         ((0.3, 7.0, 2.2), (33, 1, 64), 0.7)])
def test_acui_grid_bit_exact(size, grid, d):
    import torch
    import paper_2403_04116_amd as P
    note(f"acui grid {size} {grid} {d}")
    m = P.acui_means(size, grid, d)
    torch.cuda.synchronize()
    ref = acui.points(size, grid, d)
    got = m.cpu().numpy()
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


def _scene(size, grid, d, seed, gpu: bool):
    """ACUI centres (GPU kernel or oracle) + seeded attributes."""
    w = S.workload(6)
    if gpu:
        import paper_2403_04116_amd as P
        means = P.acui_means(size, grid, d).cpu().numpy()
    else:
        means = acui.points(size, grid, d)
    g = S.attributes(len(means), w.log_scale_mean, w.log_scale_std, seed)
    g["means"] = means
    return g


def test_acui_reduced_scan_forward():
    size, grid, d = S.ACUI_SIZE, (64, 64, 64), 8.0
    sizes = [(96, 80), (64, 64), (130, 70), (48, 112)] * 3
    angles = [math.pi * k / len(sizes) for k in range(len(sizes))]
    note("acui reduced scan: 12 views, 11^3 grid")
    g_gpu = _scene(size, grid, d, 61, gpu=True)
    g_ref = _scene(size, grid, d, 61, gpu=False)
    np.testing.assert_array_equal(g_gpu["means"], g_ref["means"])
    gpu = gpu_run(g_gpu, angles, sizes, backward=False)
    ref = oracle_run(g_ref, angles, sizes)
    assert gpu["status"] == 0
    compare_forward(gpu, ref, label="acui reduced scan")


def test_acui_full_scan_keys_and_sampled_pixels():
    w = S.workload(6)
    note("acui full scan: 100 views of 512x512, 35^3 grid")
    g_gpu = _scene(S.ACUI_SIZE, S.ACUI_GRID, S.ACUI_D, w.seeds["scene"], gpu=True)
    g_ref = _scene(S.ACUI_SIZE, S.ACUI_GRID, S.ACUI_D, w.seeds["scene"], gpu=False)
    np.testing.assert_array_equal(g_gpu["means"], g_ref["means"])
    gpu = gpu_run(g_gpu, w.angles, w.sizes, backward=False)
    assert gpu["status"] == 0
    st = O.Settings(tile=16)
    cams = oracle_cams(w.angles, w.sizes)
    note("acui full scan: oracle pairs")
    pr = O.pairs(g_ref, cams, st)
    np.testing.assert_array_equal(gpu["keys"], pr["keys"])
    np.testing.assert_array_equal(gpu["values"], pr["values"])
    np.testing.assert_array_equal(gpu["ranges"], pr["ranges"])
    note(f"acui full scan: {len(pr['keys'])} pairs bit-exact; brute-force sampled pixels")
    rng = np.random.default_rng(23)
    off = 0
    for v, c in enumerate(cams):
        npx = c.width * c.height
        # 8 anywhere, 8 in the central quarter (inside the object's projection)
        cx, cy = c.width // 4 + rng.integers(0, c.width // 2, 8), c.height // 4 + rng.integers(0, c.height // 2, 8)
        pix = np.concatenate([rng.choice(npx, 8, replace=False), cy * c.width + cx]).astype(np.int32)
        compare_pixels(gpu["image"][off + pix], gpu["final_t"][off + pix], g_ref, c, st, pix,
                       label=f"acui view {v}")
        off += npx
