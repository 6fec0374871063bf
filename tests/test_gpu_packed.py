"""Packed tile-sorted pairs at the boundary of the packing: 2^19 Gaussians
(19 index bits) over 8 views of 512 x 512 with 16 x 16 tiles (8192 tiles,
13 bits) fill the 32-bit word, the tile id reaching its top bit.  Keys,
values and tile ranges bit-exact against the oracle's sorted lists;
sampled pixels against the brute-force renderer."""
import math

import numpy as np
import pytest

import oracle as O
import scenes as S
from _gpu import compare_pixels, gpu_run, note, oracle_cams

pytestmark = pytest.mark.gpu


def test_packed_pairs_fill_the_word():
    n = 1 << 19
    w = S.workload(3)
    g = S.gaussians(n, math.log(0.006), 0.3, 19)
    note("packed pairs: 2^19 Gaussians x 8 views of 512^2")
    gpu = gpu_run(g, w.angles, w.sizes, backward=False)
    assert gpu["status"] == 0
    assert int(gpu["frame"].layout.pair_index_bits) == 19
    st = O.Settings(tile=16)
    cams = oracle_cams(w.angles, w.sizes)
    note("packed pairs: oracle pairs")
    pr = O.pairs(g, cams, st)
    assert pr["keys"].size > 1_000_000
    assert (pr["keys"] >> 32).max() >= 4096            # tile ids use all 13 bits
    np.testing.assert_array_equal(gpu["keys"], pr["keys"])
    np.testing.assert_array_equal(gpu["values"], pr["values"])
    np.testing.assert_array_equal(gpu["ranges"], pr["ranges"])
    rng = np.random.default_rng(5)
    off = 0
    for v, c in enumerate(cams[:3]):
        npx = c.width * c.height
        pix = rng.choice(npx, 32, replace=False).astype(np.int32)
        compare_pixels(gpu["image"][off + pix], gpu["final_t"][off + pix], g, c, st, pix,
                       label=f"packed view {v}")
        off += npx
