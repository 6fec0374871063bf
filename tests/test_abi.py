"""C ABI checks that need no GPU: the library loads, exports every entry
point declared in include/xg.h, and validates arguments on the host before
any HIP call.  Also: the host camera (Eq. 12) equals the oracle's bit for bit.
"""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import scenes as S

P = pytest.importorskip("paper_2403_04116_amd")
X = P._lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xg_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 11
    lib = C.CDLL(X.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(X.EXPORTED)


def test_abi_version_and_status_strings():
    assert P.xg_abi_version() == 4
    for st in (0, 1, 2, 3):
        assert X.status_string(st).startswith("XG_")


def test_struct_sizes_match_header():
    assert C.sizeof(X.XgCamera) == 80
    assert C.sizeof(X.XgSettings) == 32
    assert C.sizeof(X.XgFrame) == 80
    assert C.sizeof(X.XgAdam) == 56
    assert X.XgAdam.beta1.offset == 40
    assert C.sizeof(X.XgParams) == 56
    assert C.sizeof(X.XgGrads) == 40


def _adam_cfg(**kw):
    c = dict(lr_means_start=1.9e-4, lr_means_end=1.9e-6, lr_means_steps=20000, lr_scales=5e-3,
             lr_quats=1e-3, lr_opacity=8e-3, lr_feature=2e-3, eps=1e-15,
             reserved=0, beta1=0.9, beta2=0.999)
    c.update(kw)
    return X.XgAdam(**c)


@pytest.mark.parametrize("bad", [dict(beta2=1.0), dict(beta1=-0.1), dict(eps=-1.0),
                                 dict(lr_means_steps=0), dict(lr_means_end=0.0),
                                 dict(lr_quats=float("nan")), dict(reserved=1)])
def test_invalid_adam_settings_rejected_before_any_hip_call(bad):
    fake = 4096          # never dereferenced: validation fails first
    p = X.XgParams(fake, fake, fake, fake, fake, fake, 10, 16)
    g = X.XgGrads(fake, fake, fake, fake, fake)
    with pytest.raises(X.XgError) as e:
        X.xg_adam_step(p, g, fake, fake, fake, _adam_cfg(**bad), fake, fake, fake, 0, 0)
    assert e.value.status == X.XG_EINVAL


@pytest.mark.parametrize("phi", [0.0, 0.7, math.pi / 2, math.pi, 5.5, 2 * math.pi])
@pytest.mark.parametrize("wh", [(64, 64), (512, 512), (100, 37)])
def test_camera_matches_oracle_bitwise(phi, wh):
    w, h = wh
    c = P.xg_camera_from_scanner(phi, 4.0, 6.0, w, h, S.DETECTOR_SIDE, 0.9 * S.DETECTOR_SIDE)
    o = O.camera(phi, 4.0, 6.0, w, h, S.DETECTOR_SIDE, 0.9 * S.DETECTOR_SIDE)
    # the first 72 bytes share one layout (rotation, translation, intrinsics, size)
    assert bytes(c)[:72] == bytes(o)[:72]
    assert c.pixel_offset == 0 and c.tile_offset == 0


def test_layout_views():
    cams = (X.XgCamera * 3)(*[P.xg_camera_from_scanner(0.1 * k, 4, 6, w, h, 5, 5)
                             for k, (w, h) in enumerate([(64, 64), (37, 20), (128, 96)])])
    px, tl = P.xg_layout_views(cams, 16)
    assert px == 64 * 64 + 37 * 20 + 128 * 96
    assert tl == 16 + 3 * 2 + 8 * 6
    assert [c.pixel_offset for c in cams] == [0, 4096, 4096 + 740]
    assert [c.tile_offset for c in cams] == [0, 16, 22]
    px8, tl8 = P.xg_layout_views(cams, 8)
    assert tl8 == 64 + 5 * 3 + 16 * 12


def _frame(n=100, views=((64, 64),), tile=16, cap=1 << 16, **kw):
    cams = (X.XgCamera * len(views))(*[P.xg_camera_from_scanner(0.3, 4, 6, w, h, 5, 5)
                                       for w, h in views])
    P.xg_layout_views(cams, tile if tile in (8, 16, 32) else 16)
    st = P.settings(tile=16)
    st.tile = tile
    for k, v in kw.items():
        setattr(st, k, v)
    return X.XgFrame(n, len(views), cams, 0, st, 0, 0, cap), cams


def test_workspace_size_grows_with_capacity_and_views():
    f1, _ = _frame(cap=1000)
    f2, _ = _frame(cap=100000)
    f3, _ = _frame(cap=1000, views=((64, 64), (64, 64)))
    s1, s2, s3 = (P.xg_workspace_size(f) for f in (f1, f2, f3))
    # two buffers of 4 bytes per pair (packed tile | index), or 2 x 8 when unpacked
    per_pair = 8 if P.xg_ws_layout_of(f1).pair_index_bits else 16
    assert s2 > s1 + per_pair * (100000 - 1000) - 1
    assert s3 > s1
    lay = P.xg_ws_layout_of(f1)
    assert lay.total == s1
    offs = [lay.records, lay.counts, lay.offsets, min(lay.pair_tiles, lay.pair_values),
            lay.ranges, lay.grad2d]
    assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)


@pytest.mark.parametrize("field,value", [
    ("tile", 12), ("lds_batch", 100), ("lowpass", -1.0), ("alpha_min", 1.0),
    ("alpha_max", 0.0), ("alpha_max", 1.0), ("t_min", 1.0), ("near_z", float("nan")),
    ("flags", 8)])
def test_invalid_settings_rejected(field, value):
    f, _ = _frame(**{field: value})
    with pytest.raises(X.XgError) as e:
        P.xg_workspace_size(f)
    assert e.value.status == X.XG_EINVAL


def test_invalid_frames_rejected_before_any_hip_call():
    g = X.XgGaussians(0, 0, 0, 0, 0, 100)
    f, cams = _frame()
    # no device workspace / cameras: EINVAL
    with pytest.raises(X.XgError):
        P.xg_preprocess(f, g)
    # inconsistent offsets
    f2, cams2 = _frame(views=((64, 64), (32, 32)))
    cams2[1].tile_offset = 3
    with pytest.raises(X.XgError):
        P.xg_workspace_size(f2)
    # capacity out of range
    for cap in (0, -5, 1 << 31):
        f3, _ = _frame(cap=cap)
        with pytest.raises(X.XgError):
            P.xg_workspace_size(f3)
    # bad detector sizes
    with pytest.raises(X.XgError):
        P.xg_camera_from_scanner(0.0, 4, 6, 0, 10, 5, 5)
    with pytest.raises(X.XgError):
        P.xg_camera_from_scanner(0.0, -4, 6, 10, 10, 5, 5)
    # misaligned workspace pointer and too-small workspace
    f4, _ = _frame()
    need = P.xg_workspace_size(f4)
    f4.cams_dev = 256
    f4.ws = 256 + 8
    f4.ws_bytes = need
    with pytest.raises(X.XgError):
        P.xg_bin_sort(f4)
    f4.ws = 512
    f4.ws_bytes = need - 1
    with pytest.raises(X.XgError):
        P.xg_bin_sort(f4)
    # Gaussian count mismatch and null parameter pointers
    f4.ws_bytes = need
    with pytest.raises(X.XgError):
        P.xg_preprocess(f4, X.XgGaussians(0, 0, 0, 0, 0, 99))
    with pytest.raises(X.XgError):
        P.xg_preprocess(f4, X.XgGaussians(0, 0, 0, 0, 0, 100))
    with pytest.raises(X.XgError):
        P.xg_l1_grad(0, 0, 0, 10, 1.0)
    # loss gradient: null images and gamma outside [0, 1] fail before any HIP call
    with pytest.raises(X.XgError) as e:
        X.xg_loss_grad(f4, 0, 4096, 0.2, 8192)
    assert e.value.status == X.XG_EINVAL
    for gamma in (-0.1, 1.5, float("nan")):
        with pytest.raises(X.XgError) as e:
            X.xg_loss_grad(f4, 4096, 4096, gamma, 8192)
        assert e.value.status == X.XG_EINVAL
    # the allocation-free form: no workspace needed, but device cameras and
    # images are; maps beyond the static array are refused before any HIP call
    f5, _ = _frame()
    with pytest.raises(X.XgError) as e:
        X.xg_loss_grad_static(f5, 4096, 4096, 0.2, 8192)
    assert e.value.status == X.XG_EINVAL
    f5.cams_dev = 256
    for args in ((0, 4096, 0.2, 8192), (4096, 4096, 1.5, 8192), (4096, 4096, 0.2, 0)):
        with pytest.raises(X.XgError) as e:
            X.xg_loss_grad_static(f5, *args)
        assert e.value.status == X.XG_EINVAL
    big, _ = _frame(views=((2048, 2048),))
    big.cams_dev = 256
    with pytest.raises(X.XgError) as e:
        X.xg_loss_grad_static(big, 4096, 4096, 0.2, 8192)
    assert e.value.status == X.XG_ECAPACITY
    assert 12 * 2048 * 2048 > X.STATIC_SCRATCH_BYTES >= 12 * 8 * 512 * 512 + 4 * 8 * 11 * 64


def test_package_fails_loudly_without_library(tmp_path):
    """The binding raises ImportError when libxg.so is absent (no CPU fallback)."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2403_04116_amd"
    shutil.copytree(os.path.join(ROOT, "paper_2403_04116_amd"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__"))
    r = subprocess.run([sys.executable, "-c", "import paper_2403_04116_amd"], cwd=tmp_path,
                       capture_output=True, text=True)
    assert r.returncode != 0 and "not built" in r.stderr


def test_store_size_and_validation():
    f, _ = _frame(views=((64, 64), (40, 24)))
    px_tiles = (16 + 3 * 2) * 256
    s8 = X.xg_store_size(f, 8)
    s9 = X.xg_store_size(f, 9)
    assert s9 - s8 == px_tiles * 4
    assert s8 >= px_tiles * 4 * 9 and s8 % 256 == 0
    for bad in (0, -1, X.MAX_STORE_SLOTS + 1):
        with pytest.raises(X.XgError) as e:
            X.xg_store_size(f, bad)
        assert e.value.status == X.XG_EINVAL
    # a frame with (fake) device pointers: the store checks fail before any HIP call
    need = P.xg_workspace_size(f)
    f.cams_dev = 256
    f.ws = 256
    f.ws_bytes = need
    g = X.XgGaussians(256, 256, 256, 256, 256, 100)
    for store, slots, nbytes in ((0, 8, s8), (256 + 4, 8, s8), (256, 8, s8 - 256), (256, 0, s8)):
        with pytest.raises(X.XgError) as e:
            X.xg_render_fwd_store(f, g, 256, 256, 256, store, slots, nbytes, 0)
        assert e.value.status == X.XG_EINVAL
        with pytest.raises(X.XgError) as e:
            X.xg_render_bwd_store_2d(f, 256, 256, 256, store, slots, nbytes, 0)
        assert e.value.status == X.XG_EINVAL
        with pytest.raises(X.XgError) as e:
            X.xg_render_bwd_store(f, g, 256, 256, 256, store, slots, nbytes,
                                  X.XgGrads(256, 256, 256, 256, 256), 0)
        assert e.value.status == X.XG_EINVAL
    f.settings.flags = 1           # the persistent queue has no stored variant
    with pytest.raises(X.XgError) as e:
        X.xg_render_fwd_store(f, g, 256, 256, 256, 256, 8, s8, 0)
    assert e.value.status == X.XG_EINVAL


def test_invalid_feature_counts_rejected_before_any_hip_call():
    fake = 4096
    for nf in (0, -3, X.MAX_FEATURES + 1):
        with pytest.raises(X.XgError) as e:
            X.xg_rirf_fwd(fake, fake, 10, nf, fake, 0)
        assert e.value.status == X.XG_EINVAL
        with pytest.raises(X.XgError) as e:
            X.xg_rirf_bwd(fake, fake, 10, nf, fake, fake, 0)
        assert e.value.status == X.XG_EINVAL
        p = X.XgParams(fake, fake, fake, fake, fake, fake, 10, nf)
        g = X.XgGrads(fake, fake, fake, fake, fake)
        with pytest.raises(X.XgError) as e:
            X.xg_adam_step(p, g, fake, fake, fake, _adam_cfg(), fake, fake, fake, 0, 0)
        assert e.value.status == X.XG_EINVAL
    with pytest.raises(X.XgError):
        X.xg_rirf_fwd(0, fake, 10, 16, fake, 0)          # null features


@pytest.mark.parametrize("size,grid,d", [((2, 2, 2), (256, 256, 256), 8.0),
                                         ((3.0, 1.5, 0.75), (100, 60, 30), 3.5),
                                         ((1, 1, 1), (4, 4, 4), 3.0),
                                         ((2.0, 1.0, 0.5), (7, 9, 11), 1.0)])
def test_acui_count_matches_oracle(size, grid, d):
    from oracle import acui
    assert X.xg_acui_count(size, grid, d) == acui.count(size, grid, d)


def test_acui_validation():
    """Bad ACUI parameters fail on the host, before any HIP call."""
    good = ((2, 2, 2), (256, 256, 256), 8.0)
    bad = [((0, 2, 2), (256, 256, 256), 8.0), ((2, float("inf"), 2), (256, 256, 256), 8.0),
           ((2, 2, 2), (256, 0, 256), 8.0), ((2, 2, 2), (256, 256, 256), 0.0),
           ((2, 2, 2), (256, 256, 256), float("nan")), ((2, 2, 2), (4096, 4096, 4096), 1.0)]
    for size, grid, d in bad:
        with pytest.raises(X.XgError) as e:
            X.xg_acui_count(size, grid, d)
        assert e.value.status == X.XG_EINVAL
    n = X.xg_acui_count(*good)
    for ptr, cap in ((0, n), (4096, n - 1)):
        with pytest.raises(X.XgError) as e:
            X.xg_acui_grid(*good, ptr, cap)
        assert e.value.status == X.XG_EINVAL


def test_rgb_validation():
    """The comparison model's entry points reject a null coefficient array, a
    degree outside 0..3 and the persistent flag before any HIP call."""
    f, _ = _frame()
    need = P.xg_workspace_size(f)
    f.cams_dev = 256
    f.ws = 512
    f.ws_bytes = need
    g = X.XgGaussians(4096, 4096, 4096, 4096, 4096, 100)
    for sh, deg in ((0, 3), (4096, -1), (4096, 4)):
        with pytest.raises(X.XgError) as e:
            X.xg_preprocess_rgb(f, g, sh, deg)
        assert e.value.status == X.XG_EINVAL
    fp, _ = _frame(flags=X.XG_F_PERSISTENT)
    fp.cams_dev, fp.ws, fp.ws_bytes = 256, 512, P.xg_workspace_size(fp)
    with pytest.raises(X.XgError) as e:
        X.xg_render_fwd_rgb(fp, g, 4096, 4096, 4096)
    assert e.value.status == X.XG_EINVAL


def test_pair_packing_decision():
    """Tile id and Gaussian index share one word exactly when they fit 32 bits."""
    small, _ = _frame(n=100, views=((64, 64),))                 # 16 tiles, 7 index bits
    lay = P.xg_ws_layout_of(small)
    assert lay.pair_index_bits == 7 and lay.pair_values == lay.pair_tiles
    big, _ = _frame(n=1 << 20, views=((4096, 4096),) * 16)     # 2^20 tiles + 20 index bits
    lay = P.xg_ws_layout_of(big)
    assert lay.pair_index_bits == 0 and lay.pair_values != lay.pair_tiles
    one, _ = _frame(n=1, views=((64, 64),))
    assert P.xg_ws_layout_of(one).pair_index_bits == 1


def test_render_bwd_validation():
    """The one-call backward (2-D stage + projection adjoint) checks all its
    arguments before enqueueing either stage."""
    f, _ = _frame()
    need = P.xg_workspace_size(f)
    f.cams_dev, f.ws, f.ws_bytes = 256, 512, need
    g = X.XgGaussians(4096, 4096, 4096, 4096, 4096, 100)
    gr = X.XgGrads(4096, 4096, 4096, 4096, 4096)
    bad = [(g, 0, 4096, 4096, gr), (g, 4096, 0, 4096, gr), (g, 4096, 4096, 0, gr),
           (g, 4096, 4096, 4096, X.XgGrads(4096, 0, 4096, 4096, 4096)),
           (X.XgGaussians(4096, 4096, 4096, 4096, 4096, 99), 4096, 4096, 4096, gr)]
    for gg, dl, ft, nc, grads in bad:
        with pytest.raises(X.XgError) as e:
            X.xg_render_bwd(f, gg, dl, ft, nc, grads)
        assert e.value.status == X.XG_EINVAL


def test_ws_inspect_matches_layout():
    """xg_ws_inspect returns the workspace addresses the layout describes
    (host arithmetic only: the workspace pointer is never dereferenced)."""
    f, _ = _frame(views=((64, 64), (40, 24)))
    lay = P.xg_ws_layout_of(f)
    base = 1 << 20
    f.cams_dev, f.ws, f.ws_bytes = 256, base, lay.total
    v = X.xg_ws_inspect(f)
    assert v.status == base + lay.status and v.n_pairs == base + lay.n_pairs
    assert v.pair_tiles == base + lay.pair_tiles and v.pair_values == base + lay.pair_values
    assert v.ranges == base + lay.ranges and v.records == base + lay.records
    assert v.grad2d == base + lay.grad2d and v.pair_index_bits == lay.pair_index_bits
    assert v.total_tiles == 16 + 3 * 2 and v.total_pixels == 64 * 64 + 40 * 24
    # the blend launches' tile order: int32 per tile, inside the workspace,
    # clear of the public sub-buffers
    assert base <= v.tile_order and v.tile_order + 4 * v.total_tiles <= base + lay.total
    for off in (lay.status, lay.records, lay.counts, lay.offsets, lay.pair_tiles, lay.pair_values,
                lay.ranges, lay.grad2d):
        assert v.tile_order != base + off
    f.ws = 0
    with pytest.raises(X.XgError):
        X.xg_ws_inspect(f)
    for keys, vals, cap in ((0, 4096, 10), (4096, 0, 10), (4096, 4096, -1)):
        f.ws = base
        with pytest.raises(X.XgError) as e:
            X.xg_pair_keys(f, keys, vals, cap)
        assert e.value.status == X.XG_EINVAL

