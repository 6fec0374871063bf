"""ctypes binding of libxg (include/xg.h): argument marshalling only.

Every function here has the name of the C entry point it calls and raises
XgError on a non-XG_OK status.  Device pointers are passed as integers
(e.g. ``tensor.data_ptr()``); ``stream`` is a hipStream_t as an integer
(``torch.cuda.current_stream().cuda_stream``) or 0.  There is no fallback:
if libxg.so is missing the import of this module fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

# torch ships its own HIP runtime (libamdhip64.so, SONAME libamdhip64.so.7).
# Loading it before libxg.so makes libxg's libamdhip64.so.7 dependency bind
# to that same copy; loading libxg first would bring in a second HIP/HSA
# runtime that does not know torch's device pointers and streams.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxg.so")

XG_OK, XG_EINVAL, XG_ECAPACITY, XG_EHIP = 0, 1, 2, 3
XG_F_PERSISTENT = 1
ABI_VERSION = 4
COUNT_ROWS = 8
MAX_FEATURES = 64


class XgError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = f"{where}: {status_string(status)}"
        if status == XG_EHIP:
            msg += f" ({_L.xg_last_error().decode()})"
        super().__init__(msg)
        self.status = status


class XgCamera(C.Structure):
    _fields_ = [("rot", C.c_float * 9), ("trans", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32),
                ("pixel_offset", C.c_int32), ("tile_offset", C.c_int32)]


class XgSettings(C.Structure):
    _fields_ = [("tile", C.c_int32), ("lds_batch", C.c_int32), ("lowpass", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("near_z", C.c_float), ("flags", C.c_uint32)]


class XgGaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("intensity", C.c_void_p), ("n", C.c_int32)]


class XgGrads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("intensity", C.c_void_p)]


class XgParams(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("features", C.c_void_p), ("weights", C.c_void_p),
                ("n", C.c_int32), ("n_features", C.c_int32)]


class XgAdam(C.Structure):
    _fields_ = [("lr_means_start", C.c_float), ("lr_means_end", C.c_float),
                ("lr_means_steps", C.c_int32), ("lr_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_opacity", C.c_float), ("lr_feature", C.c_float), ("eps", C.c_float),
                ("reserved", C.c_int32), ("beta1", C.c_double), ("beta2", C.c_double)]


class XgFrame(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_views", C.c_int32), ("cams", C.POINTER(XgCamera)),
                ("cams_dev", C.c_void_p), ("settings", XgSettings), ("ws", C.c_void_p),
                ("ws_bytes", C.c_size_t), ("pair_capacity", C.c_int64)]


class XgWsLayout(C.Structure):
    _fields_ = [(k, C.c_size_t) for k in (
        "status", "n_pairs", "depth_range", "records", "counts", "offsets", "pair_tiles",
        "pair_values", "ranges", "grad2d", "total", "pair_index_bits")]


class XgWsView(C.Structure):
    _fields_ = [("status", C.c_void_p), ("n_pairs", C.c_void_p), ("pair_tiles", C.c_void_p),
                ("pair_values", C.c_void_p), ("ranges", C.c_void_p), ("records", C.c_void_p),
                ("grad2d", C.c_void_p), ("pair_index_bits", C.c_int32), ("total_tiles", C.c_int64),
                ("total_pixels", C.c_int64), ("tile_order", C.c_void_p)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(the DRR path has no CPU fallback)")

_L = C.CDLL(LIB_PATH)
_P = C.c_void_p
_S = C.c_int

_L.xg_abi_version.restype = C.c_int32
_L.xg_status_string.restype = C.c_char_p
_L.xg_status_string.argtypes = [_S]
_L.xg_default_settings.restype = XgSettings
_L.xg_camera_from_scanner.restype = _S
_L.xg_camera_from_scanner.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                      C.c_double, C.c_double, C.POINTER(XgCamera)]
_L.xg_layout_views.restype = _S
_L.xg_layout_views.argtypes = [C.POINTER(XgCamera), C.c_int32, C.c_int32,
                               C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
_L.xg_ws_layout_of.restype = _S
_L.xg_ws_layout_of.argtypes = [C.POINTER(XgFrame), C.POINTER(XgWsLayout)]
_L.xg_workspace_size.restype = _S
_L.xg_workspace_size.argtypes = [C.POINTER(XgFrame), C.POINTER(C.c_size_t)]
_L.xg_preprocess.restype = _S
_L.xg_preprocess.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), _P]
_L.xg_bin_sort.restype = _S
_L.xg_bin_sort.argtypes = [C.POINTER(XgFrame), _P]
_L.xg_render_fwd.restype = _S
_L.xg_render_fwd.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), _P, _P, _P, _P]
_L.xg_render_bwd.restype = _S
_L.xg_render_bwd.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), _P, _P, _P,
                             C.POINTER(XgGrads), _P]
_L.xg_render_bwd_2d.restype = _S
_L.xg_render_bwd_2d.argtypes = [C.POINTER(XgFrame), _P, _P, _P, _P]
_L.xg_ws_inspect.restype = _S
_L.xg_ws_inspect.argtypes = [C.POINTER(XgFrame), C.POINTER(XgWsView)]
_L.xg_pair_keys.restype = _S
_L.xg_pair_keys.argtypes = [C.POINTER(XgFrame), _P, _P, C.c_int64, _P]
_L.xg_preprocess_bwd.restype = _S
_L.xg_preprocess_bwd.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), C.POINTER(XgGrads), _P]
_L.xg_render_counts.restype = _S
_L.xg_render_counts.argtypes = [C.POINTER(XgFrame), _P, _P]
_L.xg_last_error.restype = C.c_char_p
_L.xg_adam_step.restype = _S
_L.xg_adam_step.argtypes = [C.POINTER(XgParams), C.POINTER(XgGrads), _P, _P, _P, C.POINTER(XgAdam),
                            _P, _P, _P, _P, _P]
_L.xg_store_size.restype = _S
_L.xg_store_size.argtypes = [C.POINTER(XgFrame), C.c_int32, C.POINTER(C.c_int64)]
_L.xg_render_fwd_store.restype = _S
_L.xg_render_fwd_store.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), _P, _P, _P, _P,
                                   C.c_int32, C.c_int64, _P]
_L.xg_render_bwd_store.restype = _S
_L.xg_render_bwd_store.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), _P, _P, _P, _P,
                                   C.c_int32, C.c_int64, C.POINTER(XgGrads), _P]
_L.xg_render_bwd_store_2d.restype = _S
_L.xg_render_bwd_store_2d.argtypes = [C.POINTER(XgFrame), _P, _P, _P, _P, C.c_int32, C.c_int64, _P]
_L.xg_rirf_fwd.restype = _S
_L.xg_rirf_fwd.argtypes = [_P, _P, C.c_int32, C.c_int32, _P, _P]
_L.xg_rirf_bwd.restype = _S
_L.xg_rirf_bwd.argtypes = [_P, _P, C.c_int32, C.c_int32, _P, _P, _P]
_L.xg_render_fwd_l1.restype = _S
_L.xg_render_fwd_l1.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), _P, _P, _P, _P, C.c_float,
                                _P, _P]
_L.xg_preprocess_bwd_write.restype = _S
_L.xg_preprocess_bwd_write.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), C.POINTER(XgGrads),
                                       _P]
_L.xg_preprocess_rgb.restype = _S
_L.xg_preprocess_rgb.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), _P, C.c_int32, _P]
_L.xg_render_fwd_rgb.restype = _S
_L.xg_render_fwd_rgb.argtypes = [C.POINTER(XgFrame), C.POINTER(XgGaussians), _P, _P, _P, _P]
_L.xg_acui_count.restype = _S
_L.xg_acui_count.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_double,
                             C.POINTER(C.c_int64)]
_L.xg_acui_grid.restype = _S
_L.xg_acui_grid.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_double, _P, C.c_int64, _P]
_L.xg_loss_grad.restype = _S
_L.xg_loss_grad.argtypes = [C.POINTER(XgFrame), _P, _P, C.c_float, _P, _P, _P]
_L.xg_loss_grad_static.restype = _S
_L.xg_loss_grad_static.argtypes = [C.POINTER(XgFrame), _P, _P, C.c_float, _P, _P, _P]
_L.xg_l1_grad.restype = _S
_L.xg_l1_grad.argtypes = [_P, _P, _P, C.c_int64, C.c_float, _P]

if _L.xg_abi_version() != ABI_VERSION:
    raise ImportError("libxg.so ABI version mismatch; rebuild it")

EXPORTED = ("xg_abi_version", "xg_status_string", "xg_default_settings", "xg_camera_from_scanner",
            "xg_layout_views", "xg_ws_layout_of", "xg_workspace_size", "xg_preprocess",
            "xg_bin_sort", "xg_render_fwd", "xg_render_bwd", "xg_preprocess_bwd",
            "xg_render_counts", "xg_l1_grad", "xg_last_error", "xg_adam_step", "xg_store_size",
            "xg_render_fwd_store", "xg_render_bwd_store", "xg_rirf_fwd", "xg_rirf_bwd",
            "xg_loss_grad", "xg_acui_count", "xg_acui_grid", "xg_preprocess_rgb",
            "xg_render_fwd_rgb", "xg_render_fwd_l1", "xg_preprocess_bwd_write", "xg_render_bwd_2d",
            "xg_render_bwd_store_2d", "xg_ws_inspect", "xg_pair_keys", "xg_loss_grad_static")
STATIC_SCRATCH_BYTES = 32 << 20
MAX_STORE_SLOTS = 4096


def lib() -> C.CDLL:
    return _L


def _check(st: int, where: str) -> None:
    if st != XG_OK:
        raise XgError(st, where)


def status_string(st: int) -> str:
    return _L.xg_status_string(st).decode()


def xg_abi_version() -> int:
    return int(_L.xg_abi_version())


def xg_default_settings() -> XgSettings:
    return _L.xg_default_settings()


def xg_camera_from_scanner(phi, l_so, l_sd, width, height, det_w, det_h) -> XgCamera:
    c = XgCamera()
    _check(_L.xg_camera_from_scanner(phi, l_so, l_sd, width, height, det_w, det_h, C.byref(c)),
           "xg_camera_from_scanner")
    return c


def xg_layout_views(cams, tile: int):
    """cams: ctypes array of XgCamera (modified in place).  Returns (pixels, tiles)."""
    px, tl = C.c_int64(), C.c_int64()
    _check(_L.xg_layout_views(cams, len(cams), tile, C.byref(px), C.byref(tl)), "xg_layout_views")
    return px.value, tl.value


def xg_ws_layout_of(frame: XgFrame) -> XgWsLayout:
    out = XgWsLayout()
    _check(_L.xg_ws_layout_of(C.byref(frame), C.byref(out)), "xg_ws_layout_of")
    return out


def xg_workspace_size(frame: XgFrame) -> int:
    b = C.c_size_t()
    _check(_L.xg_workspace_size(C.byref(frame), C.byref(b)), "xg_workspace_size")
    return b.value


def xg_preprocess(frame: XgFrame, g: XgGaussians, stream: int = 0) -> None:
    _check(_L.xg_preprocess(C.byref(frame), C.byref(g), stream), "xg_preprocess")


def xg_bin_sort(frame: XgFrame, stream: int = 0) -> None:
    _check(_L.xg_bin_sort(C.byref(frame), stream), "xg_bin_sort")


def xg_render_fwd(frame: XgFrame, g: XgGaussians, image: int, final_t: int, n_contrib: int,
                  stream: int = 0) -> None:
    _check(_L.xg_render_fwd(C.byref(frame), C.byref(g), image, final_t, n_contrib, stream),
           "xg_render_fwd")


def xg_rirf_fwd(features: int, weights: int, n: int, n_features: int, intensity: int,
                stream: int = 0) -> None:
    _check(_L.xg_rirf_fwd(features, weights, n, n_features, intensity, stream), "xg_rirf_fwd")


def xg_rirf_bwd(features: int, weights: int, n: int, n_features: int, dl_dintensity: int,
                grad_features: int, stream: int = 0) -> None:
    _check(_L.xg_rirf_bwd(features, weights, n, n_features, dl_dintensity, grad_features, stream),
           "xg_rirf_bwd")


def xg_store_size(frame: XgFrame, slots: int) -> int:
    b = C.c_int64()
    _check(_L.xg_store_size(C.byref(frame), slots, C.byref(b)), "xg_store_size")
    return b.value


def xg_render_fwd_store(frame: XgFrame, g: XgGaussians, image: int, final_t: int, n_contrib: int,
                        store: int, slots: int, store_bytes: int, stream: int = 0) -> None:
    _check(_L.xg_render_fwd_store(C.byref(frame), C.byref(g), image, final_t, n_contrib, store,
                                  slots, store_bytes, stream), "xg_render_fwd_store")


def xg_render_bwd_store(frame: XgFrame, g: XgGaussians, dl_dimage: int, final_t: int,
                        n_contrib: int, store: int, slots: int, store_bytes: int, grads: XgGrads,
                        stream: int = 0) -> None:
    _check(_L.xg_render_bwd_store(C.byref(frame), C.byref(g), dl_dimage, final_t, n_contrib, store,
                                  slots, store_bytes, C.byref(grads), stream), "xg_render_bwd_store")


def xg_render_bwd_store_2d(frame: XgFrame, dl_dimage: int, final_t: int, n_contrib: int, store: int,
                           slots: int, store_bytes: int, stream: int = 0) -> None:
    _check(_L.xg_render_bwd_store_2d(C.byref(frame), dl_dimage, final_t, n_contrib, store, slots,
                                     store_bytes, stream), "xg_render_bwd_store_2d")


def xg_render_bwd(frame: XgFrame, g: XgGaussians, dl_dimage: int, final_t: int, n_contrib: int,
                  grads: XgGrads, stream: int = 0) -> None:
    _check(_L.xg_render_bwd(C.byref(frame), C.byref(g), dl_dimage, final_t, n_contrib,
                            C.byref(grads), stream), "xg_render_bwd")


def xg_render_bwd_2d(frame: XgFrame, dl_dimage: int, final_t: int, n_contrib: int,
                     stream: int = 0) -> None:
    _check(_L.xg_render_bwd_2d(C.byref(frame), dl_dimage, final_t, n_contrib, stream),
           "xg_render_bwd_2d")


def xg_ws_inspect(frame: XgFrame) -> XgWsView:
    out = XgWsView()
    _check(_L.xg_ws_inspect(C.byref(frame), C.byref(out)), "xg_ws_inspect")
    return out


def xg_pair_keys(frame: XgFrame, keys: int, values: int, capacity: int, stream: int = 0) -> None:
    _check(_L.xg_pair_keys(C.byref(frame), keys, values, capacity, stream), "xg_pair_keys")


def xg_preprocess_bwd(frame: XgFrame, g: XgGaussians, grads: XgGrads, stream: int = 0) -> None:
    _check(_L.xg_preprocess_bwd(C.byref(frame), C.byref(g), C.byref(grads), stream),
           "xg_preprocess_bwd")


def xg_render_counts(frame: XgFrame, counts: int, stream: int = 0) -> None:
    _check(_L.xg_render_counts(C.byref(frame), counts, stream), "xg_render_counts")


def xg_l1_grad(image: int, target: int, dl_dimage: int, n_pixels: int, scale: float,
               stream: int = 0) -> None:
    _check(_L.xg_l1_grad(image, target, dl_dimage, n_pixels, scale, stream), "xg_l1_grad")


def xg_render_fwd_l1(frame: XgFrame, g: XgGaussians, image: int, final_t: int, n_contrib: int,
                     target: int, scale: float, dl_dimage: int, stream: int = 0) -> None:
    _check(_L.xg_render_fwd_l1(C.byref(frame), C.byref(g), image, final_t, n_contrib, target, scale,
                               dl_dimage, stream), "xg_render_fwd_l1")


def xg_preprocess_bwd_write(frame: XgFrame, g: XgGaussians, grads: XgGrads, stream: int = 0) -> None:
    _check(_L.xg_preprocess_bwd_write(C.byref(frame), C.byref(g), C.byref(grads), stream),
           "xg_preprocess_bwd_write")


def xg_preprocess_rgb(frame: XgFrame, g: XgGaussians, sh: int, degree: int, stream: int = 0) -> None:
    _check(_L.xg_preprocess_rgb(C.byref(frame), C.byref(g), sh, degree, stream), "xg_preprocess_rgb")


def xg_render_fwd_rgb(frame: XgFrame, g: XgGaussians, image: int, final_t: int, n_contrib: int,
                      stream: int = 0) -> None:
    _check(_L.xg_render_fwd_rgb(C.byref(frame), C.byref(g), image, final_t, n_contrib, stream),
           "xg_render_fwd_rgb")


def _acui_args(size, grid, d):
    return (C.c_double * 3)(*map(float, size)), (C.c_int32 * 3)(*map(int, grid)), float(d)


def xg_acui_count(size, grid, d: float) -> int:
    out = C.c_int64(0)
    _check(_L.xg_acui_count(*_acui_args(size, grid, d), C.byref(out)), "xg_acui_count")
    return int(out.value)


def xg_acui_grid(size, grid, d: float, means: int, capacity: int, stream: int = 0) -> None:
    _check(_L.xg_acui_grid(*_acui_args(size, grid, d), means, capacity, stream), "xg_acui_grid")


def xg_loss_grad(frame: XgFrame, image: int, target: int, gamma: float, dl_dimage: int,
                 loss: int = 0, stream: int = 0) -> None:
    _check(_L.xg_loss_grad(C.byref(frame), image, target, gamma, dl_dimage, loss or None, stream),
           "xg_loss_grad")


def xg_loss_grad_static(frame: XgFrame, image: int, target: int, gamma: float, dl_dimage: int,
                        loss: int = 0, stream: int = 0) -> None:
    _check(_L.xg_loss_grad_static(C.byref(frame), image, target, gamma, dl_dimage, loss or None,
                                  stream), "xg_loss_grad_static")


def xg_adam_step(params: XgParams, grads: XgGrads, m: int, v: int, step: int, cfg: XgAdam,
                 scales: int, opacity: int, intensity: int, gate: int = 0, stream: int = 0) -> None:
    _check(_L.xg_adam_step(C.byref(params), C.byref(grads), m, v, step, C.byref(cfg), scales,
                           opacity, intensity, gate or None, stream), "xg_adam_step")
