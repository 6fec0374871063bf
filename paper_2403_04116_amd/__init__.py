"""MI355X (gfx950) Differentiable Radiative Rasterization.

The rendering path is the HIP library libxg.so behind the C ABI of
include/xg.h; ``_lib`` binds it with ctypes and ``drr`` adds torch memory,
streams and autograd around it.  Importing this package fails loudly if
the library has not been built: there is no CPU fallback.
"""
from . import _lib  # noqa: F401  (loads libxg.so or raises)
from ._lib import (XgCamera, XgError, XgFrame, XgGaussians, XgGrads, XgSettings,  # noqa: F401
                   xg_abi_version, xg_bin_sort, xg_camera_from_scanner, xg_default_settings,
                   xg_l1_grad, xg_layout_views, xg_preprocess, xg_preprocess_bwd, xg_render_bwd,
                   xg_render_bwd_2d, xg_render_counts, xg_render_fwd, xg_pair_keys, xg_ws_inspect,
                   xg_workspace_size, xg_ws_layout_of)
from .drr import (DRRFunction, Frame, RIRFFunction, acui_means, cameras, l1_grad, render,  # noqa: F401
                  rirf, settings)
