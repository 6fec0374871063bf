"""Torch-facing wrapper of the DRR library: frames, workspaces, autograd.

PyTorch supplies device memory, streams and autograd here; every step of
the rendering runs in libxg's HIP kernels (see include/xg.h).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from . import _lib as X

PARAMS = ("means", "scales", "quats", "opacity", "intensity")


def settings(tile: int = 16, lds_batch: int = 256, lowpass: float = 0.3,
             alpha_min: float = 1.0 / 255.0, alpha_max: float = 0.99, t_min: float = 1e-4,
             near_z: float = 0.2, persistent: bool = False) -> X.XgSettings:
    s = X.xg_default_settings()
    s.tile, s.lds_batch, s.lowpass = tile, lds_batch, lowpass
    s.alpha_min, s.alpha_max, s.t_min, s.near_z = alpha_min, alpha_max, t_min, near_z
    s.flags = X.XG_F_PERSISTENT if persistent else 0
    return s


def cameras(angles, sizes, l_so: float, l_sd: float, det_w: float, det_h: float | None = None):
    """One cone-beam camera per (azimuth, (width, height)) (Eq. 12)."""
    det_h = det_w if det_h is None else det_h
    return [X.xg_camera_from_scanner(float(a), l_so, l_sd, int(w), int(h), det_w, det_h)
            for a, (w, h) in zip(angles, sizes)]


def gaussians_struct(g: dict) -> X.XgGaussians:
    n = g["means"].shape[0]
    for k in PARAMS:
        t = g[k]
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{k} must be a contiguous float32 CUDA tensor")
    return X.XgGaussians(g["means"].data_ptr(), g["scales"].data_ptr(), g["quats"].data_ptr(),
                         g["opacity"].data_ptr(), g["intensity"].data_ptr(), n)


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Grads(dict):
    """Gradient tensors of the Gaussian parameters as views of one flat
    buffer, so clearing them is a single fill (``zero_()``)."""

    @staticmethod
    def like(g: dict) -> "Grads":
        sizes = [g[k].numel() for k in PARAMS]
        flat = torch.zeros(sum(sizes), dtype=torch.float32, device=g["means"].device)
        out = Grads()
        off = 0
        for k, n in zip(PARAMS, sizes):
            out[k] = flat[off:off + n].view(g[k].shape)
            off += n
        out.flat = flat
        return out

    def zero_(self) -> None:
        self.flat.zero_()


class TStore:
    """Stored transmittances between a forward and its backward."""

    def __init__(self, buf: torch.Tensor, view: torch.Tensor, slots: int, tile: int):
        self.buf, self.view, self.slots, self.tile = buf, view, int(slots), int(tile)

    def contributors(self, frame: "Frame") -> torch.Tensor:
        """Per-pixel contributor counts written by the forward, in tile order."""
        n = frame.total_tiles * self.tile * self.tile
        return self.view[:4 * n].view(torch.int32)


class Frame:
    """n Gaussians rendered into a fixed list of views, with its workspace.

    The workspace holds the sorted per-tile lists between the forward and
    the backward call, so a Frame serves one forward/backward at a time.
    """

    def __init__(self, n: int, cams, st: X.XgSettings | None = None, pair_capacity: int | None = None,
                 device: str | torch.device = "cuda"):
        self.n = int(n)
        self.settings = st if st is not None else settings()
        self.cams = (X.XgCamera * len(cams))(*cams)
        self.total_pixels, self.total_tiles = X.xg_layout_views(self.cams, self.settings.tile)
        self.device = torch.device(device)
        self.cams_dev = torch.frombuffer(bytearray(bytes(self.cams)), dtype=torch.uint8).to(self.device)
        self.n_views = len(cams)
        self.sizes = [(c.width, c.height) for c in cams]
        self.capacity = int(pair_capacity) if pair_capacity else max(1 << 16, 6 * self.n * self.n_views)
        # bumped by every preprocess: a backward checks that the lists it walks
        # are those of its own forward
        self.generation = 0
        # whether a backward has added into the 2-D gradient accumulators since
        # the last preprocess (which clears them)
        self.accumulated = False
        self._allocate()

    # -- workspace -----------------------------------------------------------
    def _frame(self, ws_ptr: int = 0, ws_bytes: int = 0) -> X.XgFrame:
        return X.XgFrame(self.n, self.n_views, self.cams, self.cams_dev.data_ptr(), self.settings,
                         ws_ptr, ws_bytes, self.capacity)

    def _allocate(self) -> None:
        probe = self._frame()
        self.layout = X.xg_ws_layout_of(probe)
        size = self.layout.total
        self._ws_buf = torch.empty(size + 256, dtype=torch.uint8, device=self.device)
        base = self._ws_buf.data_ptr()
        self._ws_off = (-base) % 256
        self.ws = self._ws_buf[self._ws_off:self._ws_off + size]
        self.frame = self._frame(self.ws.data_ptr(), size)

    def set_capacity(self, cap: int) -> None:
        if cap != self.capacity:
            self.capacity = int(cap)
            self._allocate()

    def ws_tensor(self, offset: int, dtype: torch.dtype, count: int) -> torch.Tensor:
        itemsize = torch.empty((), dtype=dtype).element_size()
        return self.ws[offset:offset + count * itemsize].view(dtype)

    def status(self) -> int:
        return int(self.ws_tensor(self.layout.status, torch.int32, 1).item())

    def status_ptr(self) -> int:
        """Device address of the status word (valid until the next reallocation)."""
        return self.ws.data_ptr() + self.layout.status

    def n_pairs(self) -> int:
        return int(self.ws_tensor(self.layout.n_pairs, torch.int32, 1).item())

    def sorted_pairs(self, stream=None):
        """(keys, values, ranges) of the sorted lists, for inspection
        (synchronises): keys[p] = tile << 32 | depth bits and values[p] =
        Gaussian index as written by xg_pair_keys."""
        p = self.n_pairs()
        if self.status() != X.XG_OK:
            p = 0
        keys = torch.empty(max(p, 1), dtype=torch.int64, device=self.device)
        vals = torch.empty(max(p, 1), dtype=torch.int32, device=self.device)
        X.xg_pair_keys(self.frame, keys.data_ptr(), vals.data_ptr(), p, _stream(stream))
        torch.cuda.synchronize(self.device)
        ranges = self.ws_tensor(self.layout.ranges, torch.int32, 2 * self.total_tiles)
        return keys[:p], vals[:p], ranges.view(self.total_tiles, 2)

    # -- stages --------------------------------------------------------------
    def preprocess_sort(self, g: dict, stream=None) -> None:
        gs = gaussians_struct(g)
        s = _stream(stream)
        X.xg_preprocess(self.frame, gs, s)
        X.xg_bin_sort(self.frame, s)
        self.generation += 1
        self.accumulated = False

    def clear_2d_grads(self) -> None:
        """Zeroes the per-(view, Gaussian) 2-D gradient accumulators (what the
        preprocess does), so that a second backward of the same forward does
        not add to the first one's sums."""
        self.ws_tensor(self.layout.grad2d, torch.float32, 8 * self.n * self.n_views).zero_()
        self.accumulated = False

    def fit_capacity(self, g: dict, headroom: float = 1.25) -> int:
        """Runs preprocess + sort, grows the workspace if the pairs did not fit
        (synchronises).  Returns the pair count."""
        self.preprocess_sort(g)
        p = self.n_pairs()
        if self.status() == X.XG_ECAPACITY or p > self.capacity:
            self.set_capacity(int(math.ceil(p * headroom)) + 1024)
            self.preprocess_sort(g)
            p = self.n_pairs()
        if self.status() != X.XG_OK:
            raise X.XgError(self.status(), "fit_capacity")
        return p

    def new_outputs(self):
        px = self.total_pixels
        return (torch.empty(px, dtype=torch.float32, device=self.device),
                torch.empty(px, dtype=torch.float32, device=self.device),
                torch.empty(px, dtype=torch.int32, device=self.device))

    def render_fwd(self, g: dict, out=None, stream=None):
        image, final_t, n_contrib = out if out is not None else self.new_outputs()
        X.xg_render_fwd(self.frame, gaussians_struct(g), image.data_ptr(), final_t.data_ptr(),
                        n_contrib.data_ptr(), _stream(stream))
        return image, final_t, n_contrib

    def forward_rgb(self, g: dict, sh: torch.Tensor, degree: int, out=None, stream=None):
        """Forward of the comparison model (RGB Gaussians, SH colours of Eq. 2):
        preprocess with colours, binning, three-channel blend.  Returns the
        planar [3, total_pixels] image, final T and the last contributor."""
        if sh.dtype != torch.float32 or not sh.is_contiguous() or \
                sh.numel() != self.n * (degree + 1) ** 2 * 3:
            raise ValueError("sh must be contiguous float32 [n, (degree+1)^2, 3]")
        sid = _stream(stream)
        gs = gaussians_struct(g)
        if out is None:
            out = (torch.empty((3, self.total_pixels), dtype=torch.float32, device=self.device),
                   torch.empty(self.total_pixels, dtype=torch.float32, device=self.device),
                   torch.empty(self.total_pixels, dtype=torch.int32, device=self.device))
        image, final_t, n_contrib = out
        X.xg_preprocess_rgb(self.frame, gs, sh.data_ptr(), degree, sid)
        X.xg_bin_sort(self.frame, sid)
        X.xg_render_fwd_rgb(self.frame, gs, image.data_ptr(), final_t.data_ptr(), n_contrib.data_ptr(),
                            sid)
        return image, final_t, n_contrib

    def forward(self, g: dict, out=None, stream=None):
        self.preprocess_sort(g, stream)
        return self.render_fwd(g, out, stream)

    def new_grads(self, g: dict) -> "Grads":
        return Grads.like(g)

    def backward(self, g: dict, dl_dimage: torch.Tensor, final_t: torch.Tensor,
                 n_contrib: torch.Tensor, grads: dict | None = None, stream=None) -> dict:
        """Adjoint of forward() (xg_render_bwd), added to ``grads`` (new
        zeroed tensors if None).  A repeated backward of the same forward
        clears the 2-D accumulators first."""
        grads = self.new_grads(g) if grads is None else grads
        gr = X.XgGrads(*(grads[k].data_ptr() for k in PARAMS))
        if self.accumulated:
            self.clear_2d_grads()
        X.xg_render_bwd(self.frame, gaussians_struct(g), dl_dimage.data_ptr(), final_t.data_ptr(),
                        n_contrib.data_ptr(), gr, _stream(stream))
        self.accumulated = True
        return grads

    # -- stored-transmittance variant ------------------------------------------
    def new_store(self, slots: int) -> "TStore":
        """A buffer for the transmittances of the first ``slots`` contributors
        of every pixel (256-byte aligned view of a torch allocation)."""
        nbytes = X.xg_store_size(self.frame, slots)
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        return TStore(buf, buf[off:off + nbytes], slots, self.settings.tile)

    def render_fwd_store(self, g: dict, store: "TStore", out=None, stream=None):
        image, final_t, n_contrib = out if out is not None else self.new_outputs()
        X.xg_render_fwd_store(self.frame, gaussians_struct(g), image.data_ptr(), final_t.data_ptr(),
                              n_contrib.data_ptr(), store.view.data_ptr(), store.slots,
                              store.view.numel(), _stream(stream))
        return image, final_t, n_contrib

    def backward_store(self, g: dict, dl_dimage: torch.Tensor, final_t: torch.Tensor,
                       n_contrib: torch.Tensor, store: "TStore", grads: dict | None = None,
                       stream=None) -> dict:
        grads = self.new_grads(g) if grads is None else grads
        gr = X.XgGrads(*(grads[k].data_ptr() for k in PARAMS))
        if self.accumulated:
            self.clear_2d_grads()
        X.xg_render_bwd_store(self.frame, gaussians_struct(g), dl_dimage.data_ptr(),
                              final_t.data_ptr(), n_contrib.data_ptr(), store.view.data_ptr(),
                              store.slots, store.view.numel(), gr, _stream(stream))
        self.accumulated = True
        return grads

    def render_counts(self, stream=None) -> torch.Tensor:
        """Work counts of the current sorted lists (int32 [XG_COUNT_ROWS,
        pixels], rows as documented at xg_render_counts): per-pixel
        evaluations, contributors, revisited evaluations; per 8 x 8 block the
        backward's wavefront reductions and the entries the backward and the
        forward visit; per-pixel evaluations inside those visits."""
        out = torch.empty((X.COUNT_ROWS, self.total_pixels), dtype=torch.int32, device=self.device)
        X.xg_render_counts(self.frame, out.data_ptr(), _stream(stream))
        return out

    def loss_grad(self, image: torch.Tensor, target: torch.Tensor, gamma: float = 0.2, out=None,
                  loss: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """dL/dI of the Eq. 11 objective (1 - gamma) L1 + gamma L_SSIM over all
        views; writes L into ``loss`` (one device float) when given."""
        for t in (image, target):
            if t.dtype != torch.float32 or t.numel() != self.total_pixels or not t.is_contiguous():
                raise ValueError("image and target must be contiguous float32 of total_pixels")
        out = torch.empty_like(image) if out is None else out
        X.xg_loss_grad(self.frame, image.data_ptr(), target.data_ptr(), gamma, out.data_ptr(),
                       loss.data_ptr() if loss is not None else 0, _stream(stream))
        return out

    def split(self, flat: torch.Tensor):
        """Per-view (H, W) views of a concatenated per-pixel buffer."""
        out, o = [], 0
        for w, h in self.sizes:
            out.append(flat[o:o + w * h].view(h, w))
            o += w * h
        return out


def acui_means(size, grid, d: float, device="cuda", stream=None) -> torch.Tensor:
    """ACUI Gaussian centres (Sec. 3.3, Eq. 13) generated on the GPU: a
    float32 [count, 3] tensor, n1 slowest and n3 fastest."""
    n = X.xg_acui_count(size, grid, d)
    out = torch.empty((n, 3), dtype=torch.float32, device=device)
    X.xg_acui_grid(size, grid, d, out.data_ptr(), n, _stream(stream))
    return out


def l1_grad(image: torch.Tensor, target: torch.Tensor, scale: float, out: torch.Tensor | None = None,
            stream=None) -> torch.Tensor:
    """dL/dI of the L1 term of Eq. 11: scale * sign(image - target)."""
    out = torch.empty_like(image) if out is None else out
    X.xg_l1_grad(image.data_ptr(), target.data_ptr(), out.data_ptr(), image.numel(), scale,
                 _stream(stream))
    return out


class DRRFunction(torch.autograd.Function):
    """I = F_DRR(M_ext, M_int, {G_i}) (Eq. 5) with the hand-written backward.

    Saves only the final transmittance and the last contributor per pixel;
    the backward recomputes the transmittance by division.  The sorted lists
    stay in the frame's workspace between forward and backward, so the
    backward must come before the frame renders again (checked: RuntimeError
    otherwise).  The forward reads the device status word (one
    synchronisation): on a pair overflow it grows the workspace and renders
    again; any other failure raises XgError.  A second backward of the same
    forward (retain_graph) gives the same gradients again.
    """

    @staticmethod
    def forward(ctx, means, scales, quats, opacity, intensity, frame: Frame):
        g = {"means": means.detach().contiguous(), "scales": scales.detach().contiguous(),
             "quats": quats.detach().contiguous(), "opacity": opacity.detach().contiguous(),
             "intensity": intensity.detach().contiguous()}
        frame.fit_capacity(g)          # preprocess + lists; grows the workspace on overflow
        image, final_t, n_contrib = frame.render_fwd(g)
        ctx.frame = frame
        ctx.generation = frame.generation
        ctx.save_for_backward(g["means"], g["scales"], g["quats"], g["opacity"], g["intensity"],
                              final_t, n_contrib)
        ctx.mark_non_differentiable(final_t, n_contrib)
        return image, final_t, n_contrib

    @staticmethod
    def backward(ctx, dl_dimage, _dt, _dn):
        frame = ctx.frame
        if frame.generation != ctx.generation:
            raise RuntimeError("DRRFunction.backward: the frame rendered again after this forward; "
                               "its sorted lists belong to the later render")
        means, scales, quats, opacity, intensity, final_t, n_contrib = ctx.saved_tensors
        g = {"means": means, "scales": scales, "quats": quats, "opacity": opacity,
             "intensity": intensity}
        grads = frame.backward(g, dl_dimage.contiguous(), final_t, n_contrib)
        return (grads["means"], grads["scales"], grads["quats"], grads["opacity"],
                grads["intensity"], None)


def rirf(features: torch.Tensor, weights: torch.Tensor, stream=None) -> torch.Tensor:
    """Eq. 3: intensity = sigmoid(weights . features) (xg_rirf_fwd)."""
    n, nf = features.shape
    out = torch.empty(n, dtype=torch.float32, device=features.device)
    X.xg_rirf_fwd(features.data_ptr(), weights.data_ptr(), n, nf, out.data_ptr(), _stream(stream))
    return out


class RIRFFunction(torch.autograd.Function):
    """Autograd wrapper of the radiation intensity response (weights are
    constants, no gradient)."""

    @staticmethod
    def forward(ctx, features, weights):
        features = features.contiguous()
        weights = weights.contiguous()
        ctx.save_for_backward(features, weights)
        return rirf(features, weights)

    @staticmethod
    def backward(ctx, dl_di):
        features, weights = ctx.saved_tensors
        n, nf = features.shape
        gf = torch.zeros_like(features)
        X.xg_rirf_bwd(features.data_ptr(), weights.data_ptr(), n, nf, dl_di.contiguous().data_ptr(),
                      gf.data_ptr(), _stream(None))
        return gf, None


def render(g: dict, frame: Frame):
    """Differentiable render of all views; returns the concatenated image."""
    image, _, _ = DRRFunction.apply(g["means"], g["scales"], g["quats"], g["opacity"],
                                    g["intensity"], frame)
    return image
