"""A complete DRR training step on persistent buffers, eager or captured as
one HIP graph.

The step is: preprocess (Eq. 7-9), per-tile depth-sorted lists (Sec. 3.2),
forward blending (Eq. 10) with the L1 upstream gradient (Eq. 11) in the
same launch, reverse blending and the projection adjoint (writing fresh
gradients, so no clearing launch), optionally followed by the fused Adam
update of the raw parameters.  Every stage is a libxg kernel launch on one
stream with no allocation, memset or synchronisation, so the whole
sequence is captured once (torch.cuda.CUDAGraph is a hipGraph on ROCm) and
replayed per step.  The pair capacity is data dependent: after replays the
caller checks the device status word with ``check()``, which grows the
workspace and re-captures when the pairs no longer fit.
"""
from __future__ import annotations

import torch

from . import _lib as X
from .drr import PARAMS, Frame, gaussians_struct


class TrainStep:
    def __init__(self, frame: Frame, g: dict, target: torch.Tensor, scale: float,
                 grads: dict | None = None, zero_grads: bool = True, optimizer=None,
                 store=None):
        self.frame = frame
        self.g = g
        self.target = target
        self.scale = float(scale)
        self.zero_grads = zero_grads
        self.image, self.final_t, self.n_contrib = frame.new_outputs()
        self.dl = torch.empty_like(self.image)
        self.grads = frame.new_grads(g) if grads is None else grads
        self.graph = None
        self.post = []   # extra enqueue callables run after the backward
        # FusedAdam over the Gaussians in ``g`` (its activated copies are ``g``);
        # gated by the frame's status word, so an overflowed step changes nothing
        self.optimizer = optimizer
        # stored-transmittance variant: a Frame.new_store() buffer (None = divide back)
        self.store = store

    def run(self, stream=None, optimize: bool = True) -> None:
        """Enqueues one step on ``stream`` (default: the current stream);
        ``optimize=False`` leaves the optimiser out."""
        s = int((stream or torch.cuda.current_stream()).cuda_stream)
        f = self.frame
        gs = gaussians_struct(self.g)
        gr = X.XgGrads(*(self.grads[k].data_ptr() for k in PARAMS))
        X.xg_preprocess(f.frame, gs, s)
        X.xg_bin_sort(f.frame, s)
        st = self.store
        if st is None:
            # forward blend and the L1 gradient in one launch
            X.xg_render_fwd_l1(f.frame, gs, self.image.data_ptr(), self.final_t.data_ptr(),
                               self.n_contrib.data_ptr(), self.target.data_ptr(), self.scale,
                               self.dl.data_ptr(), s)
        else:
            X.xg_render_fwd_store(f.frame, gs, self.image.data_ptr(), self.final_t.data_ptr(),
                                  self.n_contrib.data_ptr(), st.view.data_ptr(), st.slots,
                                  st.view.numel(), s)
            X.xg_l1_grad(self.image.data_ptr(), self.target.data_ptr(), self.dl.data_ptr(),
                         self.image.numel(), self.scale, s)
        # the 2-D stage, then the projection adjoint writing (or adding) the
        # parameter gradients
        if st is None:
            X.xg_render_bwd_2d(f.frame, self.dl.data_ptr(), self.final_t.data_ptr(),
                               self.n_contrib.data_ptr(), s)
        else:
            X.xg_render_bwd_store_2d(f.frame, self.dl.data_ptr(), self.final_t.data_ptr(),
                                     self.n_contrib.data_ptr(), st.view.data_ptr(), st.slots,
                                     st.view.numel(), s)
        if self.zero_grads:
            X.xg_preprocess_bwd_write(f.frame, gs, gr, s)   # this step's gradients only
        else:
            X.xg_preprocess_bwd(f.frame, gs, gr, s)         # added to the caller's
        if optimize and self.optimizer is not None:
            self.optimizer.step(self.grads, s, gate=f.status_ptr())
        for fn in self.post:
            fn(s)

    def capture(self) -> None:
        """Captures run() into a graph (after one eager warm-up on a side
        stream, which leaves the optimiser out so the parameters do not move)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run(optimize=False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()

    def replay(self) -> None:
        self.graph.replay()

    def check(self, headroom: float = 1.25) -> bool:
        """Synchronises and reads the status word.  On pair overflow, grows the
        workspace (re-running the stages eagerly) and re-captures if a graph
        was in use; returns False in that case (the last step's outputs are
        invalid and the step should be repeated)."""
        torch.cuda.synchronize()
        st = self.frame.status()
        if st == X.XG_OK:
            return True
        if st != X.XG_ECAPACITY:
            raise X.XgError(st, "TrainStep")
        had_graph = self.graph is not None
        self.graph = None
        self.frame.fit_capacity(self.g, headroom)
        if had_graph:
            self.capture()
        return False
