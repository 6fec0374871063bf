"""Fused Adam over the raw Gaussian parameters (xg_adam_step).

The renderer consumes activated parameters (scales, opacity, intensity);
the optimiser keeps the raw ones (log-scales, opacity logits, the feature
vectors of the radiation intensity response) and rewrites the activated
copies after every step.  Means and quaternions are shared between the two
views (identity activation).  The step counter lives on the device, so an
optimiser step inside a captured graph replays correctly.
"""
from __future__ import annotations

import torch

from . import _lib as X

# Sec. 4.1 of the paper; 16 features per Gaussian (its choice of N_f)
PAPER_ADAM = {"lr_means_start": 1.9e-4, "lr_means_end": 1.9e-6, "lr_means_steps": 20000,
              "lr_scales": 5e-3, "lr_quats": 1e-3, "lr_opacity": 8e-3, "lr_feature": 2e-3,
              "beta1": 0.9, "beta2": 0.999, "eps": 1e-15}
PAPER_FEATURES = 16


class FusedAdam:
    def __init__(self, raw: dict, act: dict, weights: torch.Tensor, **overrides):
        n = raw["means"].shape[0]
        nf = raw["features"].shape[1]
        if weights.numel() != nf:
            raise ValueError("one weight per feature")
        self.n, self.n_features = n, nf
        self.raw = raw
        self.act = act
        self.weights = weights.contiguous()
        cfg = dict(PAPER_ADAM)
        cfg.update(overrides)
        self.cfg = X.XgAdam(cfg["lr_means_start"], cfg["lr_means_end"], int(cfg["lr_means_steps"]),
                            cfg["lr_scales"], cfg["lr_quats"], cfg["lr_opacity"], cfg["lr_feature"],
                            cfg["eps"], 0, cfg["beta1"], cfg["beta2"])
        dev = raw["means"].device
        self.m = torch.zeros((11 + nf) * n, dtype=torch.float32, device=dev)
        self.v = torch.zeros((11 + nf) * n, dtype=torch.float32, device=dev)
        self.step_count = torch.zeros(1, dtype=torch.int32, device=dev)
        self._params = X.XgParams(raw["means"].data_ptr(), raw["log_scales"].data_ptr(),
                                  raw["quats"].data_ptr(), raw["opacity_logit"].data_ptr(),
                                  raw["features"].data_ptr(), self.weights.data_ptr(), n, nf)

    @staticmethod
    def from_activated(g: dict, n_features: int = PAPER_FEATURES, weights: torch.Tensor | None = None,
                       **overrides) -> "FusedAdam":
        """Raw parameters from activated ones (features: the minimum-norm
        vector with sigmoid(weights . f) = intensity); the returned
        optimiser's ``act`` dict is the render input (means/quats shared
        with raw).  Default weights: all ones."""
        dev = g["means"].device
        w = (torch.ones(n_features, dtype=torch.float32, device=dev) if weights is None
             else weights.to(dev, torch.float32).contiguous())
        means = g["means"].clone().contiguous()
        quats = g["quats"].clone().contiguous()
        logit_i = torch.logit(g["intensity"].double().clamp(1e-7, 1 - 1e-7))
        wd = w.double()
        features = (logit_i[:, None] * wd[None, :] / (wd @ wd)).float().contiguous()
        raw = {"means": means, "log_scales": torch.log(g["scales"]).contiguous(), "quats": quats,
               "opacity_logit": torch.logit(g["opacity"].double()).float().contiguous(),
               "features": features}
        act = {"means": means, "scales": g["scales"].clone().contiguous(), "quats": quats,
               "opacity": g["opacity"].clone().contiguous(),
               "intensity": g["intensity"].clone().contiguous()}
        return FusedAdam(raw, act, w, **overrides)

    def step(self, grads: dict, stream=None, gate: int = 0) -> None:
        """Enqueues one Adam step with gradients of the activated parameters.
        ``stream``: a torch stream or a raw HIP stream handle.  ``gate``:
        device address of an int32 that skips the step when nonzero (a
        frame's status word)."""
        if isinstance(stream, int):
            s = stream
        else:
            s = int((stream or torch.cuda.current_stream()).cuda_stream)
        gr = X.XgGrads(grads["means"].data_ptr(), grads["scales"].data_ptr(),
                       grads["quats"].data_ptr(), grads["opacity"].data_ptr(),
                       grads["intensity"].data_ptr())
        X.xg_adam_step(self._params, gr, self.m.data_ptr(), self.v.data_ptr(),
                       self.step_count.data_ptr(), self.cfg, self.act["scales"].data_ptr(),
                       self.act["opacity"].data_ptr(), self.act["intensity"].data_ptr(), gate, s)

    def state_dict(self) -> dict:
        return {"raw": {k: t.detach().cpu() for k, t in self.raw.items()},
                "weights": self.weights.cpu(), "m": self.m.cpu(), "v": self.v.cpu(),
                "step": int(self.step_count.item())}

    def load_state_dict(self, sd: dict) -> None:
        for k, t in self.raw.items():
            t.copy_(sd["raw"][k])
        self.weights.copy_(sd["weights"])
        self.m.copy_(sd["m"])
        self.v.copy_(sd["v"])
        self.step_count.fill_(int(sd["step"]))
