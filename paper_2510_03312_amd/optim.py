"""Optimiser step (``ubs_adam_step``): the Sec. 4.5 regularisers and spatial
noise, Adam with the Sec. 5.1 per-group learning rates, in one kernel over a
scene's [F][n] parameters.  Argument marshalling only."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib


@dataclass
class AdamConfig:
    lr_mu_x: float = 1.6e-4
    lr_opacity: float = 5e-2
    lr_scale: float = 5e-3
    lr_other: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    lambda_o: float = 0.01
    lambda_s: float = 0.01
    lambda_eps: float = 1.0

    def to_c(self, step: int) -> _lib.UbsAdam:
        return _lib.UbsAdam(self.lr_mu_x, self.lr_opacity, self.lr_scale, self.lr_other,
                            self.beta1, self.beta2, self.eps, self.lambda_o, self.lambda_s,
                            self.lambda_eps, int(step), 0)


def _check_tensor(name: str, t: torch.Tensor, shape) -> None:
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
        raise ValueError(f"{name}: expected a contiguous float32 device tensor of shape {shape}")


def adam_step(params: torch.Tensor, dparams: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
              step: int, dim: int, rot: int, noise: Optional[torch.Tensor] = None,
              cfg: Optional[AdamConfig] = None) -> None:
    """Updates params, m and v in place on the current stream (step is 1-based)."""
    F = _lib.ubs_param_count(dim, rot)
    if F <= 0:
        raise ValueError(f"unsupported dim {dim} / rot {rot}")
    n = params.shape[1] if params.dim() == 2 else -1
    for name, t in (("params", params), ("dparams", dparams), ("m", m), ("v", v)):
        _check_tensor(name, t, (F, n))
    if noise is not None:
        _check_tensor("noise", noise, (3, n))
    cfg = cfg or AdamConfig()
    stream = torch.cuda.current_stream().cuda_stream
    _lib.ubs_adam_step(cfg.to_c(step), dim, rot, n, params.data_ptr(), dparams.data_ptr(),
                       m.data_ptr(), v.data_ptr(), 0 if noise is None else noise.data_ptr(),
                       stream)
