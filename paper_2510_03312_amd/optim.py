"""Training-step pieces around the renderer: the image loss with D-SSIM
(``ubs_ssim_loss``), the optimiser step (``ubs_adam_step``: the Sec. 4.5
regularisers and spatial noise, Adam with the Sec. 5.1 per-group learning
rates, in one kernel over a scene's [F][n] parameters) and the relocation
of dead primitives (``ubs_relocate``: Sec. 4.5 cloning rule).  Argument
marshalling only."""
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


def relocate(params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, uniforms: torch.Tensor,
             dim: int, rot: int, o_min: float = 0.005):
    """Relocates dead primitives in place (params, m, v) on the current
    stream; uniforms: float64 [n] in [0, 1).  Returns (targets, n_dead):
    device tensors, the pick of each dead slot (first n_dead entries) and
    the number of dead slots."""
    F = _lib.ubs_param_count(dim, rot)
    if F <= 0:
        raise ValueError(f"unsupported dim {dim} / rot {rot}")
    n = params.shape[1] if params.dim() == 2 else -1
    for name, t in (("params", params), ("m", m), ("v", v)):
        _check_tensor(name, t, (F, n))
    if uniforms.dtype != torch.float64 or not uniforms.is_cuda or tuple(uniforms.shape) != (n,):
        raise ValueError("uniforms: expected a float64 device tensor of shape (n,)")
    need = _lib.ubs_relocate(dim, rot, n, 0, 0, 0, 0, o_min, 0, 0, 0, 0, 0)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=params.device)
    targets = torch.zeros(max(n, 1), dtype=torch.int32, device=params.device)
    n_dead = torch.zeros(1, dtype=torch.int64, device=params.device)
    stream = torch.cuda.current_stream().cuda_stream
    _lib.ubs_relocate(dim, rot, n, params.data_ptr(), m.data_ptr(), v.data_ptr(),
                      uniforms.data_ptr(), o_min, ws.data_ptr(), ws.numel(), targets.data_ptr(),
                      n_dead.data_ptr(), stream)
    return targets, n_dead


def ssim_loss(image: torch.Tensor, target: torch.Tensor, views, lambda_ssim: float = 0.2):
    """(1 - lambda) L1 + lambda (1 - SSIM) over the views of a frame (image,
    target: float32 [sum H W, 3] as the renderer produces).  Returns (loss,
    d_image): a float64 device scalar and the image gradient."""
    sizes = [(v.width, v.height) for v in views]
    A = sum(w * h for w, h in sizes)
    for name, t in (("image", image), ("target", target)):
        _check_tensor(name, t, (A, 3))
    need = _lib.ubs_ssim_loss(sizes, 0, 0, lambda_ssim, 0, 0, 0, 0, 0)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=image.device)
    d_image = torch.empty_like(image)
    loss = torch.zeros(1, dtype=torch.float64, device=image.device)
    _lib.ubs_ssim_loss(sizes, image.data_ptr(), target.data_ptr(), lambda_ssim,
                       d_image.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel(),
                       torch.cuda.current_stream().cuda_stream)
    return loss, d_image
