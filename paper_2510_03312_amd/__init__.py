"""MI355X-native Universal Beta Splatting renderer (HIP kernels for gfx950).

The rendering path is the C ABI of ``libubs.so`` (include/ubs.h); this package
wraps it for PyTorch.  Importing the package does not need a GPU; using the
renderer requires the built library and raises if it is missing.
"""
from ._lib import (UBS_ROT_QUAT, UBS_ROT_SKEW, UBS_TUNE_NO_BETA_COND,  # noqa: F401
                   UBS_TUNE_NO_BETA_OPACITY, UBS_TUNE_PERSISTENT, UBS_TUNE_PRE_FP32, UbsError,
                   load)
from .renderer import (Renderer, SceneRef, Tuning, UBSRenderFunction, render,  # noqa: F401
                       split_views)

from .optim import AdamConfig, adam_step, relocate, ssim_loss  # noqa: F401,E402

__all__ = ["AdamConfig", "adam_step", "relocate", "ssim_loss", "Renderer", "SceneRef", "Tuning", "UBSRenderFunction", "render", "split_views",
           "UBS_ROT_QUAT", "UBS_ROT_SKEW", "UBS_TUNE_PERSISTENT", "UBS_TUNE_PRE_FP32",
           "UBS_TUNE_NO_BETA_COND", "UBS_TUNE_NO_BETA_OPACITY",
           "UbsError", "load"]
