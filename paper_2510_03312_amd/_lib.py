"""ctypes binding of ``libubs.so`` (include/ubs.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of the method; the kernels do all of it.  Loading fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libubs.so")

UBS_OK = 0
UBS_ERR_ARG = 1
UBS_ERR_UNSUPPORTED = 2
UBS_ERR_CAPACITY = 3
UBS_ERR_HIP = 4
STATUS_NAMES = {0: "UBS_OK", 1: "UBS_ERR_ARG", 2: "UBS_ERR_UNSUPPORTED", 3: "UBS_ERR_CAPACITY",
                4: "UBS_ERR_HIP"}

UBS_ROT_QUAT = 0
UBS_ROT_SKEW = 1
UBS_TUNE_PERSISTENT = 1
UBS_TUNE_PRE_FP32 = 2
UBS_TUNE_NO_BETA_COND = 4
UBS_TUNE_NO_BETA_OPACITY = 8
UBS_RELOCATE_NOALLOC_MAX_N = 1 << 21

EXPORTS = ("ubs_preprocess", "ubs_bin_sort", "ubs_render_fwd", "ubs_render_bwd",
           "ubs_adam_step", "ubs_relocate", "ubs_relocate_noalloc", "ubs_ssim_loss",
           "ubs_param_count", "ubs_abi_version")


class UbsScene(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("rot", c_int32), ("n", c_int64),
                ("params", c_void_p), ("dparams", c_void_p)]


class UbsView(ctypes.Structure):
    _fields_ = [("scene", c_int32), ("width", c_int32), ("height", c_int32), ("_pad0", c_int32),
                ("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("time", c_float), ("query", c_float * 3)]


class UbsTuning(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("batch_depth", c_int32),
                ("digit_bits", c_int32), ("pair_capacity", c_int64), ("flags", c_uint32),
                ("tile_slots", c_int32)]


class UbsFrame(ctypes.Structure):
    _fields_ = [("scenes", POINTER(UbsScene)), ("n_scenes", c_int32), ("n_views", c_int32),
                ("views", POINTER(UbsView)), ("tuning", UbsTuning),
                ("stage_events", POINTER(c_void_p))]


STAGES = ("preprocess", "bin_count", "scan", "bin_emit", "sort", "ranges", "raster_fwd",
          "grad_clear", "raster_bwd", "pre_bwd")
N_STAGES = len(STAGES)


class UbsLayout(ctypes.Structure):
    _fields_ = [("bytes", c_uint64), ("n_records", c_int64), ("n_tiles", c_int64),
                ("n_pixels", c_int64), ("pair_capacity", c_int64), ("key_bits", c_int32),
                ("n_views", c_int32), ("off_status", c_uint64), ("off_records", c_uint64),
                ("off_keys", c_uint64), ("off_values", c_uint64), ("off_ranges", c_uint64),
                ("off_ncontrib", c_uint64), ("off_grad2d", c_uint64),
                ("off_live", c_uint64)]


class UbsStatusBlock(ctypes.Structure):
    _fields_ = [("pairs_needed", c_uint64), ("overflow", c_uint32), ("n_nonfinite", c_uint32),
                ("n_visible", c_uint32), ("sort_stalled", c_uint32),
                ("_reserved", c_uint32 * 3), ("spill", c_uint32), ("_pad", c_uint32 * 6)]


class UbsAdam(ctypes.Structure):
    _fields_ = [("lr_mu_x", c_float), ("lr_opacity", c_float), ("lr_scale", c_float),
                ("lr_other", c_float), ("beta1", c_float), ("beta2", c_float), ("eps", c_float),
                ("lambda_o", c_float), ("lambda_s", c_float), ("lambda_eps", c_float),
                ("step", c_int32), ("_pad", c_int32)]


class UbsError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} returned {STATUS_NAMES.get(code, code)}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2510_03312_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        fp = POINTER(UbsFrame)
        L.ubs_preprocess.argtypes = [fp, c_void_p, c_uint64, POINTER(UbsLayout), c_void_p]
        L.ubs_bin_sort.argtypes = [fp, c_void_p, c_uint64, c_void_p]
        L.ubs_render_fwd.argtypes = [fp, c_void_p, c_uint64, c_void_p, c_void_p, c_void_p]
        L.ubs_render_bwd.argtypes = [fp, c_void_p, c_uint64, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p]
        for fn in ("ubs_preprocess", "ubs_bin_sort", "ubs_render_fwd", "ubs_render_bwd"):
            getattr(L, fn).restype = c_int32
        L.ubs_adam_step.argtypes = [POINTER(UbsAdam), c_int32, c_int32, c_int64, c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.ubs_adam_step.restype = c_int32
        L.ubs_relocate.argtypes = [c_int32, c_int32, c_int64, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_float, c_void_p, c_uint64, POINTER(c_uint64),
                                   c_void_p, c_void_p, c_void_p]
        L.ubs_relocate.restype = c_int32
        L.ubs_relocate_noalloc.argtypes = [c_int32, c_int32, c_int64, c_void_p, c_void_p,
                                           c_void_p, c_void_p, c_float, c_void_p, c_void_p,
                                           c_void_p]
        L.ubs_relocate_noalloc.restype = c_int32
        L.ubs_ssim_loss.argtypes = [c_int32, POINTER(c_int32), c_void_p, c_void_p, c_float,
                                    c_void_p, c_void_p, c_void_p, c_uint64, POINTER(c_uint64),
                                    c_void_p]
        L.ubs_ssim_loss.restype = c_int32
        L.ubs_param_count.argtypes = [c_int32, c_int32]
        L.ubs_param_count.restype = c_int32
        L.ubs_abi_version.argtypes = []
        L.ubs_abi_version.restype = c_int32
        _lib = L
    return _lib


def _check(fn: str, code: int) -> int:
    if code != UBS_OK:
        raise UbsError(fn, code)
    return code


def ubs_preprocess(frame: UbsFrame, ws: int, ws_bytes: int, layout: UbsLayout | None,
                   stream: int, check: bool = True) -> int:
    code = load().ubs_preprocess(ctypes.byref(frame), ws or None, ws_bytes,
                                 ctypes.byref(layout) if layout is not None else None, stream or None)
    return _check("ubs_preprocess", code) if check else code


def ubs_bin_sort(frame: UbsFrame, ws: int, ws_bytes: int, stream: int, check: bool = True) -> int:
    code = load().ubs_bin_sort(ctypes.byref(frame), ws or None, ws_bytes, stream or None)
    return _check("ubs_bin_sort", code) if check else code


def ubs_render_fwd(frame: UbsFrame, ws: int, ws_bytes: int, image: int, t_final: int,
                   stream: int, check: bool = True) -> int:
    code = load().ubs_render_fwd(ctypes.byref(frame), ws or None, ws_bytes, image or None,
                                 t_final or None, stream or None)
    return _check("ubs_render_fwd", code) if check else code


def ubs_render_bwd(frame: UbsFrame, ws: int, ws_bytes: int, d_image: int, d_t_final: int,
                   l1_image: int, l1_target: int, stream: int, check: bool = True) -> int:
    code = load().ubs_render_bwd(ctypes.byref(frame), ws or None, ws_bytes, d_image or None,
                                 d_t_final or None, l1_image or None, l1_target or None,
                                 stream or None)
    return _check("ubs_render_bwd", code) if check else code


def ubs_adam_step(cfg: UbsAdam, dim: int, rot: int, n: int, params: int, dparams: int, m: int,
                  v: int, noise: int, stream: int, check: bool = True) -> int:
    code = load().ubs_adam_step(ctypes.byref(cfg), dim, rot, n, params, dparams, m, v, noise,
                                stream)
    return _check("ubs_adam_step", code) if check else code


def ubs_relocate(dim: int, rot: int, n: int, params: int, m: int, v: int, uniforms: int,
                 o_min: float, ws: int, ws_bytes: int, targets_out: int, n_dead_out: int,
                 stream: int, check: bool = True):
    """Returns the workspace bytes needed when ws == 0 (size query), else the code."""
    need = c_uint64(0)
    code = load().ubs_relocate(dim, rot, n, params, m, v, uniforms, o_min, ws, ws_bytes,
                               ctypes.byref(need), targets_out, n_dead_out, stream)
    if check:
        _check("ubs_relocate", code)
    return int(need.value) if not ws else code


def ubs_relocate_noalloc(dim: int, rot: int, n: int, params: int, m: int, v: int, uniforms: int,
                         o_min: float, targets_out: int, n_dead_out: int, stream: int,
                         check: bool = True) -> int:
    code = load().ubs_relocate_noalloc(dim, rot, n, params, m, v, uniforms, o_min,
                                       targets_out or None, n_dead_out or None, stream or None)
    return _check("ubs_relocate_noalloc", code) if check else code


def ubs_ssim_loss(sizes, image: int, target: int, lambda_ssim: float, d_image: int, loss: int,
                  ws: int, ws_bytes: int, stream: int, check: bool = True):
    """sizes: sequence of (width, height).  Returns the workspace bytes needed
    when ws == 0 (size query), else the code."""
    arr = (c_int32 * (2 * max(len(sizes), 1)))(*[int(x) for wh in sizes for x in wh])
    need = c_uint64(0)
    code = load().ubs_ssim_loss(len(sizes), arr, image, target, lambda_ssim, d_image, loss, ws,
                                ws_bytes, ctypes.byref(need), stream)
    if check:
        _check("ubs_ssim_loss", code)
    return int(need.value) if not ws else code


def ubs_param_count(dim: int, rot: int) -> int:
    return int(load().ubs_param_count(dim, rot))


def ubs_abi_version() -> int:
    return int(load().ubs_abi_version())
