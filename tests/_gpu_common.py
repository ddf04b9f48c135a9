"""Shared helpers of the GPU tests: run a workload through the HIP path and
through the oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import raster as oraster
from oracle import render as orender

GRAD_BLOCKS = ("mu_x", "mu_q", "rot", "log_s_x", "L_qx", "L_q", "b_x", "b_q", "o", "rgb")


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_ready() -> bool:
    return torch.cuda.is_available()


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def live_records(r):
    """The frame's records with the culled ones zeroed, after checking that
    every record marked live has rho > 0 (the preprocess writes the fields
    of the live records only)."""
    live = r.record_live().cpu().numpy()
    assert set(np.unique(live)) <= {0, 1}
    rec = r.live_records().cpu().numpy()
    assert (rec[live == 1, 5] > 0).all()
    return rec


def gpu_render(cfg: dict, tuning=None, *, want_grad: bool = False, d_images=None, l1: bool = False,
               d_tfinals=None, l1_targets=None):
    """Render every view of a workload on the GPU in one frame.  Backward
    (``want_grad``) takes ``d_images`` (and optionally ``d_tfinals``) per view,
    or with ``l1`` the fused L1 loss against ``l1_targets`` (default: the
    workload's targets)."""
    from paper_2510_03312_amd import Renderer, SceneRef, Tuning, split_views
    r = Renderer(tuning or Tuning())
    scenes = [SceneRef(to_dev(s.params), s.dim, s.rot) for s in cfg["scenes"]]
    image, tfin = r.forward(scenes, cfg["views"])
    out = {"renderer": r, "image_flat": image, "t_flat": tfin,
           "images": [x.cpu().numpy() for x in split_views(image, cfg["views"])],
           "t_final": [x.cpu().numpy() for x in split_views(tfin, cfg["views"])],
           "status": r.status(), "records": live_records(r)}
    if want_grad:
        if l1:
            tg = cfg["targets"] if l1_targets is None else l1_targets
            target = torch.cat([to_dev(np.asarray(t, dtype=np.float32)).view(-1, 3) for t in tg])
            grads = r.backward(l1_image=image, l1_target=target)
        else:
            d = torch.cat([to_dev(np.asarray(g, dtype=np.float32)).view(-1, 3) for g in d_images])
            dt = None
            if d_tfinals is not None:
                dt = torch.cat([to_dev(np.asarray(g, dtype=np.float32)).view(-1) for g in d_tfinals])
            grads = r.backward(d, dt)
        torch.cuda.synchronize()
        out["dparams"] = [g.cpu().numpy() for g in grads]
        out["grad2d"] = r.grad2d().cpu().numpy()
    return out


def oracle_view(cfg: dict, v: int, **kw):
    """The oracle's render of view v, compositing float32-rounded records (the
    record precision of the renderer's interface)."""
    view = cfg["views"][v]
    sc = cfg["scenes"][view.scene]
    kw.setdefault("record_f32", True)
    return orender.render(sc.params, sc.dim, sc.rot, view, **kw)


def compare_images(img_gpu, img_or, flags, tol=1e-4):
    """Max |diff| over unflagged pixels; returns (max_err, n_flagged, n_bad)."""
    ok = flags == 0
    diff = np.abs(img_gpu.astype(np.float64) - img_or)
    if diff.ndim == 3:
        diff = diff.max(axis=2)
    bad = (diff > tol) & ok
    return float(diff[ok].max() if ok.any() else 0.0), int((~ok).sum()), int(bad.sum())


# Float32 summation budget: a float32 sum of terms t_k (wavefront trees plus
# atomics) is within about n_ulp * 2^-24 * sum |t_k| of the exact sum; 1e-5
# (~170 ulps) also covers the float32 evaluation of each term.  Only the
# float32 per-primitive option's test adds it; every float64 gradient meets
# the bar without it.
FP32_SUM_BUDGET = 1e-5


def grad_violations(g, g_ref, rtol=1e-3, floor=1e-3, noise=None):
    """|g - g_ref| <= rtol * max(|g_ref|, floor * max|g_ref|) elementwise
    (+ FP32_SUM_BUDGET * noise if given, the oracle's sum of |per-pixel
    terms| carried through |Jacobian|)."""
    scale = np.abs(g_ref).max() if g_ref.size else 0.0
    bound = rtol * np.maximum(np.abs(g_ref), floor * scale)
    if noise is not None:
        bound = bound + FP32_SUM_BUDGET * noise
    viol = np.abs(g.astype(np.float64) - g_ref) > bound + 1e-30
    return viol


def bin_reference(records: np.ndarray, views, tile_w=16, tile_h=16):
    """Oracle binning over a frame's records (views in order)."""
    keys, vals = [], []
    rec_base = tile_base = 0
    n_tiles = 0
    for v in views:
        n = int(v.n_records)
        k, vv = oraster.bin_view(records[rec_base:rec_base + n], v.width, v.height, tile_w, tile_h,
                                 tile_base=tile_base, rec_base=rec_base)
        keys.append(k)
        vals.append(vv)
        nt = ((v.width + tile_w - 1) // tile_w) * ((v.height + tile_h - 1) // tile_h)
        tile_base += nt
        rec_base += n
    keys = np.concatenate(keys) if keys else np.zeros(0, np.uint64)
    vals = np.concatenate(vals) if vals else np.zeros(0, np.uint32)
    return oraster.sort_and_ranges(keys, vals, tile_base)
