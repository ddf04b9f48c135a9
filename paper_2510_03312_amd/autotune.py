"""Autotuner: picks the raster tile shape, LDS batch depth and launch mode
(one wavefront per tile, or a persistent grid with a tile queue) for a
frame by timing each candidate on the device with HIP events, and caches the
winner per frame signature (architecture, dimensions, primitive and pixel
counts bucketed by powers of two, number of views).
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from ._lib import UBS_TUNE_PERSISTENT
from .renderer import Renderer, SceneRef, Tuning

TILES = ((16, 16), (16, 8), (8, 8), (32, 16))
BATCHES = (64, 128, 256)
PERSISTENT = (False, True)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ubs_autotune.json")


def _bucket(x: int) -> int:
    return 0 if x <= 0 else int(math.ceil(math.log2(x)))


def signature(scenes: Sequence[SceneRef], views: Sequence, backward: bool) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
    dims = ",".join(str(s.dim) for s in scenes)
    n_rec = sum(scenes[int(getattr(v, "scene", 0))].n for v in views)
    n_pix = sum(int(v.width) * int(v.height) for v in views)
    return (f"{arch}|dims={dims}|rec=2^{_bucket(n_rec)}|px=2^{_bucket(n_pix)}|views={len(views)}"
            f"|{'fwdbwd' if backward else 'fwd'}")


def candidates(base: Optional[Tuning] = None) -> List[Tuning]:
    base = base or Tuning()
    out = []
    for (tw, th) in TILES:
        for b in BATCHES:
            for p in PERSISTENT:
                out.append(Tuning(tile_w=tw, tile_h=th, batch_depth=b, digit_bits=base.digit_bits,
                                  flags=(base.flags & ~UBS_TUNE_PERSISTENT) | (UBS_TUNE_PERSISTENT if p else 0),
                                  tile_slots=base.tile_slots))
    return out


def time_frame(tuning: Tuning, scenes: Sequence[SceneRef], views: Sequence, *, backward: bool,
               l1_target: Optional[torch.Tensor], steps: int = 3) -> float:
    """Median ms of a frame (eager calls) under one tuning."""
    r = Renderer(tuning)
    image, t_final = r.forward(scenes, views)
    frame = r.frame
    for k, s in enumerate(frame.scenes):
        frame.set_dparams(k, torch.empty_like(s.params))
    ms = []
    for i in range(steps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r.preprocess(frame)
        r.bin_sort(frame)
        r.render_fwd(frame, image, t_final)
        if backward:
            r.render_bwd(frame, l1_image=image, l1_target=l1_target)
        e1.record()
        torch.cuda.synchronize()
        if i:
            ms.append(e0.elapsed_time(e1))
    ms.sort()
    return ms[len(ms) // 2]


def autotune(scenes: Sequence[SceneRef], views: Sequence, *, backward: bool = True,
             l1_target: Optional[torch.Tensor] = None, base: Optional[Tuning] = None,
             cache_path: Optional[str] = DEFAULT_CACHE, steps: int = 3,
             cands: Optional[List[Tuning]] = None) -> Tuple[Tuning, Dict[str, float]]:
    """Best tuning for this frame (from the cache if present) and the timings."""
    key = signature(scenes, views, backward)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        t = cache[key]["tuning"]
        return Tuning(**t), cache[key].get("ms", {})
    if backward and l1_target is None:
        n_pix = sum(int(v.width) * int(v.height) for v in views)
        l1_target = torch.full((n_pix, 3), 0.5, device="cuda")
    timings: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    for t in (cands or candidates(base)):
        name = f"{t.tile_w}x{t.tile_h}/b{t.batch_depth}/{'persistent' if t.flags & UBS_TUNE_PERSISTENT else 'grid'}"
        ms = time_frame(t, scenes, views, backward=backward, l1_target=l1_target, steps=steps)
        timings[name] = ms
        if ms < best_ms:
            best, best_ms = t, ms
    if cache_path:
        cache[key] = {"tuning": best.__dict__, "ms": timings}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return best, timings
