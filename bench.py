#!/usr/bin/env python
"""Benchmark of the Universal Beta Splatting hot path on one MI355X.

One step = one full forward+backward frame through the four C entry points
(preprocess -> bin_sort -> render_fwd -> render_bwd with the fused L1 loss
gradient), on inputs already resident in HBM.  Default workload: 1,000,000
7-D Beta primitives (quaternion rotation), one 1920x1080 view at t = 0.5,
L1 loss against a seeded U(0,1) target.  The timed steps replay HIP graphs
of the frame (``--eager`` times the plain calls instead).

Prints ONE JSON line.  Per-stage kernel durations come from HIP events that
the library records around each stage inside the timed region (on the stream
the kernels run on); the roofline object reports the dominant stage.

``--workload cfg3`` / ``cfg4`` time the batched multi-view frames (views/s),
``cfg4`` with the autotuner's tuning, each beside the same views rendered one
per frame through the single-view path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd frames/s at 1M 7-D Beta prims, 1080p, 1 MI355X; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# Vector ALU peak in lane-operations: 256 CUs x 64 lanes per clock x 2.4 GHz
# (non-packed fp32; the kernels are built without packed fp32 instructions).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic VALU lane-operations of the rasters per unit of work, counted
# from the arithmetic itself (an FMA, add, mul, min or compare = 1; exp2,
# log2 and reciprocal = 4, they issue at quarter rate).  Only work the
# method needs is counted: the cross-lane sums, the LDS staging and the
# lanes idle under divergence are overheads of the implementation.
# Backward raster:
#   eval     (pixel, record) visited before the pixel's last contributor:
#            dy, r = A + dy (B + c dy), support test                      4
#   support  r <= rho: 1 - r, log2, fma with beta and log2 o, exp2,
#            min 0.99, alpha test                                         12
#   contrib  alpha >= 1/255: 1 - alpha, rcp (4), T/(1-alpha), weight
#            alpha T, three colour-gradient sums (3), g.c (3), g.c - g.S
#            with g.S kept per pixel, g.S += alpha (g.c - g.S)             15
#   grad     sigma < 0.99 as well: d alpha = T (g.c - g.S), s = sigma
#            d alpha, opacity and beta sums, rcp of 1 - r (4), s/(1 - r),
#            the three moment sums (4)                                    13
#   pair     per (tile, record): dx and the column terms of the tile's 16
#            pixel columns (4 each), 1/o, the ten sums turned into the
#            record-field gradients (14)                                  64 + 4 + 14
BWD_OPS = {"eval": 4, "support": 12, "contrib": 15, "grad": 13, "pair": 82}
# Forward raster: eval and support as above; contrib: T (1 - alpha) and its
# stop test, weight alpha T, three colour FMAs, the contributor count (8);
# pair: the column terms (64) and log2 o (4).
FWD_OPS = {"eval": 4, "support": 12, "contrib": 8, "pair": 68}

WORKLOADS = {
    "headline": ("headline", "1,000,000 7-D Beta primitives (quaternion rotation), one "
                             "1920x1080 view at t=0.5, forward+backward, L1 loss"),
    "cfg2": ("cfg2", "1,000,000 6-D Beta primitives, one 1920x1080 view, forward+backward, L1 loss"),
    "cfg1": ("cfg1", "500,000 6-D Beta primitives, one 1264x832 view, forward only"),
    "cfg0": ("cfg0", "2,000 3-D Beta primitives, one 128x128 view, forward+backward, L1 loss"),
    "dim10": ("dim10", "1,000,000 10-D Beta primitives (query [t, d, e0..e2], e from the view), "
                       "one 1920x1080 view at t=0.5, forward+backward, L1 loss"),
    "cfg3": ("cfg3", "2,000,000 7-D Beta primitives, 8 views of 1352x1014 (cameras on a circle, "
                     "t = k/7) in one batched frame, forward+backward, L1 loss"),
    "cfg4": ("cfg4", "4 scenes of 7-D Beta primitives (100k/500k/1.5M/3M), 32 views of uneven "
                     "resolution in one batched frame, autotuned, forward+backward, L1 loss"),
    "adam": ("headline", "optimiser step (regularisers, Adam, spatial noise) over the parameters "
                         "of 1,000,000 7-D primitives (45 rows)"),
    "relocate": ("headline", "relocation of dead primitives (opacity < 0.005, 30% of 1,000,000 "
                             "7-D primitives) to live ones drawn by opacity"),
    "ssim": ("headline", "image loss (0.8 L1 + 0.2 D-SSIM, 11x11 Gaussian window) and its gradient "
                         "on one 1920x1080 view"),
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_sources_digest() -> str:
    """sha256 over the HIP sources and the ABI header (a profile's counters
    describe the kernels built from exactly these sources)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_03312_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".hpp")))
    files.append(os.path.join(ROOT, "include", "ubs.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary in profiles/, if it was taken on the current sources."""
    import re
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    digest = kernel_sources_digest()
    for m in re.finditer(r"<!-- traffic kernel=(\w+) bytes=(\d+) sources=(\w+) -->", open(path).read()):
        if m.group(1) == kernel and m.group(3) == digest:
            return int(m.group(2))
    return None


def stage_bytes(stage: str, c: dict) -> float:
    """Algorithmic HBM bytes of one launch of a stage: the bytes its inputs and
    outputs must move at least once (records 48 B, pairs 8-12 B, pixels 12-32 B,
    parameters 4 B per row entry)."""
    P, F, R, Pv, K, A, G = c["P"], c["F"], c["R"], c["Pv"], c["K"], c["A"], c["G"]
    return {
        "preprocess": 4.0 * F * P + 48.0 * R,
        "bin_count": 36.0 * R + 12.0 * K + 4.0 * G,
        "scan": 12.0 * G,
        # the emitting pass runs only when a tile outgrew its slot block
        "bin_emit": (36.0 * R + 12.0 * K) * c.get("spill", 1),
        "sort": 20.0 * K + 16.0 * G,
        "raster_fwd": 52.0 * K + 20.0 * A + 8.0 * G,
        "grad_clear": 40.0 * R,
        "raster_bwd": 92.0 * K + 32.0 * A + 8.0 * G,
        # live primitives' parameters read (Pv bounds them), every gradient
        # written, liveness flags and the live records' gradients read
        "pre_bwd": 4.0 * F * Pv + 4.0 * F * P + 8.0 * R + 40.0 * Pv,
    }[stage]


def raster_bwd_work(r, view, n_pairs: int, tile: int = 16, chunk: int = 8192) -> dict:
    """Counts the backward raster's units of work on the frame left in the
    workspace (one view, 16x16 tiles), with the same per-pixel decisions in
    float32 torch ops on the device, outside the timed region."""
    import torch
    rec = r.records()
    rng = r.ranges().long()
    vals = r.sorted_pairs(n_pairs)[1].long()
    last = r.ncontrib().long()
    W, H = view.width, view.height
    tiles_x = (W + tile - 1) // tile
    counts = rng[:, 1] - rng[:, 0]
    tile_of = torch.repeat_interleave(torch.arange(rng.shape[0], device=rec.device), counts)
    pos_all = torch.arange(n_pairs, device=rec.device) - rng[tile_of, 0]
    lane = torch.arange(tile * tile, device=rec.device)
    lx, ly = lane % tile, lane // tile
    tot = {k: 0 for k in ("eval", "support", "contrib", "grad", "pair", "pairs_active")}
    tot["pair"] = n_pairs
    for c0 in range(0, n_pairs, chunk):
        t = tile_of[c0:c0 + chunk]
        pos = pos_all[c0:c0 + chunk, None]
        g = rec[vals[c0:c0 + chunk]]
        px = (t % tiles_x)[:, None] * tile + lx[None]
        py = (t // tiles_x)[:, None] * tile + ly[None]
        inside = (px < W) & (py < H)
        pix = (py.clamp(max=H - 1) * W + px.clamp(max=W - 1))
        ev = inside & (pos < last[pix])
        dx = px.float() + 0.5 - g[:, 0:1]
        dy = py.float() + 0.5 - g[:, 1:2]
        rr = g[:, 2:3] * dx * dx + 2.0 * g[:, 3:4] * dx * dy + g[:, 4:5] * dy * dy
        sup = ev & (rr <= g[:, 5:6])
        sigma = g[:, 6:7] * torch.clamp(1.0 - rr, min=0.0) ** g[:, 7:8]
        con = sup & (torch.clamp(sigma, max=0.99) >= 1.0 / 255.0)
        tot["eval"] += int(ev.sum())
        tot["support"] += int(sup.sum())
        tot["contrib"] += int(con.sum())
        tot["grad"] += int((con & (sigma < 0.99)).sum())
        tot["pairs_active"] += int(con.any(dim=1).sum())
    tot["lane_ops"] = sum(BWD_OPS[k] * tot[k] for k in BWD_OPS)
    # every visit is of a record before its pixel's last contributor: the
    # visits must add up to the sum of the per-pixel contributor counts
    tot["sum_ncontrib"] = int(last[:W * H].sum())
    return tot


def _oracle_band(job):
    """One row band of the oracle's compositing, forward and adjoint, in a
    worker process of its own (the oracle's C code is single-threaded);
    returns the seconds it took."""
    path, W, H, y0, y1 = job
    import numpy as np
    from oracle import raster as oraster
    rec = np.load(path)
    dimg = np.zeros((H, W, 3))
    dimg[y0:y1] = np.random.default_rng(y0).normal(size=(y1 - y0, W, 3)) * 1e-6
    t0 = time.perf_counter()
    oraster.render_fwd(rec, W, H, rows=(y0, y1))
    oraster.render_bwd(rec, W, H, dimg, rows=(y0, y1))
    return time.perf_counter() - t0


def host_cpu() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable": usable}


def cpu_baseline(cfg, rows: int = 32, sub: int = 100_000, max_workers: int = 16) -> dict:
    """The oracle timed on a bounded sample of the same frame, on one host
    thread and on all the host threads this process may use (at most
    max_workers): the per-primitive steps (torch float64, forward and
    backward) on `sub` primitives, and the compositing (C, forward and
    adjoint) on `rows` rows in one band per worker, spread evenly over the
    image; both scaled linearly to the whole frame."""
    import multiprocessing as mp
    import tempfile

    import numpy as np
    import torch
    from oracle import preprocess as opp

    cpu = host_cpu()
    workers = max(1, min(max_workers, cpu["usable"] or 1))
    sc, view = cfg["scenes"][0], cfg["views"][0]
    n = sc.n
    sub = min(sub, n)
    t_pre = {}
    for threads in (1, workers):
        torch.set_num_threads(threads)
        Ps = torch.tensor(sc.params[:, :sub].astype(np.float64), requires_grad=True)
        t0 = time.perf_counter()
        out = opp.preprocess(Ps, sc.dim, sc.rot, view)
        out["rec"].backward(torch.ones_like(out["rec"]))
        t_pre[threads] = (time.perf_counter() - t0) * (n / sub)
    # records of every primitive (setup for the compositing sample, untimed)
    recs = []
    with torch.no_grad():
        for k in range(0, n, 200_000):
            P = torch.tensor(sc.params[:, k:k + 200_000].astype(np.float64))
            recs.append(opp.preprocess(P, sc.dim, sc.rot, view)["rec"].numpy())
    H, W = view.height, view.width
    per = max(1, rows // workers)
    starts = [int(round((k + 0.5) * H / workers - per / 2)) for k in range(workers)]
    jobs_rows = [(max(0, y), min(H, max(0, y) + per)) for y in starts]
    sampled = sum(y1 - y0 for y0, y1 in jobs_rows)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "records.npy")
        np.save(path, np.concatenate(recs))
        jobs = [(path, W, H, y0, y1) for y0, y1 in jobs_rows]
        with mp.get_context("spawn").Pool(workers) as pool:
            pool.map(_oracle_band, jobs[:1])          # start-up of the workers, untimed
            t0 = time.perf_counter()
            band_s = pool.map(_oracle_band, jobs)
            wall = time.perf_counter() - t0
    scale = H / sampled
    one = t_pre[1] + sum(band_s) * scale
    many = t_pre[workers] + wall * scale
    return {"value": 1.0 / many, "unit": "frames/s", "cores": workers, "kind": "oracle",
            "single_thread_value": 1.0 / one, "cpu_model": cpu["model"], "nproc": cpu["nproc"],
            "usable_cpus": cpu["usable"],
            "sample": (f"per-primitive steps fwd+bwd (torch float64) on {sub:,} of {n:,} primitives "
                       f"scaled x{n / sub:g}; compositing fwd+bwd (C float64, one process per band) "
                       f"on {len(jobs_rows)} bands of {per} rows spread over {H} scaled "
                       f"x{scale:.1f}; value: {workers} threads/processes, single_thread_value: "
                       f"the same sample on one thread")}


def timed_steps(gf, steps: int, eager: bool):
    """Times `steps` frames; returns ms per step.  Graph replays or plain calls."""
    import torch
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        gf.step() if eager else gf.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def timed_stages(gf, steps: int):
    """Per-stage durations (mean ms) of `steps` plain-call frames, from HIP
    events the library records around each stage on the frame's stream; also
    returns the ms per step of those frames."""
    import numpy as np
    import torch
    from paper_2510_03312_amd.timing import StageTimer

    timer = StageTimer(steps)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(steps):
        timer.attach(gf.frame.c, k)
        gf.step()
    e1.record(stream)
    torch.cuda.synchronize()
    timer.detach(gf.frame.c)
    stages = {}
    for k in range(steps):
        for s, v in timer.elapsed_ms(k).items():
            stages.setdefault(s, []).append(v)
    timer.close()
    return e0.elapsed_time(e1) / steps, {s: float(np.mean(v)) for s, v in stages.items()}


def run_single(args, name, desc):
    import torch
    from paper_2510_03312_amd import Renderer, SceneRef, Tuning, UBS_TUNE_PRE_FP32
    from paper_2510_03312_amd.renderer import GraphFrame
    from synth import make_config

    cfg = make_config(name)
    sc, view = cfg["scenes"][0], cfg["views"][0]
    dev = torch.device("cuda:0")
    params = torch.from_numpy(sc.params).to(dev)
    target = torch.from_numpy(cfg["targets"][0]).to(dev).view(-1, 3).contiguous()
    backward = cfg["mode"] == "fwdbwd"
    r = Renderer(Tuning(flags=UBS_TUNE_PRE_FP32 if args.pre_fp32 else 0))
    log("[bench] sizing and capturing the frame")
    gf = GraphFrame(r, [SceneRef(params, sc.dim, sc.rot)], [view],
                    l1_target=target if backward else None, backward=backward)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        gf.step() if args.eager else gf.replay()
    torch.cuda.synchronize()
    st = r.status()
    assert not st["overflow"] and not st["sort_stalled"], st
    log(f"[bench] pairs {st['pairs_needed']:,} visible {st['n_visible']:,}; timing {args.steps} steps")
    t_wall = time.perf_counter()
    ms = timed_steps(gf, args.steps, args.eager)
    t_wall = time.perf_counter() - t_wall
    # per-stage kernel durations: the same frame as plain calls with the
    # library's stage events (kernel durations do not depend on the launch
    # mode; graph replays only remove the launch gaps between them)
    log("[bench] per-stage timing")
    eager_ms, stages_ms = timed_stages(gf, args.steps)
    st = r.status()
    assert not st["overflow"] and not st["sort_stalled"], st
    lay = r.layout
    c = {"P": sc.n, "F": int(sc.params.shape[0]), "R": lay.n_records, "Pv": st["n_visible"],
         "K": st["pairs_needed"], "A": lay.n_pixels, "G": lay.n_tiles, "spill": st["spill"]}
    dom = max(stages_ms, key=stages_ms.get)
    ach = stage_bytes(dom, c) / (stages_ms[dom] * 1e-3) / 1e9
    frame_bytes = sum(stage_bytes(s, c) for s in stages_ms)
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5),
            "traffic": recorded_traffic(name, dom)}
    work = raster_bwd_work(r, view, c["K"]) if view.width * view.height > 0 else None
    if dom == "raster_bwd" and work is not None:
        # the backward raster is bound by vector ALU work, not by bytes
        tops = work["lane_ops"] / (stages_ms[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(tops, 3), "peak": VALU_PEAK_TOPS,
                "unit": "T lane-ops/s", "frac": round(tops / VALU_PEAK_TOPS, 4),
                "traffic": recorded_traffic(name, dom), "work": work,
                "hbm": {"achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 5)}}
    # the frame against both rooflines: B = compulsory HBM bytes of the
    # frame (8 F P for params in and dparams out, Pv (176 + 4 F) for the
    # records, 2-D gradients and the visible parameters read again, 172 K
    # for keys, values, record gathers and atomics, 76 A for the pixels,
    # 16 G for the tile ranges); ALU = the rasters' algorithmic lane-ops
    # (the per-primitive float64 work is left out, so T_bound is a lower
    # bound of the frame time)
    F, P, Pv, K, A, G = c["F"], c["P"], c["Pv"], c["K"], c["A"], c["G"]
    B = (8.0 * F * P if backward else 4.0 * F * P) + Pv * (176.0 + 4.0 * F) + 172.0 * K + 76.0 * A + 16.0 * G
    alu = 0.0
    if work is not None:
        alu = sum(FWD_OPS[k] * work[k] for k in FWD_OPS)
        if backward:
            alu += work["lane_ops"]
    t_s = ms * 1e-3
    t_hbm, t_alu = B / (HBM_PEAK_GBS * 1e9), alu / (VALU_PEAK_TOPS * 1e12)
    frame = {"bytes": B, "hbm_frac": round(t_hbm / t_s, 4), "alu_lane_ops": alu,
             "alu_frac": round(t_alu / t_s, 4), "t_bound_ms": round(max(t_hbm, t_alu) * 1e3, 4),
             "t_bound_frac": round(max(t_hbm, t_alu) / t_s, 4)}
    res = {
        "metric": METRIC if name == "headline" else f"{'fwd+bwd' if backward else 'fwd'} frames/s ({name})",
        "value": round(1000.0 / ms, 3), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "primitives": sc.n, "dim": sc.dim, "params_per_prim": c["F"],
                   "width": view.width, "height": view.height, "views": 1, "pairs": c["K"],
                   "visible": c["Pv"], "launch": "eager" if args.eager else "hip-graph"},
        "roofline": roof,
        "kernel_sources": kernel_sources_digest(),
        "frame_hbm_frac": round(frame_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
        "frame": frame,
        "stages_ms": {k: round(v, 4) for k, v in stages_ms.items()},
        "eager_ms_per_step": round(eager_ms, 4),
        "per_primitive_math": "f32" if args.pre_fp32 else "f64",
        "wall_s": round(t_wall, 3),
    }
    if not args.no_cpu_baseline and name == "headline":
        log("[bench] timing the oracle on a bounded CPU sample")
        res["cpu_baseline"] = cpu_baseline(cfg)
        for k in ("value", "single_thread_value"):
            res["cpu_baseline"][k] = round(res["cpu_baseline"][k], 6)
    return res


def run_batched(args, name, desc):
    import torch
    from paper_2510_03312_amd import Renderer, SceneRef, Tuning
    from paper_2510_03312_amd.autotune import autotune
    from paper_2510_03312_amd.renderer import GraphFrame
    from synth import make_config

    cfg = make_config(name)
    dev = torch.device("cuda:0")
    scenes = [SceneRef(torch.from_numpy(s.params).to(dev), s.dim, s.rot) for s in cfg["scenes"]]
    views = cfg["views"]
    target = torch.cat([torch.from_numpy(t).view(-1, 3) for t in cfg["targets"]]).to(dev)
    tuning, tune_ms = Tuning(), None
    if name == "cfg4":
        log("[bench] autotuning")
        tuning, tune_ms = autotune(scenes, views, l1_target=target, steps=2)
    batched, single = {}, {}
    for mode in ("fwdbwd", "fwd"):
        backward = mode == "fwdbwd"
        log(f"[bench] batched {mode}")
        gf = GraphFrame(Renderer(Tuning(**tuning.__dict__)), scenes, views,
                        l1_target=target if backward else None, backward=backward)
        for _ in range(args.warmup):
            gf.replay()
        ms = timed_steps(gf, args.steps, args.eager)
        _, stages = timed_stages(gf, max(2, args.steps // 2))
        st = gf.status()
        assert not st["overflow"] and not st["sort_stalled"], st
        batched[mode] = {"views_per_s": round(len(views) * 1000.0 / ms, 2), "ms_per_frame": round(ms, 4),
                         "stages_ms": {k: round(v, 4) for k, v in stages.items()},
                         "tile_slots": gf.r.tile_slots or 256, "spill": st["spill"]}
        del gf
        torch.cuda.empty_cache()
        # the same views one per frame through the single-view path
        log(f"[bench] single-view path {mode}")
        frames, base = [], 0
        for v in views:
            n = v.width * v.height
            tv = target[base:base + n].contiguous()
            base += n
            frames.append(GraphFrame(Renderer(Tuning(**tuning.__dict__)), scenes, [v],
                                     l1_target=tv if backward else None, backward=backward))
        reps = max(1, args.steps // 4)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            for f in frames:
                f.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        single[mode] = {"views_per_s": round(len(views) * 1000.0 / ms, 2), "ms_per_batch": round(ms, 4)}
        del frames
        torch.cuda.empty_cache()
    return {
        "metric": f"batched fwd+bwd views/s ({name})", "value": batched["fwdbwd"]["views_per_s"],
        "unit": "views/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": batched["fwdbwd"]["ms_per_frame"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "views": len(views), "scenes": len(scenes),
                   "primitives": [s.n for s in scenes],
                   "tuning": {"tile": [tuning.tile_w, tuning.tile_h],
                              "batch_depth": tuning.batch_depth, "persistent": bool(tuning.flags & 1)}},
        "batched": batched, "single_view_path": single, "autotune_ms": tune_ms,
    }


def run_adam(args, name, desc):
    """The optimiser step alone: one streaming pass over params, dparams, m,
    v (and three noise rows), writing params, m, v."""
    import torch
    from paper_2510_03312_amd.optim import adam_step
    from synth import make_config

    cfg = make_config(name)
    sc = cfg["scenes"][0]
    dev = torch.device("cuda:0")
    F, n = sc.params.shape
    params = torch.from_numpy(sc.params).to(dev)
    g = torch.randn(F, n, device=dev) * 1e-3
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    noise = torch.randn(3, n, device=dev)
    for t in range(1, args.warmup + 1):
        adam_step(params, g, m, v, t, sc.dim, sc.rot, noise=noise)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for t in range(args.warmup + 1, args.warmup + 1 + args.steps):
        adam_step(params, g, m, v, t, sc.dim, sc.rot, noise=noise)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nbytes = 4.0 * F * n * 7 + 4.0 * 3 * n   # read p, g, m, v; write p, m, v; read noise
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {
        "metric": "optimiser steps/s (Adam + regularisers + noise, 1M 7-D prims)",
        "value": round(1000.0 / ms, 2), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "primitives": n, "rows": F},
        "roofline": {"bound": "hbm", "kernel": "adam", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_step": nbytes},
    }


def run_relocate(args, name, desc):
    """Relocation alone, on a fresh copy of the same state each step (the
    copy is outside the timed region: one stream, events around the call)."""
    import numpy as np
    import torch
    from paper_2510_03312_amd.optim import relocate
    from synth import make_config

    cfg = make_config(name)
    sc = cfg["scenes"][0]
    dev = torch.device("cuda:0")
    F, n = sc.params.shape
    P = sc.params.copy()
    rng = np.random.default_rng(7)
    o_row = F - 4          # the opacity row: followed only by the three colour rows
    P[o_row] = np.where(rng.uniform(size=n) < 0.3, 0.001, P[o_row]).astype(np.float32)
    base = torch.from_numpy(P).to(dev)
    params = base.clone()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    u = torch.from_numpy(rng.uniform(size=n)).to(dev)
    total = 0.0
    n_dead = 0
    for k in range(args.warmup + args.steps):
        params.copy_(base)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, nd = relocate(params, m, v, u, sc.dim, sc.rot)
        e1.record()
        torch.cuda.synchronize()
        if k >= args.warmup:
            total += e0.elapsed_time(e1)
        n_dead = int(nd.item())
    ms = total / args.steps
    # every row read once, cdf / flags / scans, and per dead slot its source
    # column read and its own column plus both columns' moments written
    nbytes = 4.0 * F * n + 40.0 * n + n_dead * (4.0 * F * 6 + 24.0)
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {
        "metric": "relocation passes/s (1M 7-D prims, 30% dead)", "value": round(1000.0 / ms, 2),
        "unit": "passes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "primitives": n, "rows": F, "dead": n_dead},
        "roofline": {"bound": "hbm", "kernel": "relocate", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_step": nbytes},
    }


def run_ssim(args, name, desc):
    """The image loss alone on a 1080p image / target pair."""
    import numpy as np
    import torch
    from paper_2510_03312_amd.optim import ssim_loss
    from synth import make_config

    cfg = make_config(name)
    view = cfg["views"][0]
    A = view.width * view.height
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(3)
    img = torch.from_numpy(rng.uniform(size=(A, 3)).astype(np.float32)).to(dev)
    tgt = torch.from_numpy(cfg["targets"][0].reshape(-1, 3).astype(np.float32)).to(dev)
    for _ in range(args.warmup):
        ssim_loss(img, tgt, [view])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ssim_loss(img, tgt, [view])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # image and target read, gradient written, the per-pixel partials
    # written once and read once
    nbytes = A * (24.0 + 12.0 + 72.0)
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {
        "metric": "image loss + gradient evaluations/s (L1 + D-SSIM, 1080p)",
        "value": round(1000.0 / ms, 2), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "width": view.width, "height": view.height},
        "roofline": {"bound": "hbm", "kernel": "ssim", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_step": nbytes},
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="headline", choices=sorted(WORKLOADS))
    ap.add_argument("--eager", action="store_true", help="time plain calls instead of graph replays")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pre-fp32", action="store_true",
                    help="per-primitive math in float32 instead of float64")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="before timing, run a 256 MiB device copy (torch) whose known "
                         "traffic calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested): this build runs "
              "and reports a single MI355X; multi-GPU sharding by view is a design note only.",
              file=sys.stderr)
        return 2
    import torch
    torch.cuda.set_device(0)
    name, desc = WORKLOADS[args.workload]
    log(f"[bench] workload {args.workload}")
    if args.workload == "adam":
        res = run_adam(args, name, desc)
    elif args.workload == "relocate":
        res = run_relocate(args, name, desc)
    elif args.workload == "ssim":
        res = run_ssim(args, name, desc)
    elif name in ("cfg3", "cfg4"):
        res = run_batched(args, name, desc)
    else:
        res = run_single(args, name, desc)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
