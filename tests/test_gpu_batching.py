"""Batching, launch modes, graph capture and the autotuner, through the C ABI.

Per-pixel arithmetic does not depend on the tile shape, the LDS batch depth
or the launch mode, so images must be bit-identical across them; gradients
are sums of float atomics in different orders and agree to 1e-4.
"""
import numpy as np
import pytest
import torch

from _gpu_common import gpu_ready, gpu_render, grad_violations, log, to_dev
from synth import make_config

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def _grads_close(a, b):
    return grad_violations(a, b.astype(np.float64), rtol=1e-4, floor=1e-3).sum() == 0


@pytest.mark.parametrize("tile", [(16, 16), (16, 8), (8, 8), (32, 16)])
@pytest.mark.parametrize("batch", [64, 128, 256])
@pytest.mark.parametrize("persistent", [False, True])
def test_tuning_variants_render_identically(tile, batch, persistent):
    from paper_2510_03312_amd import UBS_TUNE_PERSISTENT, Tuning
    log(f"[tuning] tile {tile} batch {batch} persistent {persistent}")
    cfg = make_config("headline", n=30000, width=240, height=135)
    d = [np.full((135, 240, 3), 1e-3)]
    ref = gpu_render(cfg, want_grad=True, d_images=d)
    t = Tuning(tile_w=tile[0], tile_h=tile[1], batch_depth=batch,
               flags=UBS_TUNE_PERSISTENT if persistent else 0)
    g = gpu_render(cfg, t, want_grad=True, d_images=d)
    np.testing.assert_array_equal(g["images"][0], ref["images"][0])
    np.testing.assert_array_equal(g["t_final"][0], ref["t_final"][0])
    assert _grads_close(g["dparams"][0], ref["dparams"][0])


def test_persistent_multi_view_batch_matches_grid_launch():
    from paper_2510_03312_amd import UBS_TUNE_PERSISTENT, Tuning
    log("[tuning] persistent, 8 views")
    cfg = make_config("cfg3", n=20000, width=200, height=150)
    d = [np.full((150, 200, 3), 1e-3)] * 8
    a = gpu_render(cfg, want_grad=True, d_images=d)
    b = gpu_render(cfg, Tuning(flags=UBS_TUNE_PERSISTENT), want_grad=True, d_images=d)
    for k in range(8):
        np.testing.assert_array_equal(a["images"][k], b["images"][k])
    assert _grads_close(b["dparams"][0], a["dparams"][0])


def test_graph_replays_match_eager_frames():
    """Replays with eager work and synchronisations in between; every replay
    is checked against the eager result."""
    from paper_2510_03312_amd import Renderer, SceneRef
    from paper_2510_03312_amd.renderer import GraphFrame
    log("[graph] replays")
    cfg = make_config("headline", n=40000, width=320, height=180)
    sc = cfg["scenes"][0]
    params = to_dev(sc.params)
    target = to_dev(cfg["targets"][0]).view(-1, 3).contiguous()
    eager = gpu_render(cfg, want_grad=True, l1=True)
    gf = GraphFrame(Renderer(), [SceneRef(params, sc.dim, sc.rot)], cfg["views"], l1_target=target)
    for rep in range(4):
        gf.replay()
        torch.cuda.synchronize()
        img = gf.image.view(180, 320, 3).cpu().numpy()
        np.testing.assert_array_equal(img, eager["images"][0])
        assert _grads_close(gf.dparams[0].cpu().numpy(), eager["dparams"][0])
        assert not gf.status()["overflow"]
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        float((x * 2).sum())
        torch.cuda.synchronize()
    # parameters changed in place: the next replay renders the new values
    with torch.no_grad():
        params[sc.params.shape[0] - 3:] = 0.25      # all colours
    gf.replay()
    torch.cuda.synchronize()
    cfg2 = make_config("headline", n=40000, width=320, height=180)
    cfg2["scenes"][0].params[sc.params.shape[0] - 3:] = 0.25
    ref2 = gpu_render(cfg2)
    np.testing.assert_array_equal(gf.image.view(180, 320, 3).cpu().numpy(), ref2["images"][0])


def test_autotuner_picks_a_valid_tuning(tmp_path):
    from paper_2510_03312_amd import SceneRef
    from paper_2510_03312_amd.autotune import autotune, candidates
    log("[autotune]")
    cfg = make_config("cfg4", scene_sizes=(2000, 4000, 6000, 8000), n_views=4)
    for v in cfg["views"]:
        v.width, v.height, v.cx, v.cy = 128, 96, 64.0, 48.0
        v.fx = v.fy = float(np.float32(64.0 / np.tan(np.radians(30))))
    scenes = [SceneRef(to_dev(s.params), s.dim, s.rot) for s in cfg["scenes"]]
    cands = candidates()[:6]
    best, timings = autotune(scenes, cfg["views"], cache_path=str(tmp_path / "c.json"),
                             steps=1, cands=cands)
    assert len(timings) == 6 and all(t > 0 for t in timings.values())
    best2, _ = autotune(scenes, cfg["views"], cache_path=str(tmp_path / "c.json"))
    assert best2 == best
