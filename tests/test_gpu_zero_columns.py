"""Every column of dparams is written by ubs_render_bwd: the gradients of the
primitives some view kept, zeros for the others (culled in every view, or
in a scene no view sees).  dparams starts as NaN here, so a column that
nobody writes shows up; the written values must match a plain backward."""
import numpy as np
import pytest
import torch

from _gpu_common import gpu_ready, grad_violations, log, to_dev
from synth import make_config, make_scene, make_view

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def _backward_twice(cfg, tuning=None):
    """(dparams written over NaN, dparams of a plain backward, live flags)."""
    from paper_2510_03312_amd import Renderer, SceneRef, Tuning
    r = Renderer(tuning or Tuning())
    scenes = [SceneRef(to_dev(s.params), s.dim, s.rot) for s in cfg["scenes"]]
    image, _ = r.forward(scenes, cfg["views"])
    d = torch.full_like(image, 1e-3)
    plain = [g.cpu().numpy() for g in r.backward(d)]
    frame = r.frame
    nan = []
    for k, s in enumerate(frame.scenes):
        g = torch.full_like(s.params, float("nan"))
        frame.set_dparams(k, g)
        nan.append(g)
    r.render_bwd(frame, d, None, None, None)
    torch.cuda.synchronize()
    rec = r.live_records().cpu().numpy()
    live = [np.zeros(s.n, dtype=bool) for s in cfg["scenes"]]
    base = 0
    for v in cfg["views"]:
        n = cfg["scenes"][v.scene].n
        live[v.scene] |= rec[base:base + n, 5] > 0
        base += n
    return [g.cpu().numpy() for g in nan], plain, live


def _check(cfg, tuning=None):
    got, plain, live = _backward_twice(cfg, tuning)
    for k, (g, p, lv) in enumerate(zip(got, plain, live)):
        assert np.isfinite(g).all(), (k, np.argwhere(~np.isfinite(g))[:5])
        assert np.all(g[:, ~lv] == 0.0), k
        assert grad_violations(g, p.astype(np.float64), rtol=1e-4, floor=1e-3).sum() == 0, k
    return live


def test_single_scene_every_column_written():
    log("[zero] single scene")
    live = _check(make_config("headline", n=30000, width=240, height=135))
    assert 0 < live[0].sum() < live[0].size


def test_persistent_raster_every_column_written():
    from paper_2510_03312_amd import UBS_TUNE_PERSISTENT, Tuning
    log("[zero] persistent")
    _check(make_config("headline", n=30000, width=240, height=135), Tuning(flags=UBS_TUNE_PERSISTENT))


def test_eleven_scenes_one_unseen_every_column_written():
    log("[zero] 11 scenes, one unseen")
    scenes = [make_scene(7, 3000 + 100 * k, 10 + k, dist="cfg3") for k in range(11)]
    views = [make_view(96, 64, scene=k, time=0.1 * k) for k in range(10)]
    cfg = {"scenes": scenes, "views": views}
    live = _check(cfg)
    assert not live[10].any()
    assert all(0 < lv.sum() < lv.size for lv in live[:10])


def test_one_tile_many_primitives_every_column_written():
    log("[zero] one tile, 40k primitives")
    live = _check(make_config("headline", n=40000, width=16, height=16))
    assert live[0].sum() < live[0].size
