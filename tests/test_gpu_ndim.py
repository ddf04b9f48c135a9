"""Primitives beyond 7-D (query [t, d, e], e from the view) on the GPU,
through the C ABI, against the fp64 oracle: records, pixels and gradients
to the frame's bars, and the reduction of uncorrelated further dimensions
queried at their mean to the 7-D primitive."""
import math

import numpy as np
import pytest

from _gpu_common import (compare_images, gpu_ready, gpu_render, grad_violations, log,
                         oracle_view)
from oracle import preprocess as opp
from synth import make_scene, make_view

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]

CASES = {
    "8d_quat": (8, 0, 20000, 240, 135, (0.4, 0.0, 0.0)),
    "9d_skew": (9, 1, 15000, 200, 136, (0.3, 0.8, 0.0)),
    "10d_quat_ragged": (10, 0, 12000, 150, 90, (0.2, 0.7, 0.5)),
}


def _cfg(case):
    dim, rot, n, W, H, q = CASES[case]
    view = make_view(W, H, time=0.5)
    view.query = q
    return {"scenes": [make_scene(dim, n, seed=dim + 10 * rot, dist="cfg3", rot=rot)],
            "views": [view]}


@pytest.mark.parametrize("case", list(CASES))
def test_ndim_records_pixels_and_gradients_match_oracle(case):
    log(f"[ndim] {case}")
    cfg = _cfg(case)
    view, sc = cfg["views"][0], cfg["scenes"][0]
    o0 = oracle_view(cfg, 0)
    rng = np.random.default_rng(5)
    ok = o0["flags"] == 0
    dimg = rng.normal(size=(view.height, view.width, 3)) * ok[..., None] / math.sqrt(ok.size)
    o = oracle_view(cfg, 0, d_image=dimg)
    g = gpu_render(cfg, want_grad=True, d_images=[dimg])
    # records
    rg, ro = g["records"], o0["rec"]
    vg, vo, amb = rg[:, 5] > 0, o0["valid"], o0["amb"]
    assert ((vg != vo) & ~amb).sum() == 0
    both = vg & vo
    assert both.sum() > 50
    for k, name in enumerate(opp.REC_FIELDS):
        a, b = rg[both, k].astype(np.float64), ro[both, k]
        scale = np.median(np.abs(b)) + 1e-12
        assert (np.abs(a - b) / (np.abs(b) + scale)).max() < 2e-5, name
    # pixels
    err, nflag, nbad = compare_images(g["images"][0], o0["image"], o0["flags"], 1e-4)
    log(f"  pixels: max err {err:.3g}, flagged {nflag}")
    assert nbad == 0
    # gradients, every parameter block
    sl = opp.field_slices(sc.dim, sc.rot)
    bad = 0
    for name, s in sl.items():
        if name == "_F" or s.stop == s.start:
            continue
        v = grad_violations(g["dparams"][0][s], o["dparams"][s])
        log(f"  {name}: violations {int(v.sum())}")
        bad += int(v.sum())
    assert bad == 0


def test_uncorrelated_dimension_at_its_mean_renders_like_7d():
    log("[ndim] 8-D reduction to 7-D")
    sc7 = make_scene(7, 20000, seed=3, dist="cfg3")
    view = make_view(200, 150, time=0.35)
    P7 = sc7.params.astype(np.float64)
    s7, s8 = opp.field_slices(7, 0), opp.field_slices(8, 0)
    n = sc7.n
    P8 = np.zeros((opp.n_params(8, 0), n))
    for k in ("mu_x", "rot", "log_s_x", "b_x", "o", "rgb"):
        P8[s8[k]] = P7[s7[k]]
    P8[s8["mu_q"]] = np.concatenate([P7[s7["mu_q"]], np.full((1, n), 0.6)])
    P8[s8["b_q"]] = np.concatenate([P7[s7["b_q"]], np.full((1, n), 0.5)])
    P8[s8["L_qx"]] = np.concatenate([P7[s7["L_qx"]], np.zeros((3, n))])
    P8[s8["L_q"]] = np.concatenate([P7[s7["L_q"]], np.zeros((4, n)), np.full((1, n), np.log(0.7))])
    view.query = (0.6, 0.0, 0.0)
    sc8 = type(sc7)(dim=8, rot=0, params=P8.astype(np.float32))
    a = gpu_render({"scenes": [sc7], "views": [view]})
    b = gpu_render({"scenes": [sc8], "views": [view]})
    assert np.abs(a["images"][0] - b["images"][0]).max() <= 1e-5
    assert np.abs(a["t_final"][0] - b["t_final"][0]).max() <= 1e-5
