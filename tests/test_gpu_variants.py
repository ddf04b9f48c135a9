"""Parity of the Sec. 5.3 ablation variants (tuning flags
UBS_TUNE_NO_BETA_COND / UBS_TUNE_NO_BETA_OPACITY) with the oracle's
variants, through the C ABI: records, pixels and parameter gradients, to
the bars of test_gpu_parity.py."""
import math

import numpy as np
import pytest

from _gpu_common import (GRAD_BLOCKS, compare_images, gpu_ready, gpu_render, grad_violations,
                         log, oracle_view)
from oracle import preprocess as opp
from synth import make_config

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]

VARIANTS = {
    "no_beta_cond": (4, (opp.NO_BETA_CONDITION,)),
    "no_beta_opacity": (8, (opp.NO_BETA_OPACITY,)),
    "both": (12, (opp.NO_BETA_CONDITION, opp.NO_BETA_OPACITY)),
}
CASES = {
    "headline_7d": ("headline", dict(n=30000, width=240, height=135)),
    "cfg1_6d_skew": ("cfg1", dict(n=12000, width=96, height=160, rot=1)),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("variant", list(VARIANTS))
def test_variant_parity(case, variant):
    from paper_2510_03312_amd import Tuning
    flags, ovar = VARIANTS[variant]
    base, kw = CASES[case]
    log(f"[variant] {variant} {case}")
    cfg = make_config(base, **kw)
    sc, view = cfg["scenes"][0], cfg["views"][0]
    o0 = oracle_view(cfg, 0, variant=ovar)
    # records
    g0 = gpu_render(cfg, Tuning(flags=flags))
    rg, ro = g0["records"], o0["rec"]
    vg, vo, amb = rg[:, 5] > 0, o0["valid"], o0["amb"]
    assert ((vg != vo) & ~amb).sum() == 0
    both = vg & vo
    for k, name in enumerate(opp.REC_FIELDS):
        a, b = rg[both, k].astype(np.float64), ro[both, k]
        err = np.abs(a - b) / (np.abs(b) + np.median(np.abs(b)) + 1e-12)
        assert err.max() < 2e-5, (name, err.max())
    # pixels
    err, nflag, nbad = compare_images(g0["images"][0], o0["image"], o0["flags"], 1e-4)
    log(f"  pixels max err {err:.3g}, flagged {nflag}")
    assert nbad == 0 and nflag <= 0.01 * o0["flags"].size
    # gradients
    rng = np.random.default_rng(3)
    ok = o0["flags"] == 0
    dimg = rng.normal(size=(view.height, view.width, 3)) * ok[..., None] / math.sqrt(ok.size)
    o = oracle_view(cfg, 0, d_image=dimg, variant=ovar)
    g = gpu_render(cfg, Tuning(flags=flags), want_grad=True, d_images=[dimg])
    sl = opp.field_slices(sc.dim, sc.rot)
    bad = 0
    for name in GRAD_BLOCKS:
        s = sl[name]
        if s.stop <= s.start:
            continue
        v = grad_violations(g["dparams"][0][s], o["dparams"][s])
        if v.sum():
            log(f"  {name}: {int(v.sum())} violations")
        bad += int(v.sum())
    assert bad == 0
    if ovar == (opp.NO_BETA_CONDITION, opp.NO_BETA_OPACITY):
        # neither modulation: b_q has no influence at all
        assert np.all(g["dparams"][0][sl["b_q"]] == 0.0)
