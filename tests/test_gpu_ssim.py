"""Parity of the fused loss (ubs_ssim_loss: (1 - lambda) L1 + lambda D-SSIM,
Sec. 4.5) with the float64 oracle, through the C ABI, on ragged multi-view
frames and a 1080p view.

Bar (float32 statistics: the local variances subtract squares, so they carry
~1e-7 absolute error against the C2 = 9e-4 floor of the denominator): loss
within 1e-5 relative, gradient within 1e-3 of its largest entry (plus 1e-3
relative); the L1 sign at exact ties is not compared (sign(0) = 0 on both
sides only for bit-equal inputs)."""
import numpy as np
import pytest
import torch

from _gpu_common import gpu_ready, log, to_dev
from oracle import ssim as oss

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


class _V:
    def __init__(self, w, h):
        self.width, self.height = w, h


def _check(sizes, seed, lam, noise=0.15):
    from paper_2510_03312_amd.optim import ssim_loss
    rng = np.random.default_rng(seed)
    imgs = [rng.uniform(size=(h, w, 3)).astype(np.float32) for w, h in sizes]
    tgts = [np.clip(x + noise * rng.normal(size=x.shape), 0, 1).astype(np.float32) for x in imgs]
    flat = lambda xs: to_dev(np.concatenate([x.reshape(-1, 3) for x in xs]))  # noqa: E731
    loss, d = ssim_loss(flat(imgs), flat(tgts), [_V(w, h) for w, h in sizes], lam)
    torch.cuda.synchronize()
    ref_loss, ref_g = oss.loss_and_grad(imgs, tgts, lam)
    got = float(loss.cpu().numpy()[0])
    assert abs(got - ref_loss) <= 1e-5 * abs(ref_loss) + 1e-9, (got, ref_loss)
    dg = d.cpu().numpy().astype(np.float64)
    ref = np.concatenate([g.reshape(-1, 3) for g in ref_g])
    scale = np.abs(ref).max()
    ties = np.concatenate([(x == y).reshape(-1, 3) for x, y in zip(imgs, tgts)])
    err = np.abs(dg - ref) * ~ties
    assert np.all(err <= 1e-3 * scale + 1e-3 * np.abs(ref)), err.max() / scale
    return got


@pytest.mark.parametrize("sizes,lam", [([(37, 23), (64, 48), (5, 3)], 0.2), ([(17, 40)], 1.0),
                                       ([(96, 64)], 0.0)])
def test_ssim_loss_matches_oracle(sizes, lam):
    log(f"[ssim] {sizes} lambda {lam}")
    _check(sizes, len(sizes) * 7, lam)


def test_ssim_loss_full_hd():
    log("[ssim] 1920x1080")
    _check([(1920, 1080)], 3, 0.2)


def test_identical_images_have_zero_loss():
    from paper_2510_03312_amd.optim import ssim_loss
    x = to_dev(np.random.default_rng(5).uniform(size=(40 * 30, 3)).astype(np.float32))
    loss, d = ssim_loss(x, x.clone(), [_V(40, 30)], 0.2)
    torch.cuda.synchronize()
    assert abs(float(loss.cpu().numpy()[0])) < 1e-6
    assert float(d.abs().max()) < 1e-6
