"""Pins of the D-SSIM oracle (Sec. 4.5 loss): the window, the SSIM map
against explicit window sums (borders included), identity and constant-
image closed forms, and finite differences of the combined loss."""
import numpy as np
import pytest
import torch

from oracle import ssim as oss


def test_window_taps():
    g = oss.gaussian_taps()
    assert g.size == 11 and abs(g.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(g, g[::-1], rtol=0, atol=0)
    x = np.arange(11) - 5.0
    assert abs(np.sqrt((g * x * x).sum()) - 1.5) < 0.01   # the truncated Gaussian's spread


def test_ssim_map_matches_explicit_window_sums():
    rng = np.random.default_rng(0)
    X = rng.uniform(size=(23, 17, 3))
    Y = np.clip(X + 0.1 * rng.normal(size=X.shape), 0, 1)
    S = oss.ssim_map(torch.tensor(X), torch.tensor(Y)).numpy()
    for (i, j, c) in [(0, 0, 0), (22, 16, 2), (11, 8, 1), (3, 15, 0), (20, 2, 2), (5, 5, 1)]:
        assert abs(S[i, j, c] - oss.ssim_brute(X, Y, i, j, c)) < 1e-12


def test_identical_images_give_ssim_one_and_zero_gradient():
    X = np.random.default_rng(1).uniform(size=(12, 20, 3))
    S = oss.ssim_map(torch.tensor(X), torch.tensor(X)).numpy()
    np.testing.assert_allclose(S, 1.0, rtol=0, atol=1e-12)
    loss, (g,) = oss.loss_and_grad([X], [X], lam=1.0)
    assert abs(loss) < 1e-12 and np.abs(g).max() < 1e-10


def test_constant_images_interior_closed_form():
    a, b = 0.7, 0.3
    X = np.full((30, 30, 3), a)
    Y = np.full((30, 30, 3), b)
    S = oss.ssim_map(torch.tensor(X), torch.tensor(Y)).numpy()
    want = (2 * a * b + oss.C1) / (a * a + b * b + oss.C1)     # variances 0 in the interior
    np.testing.assert_allclose(S[5:25, 5:25], want, rtol=1e-12)


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    imgs = [rng.uniform(size=(9, 13, 3)), rng.uniform(size=(6, 7, 3))]
    tgts = [rng.uniform(size=x.shape) for x in imgs]
    loss, grads = oss.loss_and_grad(imgs, tgts, lam=0.2)
    h = 1e-6
    for v, (i, j, c) in [(0, (4, 6, 1)), (0, (0, 12, 2)), (1, (5, 0, 0)), (1, (2, 3, 2))]:
        P = [x.copy() for x in imgs]
        M = [x.copy() for x in imgs]
        P[v][i, j, c] += h
        M[v][i, j, c] -= h
        fd = (oss.loss_and_grad(P, tgts)[0] - oss.loss_and_grad(M, tgts)[0]) / (2 * h)
        assert abs(fd - grads[v][i, j, c]) <= 1e-7 * max(1.0, abs(fd)), (v, i, j, c, fd)
