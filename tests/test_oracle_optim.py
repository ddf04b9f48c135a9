"""Pins of the optimiser-step oracle (Sec. 4.5 loss regularisers, Adam with
the Sec. 5.1 rates, spatial noise): the printed constants, the closed form
of Adam's first step, torch.optim.Adam over several steps, finite
differences of the regularisers, and where the noise goes."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import optim
from oracle.preprocess import field_slices, n_params

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _state(dim, rot, n, seed):
    rng = np.random.default_rng(seed)
    F = n_params(dim, rot)
    P = rng.normal(size=(F, n))
    P[field_slices(dim, rot)["o"]] = rng.uniform(0.05, 0.95, size=(1, n))
    return P, rng


def test_rates_and_weights_are_the_papers():
    g = GOLDEN["optimiser_sec5_1"]
    assert optim.PAPER_LR == {"mu_x": g["lr_positions"], "o": g["lr_opacity"],
                              "log_s": g["lr_scales"], "other": g["lr_other"]}
    assert (optim.LAMBDA_O, optim.LAMBDA_S, optim.LAMBDA_EPS) == (
        g["lambda_o"], g["lambda_sigma"], g["lambda_eps"])


@pytest.mark.parametrize("dim,rot", [(3, 0), (6, 1), (7, 0)])
def test_row_groups_cover_the_layout(dim, rot):
    grp = optim.row_groups(dim, rot)
    sl = field_slices(dim, rot)
    assert len(grp) == n_params(dim, rot)
    assert [i for i, x in enumerate(grp) if x == "mu_x"] == list(range(sl["mu_x"].start, sl["mu_x"].stop))
    assert [i for i, x in enumerate(grp) if x == "log_s"] == list(range(sl["log_s_x"].start, sl["log_s_x"].stop))
    assert [i for i, x in enumerate(grp) if x == "o"] == [sl["o"].start]


def test_first_step_moves_every_entry_by_its_rate():
    """From zero moments, m_hat = g and v_hat = g^2: the step is -lr sign(g)."""
    P, rng = _state(7, 0, 50, 0)
    g = rng.normal(size=P.shape)
    Z = np.zeros_like(P)
    P1, M, V = optim.adam_step(P, g, Z, Z, 1, 7, 0, lambda_o=0.0, lambda_s=0.0, noise=None)
    rate = np.array([optim.PAPER_LR[x] for x in optim.row_groups(7, 0)])[:, None]
    np.testing.assert_allclose(P1 - P, -rate * np.sign(g), rtol=1e-9, atol=1e-16)
    np.testing.assert_allclose(M, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(V, 0.001 * g * g, rtol=1e-14)


def test_matches_torch_adam_over_steps():
    dim, rot = 6, 1
    P, rng = _state(dim, rot, 40, 1)
    grp = optim.row_groups(dim, rot)
    rows = {k: [i for i, x in enumerate(grp) if x == k] for k in ("mu_x", "o", "log_s", "other")}
    tens = {k: torch.tensor(P[rows[k]], dtype=torch.float64, requires_grad=True) for k in rows}
    opt = torch.optim.Adam([{"params": [tens[k]], "lr": optim.PAPER_LR[k]} for k in rows],
                           betas=(0.9, 0.999), eps=1e-15)
    M = np.zeros_like(P)
    V = np.zeros_like(P)
    Q = P.copy()
    for t in range(1, 6):
        g = rng.normal(size=P.shape)
        Q, M, V = optim.adam_step(Q, g, M, V, t, dim, rot, lambda_o=0.0, lambda_s=0.0)
        opt.zero_grad()
        for k in rows:
            tens[k].grad = torch.tensor(g[rows[k]], dtype=torch.float64)
        opt.step()
    for k in rows:
        np.testing.assert_allclose(Q[rows[k]], tens[k].detach().numpy(), rtol=1e-12, atol=1e-14)


def test_regulariser_gradient_is_the_derivative_of_its_value():
    dim, rot = 7, 0
    P, _ = _state(dim, rot, 6, 2)
    G = optim.regulariser_grad(P, dim, rot, 0.01, 0.01)
    sl = field_slices(dim, rot)
    h = 1e-6
    for r in list(range(sl["log_s_x"].start, sl["log_s_x"].stop)) + [sl["o"].start, 0, sl["rgb"].start]:
        for i in range(P.shape[1]):
            Pp, Pm = P.copy(), P.copy()
            Pp[r, i] += h
            Pm[r, i] -= h
            fd = (optim.regulariser_value(Pp, dim, rot, 0.01, 0.01)
                  - optim.regulariser_value(Pm, dim, rot, 0.01, 0.01)) / (2 * h)
            assert abs(fd - G[r, i]) <= 1e-8, (r, i, fd, G[r, i])


def test_noise_moves_only_the_spatial_means():
    dim, rot = 7, 0
    P, rng = _state(dim, rot, 30, 3)
    Z = np.zeros_like(P)
    eps = rng.normal(size=(3, P.shape[1]))
    P1, _, _ = optim.adam_step(P, Z, Z, Z, 1, dim, rot, lambda_o=0.0, lambda_s=0.0,
                               lambda_eps=0.5, noise=eps)
    np.testing.assert_allclose(P1[:3], P[:3] + 0.5 * eps, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(P1[3:], P[3:])
