"""Pins of the oracle's screen-space conic (Section 3, equation r) and of
the query (Section 4.4), against values fixed independently of its code:
matrices inverted by numpy, a projection Jacobian taken by central
differences, and camera geometry whose answer is known by construction.

A swap of the conic's a and c, a sign flip of b, a reversed view direction,
a wrong camera centre or the query's [t, d] order exchanged each fail one of
these tests.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import preprocess as pp
from oracle import render
from synth import look_at_view, make_view

F64 = torch.float64


def _pixel_of(view, x):
    p = view.R.astype(np.float64) @ x + view.t.astype(np.float64)
    return np.array([view.fx * p[0] / p[2] + view.cx, view.fy * p[1] / p[2] + view.cy])


def _screen_covariance(view, mu, Sigma):
    """Sigma' = Jw Sigma Jw^T + 0.3 I with Jw the derivative of the pixel
    position by the world point, taken by central differences."""
    Jw = np.zeros((2, 3))
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        Jw[:, k] = (_pixel_of(view, mu + e) - _pixel_of(view, mu - e)) / (2 * h)
    return Jw @ Sigma @ Jw.T + 0.3 * np.eye(2)


def _aniso_primitive(mu, quat_wxyz, scales, b_x, o, rgb):
    P = np.zeros((pp.n_params(3, 0), 1))
    sl = pp.field_slices(3, 0)
    P[sl["mu_x"], 0] = mu
    P[sl["rot"], 0] = quat_wxyz
    P[sl["log_s_x"], 0] = np.log(scales)
    P[sl["b_x"], 0] = b_x
    P[sl["o"], 0] = o
    P[sl["rgb"], 0] = rgb
    return P


def _sigma_x(quat_wxyz, scales):
    w, x, y, z = quat_wxyz
    R = Rotation.from_quat([x, y, z, w]).as_matrix()   # scipy is scalar-last
    return R @ np.diag(np.asarray(scales) ** 2) @ R.T


CASES = [
    # mean, quaternion (w, x, y, z), scales: rotated and strongly anisotropic,
    # so that the screen conic has a != c and b far from 0
    ((0.10, -0.05, 0.3), (0.9, 0.2, -0.3, 0.4), (0.30, 0.04, 0.10)),
    ((-0.20, 0.15, -0.5), (0.3, -0.8, 0.5, 0.1), (0.05, 0.25, 0.02)),
    ((0.05, 0.10, 0.8), (0.6, 0.1, 0.1, -0.75), (0.40, 0.06, 0.20)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_record_conic_is_inverse_of_projected_covariance(case):
    mu, q, s = CASES[case]
    view = look_at_view((0.7, -0.4, -3.5), 96, 72)
    P = _aniso_primitive(mu, q, s, 0.2, 0.8, (0.3, 0.6, 0.9))
    out = pp.preprocess(torch.as_tensor(P), 3, 0, view)
    assert bool(out["valid"][0])
    rec = out["rec"][0].numpy()
    Sp = _screen_covariance(view, np.asarray(mu), _sigma_x(q, s))
    A = np.linalg.inv(Sp)
    assert abs(A[0, 1]) > 0.1 * max(A[0, 0], A[1, 1])     # genuinely rotated
    assert abs(A[0, 0] - A[1, 1]) > 0.1 * max(A[0, 0], A[1, 1])   # genuinely anisotropic
    np.testing.assert_allclose(rec[2:5], [A[0, 0], A[0, 1], A[1, 1]], rtol=1e-7)
    np.testing.assert_allclose(rec[0:2], _pixel_of(view, np.asarray(mu)), rtol=1e-12)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_anisotropic_splat_pixels_follow_the_mahalanobis_distance(case):
    """Every pixel of a single rotated, anisotropic primitive equals
    c min(0.99, o (1 - r)^beta) with r = (s - mu')^T Sigma'^-1 (s - mu') at the
    pixel centre s (Section 3 equation r, the Beta kernel), Sigma' from a
    numerical Jacobian and numpy's inverse."""
    mu, q, s = CASES[case]
    s = tuple(2.5 * v for v in s)
    W, H = 128, 96
    view = look_at_view((0.7, -0.4, -3.5), W, H)
    b_x, o, col = -0.3, 0.85, np.array([0.25, 0.5, 0.95])
    P = _aniso_primitive(mu, q, s, b_x, o, col)
    res = render.render(P, 3, 0, view)
    mean = _pixel_of(view, np.asarray(mu))
    A = np.linalg.inv(_screen_covariance(view, np.asarray(mu), _sigma_x(q, s)))
    ys, xs = np.mgrid[0:H, 0:W]
    dx, dy = xs + 0.5 - mean[0], ys + 0.5 - mean[1]
    r = A[0, 0] * dx * dx + 2 * A[0, 1] * dx * dy + A[1, 1] * dy * dy
    beta = 4 * math.exp(b_x)
    sig = np.where(r < 1, o * np.clip(1 - r, 0, None) ** beta, 0.0)
    alpha = np.minimum(0.99, sig)
    alpha = np.where(alpha >= 1 / 255, alpha, 0.0)
    # pixels whose alpha sits at the 1/255 skip within the Jacobian's error
    # may go either way; everything else must agree closely
    clear = np.abs(sig - 1 / 255) > 1e-5
    assert clear.mean() > 0.99
    lit = (alpha > 0) & clear
    assert lit.sum() > 100, lit.sum()
    np.testing.assert_allclose(res["image"][clear], (alpha[..., None] * col)[clear], atol=2e-6)


@pytest.mark.parametrize("center", [(0.0, 0.0, -4.0), (1.2, -0.5, -4.0), (4.0, 0.3, 0.5),
                                    (-2.0, 1.0, 3.0)])
def test_camera_center_is_where_the_camera_was_placed(center):
    view = look_at_view(center, 64, 48)
    np.testing.assert_allclose(pp.camera_center(view).numpy(), center, atol=2e-6)
    # the camera centre maps to the camera-frame origin
    p = view.R.astype(np.float64) @ np.asarray(center) + view.t.astype(np.float64)
    np.testing.assert_allclose(p, 0.0, atol=2e-6)


def test_query_direction_hand_values():
    """Camera at (0, 0, -4) looking at the origin: a primitive at the origin
    is seen along +z, one level with the camera and 3 units up (world -y) or
    2 units along -x along those axes, one at (1, 1, -3) along (1, 1, 1)/sqrt 3."""
    view = make_view(64, 48, time=0.37)
    pts = np.array([[0.0, 0.0, 0.0], [0.0, -3.0, -4.0], [-2.0, 0.0, -4.0], [1.0, 1.0, -3.0]]).T
    want = np.array([[0, 0, 1], [0, -1, 0], [-1, 0, 0], [1 / math.sqrt(3)] * 3])
    d = pp.query(torch.as_tensor(pts), view, 3).numpy()
    np.testing.assert_allclose(d, want, atol=1e-6)
    q7 = pp.query(torch.as_tensor(pts), view, 4).numpy()
    np.testing.assert_allclose(q7[:, 0], 0.37, atol=1e-7)         # [t, d]: time first
    np.testing.assert_allclose(q7[:, 1:], want, atol=1e-6)
    view2 = look_at_view((4.0, 0.0, 0.0), 64, 48)
    d2 = pp.query(torch.as_tensor(np.zeros((3, 1))), view2, 3).numpy()
    np.testing.assert_allclose(d2, [[-1.0, 0.0, 0.0]], atol=1e-6)


@pytest.mark.parametrize("dim", [6, 7])
def test_query_at_the_primitive_mean_keeps_the_opacity(dim):
    """Primitives whose query mean is exactly the query of this view
    (directions known by construction, mu_t = t) have w = 0, so every factor
    (1 - tanh 0)^e is 1 and o(q) = o; the conditioned mean stays mu_x.  A
    different query order or direction moves q off mu_q and lowers o(q)."""
    C = dim - 3
    cam = np.array([0.0, 0.0, -4.0])
    view = make_view(64, 48, time=0.61)
    dirs = np.array([[0, 0, 1], [0.6, 0, 0.8], [0, -0.28, 0.96], [0.48, 0.6, 0.64]], dtype=np.float64)
    dist = np.array([4.0, 3.5, 5.0, 4.5])
    n = dirs.shape[0]
    sl = pp.field_slices(dim, 0)
    P = np.zeros((pp.n_params(dim, 0), n))
    P[sl["mu_x"]] = (cam[None, :] + dist[:, None] * dirs).T
    P[sl["mu_q"]] = dirs.T if C == 3 else np.vstack([np.full((1, n), 0.61), dirs.T])
    P[sl["rot"]] = np.array([[1.0], [0.0], [0.0], [0.0]])
    P[sl["log_s_x"]] = math.log(0.05)
    rng = np.random.default_rng(3)
    P[sl["L_qx"]] = rng.normal(0, 0.3, size=(3 * C, n))
    P[sl["L_q"]] = rng.normal(0, 0.1, size=(C * (C + 1) // 2, n))
    P[sl["b_q"]] = 0.5                       # steep opacity falloff away from mu_q
    P[sl["o"]] = 0.7
    P[sl["rgb"]] = 0.5
    out = pp.preprocess(torch.as_tensor(P), dim, 0, view)
    np.testing.assert_allclose(out["o_q"].numpy(), 0.7, rtol=1e-12)
    np.testing.assert_allclose(out["mu_c"].numpy(), P[sl["mu_x"]].T, atol=1e-12)
