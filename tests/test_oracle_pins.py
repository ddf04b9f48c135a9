"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values
printed in the paper (tests/golden/paper_values.json), textbook identities
evaluated by independent library routines, closed forms, limits, and brute
force.  None of these needs a GPU.
"""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import preprocess as pp
from oracle import raster, render
from synth import make_scene, make_splat_records, make_view, look_at_view, param_count

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
F64 = torch.float64


def _fields(params, dim, rot):
    sl = pp.field_slices(dim, rot)
    return {k: torch.as_tensor(params[s], dtype=F64) for k, s in sl.items() if k != "_F"}


# --------------------------------------------------------------------- paper values
def test_beta_map_paper_values():
    for case in GOLD["beta_map"]["cases"]:
        beta = float(pp.beta_of_b(torch.tensor(case["b"], dtype=F64)))
        assert abs(beta - case["beta"]) <= case["abs_tol"] + 1e-12, case


@pytest.mark.parametrize("key", ["ubs6d", "ubs7d"])
def test_parameter_counts(key):
    g = GOLD["param_counts"][key]
    # the paper's parameterisation uses the skew-symmetric rotation (3 values)
    assert pp.n_params(g["dim"], 1) == g["total"]
    assert param_count(g["dim"], 1) == g["total"]   # the input format agrees
    C = g["dim"] - 3
    assert 3 + 3 + 3 * C + C * (C + 1) // 2 == g["covariance"]
    assert g["covariance"] == g["dim"] * (g["dim"] + 1) // 2


def test_storage_sizes():
    for row in GOLD["storage_mb"]["rows"]:
        mb = row["num"] * pp.n_params(row["dim"], 1) * 4 / 2 ** 20
        assert round(mb, 1) == pytest.approx(row["mem"], abs=0.051), row


# --------------------------------------------------------------------- covariance
@pytest.mark.parametrize("rot", [0, 1])
@pytest.mark.parametrize("dim", [3, 6, 7])
def test_covariance_matches_appendix_blocks(dim, rot):
    sc = make_scene(dim, 64, seed=3, dist="cfg3" if dim == 7 else "cfg1", rot=rot)
    f = _fields(sc.params, dim, rot)
    L = pp.lower_factor(f, dim, rot)
    S = pp.covariance(L).numpy()
    C = dim - 3
    for i in range(sc.n):
        if rot == 0:
            w, x, y, z = sc.params[pp.field_slices(dim, rot)["rot"], i].astype(np.float64)
            R = Rotation.from_quat([x, y, z, w]).as_matrix()  # scipy is scalar-last
        else:
            om = f["rot"][:, i].numpy()
            # I + A with A v = w x v (the skew matrix of the cross product)
            R = np.eye(3) + np.stack([np.cross(om, e) for e in np.eye(3)], axis=1)
        s = np.exp(f["log_s_x"][:, i].numpy())
        Sx = R @ np.diag(s ** 2) @ R.T
        np.testing.assert_allclose(S[i, :3, :3], Sx, rtol=1e-12, atol=1e-15)
        if C:
            Lqx = f["L_qx"][:, i].numpy().reshape(C, 3)
            Lq = np.zeros((C, C))
            k = 0
            for r_ in range(C):
                for c_ in range(r_ + 1):
                    val = f["L_q"][k, i].item()
                    Lq[r_, c_] = math.exp(val) if r_ == c_ else val
                    k += 1
            np.testing.assert_allclose(S[i, :3, 3:], R @ np.diag(s) @ Lqx.T, rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(S[i, 3:, 3:], Lqx @ Lqx.T + Lq @ Lq.T, rtol=1e-12, atol=1e-15)
        assert np.linalg.eigvalsh(S[i]).min() > -1e-12


def test_quaternion_rotation_is_orthonormal():
    q = torch.as_tensor(np.random.default_rng(0).normal(size=(4, 50)))
    R = pp.rotation_matrix(q, 0).numpy()
    for i in range(50):
        np.testing.assert_allclose(R[i].T @ R[i], np.eye(3), atol=1e-13)
        assert np.linalg.det(R[i]) == pytest.approx(1.0, abs=1e-13)


def test_skew_rotation_first_order_properties():
    om = np.random.default_rng(1).normal(0, 0.4, size=(3, 20))
    R = pp.rotation_matrix(torch.as_tensor(om), 1).numpy()
    for i in range(20):
        w = om[:, i]
        # (I + A)^T (I + A) = I + A^T A = (1 + |w|^2) I - w w^T  (not orthogonal)
        np.testing.assert_allclose(R[i].T @ R[i], (1 + w @ w) * np.eye(3) - np.outer(w, w),
                                   atol=1e-13)
        np.testing.assert_allclose(R[i] @ np.ones(3) - np.ones(3), np.cross(w, np.ones(3)),
                                   atol=1e-13)


# --------------------------------------------------------------------- conditioning
def _random_full(dim, n, seed):
    sc = make_scene(dim, n, seed=seed, dist="cfg3" if dim == 7 else "cfg1", rot=0)
    f = _fields(sc.params, dim, 0)
    Sigma = pp.covariance(pp.lower_factor(f, dim, 0))
    return sc, f, Sigma


@pytest.mark.parametrize("dim", [6, 7])
def test_conditioning_is_textbook_gaussian_when_modulation_is_one(dim):
    """b_q >= 0 gives beta_tilde = 1; the result must equal the conditional
    Gaussian of the paper's Section 3 (6DGS), computed here through the
    precision matrix: Sigma_c = (Lambda_xx)^-1, mu_c = mu_x - Lambda_xx^-1 Lambda_xq v."""
    sc, f, Sigma = _random_full(dim, 40, 5)
    n = sc.n
    C = dim - 3
    b_q = torch.abs(f["b_q"].T)
    v = torch.as_tensor(np.random.default_rng(2).normal(size=(n, C)))
    mu_x = f["mu_x"].T
    mu_c, S_c = pp.condition(mu_x, Sigma, v, b_q)
    for i in range(n):
        Lam = np.linalg.inv(Sigma[i].numpy())
        Sc_ref = np.linalg.inv(Lam[:3, :3])
        mc_ref = mu_x[i].numpy() - Sc_ref @ Lam[:3, 3:] @ v[i].numpy()
        np.testing.assert_allclose(S_c[i].numpy(), Sc_ref, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(mu_c[i].numpy(), mc_ref, rtol=1e-9, atol=1e-12)


def test_conditioning_one_query_dimension_closed_form():
    """C = 1: diag(beta_tilde) is a scalar bt; mu_c = mu_x + bt Sxq v / s2 and
    Sigma_c = Sigma_x - bt Sxq Sqx / s2."""
    rng = np.random.default_rng(7)
    n = 30
    A = rng.normal(size=(n, 4, 4))
    Sigma = torch.as_tensor(A @ A.transpose(0, 2, 1) + 0.5 * np.eye(4))
    mu_x = torch.as_tensor(rng.normal(size=(n, 3)))
    v = torch.as_tensor(rng.normal(size=(n, 1)))
    b = torch.as_tensor(rng.uniform(-2, 1, size=(n, 1)))
    mu_c, S_c = pp.condition(mu_x, Sigma, v, b)
    for i in range(n):
        S = Sigma[i].numpy()
        bt = min(math.exp(b[i, 0].item()), 1.0)
        s2 = S[3, 3]
        np.testing.assert_allclose(mu_c[i].numpy(), mu_x[i].numpy() + bt * S[:3, 3] * v[i, 0].item() / s2,
                                   rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(S_c[i].numpy(), S[:3, :3] - bt * np.outer(S[:3, 3], S[3, :3]) / s2,
                                   rtol=1e-12, atol=1e-14)


def test_conditioning_diagonal_query_covariance_per_dimension_modulation():
    """Diagonal Sigma_q (orthogonal L_qx rows, diagonal L_q): the modulation
    acts per query dimension, Sigma_c = Sigma_x - sum_i bt_i Sxq_i Sqx_i / s_i."""
    rng = np.random.default_rng(11)
    n, C = 25, 3
    R = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    M = R @ np.diag(rng.uniform(0.2, 1.0, 3))
    Lqx = np.diag(rng.uniform(0.1, 0.5, C))            # rows along the axes: orthogonal
    Lq = np.diag(rng.uniform(0.3, 1.0, C))
    Lfull = np.zeros((6, 6))
    Lfull[:3, :3] = M
    Lfull[3:, :3] = Lqx
    Lfull[3:, 3:] = Lq
    S = Lfull @ Lfull.T
    Sigma = torch.as_tensor(np.repeat(S[None], n, 0))
    mu_x = torch.as_tensor(rng.normal(size=(n, 3)))
    v = torch.as_tensor(rng.normal(size=(n, C)))
    b = torch.as_tensor(rng.uniform(-2, 1, size=(n, C)))
    mu_c, S_c = pp.condition(mu_x, Sigma, v, b)
    for i in range(n):
        bt = np.minimum(np.exp(b[i].numpy()), 1.0)
        Sc_ref = S[:3, :3].copy()
        mc_ref = mu_x[i].numpy().copy()
        for k in range(C):
            Sc_ref -= bt[k] * np.outer(S[:3, 3 + k], S[3 + k, :3]) / S[3 + k, 3 + k]
            mc_ref += bt[k] * S[:3, 3 + k] * v[i, k].item() / S[3 + k, 3 + k]
        np.testing.assert_allclose(S_c[i].numpy(), Sc_ref, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(mu_c[i].numpy(), mc_ref, rtol=1e-12, atol=1e-14)


def test_conditioning_result_is_symmetric():
    sc, f, Sigma = _random_full(7, 40, 9)
    v = torch.as_tensor(np.random.default_rng(3).normal(size=(40, 4)))
    _, S_c = pp.condition(f["mu_x"].T, Sigma, v, f["b_q"].T)
    np.testing.assert_allclose(S_c.numpy(), S_c.transpose(1, 2).numpy(), atol=1e-15)


# --------------------------------------------------------------------- opacity
def test_whitening_identity_and_factor():
    """sum_i w_i^2 = v^T Sigma_q^-1 v for w = Lhat^-1 v, and the 2x2 Cholesky
    closed form for the per-dimension distances."""
    rng = np.random.default_rng(4)
    n = 30
    A = rng.normal(size=(n, 2, 2))
    Sq = A @ A.transpose(0, 2, 1) + 0.3 * np.eye(2)
    v = rng.normal(size=(n, 2))
    b = np.full((n, 2), -40.0)    # exponent 4e^-40: factors -> 1 unless d -> 1
    o = np.full(n, 0.8)
    for i in range(n):
        S = Sq[i]
        l11 = math.sqrt(S[0, 0])
        l21 = S[1, 0] / l11
        l22 = math.sqrt(S[1, 1] - l21 * l21)
        w1 = v[i, 0] / l11
        w2 = (v[i, 1] - l21 * w1) / l22
        assert w1 * w1 + w2 * w2 == pytest.approx(v[i] @ np.linalg.solve(S, v[i]), rel=1e-12)
        bb = np.array([[0.3, -0.7]])
        oq = pp.modulated_opacity(torch.tensor([0.8], dtype=F64), torch.as_tensor(S[None]),
                                  torch.as_tensor(v[i][None]), torch.as_tensor(bb))
        ref = 0.8 * (1 - math.tanh(w1 * w1)) ** (4 * math.exp(0.3)) \
            * (1 - math.tanh(w2 * w2)) ** (4 * math.exp(-0.7))
        assert float(oq[0]) == pytest.approx(ref, rel=1e-12)
    oq = pp.modulated_opacity(torch.as_tensor(o), torch.as_tensor(Sq), torch.as_tensor(v),
                              torch.as_tensor(b))
    np.testing.assert_allclose(oq.numpy(), o, rtol=1e-12)


def test_opacity_whitens_with_cholesky_of_sigma_q_not_L_q():
    """With L_qx != 0, Sigma_q != L_q L_q^T: o(q) must use chol(Sigma_q)."""
    sc = make_scene(6, 20, seed=13, dist="cfg1", rot=0)
    f = _fields(sc.params, 6, 0)
    L = pp.lower_factor(f, 6, 0)
    S = pp.covariance(L)
    v = torch.as_tensor(np.random.default_rng(5).normal(size=(20, 3)))
    oq = pp.modulated_opacity(f["o"][0], S[:, 3:, 3:], v, f["b_q"].T).numpy()
    for i in range(20):
        Sq = S[i, 3:, 3:].numpy()
        # v^T Sq^-1 v through the eigen-decomposition, a route without Cholesky
        ev, U = np.linalg.eigh(Sq)
        maha = float(((U.T @ v[i].numpy()) ** 2 / ev).sum())
        Lh = np.linalg.cholesky(Sq)
        w = np.linalg.solve(Lh, v[i].numpy())
        assert (w ** 2).sum() == pytest.approx(maha, rel=1e-10)
        e = 4 * np.exp(f["b_q"][:, i].numpy())
        ref = f["o"][0, i].item() * np.prod((1 - np.tanh(w * w)) ** e)
        if (w * w).max() < 8.0:   # direct 1 - tanh(x) is accurate to ~1e-9 relative here
            assert oq[i] == pytest.approx(ref, rel=1e-8)
        Lq_only = L[i, 3:, 3:].numpy()
        w_bad = np.linalg.solve(Lq_only, v[i].numpy())
        ref_bad = f["o"][0, i].item() * np.prod((1 - np.tanh(w_bad * w_bad)) ** e)
        if abs(ref_bad - ref) > 1e-6 * max(ref, 1e-12):
            assert abs(oq[i] - ref_bad) > 1e-9 * max(ref, 1e-12)


# --------------------------------------------------------------------- limits
@pytest.mark.parametrize("dim", [6, 7])
def test_zero_cross_correlation_and_flat_query_reduce_to_3d(dim):
    """Section 4.4: with b_q -> -inf, beta_tilde -> 0 and each opacity factor
    -> 1, so the N-D scene renders exactly like the 3-D (DBS) scene built from
    its spatial fields."""
    n = 300
    sc = make_scene(dim, n, seed=21, dist="cfg3" if dim == 7 else "cfg1", rot=0)
    sl = pp.field_slices(dim, 0)
    P = sc.params.astype(np.float64)
    P[sl["mu_x"]] = np.random.default_rng(1).uniform(-1, 1, size=(3, n))
    P[sl["b_q"]] = -60.0
    s3 = pp.field_slices(3, 0)
    P3 = np.zeros((pp.n_params(3, 0), n))
    for k in ("mu_x", "rot", "log_s_x", "b_x", "o", "rgb"):
        P3[s3[k]] = P[sl[k]]
    view = make_view(64, 48, time=0.3)
    rN = render.render(P, dim, 0, view)
    r3 = render.render(P3, 3, 0, view)
    np.testing.assert_allclose(rN["image"], r3["image"], atol=1e-12)
    np.testing.assert_allclose(rN["t_final"], r3["t_final"], atol=1e-12)


def _extend_7d(P7, rot, extra_mu, extra_logs, extra_b):
    """An N-D scene (N = 7 + m) from a 7-D one: m further query dimensions
    uncorrelated with everything else (zero rows in L_qx, zero off-diagonal
    entries of L_q), with the given means, log scales and Beta shapes."""
    m = len(extra_mu)
    s7, sN = pp.field_slices(7, rot), pp.field_slices(7 + m, rot)
    n = P7.shape[1]
    P = np.zeros((pp.n_params(7 + m, rot), n))
    for k in ("mu_x", "rot", "log_s_x", "b_x", "o", "rgb"):
        P[sN[k]] = P7[s7[k]]
    P[sN["mu_q"]] = np.concatenate([P7[s7["mu_q"]], np.repeat(np.asarray(extra_mu)[:, None], n, 1)])
    P[sN["b_q"]] = np.concatenate([P7[s7["b_q"]], np.repeat(np.asarray(extra_b)[:, None], n, 1)])
    qx7 = P7[s7["L_qx"]].reshape(4, 3, n)
    qx = np.zeros((4 + m, 3, n))
    qx[:4] = qx7
    P[sN["L_qx"]] = qx.reshape(3 * (4 + m), n)
    rows, k7 = [], 0   # L_q lower triangle, row-major
    lq7 = P7[s7["L_q"]]
    for i in range(4 + m):
        for j in range(i + 1):
            if i < 4:
                rows.append(lq7[k7]); k7 += 1
            elif i == j:
                rows.append(np.full(n, extra_logs[i - 4]))
            else:
                rows.append(np.zeros(n))
    P[sN["L_q"]] = np.stack(rows)
    return P


@pytest.mark.parametrize("m,rot", [(1, 0), (3, 1)])
def test_extra_query_dimensions_at_their_mean_reduce_to_7d(m, rot):
    """Query dimensions beyond [t, d] that are uncorrelated with the others
    and queried at their mean leave every record of the 7-D primitive
    unchanged: their block of Sigma_q^-1 does not couple (K gains zero
    columns) and each opacity factor is (1 - tanh 0)^beta = 1."""
    sc = make_scene(7, 400, seed=31 + m, dist="cfg3", rot=rot)
    P7 = sc.params.astype(np.float64)
    extra = [0.25, -0.4, 0.7][:m]
    P = _extend_7d(P7, rot, extra, [np.log(0.6), np.log(1.3), np.log(0.2)][:m], [0.8, -0.5, 0.1][:m])
    view = make_view(160, 120, time=0.45)
    view.query = tuple(extra) + (0.0,) * (3 - m)
    r7 = pp.preprocess(torch.as_tensor(P7), 7, rot, view)
    rN = pp.preprocess(torch.as_tensor(P), 7 + m, rot, view)
    assert torch.equal(r7["valid"], rN["valid"])
    np.testing.assert_allclose(rN["rec"].numpy(), r7["rec"].numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m", [1, 2])
def test_extra_query_dimension_off_its_mean_scales_the_opacity(m):
    """Off its mean, an uncorrelated further query dimension with scale s and
    shape b multiplies o(q) by (1 - tanh(w^2))^(4 e^b), w = (q_e - mu_e) / s
    (Section 4.3), and changes neither the conditioned mean nor the
    covariance (hence the projected mean and conic)."""
    sc = make_scene(7, 300, seed=41 + m, dist="cfg3", rot=0)
    P7 = sc.params.astype(np.float64)
    sl7 = pp.field_slices(7, 0)
    P7[sl7["mu_x"]] = np.random.default_rng(m).uniform(-1, 1, size=(3, 300))
    P7[sl7["o"]] = 0.9
    P7[sl7["b_q"]] = -6.0   # nearly flat in [t, d], so that most records survive
    mu_e, s_e, b_e = [0.1, 0.9][:m], [0.5, 2.0][:m], [0.3, -0.7][:m]
    P = _extend_7d(P7, 0, mu_e, list(np.log(s_e)), b_e)
    view = make_view(160, 120, time=0.6)
    q_e = [0.45, 0.2][:m]
    view.query = tuple(q_e) + (0.0,) * (3 - m)
    r7 = pp.preprocess(torch.as_tensor(P7), 7, 0, view)
    rN = pp.preprocess(torch.as_tensor(P), 7 + m, 0, view)
    factor = 1.0
    for k in range(m):
        w = (q_e[k] - mu_e[k]) / s_e[k]
        factor *= (1.0 - math.tanh(w * w)) ** (4.0 * math.exp(b_e[k]))
    both = (r7["valid"] & rN["valid"]).numpy()
    assert both.sum() > 50
    a, b = rN["rec"].numpy()[both], r7["rec"].numpy()[both]
    np.testing.assert_allclose(a[:, [0, 1, 2, 3, 4, 7, 8, 9, 10, 11]],
                               b[:, [0, 1, 2, 3, 4, 7, 8, 9, 10, 11]], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(a[:, 6], b[:, 6] * factor, rtol=1e-12)
    # rho follows o(q): 1 - (255 o(q))^(-1/beta_x)
    np.testing.assert_allclose(a[:, 5], 1.0 - (255.0 * a[:, 6]) ** (-1.0 / a[:, 7]), rtol=1e-10)


def test_zero_cross_block_leaves_spatial_part_unchanged():
    sc, f, Sigma = _random_full(6, 30, 17)
    Sg = Sigma.clone()
    Sg[:, :3, 3:] = 0
    Sg[:, 3:, :3] = 0
    v = torch.as_tensor(np.random.default_rng(6).normal(size=(30, 3)))
    mu_c, S_c = pp.condition(f["mu_x"].T, Sg, v, f["b_q"].T)
    np.testing.assert_allclose(mu_c.numpy(), f["mu_x"].T.numpy(), atol=0)
    np.testing.assert_allclose(S_c.numpy(), Sg[:, :3, :3].numpy(), atol=0)


# --------------------------------------------------------------------- projection
def test_projection_matches_numerical_jacobian():
    rng = np.random.default_rng(8)
    view = look_at_view((1.2, -0.5, -4.0), 320, 200)
    n = 20
    mu = torch.as_tensor(rng.uniform(-1, 1, size=(n, 3)))
    A = rng.normal(size=(n, 3, 3)) * 0.1
    S = torch.as_tensor(A @ A.transpose(0, 2, 1))
    mean2d, Sp, depth = pp.project(mu, S, view)
    R = view.R.astype(np.float64)
    t = view.t.astype(np.float64)

    def pix(x):
        p = R @ x + t
        return np.array([view.fx * p[0] / p[2] + view.cx, view.fy * p[1] / p[2] + view.cy])

    for i in range(n):
        x = mu[i].numpy()
        np.testing.assert_allclose(mean2d[i].numpy(), pix(x), rtol=1e-13)
        Jw = np.zeros((2, 3))
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jw[:, k] = (pix(x + e) - pix(x - e)) / (2 * h)
        ref = Jw @ S[i].numpy() @ Jw.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(Sp[i].numpy(), ref, rtol=1e-7, atol=1e-9)
        assert depth[i].item() == pytest.approx((R @ x + t)[2], rel=1e-14)


@pytest.mark.parametrize("b_x", [-0.7, 0.0, 1.3])
def test_single_isotropic_primitive_closed_form(b_x):
    """One isotropic primitive on the optical axis: Sigma' = ((f s / z)^2 + 0.3) I
    and the pixel is c * min(0.99, o (1 - r)^beta) with r = |p - mu'|^2 / that."""
    W, H = 48, 40
    view = make_view(W, H)
    s, z0, o, col = 0.06, 1.5, 0.7, np.array([0.2, 0.5, 0.9])
    P = np.zeros((pp.n_params(3, 0), 1))
    sl = pp.field_slices(3, 0)
    P[sl["mu_x"], 0] = [0.0, 0.0, z0]
    P[sl["rot"], 0] = [0.3, -0.4, 0.5, 0.2]          # any rotation: isotropic
    P[sl["log_s_x"], 0] = math.log(s)
    P[sl["b_x"], 0] = b_x
    P[sl["o"], 0] = o
    P[sl["rgb"], 0] = col
    r = render.render(P, 3, 0, view)
    z = z0 + 4.0
    var = (view.fx * s / z) ** 2 + 0.3
    beta = 4 * math.exp(b_x)
    ys, xs = np.mgrid[0:H, 0:W]
    rr = ((xs + 0.5 - W / 2) ** 2 + (ys + 0.5 - H / 2) ** 2) / var
    sig = np.where(rr < 1, o * np.clip(1 - rr, 0, None) ** beta, 0.0)
    alpha = np.minimum(0.99, sig)
    alpha = np.where(alpha >= 1 / 255, alpha, 0.0)
    np.testing.assert_allclose(r["image"], alpha[..., None] * col, atol=1e-12)
    np.testing.assert_allclose(r["t_final"], 1 - alpha, atol=1e-12)


def test_gaussian_limit_printed_bound():
    """Appendix D Property 3 (reading r = d^2): with b = 0 the profile
    (1 - r)^4 stays within 0.0433 of exp(-4.5 r) on [0, 1); checked on a
    rendered splat."""
    g = GOLD["gaussian_limit"]
    W, H = 64, 64
    view = make_view(W, H)
    P = np.zeros((pp.n_params(3, 0), 1))
    sl = pp.field_slices(3, 0)
    P[sl["mu_x"], 0] = [0.0, 0.0, 0.0]
    P[sl["rot"], 0] = [1, 0, 0, 0]
    P[sl["log_s_x"], 0] = math.log(1.0)
    P[sl["o"], 0] = 0.9
    P[sl["rgb"], 0] = 1.0
    r = render.render(P, 3, 0, view)
    var = (view.fx * 1.0 / 4.0) ** 2 + 0.3
    ys, xs = np.mgrid[0:H, 0:W]
    rr = ((xs + 0.5 - W / 2) ** 2 + (ys + 0.5 - H / 2) ** 2) / var
    lit = r["image"][..., 0] > 0
    assert lit.sum() > 300
    err = np.abs(r["image"][..., 0][lit] - 0.9 * np.exp(-g["gauss_coeff"] * rr[lit]))
    assert err.max() <= g["sup_err_max"] * 0.9 + 1e-12
    # the bound is attained: sup over r of |(1-r)^4 - exp(-4.5 r)|
    rs = np.linspace(0, 1, 200001)
    assert np.abs((1 - rs) ** g["beta"] - np.exp(-g["gauss_coeff"] * rs)).max() == \
        pytest.approx(g["sup_err_max"], abs=5e-5)


def test_exact_gaussian_limit_large_beta():
    """(1 - r_G / (2 beta))^beta -> exp(-r_G / 2) as beta grows, error O(1/beta)."""
    rG = np.linspace(0, 6, 61)
    errs = []
    for k in range(9):
        beta = float(pp.beta_of_b(torch.tensor(float(k), dtype=F64)))
        prof = np.clip(1 - rG / (2 * beta), 0, None) ** beta
        errs.append(np.abs(prof - np.exp(-rG / 2)).max())
    errs = np.array(errs)
    assert np.all(np.diff(errs) < 0)
    assert errs[-1] < 1e-3
    ratio = errs[:-1] / errs[1:]
    assert np.all(ratio > 2.0)    # beta grows by e per step


# --------------------------------------------------------------------- compositing
def _brute_composite(rec, W, H):
    """Product form of the compositing equation (Section 3) with cumulative
    products, the 1/255 skip and the 1e-4 stop: a route independent of the
    C loop."""
    n = rec.shape[0]
    order = np.lexsort((np.arange(n), rec[:, 11]))
    img = np.zeros((H, W, 3))
    tf = np.ones((H, W))
    for y in range(H):
        for x in range(W):
            dx = x + 0.5 - rec[order, 0]
            dy = y + 0.5 - rec[order, 1]
            r = rec[order, 2] * dx * dx + 2 * rec[order, 3] * dx * dy + rec[order, 4] * dy * dy
            live = (rec[order, 5] > 0) & (r <= rec[order, 5])
            sig = np.where(live, rec[order, 6] * np.clip(1 - r, 0, None) ** rec[order, 7], 0)
            a = np.minimum(0.99, sig)
            a = np.where(a >= 1 / 255, a, 0.0)
            keep = a > 0
            a = a[keep]
            c = rec[order][keep, 8:11]
            Tin = np.concatenate([[1.0], np.cumprod(1 - a)[:-1]]) if a.size else np.zeros(0)
            stop = np.flatnonzero(Tin * (1 - a) < 1e-4)
            m = stop[0] if stop.size else a.size
            img[y, x] = (c[:m] * (a[:m] * Tin[:m])[:, None]).sum(0)
            tf[y, x] = np.prod(1 - a[:m])
    return img, tf


def test_compositing_matches_product_form_brute_force():
    rec = make_splat_records(120, 40, 24, seed=3, max_extent=12.0).astype(np.float64)
    img, tf, nc, fl = raster.render_fwd(rec, 40, 24)
    img2, tf2 = _brute_composite(rec, 40, 24)
    np.testing.assert_allclose(img, img2, atol=1e-12)
    np.testing.assert_allclose(tf, tf2, atol=1e-12)


def test_compositing_invariants():
    rec = make_splat_records(400, 64, 48, seed=5, max_extent=20.0).astype(np.float64)
    img, tf, nc, fl = raster.render_fwd(rec, 64, 48)
    assert np.all(img >= 0)
    assert np.all(tf <= 1) and np.all(tf > 0)
    cmax = rec[:, 8:11].max()
    assert np.all(img <= (1 - tf)[..., None] * cmax + 1e-12)
    # permuting the record array changes nothing (order comes from depth)
    perm = np.random.default_rng(0).permutation(rec.shape[0])
    img_p, tf_p, _, _ = raster.render_fwd(rec[perm], 64, 48)
    np.testing.assert_allclose(img_p, img, atol=1e-12)
    # adding records can only lower the transmittance
    img_h, tf_h, _, _ = raster.render_fwd(rec[:200], 64, 48)
    assert np.all(tf <= tf_h + 1e-15)


def test_early_termination_golden():
    g = GOLD["early_termination"]
    n = g["n_records"]
    rec = np.zeros((n, 12))
    rec[:, 0] = 4.5
    rec[:, 1] = 3.5       # centre of pixel (4, 3): r = 0 there
    rec[:, 2] = rec[:, 4] = 1.0
    rec[:, 5] = 0.9
    rec[:, 6] = g["alpha"]
    rec[:, 7] = 4.0
    rec[:, 8:11] = 1.0
    rec[:, 11] = np.arange(n) + 1.0
    img, tf, nc, fl = raster.render_fwd(rec, 8, 6)
    assert nc[3, 4] == g["contributors"]
    assert img[3, 4, 0] == pytest.approx(g["color"], abs=1e-15)
    assert tf[3, 4] == pytest.approx(g["t_final"], abs=1e-18)


def test_stop_ends_the_pixel():
    """The pixel stops at the first record that would take T below 1e-4, and
    records behind it are not composited even when they alone would keep T
    above 1e-4: alphas 0.9, 0.9, 0.9 leave T = 1e-3; the next (0.95) would
    leave 5e-5, so the pixel ends with colour 1 - 1e-3 although a record of
    alpha 0.5 follows."""
    alphas = [0.9, 0.9, 0.9, 0.95, 0.5]
    rec = np.zeros((len(alphas), 12))
    rec[:, :5] = [4.5, 3.5, 0.2, 0.0, 0.2]
    rec[:, 5] = 0.9
    rec[:, 6] = alphas
    rec[:, 7] = 4.0
    rec[:, 8:11] = 1.0
    rec[:, 11] = np.arange(len(alphas)) + 1.0
    img, tf, nc, fl = raster.render_fwd(rec, 8, 6)
    assert nc[3, 4] == 3
    assert img[3, 4, 0] == pytest.approx(1.0 - 1e-3, abs=1e-15)
    assert tf[3, 4] == pytest.approx(1e-3, rel=1e-12)


def test_opacity_clamp_golden():
    """alpha = min(0.99, sigma) (the standard-splatting clamp the paper defers
    to): a record with o = 1 centred on a pixel centre gives alpha = 0.99
    there, so the pixel is 0.99 c with T = 0.01; at o = 0.5 it is 0.5 c."""
    for o, a in ((1.0, 0.99), (0.995, 0.99), (0.5, 0.5)):
        rec = np.zeros((1, 12))
        rec[0, :5] = [4.5, 3.5, 0.2, 0.0, 0.2]
        rec[0, 5] = 0.9
        rec[0, 6] = o
        rec[0, 7] = 4.0
        rec[0, 8:11] = [1.0, 0.5, 0.25]
        rec[0, 11] = 2.0
        img, tf, nc, fl = raster.render_fwd(rec, 8, 6)
        np.testing.assert_allclose(img[3, 4], a * np.array([1.0, 0.5, 0.25]), rtol=1e-15)
        assert tf[3, 4] == pytest.approx(1.0 - a, rel=1e-14)


# --------------------------------------------------------------------- binning
def _qp_min(rec, x0, x1, y0, y1):
    """min of the record's quadratic form over a rectangle, by scipy's
    bounded quasi-Newton solver (independent of the closed-form edge test)."""
    from scipy.optimize import minimize
    mx, my, a, b, c = rec[:5]

    def f(p):
        dx, dy = p[0] - mx, p[1] - my
        return a * dx * dx + 2 * b * dx * dy + c * dy * dy

    def g(p):
        dx, dy = p[0] - mx, p[1] - my
        return np.array([2 * (a * dx + b * dy), 2 * (b * dx + c * dy)])

    best = np.inf
    for sx in (x0, x1, 0.5 * (x0 + x1)):
        for sy in (y0, y1, 0.5 * (y0 + y1)):
            res = minimize(f, [sx, sy], jac=g, bounds=[(x0, x1), (y0, y1)], method="L-BFGS-B",
                           options={"ftol": 1e-15, "gtol": 1e-13, "maxiter": 500})
            best = min(best, res.fun)
    return best


def test_binning_is_exact_and_complete_brute_force():
    W, H, T = 64, 48, 16
    rec32 = make_splat_records(40, W, H, seed=9, max_extent=14.0)
    keys, vals = raster.bin_view(rec32, W, H, T, T)
    emitted = set(zip((keys >> np.uint64(32)).tolist(), vals.tolist()))
    rec = rec32.astype(np.float64)
    tx_n, ty_n = (W + T - 1) // T, (H + T - 1) // T
    n_hits = 0
    for i in range(rec.shape[0]):
        if not rec[i, 5] > 0:
            assert not any(v == i for _, v in emitted)
            continue
        rb = rec[i, 5] * (1 + 2.0 ** -10)
        for ty in range(ty_n):
            for tx in range(tx_n):
                x0, y0 = tx * T + 0.5, ty * T + 0.5
                x1, y1 = min(tx * T + T - 1, W - 1) + 0.5, min(ty * T + T - 1, H - 1) + 0.5
                qmin = _qp_min(rec[i], x0, x1, y0, y1)
                tile = ty * tx_n + tx
                hit = (tile, i) in emitted
                n_hits += hit
                if qmin <= rb * (1 - 1e-7):
                    assert hit, (i, tx, ty, qmin, rb)
                elif qmin > rb * (1 + 1e-7):
                    assert not hit, (i, tx, ty, qmin, rb)
                # completeness on pixel centres
                xs = np.arange(tx * T, min(tx * T + T, W)) + 0.5
                ys = np.arange(ty * T, min(ty * T + T, H)) + 0.5
                X, Y = np.meshgrid(xs, ys)
                dx, dy = X - rec[i, 0], Y - rec[i, 1]
                q = rec[i, 2] * dx * dx + 2 * rec[i, 3] * dx * dy + rec[i, 4] * dy * dy
                if (q <= rec[i, 5]).any():
                    assert hit
    assert n_hits > 20


@pytest.mark.parametrize("kind", ["ordinary", "elongated", "far"])
def test_binning_window_changes_nothing(kind):
    """The binning reference tests each record's tiles inside a float64
    window of its ellipse; scanning every tile of the view gives the same
    keys and values, for ordinary records, very elongated ones (axis ratios
    up to 1e8, some float32 conics indefinite) and records far off screen."""
    from synth import make_elongated_records
    W, H = 200, 120
    if kind == "ordinary":
        rec = make_splat_records(3000, W, H, seed=4, max_extent=50.0)
    elif kind == "elongated":
        rec = make_elongated_records(3000, W, H, seed=5, ratio=(1e3, 1e8))
    else:
        rec = make_splat_records(500, W, H, seed=6, max_extent=40.0)
        rec[:, 0] += np.float32(3 * W)
        rec[::2, 0] -= np.float32(6 * W)
        rec[::3, 1] += np.float32(1e7)
    k1, v1 = raster.bin_view(rec, W, H, 16, 16)
    k2, v2 = raster.bin_view(rec, W, H, 16, 16, full_scan=True)
    np.testing.assert_array_equal(k1, k2)
    np.testing.assert_array_equal(v1, v2)
    if kind != "far":
        assert k1.size > 1000


@pytest.mark.parametrize("a,b,c", [(1.0, 0.0, 1.0), (2.0, 0.5, 1.0), (0.5, -0.2, 3.0)])
def test_tile_test_threshold_golden(a, b, c):
    """The overlap rule (tile pixel-centre rectangle, min r <= rho (1 + 2^-10))
    at its boundary.  A record centred a distance d to the right of the
    rectangle [0.5, 15.5]^2, level with its middle row: on the right edge
    dx = -d is fixed and r is smallest at dy* = b d / c, where r equals
    (a c - b^2) d^2 / c (completing the square; dy* lies on the edge here).
    A rho just above that minimum over (1 + 2^-10) is a hit, just below it
    a miss."""
    d = 3.0
    qmin = (a * c - b * b) * d * d / c
    assert abs(b * d / c) < 7.0
    mx, my = 15.5 + d, 8.0
    for rel, want in ((1 + 1e-9, True), (1 - 1e-9, False)):
        rho = qmin / (1.0 + 2.0 ** -10) * rel
        assert raster.tile_hit(mx, my, a, b, c, rho, 0.5, 15.5, 0.5, 15.5) == want, (rel, want)
    # the same minimum seen from below the rectangle (dy fixed, dx* = b d / a)
    qmin_y = (a * c - b * b) * d * d / a
    for rel, want in ((1 + 1e-9, True), (1 - 1e-9, False)):
        rho = qmin_y / (1.0 + 2.0 ** -10) * rel
        assert raster.tile_hit(8.0, 15.5 + d, a, b, c, rho, 0.5, 15.5, 0.5, 15.5) == want


def test_binning_keys_sort_and_ranges():
    W, H = 80, 50
    rec32 = make_splat_records(300, W, H, seed=2, max_extent=10.0)
    rec32[:10, 11] = rec32[10:20, 11]     # exact depth ties between records
    keys, vals = raster.bin_view(rec32, W, H, tile_base=7, rec_base=100)
    n_tiles = 7 + ((W + 15) // 16) * ((H + 15) // 16)
    sk, sv, ranges = raster.sort_and_ranges(keys, vals, n_tiles)
    tile = (sk >> np.uint64(32)).astype(np.int64)
    depth = (sk & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    # ordered by (tile, depth), ties by the record index (lexsort is independent)
    order = np.lexsort((sv, depth, tile))
    np.testing.assert_array_equal(order, np.arange(sk.size))
    assert np.all(ranges[:7] == 0)
    for g in range(n_tiles):
        s, e = ranges[g]
        if e > s:
            assert np.all(tile[s:e] == g)
        else:
            assert not np.any(tile == g)
    assert (ranges[:, 1] - ranges[:, 0]).sum() == sk.size
    # emitted depth bits come from the records
    np.testing.assert_array_equal(depth, rec32[sv - 100, 11])


# --------------------------------------------------------------------- gradients
def _fd_check(P, dim, rot, view, rng, n_check=40, h_rel=1e-6, variant=()):
    W, H = view.width, view.height
    wimg = rng.normal(size=(H, W, 3))
    wt = rng.normal(size=(H, W))
    res = render.render(P, dim, rot, view, d_image=wimg, d_tfinal=wt, variant=variant)
    g = res["dparams"]
    F, n = P.shape
    scale = np.abs(g).max()
    checked = 0
    tries = 0
    while checked < n_check and tries < 10 * n_check:
        tries += 1
        f, i = rng.integers(F), rng.integers(n)
        if not res["valid"][i]:
            continue
        h = h_rel * max(1.0, abs(P[f, i]))
        vals = []
        for hh in (h, h / 2):
            Pp, Pm = P.copy(), P.copy()
            Pp[f, i] += hh
            Pm[f, i] -= hh
            vals.append((render.loss_value(Pp, dim, rot, view, wimg, wt, variant)
                         - render.loss_value(Pm, dim, rot, view, wimg, wt, variant)) / (2 * hh))
        if abs(vals[0] - vals[1]) > 1e-6 * max(abs(vals[1]), 1e-3 * scale):
            continue   # a threshold (skip/stop/clamp/kink) lies within h: discard
        assert abs(g[f, i] - vals[1]) <= 1e-5 * max(abs(vals[1]), 1e-3 * scale), (f, i, g[f, i], vals)
        checked += 1
    assert checked >= n_check // 2


@pytest.mark.parametrize("dim,rot,dist", [(3, 0, "cfg0"), (6, 1, "cfg1"), (7, 0, "cfg3"), (6, 0, "cfg1"),
                                          (8, 0, "cfg3"), (10, 1, "cfg3")])
def test_oracle_gradient_matches_finite_differences(dim, rot, dist):
    rng = np.random.default_rng(dim * 10 + rot)
    sc = make_scene(dim, 60, seed=dim + rot, dist=dist, rot=rot)
    P = sc.params.astype(np.float64)
    sl = pp.field_slices(dim, rot)
    # move primitives in front of the camera and make them a few pixels wide
    P[sl["mu_x"]] = rng.uniform(-0.6, 0.6, size=(3, sc.n))
    P[sl["log_s_x"]] = rng.normal(-2.2, 0.3, size=(3, sc.n))
    if dim > 3:
        P[sl["b_q"]] = rng.uniform(-1.0, 1.0, size=(dim - 3, sc.n))
    view = make_view(32, 24, time=0.4)
    view.query = (0.3, 0.6, 0.1)
    _fd_check(P, dim, rot, view, rng)


@pytest.mark.parametrize("saturated", [False, True])
def test_raster_adjoint_matches_finite_differences_on_records(saturated):
    rng = np.random.default_rng(1)
    W, H = 24, 20
    rec = make_splat_records(30, W, H, seed=4, max_extent=6.0, cull_frac=0.0).astype(np.float64)
    rec[:, 6] = rng.uniform(0.1, 0.9, size=30)
    if saturated:   # sigma above the 0.99 clamp near the centres: alpha is flat in them
        rec[::2, 6] = rng.uniform(0.995, 1.0, size=15)
    rec[:, 5] = 0.999
    wimg = rng.normal(size=(H, W, 3))
    wt = rng.normal(size=(H, W))
    d = raster.render_bwd(rec, W, H, wimg, wt)
    cols = [0, 1, 2, 3, 4, 6, 7, 8, 9, 10]

    def L(r):
        img, tf, _, _ = raster.render_fwd(r, W, H)
        return (img * wimg).sum() + (tf * wt).sum()

    scale = np.abs(d).max()
    ok = 0
    for i in range(30):
        for j, col in enumerate(cols):
            h = 1e-6 * max(1.0, abs(rec[i, col]))
            fd = []
            for hh in (h, h / 2):
                rp, rm = rec.copy(), rec.copy()
                rp[i, col] += hh
                rm[i, col] -= hh
                fd.append((L(rp) - L(rm)) / (2 * hh))
            if abs(fd[0] - fd[1]) > 1e-6 * max(abs(fd[1]), 1e-3 * scale):
                continue
            assert abs(d[i, j] - fd[1]) <= 1e-5 * max(abs(fd[1]), 1e-3 * scale), (i, col, d[i, j], fd)
            ok += 1
    assert ok > 200
