"""Pins of the oracle's Sec. 5.3 ablation variants: "w/o Beta condition"
(Gaussian conditioning) and "w/o Beta opacity" (Gaussian conditional
opacity).  Each is pinned to a plain definition computed another way and to
finite differences of the whole oracle in that variant."""
import numpy as np
import pytest
import torch

from oracle import preprocess as pp
from synth import make_scene, make_view
from test_oracle_pins import _fd_check, _fields


def _scene(dim, n, seed):
    sc = make_scene(dim, n, seed=seed, dist="cfg3" if dim == 7 else "cfg1", rot=0)
    f = _fields(sc.params, dim, 0)
    Sigma = pp.covariance(pp.lower_factor(f, dim, 0))
    return sc, f, Sigma


@pytest.mark.parametrize("dim", [6, 7])
def test_gaussian_conditioning_is_the_precision_matrix_conditional(dim):
    """Without the Beta modulation the conditional is the textbook one for
    every b_q (here mostly negative, where the full method differs)."""
    sc, f, Sigma = _scene(dim, 30, 11)
    C = dim - 3
    b_q = -torch.abs(f["b_q"].T) - 0.2
    v = torch.as_tensor(np.random.default_rng(3).normal(size=(sc.n, C)))
    mu_x = f["mu_x"].T
    mu_c, S_c = pp.condition(mu_x, Sigma, v, b_q, beta_modulated=False)
    mu_b, S_b = pp.condition(mu_x, Sigma, v, b_q, beta_modulated=True)
    assert float((mu_c - mu_b).abs().max()) > 1e-6          # the modulation matters here
    for i in range(sc.n):
        Lam = np.linalg.inv(Sigma[i].numpy())
        Sc_ref = np.linalg.inv(Lam[:3, :3])
        mc_ref = mu_x[i].numpy() - Sc_ref @ Lam[:3, 3:] @ v[i].numpy()
        np.testing.assert_allclose(S_c[i].numpy(), Sc_ref, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(mu_c[i].numpy(), mc_ref, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("dim", [6, 7])
def test_gaussian_opacity_is_the_quadratic_form(dim):
    """o exp(-v^T Sigma_q^-1 v / 2) with the inverse formed explicitly."""
    sc, f, Sigma = _scene(dim, 25, 12)
    C = dim - 3
    v = torch.as_tensor(np.random.default_rng(4).normal(size=(sc.n, C)) * 0.5)
    o = f["o"][0]
    got = pp.gaussian_opacity(o, Sigma[:, 3:, 3:], v).numpy()
    for i in range(sc.n):
        Sq = Sigma[i, 3:, 3:].numpy()
        vi = v[i].numpy()
        ref = float(o[i]) * np.exp(-0.5 * vi @ np.linalg.inv(Sq) @ vi)
        assert abs(got[i] - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("variant", [(pp.NO_BETA_CONDITION,), (pp.NO_BETA_OPACITY,),
                                     (pp.NO_BETA_CONDITION, pp.NO_BETA_OPACITY)])
def test_variant_gradient_matches_finite_differences(variant):
    dim, rot = 7, 0
    rng = np.random.default_rng(len(variant) * 7 + len(variant[0]))
    sc = make_scene(dim, 60, seed=9, dist="cfg3", rot=rot)
    P = sc.params.astype(np.float64)
    sl = pp.field_slices(dim, rot)
    P[sl["mu_x"]] = rng.uniform(-0.6, 0.6, size=(3, sc.n))
    P[sl["log_s_x"]] = rng.normal(-2.2, 0.3, size=(3, sc.n))
    P[sl["b_q"]] = rng.uniform(-1.0, 1.0, size=(dim - 3, sc.n))
    _fd_check(P, dim, rot, make_view(32, 24, time=0.4), rng, variant=variant)


def test_variants_change_the_records():
    dim, rot = 7, 0
    sc = make_scene(dim, 400, seed=3, dist="cfg3", rot=rot)
    P = torch.tensor(sc.params.astype(np.float64))
    P[pp.field_slices(dim, rot)["b_q"]] = -0.5
    view = make_view(64, 48, time=0.5)
    full = pp.preprocess(P, dim, rot, view)["rec"]
    for var in ((pp.NO_BETA_CONDITION,), (pp.NO_BETA_OPACITY,)):
        other = pp.preprocess(P, dim, rot, view, variant=var)["rec"]
        assert float((other - full).abs().max()) > 1e-6, var
