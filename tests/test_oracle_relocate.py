"""Pins of the relocation oracle (Sec. 4.5 densification rule, MCMC
relocation): the cloning rule's invariant, a hand-worked case, sampling
frequencies, exactness of the float64 CDF, and the degenerate cases."""
import numpy as np
import pytest

from oracle import relocate as orl
from oracle.preprocess import field_slices, n_params


def test_cloned_copies_composite_to_the_original_opacity():
    rng = np.random.default_rng(0)
    o = rng.uniform(0.0, 0.999, size=1000)
    N = rng.integers(1, 9, size=1000)
    op = orl.cloned_opacity(o, N)
    np.testing.assert_allclose(1.0 - (1.0 - op) ** N, o, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(orl.cloned_opacity(o, np.ones_like(N)), o, rtol=0, atol=2e-16)


def _scene(dim, rot, opac):
    F = n_params(dim, rot)
    P = np.arange(F * len(opac), dtype=np.float64).reshape(F, len(opac)) * 0.01
    P[field_slices(dim, rot)["o"].start] = opac
    return P


def test_hand_worked_case():
    """Opacities [0.5, 0.001, 0.25, 0.0, 0.25]: live 0, 2, 4 with running
    sums 0.5, 0.75, 1.0; dead slots 1 and 3 draw u = 0.6 (x = 0.6 -> index
    2) and u = 0.1 (x = 0.1 -> index 0)."""
    dim, rot = 3, 0
    P = _scene(dim, rot, [0.5, 0.001, 0.25, 0.0, 0.25])
    M = np.ones_like(P)
    V = np.full_like(P, 2.0)
    P1, M1, V1, tg = orl.relocate(P, M, V, np.array([0.6, 0.1]), dim, rot)
    assert tg.tolist() == [2, 0]
    r_o = field_slices(dim, rot)["o"].start
    o2 = 1.0 - (1.0 - 0.25) ** 0.5
    o0 = 1.0 - (1.0 - 0.5) ** 0.5
    np.testing.assert_allclose(P1[r_o], [o0, o2, o2, o0, 0.25], rtol=1e-15)
    others = [r for r in range(P.shape[0]) if r != r_o]
    np.testing.assert_array_equal(P1[others][:, 1], P[others][:, 2])
    np.testing.assert_array_equal(P1[others][:, 3], P[others][:, 0])
    np.testing.assert_array_equal(P1[others][:, [0, 2, 4]], P[others][:, [0, 2, 4]])
    for X, X1 in ((M, M1), (V, V1)):
        np.testing.assert_array_equal(X1[:, [0, 1, 2, 3]], 0.0)
        np.testing.assert_array_equal(X1[:, 4], X[:, 4])


def test_picks_are_proportional_to_opacity():
    dim, rot = 3, 0
    live_o = np.array([0.9, 0.6, 0.3, 0.1, 0.05])
    n_dead = 200000
    P = _scene(dim, rot, np.concatenate([live_o, np.zeros(n_dead)]))
    u = np.random.default_rng(1).uniform(size=n_dead)
    _, _, _, tg = orl.relocate(P, np.zeros_like(P), np.zeros_like(P), u, dim, rot)
    freq = np.bincount(tg, minlength=5) / n_dead
    expect = live_o / live_o.sum()
    assert np.all(np.abs(freq - expect) <= 5 * np.sqrt(expect * (1 - expect) / n_dead))


def test_cdf_is_exact_whatever_the_summation_order():
    """Live float32 opacities >= o_min: sums in any order agree bit for bit."""
    rng = np.random.default_rng(2)
    o = rng.uniform(orl.O_MIN, 1.0, size=300000).astype(np.float32).astype(np.float64)
    fwd = np.cumsum(o)[-1]
    rev = np.cumsum(o[::-1])[-1]
    pair = o.reshape(-1, 2).sum(axis=1).sum()
    assert fwd == rev == pair


@pytest.mark.parametrize("opac", [[0.5, 0.2, 0.9], [0.0, 0.001, 0.0]])
def test_nothing_moves_without_dead_or_without_live(opac):
    P = _scene(3, 0, opac)
    P1, M1, V1, tg = orl.relocate(P, np.ones_like(P), np.ones_like(P), np.full(3, 0.5), 3, 0)
    np.testing.assert_array_equal(P1, P)
    np.testing.assert_array_equal(M1, 1.0)
    assert tg.size == 0
