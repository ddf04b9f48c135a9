"""Parity of the relocation of dead primitives (ubs_relocate) with the
oracle, through the C ABI.  Picks are bit-exact (the float64 CDF of float32
opacities is exact, both sides round u * total once); copied parameters
are exact copies; the cloned opacity is a float64 power rounded to float32
(within one float32 ulp); reset moments are exactly zero."""
import numpy as np
import pytest
import torch

from _gpu_common import gpu_ready, log, to_dev
from oracle import relocate as orl
from oracle.preprocess import field_slices, n_params

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def _scene(dim, rot, n, dead_frac, seed):
    rng = np.random.default_rng(seed)
    F = n_params(dim, rot)
    P = rng.normal(size=(F, n)).astype(np.float32)
    o = rng.uniform(0.0, 1.0, size=n)
    o[rng.uniform(size=n) < dead_frac] = rng.uniform(0.0, orl.O_MIN, size=1)[0]
    P[field_slices(dim, rot)["o"].start] = o.astype(np.float32)
    M = rng.normal(size=(F, n)).astype(np.float32)
    V = np.abs(rng.normal(size=(F, n))).astype(np.float32)
    u = rng.uniform(size=n)
    return P, M, V, u


def _run(P, M, V, u, dim, rot):
    from paper_2510_03312_amd.optim import relocate
    p, m, v = to_dev(P), to_dev(M), to_dev(V)
    tg, nd = relocate(p, m, v, torch.from_numpy(u).cuda(), dim, rot)
    torch.cuda.synchronize()
    return (p.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), tg.cpu().numpy(),
            int(nd.cpu().numpy()[0]))


def _compare(P, M, V, u, dim, rot):
    Pg, Mg, Vg, tg, nd = _run(P, M, V, u, dim, rot)
    Pr, Mr, Vr, tr = orl.relocate(P, M, V, u, dim, rot)
    assert nd == tr.size or (tr.size == 0)
    np.testing.assert_array_equal(tg[:tr.size], tr)
    r_o = field_slices(dim, rot)["o"].start
    others = [r for r in range(P.shape[0]) if r != r_o]
    np.testing.assert_array_equal(Pg[others], Pr[others].astype(np.float32))
    ulp = np.spacing(np.abs(Pr[r_o]).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(Pg[r_o].astype(np.float64) - Pr[r_o]) <= ulp)
    np.testing.assert_array_equal(Mg, Mr.astype(np.float32))
    np.testing.assert_array_equal(Vg, Vr.astype(np.float32))
    return tr.size


@pytest.mark.parametrize("dim,rot,n,dead", [(7, 0, 100003, 0.2), (6, 1, 5000, 0.6), (3, 0, 1, 0.0),
                                            (7, 0, 1 << 20, 0.5)])
def test_relocation_matches_oracle(dim, rot, n, dead):
    log(f"[relocate] dim {dim} n {n} dead {dead}")
    P, M, V, u = _scene(dim, rot, n, dead, n)
    moved = _compare(P, M, V, u, dim, rot)
    log(f"  relocated {moved}")


def test_relocation_edge_cases():
    log("[relocate] edge cases")
    dim, rot = 7, 0
    P, M, V, u = _scene(dim, rot, 3000, 0.3, 5)
    u[:10] = np.nextafter(1.0, 0.0)                   # u * total may round to the total
    _compare(P, M, V, u, dim, rot)
    P2 = P.copy()
    P2[5, 17] = np.nan                                # non-finite: counts as dead
    P2[0, 99] = np.inf
    _compare(P2, M, V, u, dim, rot)
    Pd = P.copy()
    Pd[field_slices(dim, rot)["o"].start] = 0.001     # nothing live: nothing moves
    _compare(Pd, M, V, u, dim, rot)
    Pl = P.copy()
    Pl[field_slices(dim, rot)["o"].start] = 0.5       # nothing dead
    _compare(Pl, M, V, u, dim, rot)
