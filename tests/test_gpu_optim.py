"""Parity of the optimiser step (ubs_adam_step) with the float64 oracle,
through the C ABI: one step at a time from the GPU's own state, so that
each comparison measures one step's float32 rounding.

The oracle is given the float32 values of beta1 and beta2 the kernel
receives (0.999 as a float32 moves 1 - beta2 by 1.3e-5 relative).

Bar (derived from float32 arithmetic): parameters within 2^-21 (|p| +
|p'| + |noise|) + 1e-6 lr_row (the update and the noise are rounded in
turn, so near-cancelling sums keep the error of their larger terms),
moments within 2^-21 of their magnitude (plus the gradient scale for m, its
square for v)."""
import numpy as np
import pytest
import torch

from _gpu_common import gpu_ready, log, to_dev
from oracle import optim as oopt
from oracle.preprocess import field_slices, n_params

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]

F32_BETAS = {"beta1": float(np.float32(0.9)), "beta2": float(np.float32(0.999))}


def _init(dim, rot, n, seed):
    rng = np.random.default_rng(seed)
    F = n_params(dim, rot)
    P = rng.normal(size=(F, n)).astype(np.float32)
    P[field_slices(dim, rot)["o"]] = rng.uniform(0.0, 1.0, size=(1, n)).astype(np.float32)
    P[field_slices(dim, rot)["o"], :7] = 0.0             # sign(0) = 0
    return P, rng


@pytest.mark.parametrize("dim,rot,n", [(7, 0, 100003), (6, 1, 4097), (3, 0, 1), (7, 0, 1 << 20)])
def test_adam_steps_match_oracle(dim, rot, n):
    from paper_2510_03312_amd.optim import AdamConfig, adam_step
    log(f"[adam] dim {dim} rot {rot} n {n}")
    P, rng = _init(dim, rot, n, n)
    F = P.shape[0]
    cfg = AdamConfig()
    p_d = to_dev(P)
    m_d = torch.zeros_like(p_d)
    v_d = torch.zeros_like(p_d)
    rate = np.array([oopt.PAPER_LR[x] for x in oopt.row_groups(dim, rot)])[:, None]
    for t in range(1, 4):
        g = (rng.normal(size=(F, n)) * 10.0 ** rng.uniform(-6, 0, size=(F, 1))).astype(np.float32)
        g[:, :5] = 0.0                                   # zero gradients, and on step 1 zero moments
        noise = rng.normal(size=(3, n)).astype(np.float32) if t != 2 else None
        P0, M0, V0 = (x.cpu().numpy() for x in (p_d, m_d, v_d))
        adam_step(p_d, to_dev(g), m_d, v_d, t, dim, rot,
                  noise=None if noise is None else to_dev(noise), cfg=cfg)
        torch.cuda.synchronize()
        Pr, Mr, Vr = oopt.adam_step(P0, g, M0, V0, t, dim, rot, noise=noise, **F32_BETAS)
        Pg, Mg, Vg = (x.cpu().numpy().astype(np.float64) for x in (p_d, m_d, v_d))
        nz = np.zeros_like(Pr)
        if noise is not None:
            nz[field_slices(dim, rot)["mu_x"]] = np.abs(noise)
        tol_p = 2.0 ** -21 * (np.abs(Pr) + np.abs(P0) + nz) + 1e-6 * rate
        assert np.all(np.abs(Pg - Pr) <= tol_p), np.abs(Pg - Pr).max()
        gs = np.abs(g.astype(np.float64)) + np.abs(oopt.regulariser_grad(P0, dim, rot, 0.01, 0.01))
        assert np.all(np.abs(Mg - Mr) <= 2.0 ** -21 * (np.abs(Mr) + gs) + 1e-30)
        assert np.all(np.abs(Vg - Vr) <= 2.0 ** -21 * (np.abs(Vr) + gs * gs) + 1e-30)


def test_adam_on_a_rendered_gradient():
    """The renderer's gradient fed straight into the step, parameters updated
    in place, next frame renders from them."""
    from paper_2510_03312_amd import Renderer, SceneRef
    from paper_2510_03312_amd.optim import adam_step
    from synth import make_config
    log("[adam] after a rendered backward pass")
    cfg = make_config("headline", n=20000, width=160, height=120)
    sc = cfg["scenes"][0]
    params = to_dev(sc.params)
    r = Renderer()
    image, _ = r.forward([SceneRef(params, sc.dim, sc.rot)], cfg["views"])
    target = to_dev(cfg["targets"][0]).view(-1, 3).contiguous()
    (g,) = r.backward(l1_image=image, l1_target=target)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    P0 = params.cpu().numpy()
    G = g.cpu().numpy()
    adam_step(params, g, m, v, 1, sc.dim, sc.rot)
    torch.cuda.synchronize()
    Pr, _, _ = oopt.adam_step(P0, G, np.zeros_like(P0), np.zeros_like(P0), 1, sc.dim, sc.rot,
                              **F32_BETAS)
    rate = np.array([oopt.PAPER_LR[x] for x in oopt.row_groups(sc.dim, sc.rot)])[:, None]
    assert np.all(np.abs(params.cpu().numpy() - Pr) <= 2.0 ** -21 * (np.abs(Pr) + np.abs(P0))
                  + 1e-6 * rate)
    image2, _ = r.forward([SceneRef(params, sc.dim, sc.rot)], cfg["views"])
    assert torch.isfinite(image2).all()
