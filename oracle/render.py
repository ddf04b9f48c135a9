"""Oracle end-to-end render and gradients for one scene and one view.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Forward: ``preprocess`` (fp64 torch) -> records -> per-pixel compositing in
plain C (no tiles).  Gradients: the C adjoint gives d loss / d record, and
torch's fp64 autograd carries it back through the per-primitive steps.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import preprocess as pp
from . import raster

# relative bands for the per-primitive decisions a renderer may take
# differently from this float64 evaluation: the near plane and the
# definiteness of Sigma' (float64 on both sides in the renderer's default,
# so only rounding order separates them), o(q) against 1/255 (its scalar
# factors are float32 there); PRIM_BANDS_F32 for a renderer whose
# per-primitive math is float32 throughout
BAND_NEAR = 1e-9     # depth vs the near plane
BAND_OPACITY = raster.DEFAULT_BANDS[4]  # o(q) vs 1/255
BAND_DET = 1e-9      # det(Sigma') / (Sigma'_00 Sigma'_11) vs 0
PRIM_BANDS = (BAND_NEAR, BAND_OPACITY, BAND_DET)
PRIM_BANDS_F32 = (1e-5, 1e-4, 1e-6)

# record columns that receive a compositing gradient (d_rec order)
_GRAD_COLS = [0, 1, 2, 3, 4, 6, 7, 8, 9, 10]


def _geometry_ambiguous(out: dict, prim_bands) -> np.ndarray:
    near, _, det_band = prim_bands
    depth = out["depth"].detach().numpy()
    Sp = out["Sp"].detach().numpy()
    det = Sp[:, 0, 0] * Sp[:, 1, 1] - Sp[:, 0, 1] * Sp[:, 1, 0]
    scale = np.abs(Sp[:, 0, 0] * Sp[:, 1, 1]) + 1e-300
    geo = (np.abs(depth - pp.NEAR_PLANE) <= near * pp.NEAR_PLANE)
    geo |= (np.abs(det) / scale <= det_band) & (depth > pp.NEAR_PLANE)
    return geo


def ambiguous_records(out: dict, prim_bands=PRIM_BANDS) -> np.ndarray:
    """Primitives whose culling decision sits within a band of a threshold."""
    o_q = out["o_q"].detach().numpy()
    return _geometry_ambiguous(out, prim_bands) | (np.abs(o_q * 255.0 - 1.0) <= prim_bands[1])


def ambiguity_kinds(out: dict, prim_bands=PRIM_BANDS) -> np.ndarray:
    """uint8 per primitive for the compositing's flags: 0 unambiguous, 1 its
    culling by geometry (near plane, definiteness) is uncertain, 2 only
    o(q) against 1/255 is (see raster.c)."""
    kind = np.where(ambiguous_records(out, prim_bands), 2, 0).astype(np.uint8)
    kind[_geometry_ambiguous(out, prim_bands)] = 1
    return kind


def _amb_records(out: dict, amb: np.ndarray, rec: np.ndarray) -> np.ndarray:
    """A copy of the records ``rec`` with the would-be splat of each
    ambiguous-but-culled primitive (rho = 0: never contributes, only flags
    the pixels it could touch)."""
    rec = rec.copy()
    idx = np.flatnonzero(amb & ~out["valid"].numpy())
    if idx.size:
        Sp = out["Sp"].detach().numpy()[idx]
        m2 = out["mean2d"].detach().numpy()[idx]
        det = Sp[:, 0, 0] * Sp[:, 1, 1] - Sp[:, 0, 1] ** 2
        ok = det > 0
        dets = np.where(ok, det, 1.0)
        rec[idx, 0] = m2[:, 0]
        rec[idx, 1] = m2[:, 1]
        rec[idx, 2] = np.where(ok, Sp[:, 1, 1] / dets, 0.0)   # det <= 0: flags everything
        rec[idx, 3] = np.where(ok, -Sp[:, 0, 1] / dets, 0.0)
        rec[idx, 4] = np.where(ok, Sp[:, 0, 0] / dets, 0.0)
        rec[idx, 5] = 0.0
        rec[idx, 7] = out["beta_x"].detach().numpy()[idx]   # the reach of its flags
    return rec


def render(params: np.ndarray, dim: int, rot: int, view, *, d_image: Optional[np.ndarray] = None,
           d_tfinal: Optional[np.ndarray] = None, l1_target: Optional[np.ndarray] = None,
           rows=None, bands=raster.DEFAULT_BANDS, record_f32: bool = False,
           variant: tuple = (), prim_bands=PRIM_BANDS):
    """Render one view in float64.

    params: [F][n] (any float dtype; promoted to float64).  If ``d_image``
    (or ``l1_target``: L1-mean loss against it, sign(0) = 0) is given, also
    returns ``dparams`` [F][n].

    ``prim_bands``: (near plane, opacity, definiteness) bands of the
    primitives whose culling is counted as ambiguous.

    ``record_f32``: composite from the screen-space records rounded to
    float32, the precision the renderer's record format fixes, instead of
    their float64 values (the per-primitive steps and their derivatives stay
    float64).  Parity tests against a float32-record renderer use this so
    that rounding a record (a mean that moves by 1e-5 px next to a pixel
    centre, say) is not counted as a difference.
    """
    want_grad = d_image is not None or l1_target is not None
    P = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=want_grad)
    out = pp.preprocess(P, dim, rot, view, variant=variant)
    rec = out["rec"].detach().numpy()
    if record_f32:
        rec = rec.astype(np.float32).astype(np.float64)
    amb = ambiguous_records(out, prim_bands)
    rec_f = _amb_records(out, amb, rec) if amb.any() else rec
    W, H = view.width, view.height
    img, tf, nc, fl = raster.render_fwd(rec_f, W, H,
                                        amb=ambiguity_kinds(out, prim_bands) if amb.any() else None,
                                        rows=rows, bands=bands)
    res = {"image": img, "t_final": tf, "ncontrib": nc, "flags": fl, "rec": rec,
           "valid": out["valid"].numpy(), "amb": amb, "out": out}
    if want_grad:
        if l1_target is not None:
            d_image = np.sign(img - l1_target) / float(img.size)
            res["loss"] = float(np.abs(img - l1_target).mean())
        d_rec, d_abs = raster.render_bwd(rec, W, H, d_image, d_tfinal, with_abs=True)
        G = np.zeros_like(rec)
        G[:, _GRAD_COLS] = d_rec
        torch.autograd.backward(out["rec"], torch.from_numpy(G), retain_graph=True)
        res["dparams"] = P.grad.numpy().copy()
        res["d_rec"] = d_rec
        res["d_rec_abs"] = d_abs
        res["d_image"] = d_image
        res["dparams_noise"] = _abs_chain(P, out["rec"], d_abs)
    return res


def _abs_chain(P: torch.Tensor, rec: torch.Tensor, d_abs: np.ndarray) -> np.ndarray:
    """sum_k |d rec_k / d params| * d_abs_k per parameter entry: how far a
    float32 accumulation of the per-pixel gradient terms can move each
    parameter gradient (records depend only on their own primitive, so one
    vector-Jacobian product per record field gives that field's Jacobian)."""
    acc = np.zeros(tuple(P.shape))
    for j, col in enumerate(_GRAD_COLS):
        if not np.any(d_abs[:, j]):
            continue
        (jac,) = torch.autograd.grad(rec[:, col].sum(), P, retain_graph=True, allow_unused=True)
        if jac is not None:
            acc += np.abs(jac.numpy()) * d_abs[None, :, j]
    return acc


def loss_value(params: np.ndarray, dim: int, rot: int, view, weight_image: np.ndarray,
               weight_t: Optional[np.ndarray] = None, variant: tuple = ()) -> float:
    """Scalar <weight_image, image> + <weight_t, T_final> for finite differences."""
    r = render(params, dim, rot, view, variant=variant)
    v = float((r["image"] * weight_image).sum())
    if weight_t is not None:
        v += float((r["t_final"] * weight_t).sum())
    return v
