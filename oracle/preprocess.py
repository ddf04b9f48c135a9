"""Oracle per-primitive steps in float64 (torch CPU, differentiable).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every function follows the paper's definitions in its own order and
notation; torch's fp64 autograd supplies the derivatives.  Readings of
points where the paper is silent or garbled are marked "Reading:".
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

F64 = torch.float64

NEAR_PLANE = 0.2          # Reading: standard splatting near plane
DILATION = 0.3            # Reading: standard splatting screen-space dilation (px^2)
ALPHA_MIN = 1.0 / 255.0   # Reading: standard splatting skip threshold
ALPHA_MAX = 0.99          # Reading: standard splatting opacity clamp


# --------------------------------------------------------------------------
# parameter format (component-major [F][n]); parsed here independently
# --------------------------------------------------------------------------
def field_slices(dim: int, rot: int) -> Dict[str, slice]:
    """Row ranges of each field.  rot 0 = quaternion (w,x,y,z), 1 = skew w."""
    C = dim - 3
    sizes = [("mu_x", 3), ("mu_q", C), ("rot", 4 if rot == 0 else 3), ("log_s_x", 3),
             ("L_qx", 3 * C), ("L_q", C * (C + 1) // 2), ("b_x", 1), ("b_q", C),
             ("o", 1), ("rgb", 3)]
    out, k = {}, 0
    for name, s in sizes:
        out[name] = slice(k, k + s)
        k += s
    out["_F"] = slice(0, k)
    return out


def n_params(dim: int, rot: int) -> int:
    return field_slices(dim, rot)["_F"].stop


# --------------------------------------------------------------------------
# Section 3 (DBS) / Section 4.1: Beta exponent
# --------------------------------------------------------------------------
def beta_of_b(b: torch.Tensor) -> torch.Tensor:
    """beta(b) = 4 exp(b) (DBS kernel definition, Section 3; Section 4.1)."""
    return 4.0 * torch.exp(b)


# --------------------------------------------------------------------------
# Section 4.2 / Appendix C: spatial-orthogonal Cholesky parameterisation
# --------------------------------------------------------------------------
def rotation_matrix(rp: torch.Tensor, rot: int) -> torch.Tensor:
    """R_x per primitive, [n,3,3].

    rot 0: unit quaternion (w,x,y,z) after normalisation (the 3DGS rotation
    of Section 3).  rot 1: first-order Taylor R = I + A(w) with A the skew
    matrix of Appendix C (not exactly orthogonal).
    """
    n = rp.shape[1]
    if rot == 0:
        q = rp / torch.linalg.norm(rp, dim=0, keepdim=True)
        w, x, y, z = q[0], q[1], q[2], q[3]
        R = torch.stack([
            torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
            torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
            torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
        ], -2)
        return R
    w1, w2, w3 = rp[0], rp[1], rp[2]
    zero = torch.zeros_like(w1)
    A = torch.stack([
        torch.stack([zero, -w3, w2], -1),
        torch.stack([w3, zero, -w1], -1),
        torch.stack([-w2, w1, zero], -1),
    ], -2)
    return torch.eye(3, dtype=rp.dtype).expand(n, 3, 3) + A


def lower_factor(fields: Dict[str, torch.Tensor], dim: int, rot: int) -> torch.Tensor:
    """The full N x N lower factor L of Section 4.2, [n,N,N].

    L = [[R_x diag(s_x), 0], [L_qx, L_q]] with s_x = exp(log_s_x) and L_q
    lower triangular with a positive diagonal exp(log s_q).  Reading: the
    diagonal of L_q is stored as a log scale, the strictly-lower entries
    are free.
    """
    C = dim - 3
    R = rotation_matrix(fields["rot"], rot)
    s = torch.exp(fields["log_s_x"]).T                      # [n,3]
    n = R.shape[0]
    N = 3 + C
    blocks = [[R * s[:, None, :], torch.zeros(n, 3, C, dtype=F64)]]
    if C > 0:
        Lqx = fields["L_qx"].T.reshape(n, C, 3)
        Lq = torch.zeros(n, C, C, dtype=F64)
        k = 0
        rows = []
        for i in range(C):
            row = []
            for j in range(C):
                if j < i:
                    row.append(fields["L_q"][k + j])
                elif j == i:
                    row.append(torch.exp(fields["L_q"][k + j]))
                else:
                    row.append(torch.zeros(n, dtype=F64))
            k += i + 1
            rows.append(torch.stack(row, -1))
        Lq = torch.stack(rows, -2)
        blocks.append([Lqx, Lq])
        L = torch.cat([torch.cat(b, -1) for b in blocks], -2)
    else:
        L = blocks[0][0]
    assert L.shape == (n, N, N)
    return L


def covariance(L: torch.Tensor) -> torch.Tensor:
    """Sigma = L L^T (Section 4.2)."""
    return L @ L.transpose(-1, -2)


# --------------------------------------------------------------------------
# Section 4.4: query  q = d (6-D) or [t, d] (7-D)
# --------------------------------------------------------------------------
def camera_center(view) -> torch.Tensor:
    R = torch.as_tensor(view.R, dtype=F64)
    t = torch.as_tensor(view.t, dtype=F64)
    return -(R.T @ t)


def query(mu_x: torch.Tensor, view, C: int) -> torch.Tensor:
    """Query vector per primitive, [n,C] (Section 4.1: q holds the
    non-spatial dimensions, view direction, time, etc.).

    Reading: d is the unit direction from the camera centre to the
    (unconditioned) spatial mean, in world coordinates; for 7-D the query is
    [t, d] with the view's timestamp t; for N > 7 the further query values
    come with the view (its ``query`` attribute, zeros if absent) and follow:
    [t, d, e_0, ..., e_{N-8}].
    """
    n = mu_x.shape[1]
    if C == 0:
        return torch.zeros(n, 0, dtype=F64)
    v = mu_x.T - camera_center(view)[None, :]
    d = v / torch.linalg.norm(v, dim=1, keepdim=True)
    if C == 3:
        return d
    if C >= 4:
        t = torch.full((n, 1), float(view.time), dtype=F64)
        parts = [t, d]
        if C > 4:
            e = np.zeros(C - 4)
            given = np.asarray(getattr(view, "query", ()), dtype=np.float64).ravel()[:C - 4]
            e[:given.size] = given
            parts.append(torch.as_tensor(e, dtype=F64)[None, :].expand(n, C - 4))
        return torch.cat(parts, 1)
    raise ValueError("the camera query is defined for N = 3 and N >= 6; pass q explicitly")


# --------------------------------------------------------------------------
# Section 4.3: Beta-modulated opacity and conditioning
# --------------------------------------------------------------------------
def beta_q(b_q: torch.Tensor) -> torch.Tensor:
    """beta_qi = exp(b_qi) for the query dimensions (Section 4.3)."""
    return torch.exp(b_q)


def beta_tilde(b_q: torch.Tensor) -> torch.Tensor:
    """[beta_q]_{<=1}: elementwise min(exp(b_q), 1) (Section 4.3).

    Reading: derivative exp(b) for b < 0 and 0 for b >= 0.
    """
    return torch.where(b_q < 0, torch.exp(torch.clamp(b_q, max=0.0)), torch.ones_like(b_q))


# Ablation variants of Sec. 5.3 (Table "ablation"): the Beta modulation of
# the conditioning or of the opacity replaced by its Gaussian counterpart.
NO_BETA_CONDITION = "no_beta_condition"   # diag(bt) = I: Gaussian conditioning
NO_BETA_OPACITY = "no_beta_opacity"       # o(q) = o exp(-(q - mu_q)^T Sigma_q^-1 (q - mu_q) / 2)


def gaussian_opacity(o: torch.Tensor, Sigma_q: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """The "w/o Beta opacity" ablation (Sec. 5.3): the Gaussian conditional
    opacity of 6DGS/7DGS, o exp(-w.w / 2) with w = Lhat^-1 (q - mu_q).
    Reading: the paper names the ablation only; this is the Gaussian form the
    Beta modulation replaces (Sec. 4.3)."""
    if v.shape[1] == 0:
        return o
    Lhat = torch.linalg.cholesky(Sigma_q)
    w = torch.linalg.solve_triangular(Lhat, v[:, :, None], upper=False)[:, :, 0]
    return o * torch.exp(-0.5 * (w * w).sum(dim=1))


def modulated_opacity(o: torch.Tensor, Sigma_q: torch.Tensor, v: torch.Tensor,
                      b_q: torch.Tensor) -> torch.Tensor:
    """o(q) = o prod_i (1 - tanh(w_i^2))^(4 beta_qi), w = Lhat^-1 (q - mu_q).

    Lhat is the Cholesky factor of Sigma_q (Sigma_q = Lhat Lhat^T, Lhat lower
    with positive diagonal; the paper writes the transposes the other way
    round) -- Section 4.3, equation (d).
    Shapes: o [n], Sigma_q [n,C,C], v [n,C], b_q [n,C].
    """
    if v.shape[1] == 0:
        return o
    Lhat = torch.linalg.cholesky(Sigma_q)
    w = torch.linalg.solve_triangular(Lhat, v[:, :, None], upper=False)[:, :, 0]
    d_raw = w * w
    expo = 4.0 * beta_q(b_q)
    # (1 - d_i)^e with d_i = tanh(d_raw): evaluated as exp(e log(1 - tanh x))
    # through the exact identity log(1 - tanh x) = log 2 - 2x - log1p(e^-2x)
    # (x >= 0); the direct form rounds 1 - tanh x to 0 once x > ~19 and then
    # gives 0^e = 0 even for e -> 0.
    log1md = math.log(2.0) - 2.0 * d_raw - torch.log1p(torch.exp(-2.0 * d_raw))
    return o * torch.exp((expo * log1md).sum(dim=1))


def condition(mu_x: torch.Tensor, Sigma: torch.Tensor, v: torch.Tensor,
              b_q: torch.Tensor, beta_modulated: bool = True):
    """Beta-modulated conditional mean and covariance (Section 4.3).

    mu_{x|q} = mu_x + Sigma_xq Sigma_q^-1 diag(bt) (q - mu_q)
    Sigma_{x|q} = Sigma_x - Sigma_xq Sigma_q^-1 diag(bt) Sigma_qx
    Reading: Sigma_{x|q} is symmetrised, (M + M^T)/2, since diag(bt) does not
    commute with Sigma_q^-1 when the modulation differs per dimension.
    beta_modulated=False is the "w/o Beta condition" ablation (Sec. 5.3):
    bt = 1, the Gaussian conditional.
    Shapes: mu_x [n,3], Sigma [n,N,N], v [n,C], b_q [n,C].
    """
    C = v.shape[1]
    Sx = Sigma[:, :3, :3]
    if C == 0:
        return mu_x, Sx
    Sxq = Sigma[:, :3, 3:]
    Sq = Sigma[:, 3:, 3:]
    K = torch.linalg.solve(Sq, Sxq.transpose(-1, -2)).transpose(-1, -2)  # Sxq Sq^-1 (Sq symmetric)
    bt = beta_tilde(b_q) if beta_modulated else torch.ones_like(b_q)
    D = torch.diag_embed(bt)
    KD = K @ D
    mu_c = mu_x + (KD @ v[:, :, None])[:, :, 0]
    M = KD @ Sxq.transpose(-1, -2)
    S_c = Sx - 0.5 * (M + M.transpose(-1, -2))
    return mu_c, S_c


# --------------------------------------------------------------------------
# Section 3: projection to a screen-space splat
# --------------------------------------------------------------------------
def project(mu_c: torch.Tensor, S_c: torch.Tensor, view):
    """Pinhole projection of the conditioned 3-D kernel (Section 3).

    p = W mu + t (camera frame, OpenCV axes), J = d(pixel)/dp,
    Sigma' = J W Sigma W^T J^T + 0.3 I, conic = Sigma'^-1.
    Reading: no field-of-view clamp of J; near plane 0.2; pixel (i, j) has
    its centre at (i + 0.5, j + 0.5) with the principal point (cx, cy).
    Returns mean2d [n,2], Sigma' [n,2,2], depth [n] (= p_z).
    """
    Rw = torch.as_tensor(view.R, dtype=F64)
    tw = torch.as_tensor(view.t, dtype=F64)
    p = mu_c @ Rw.T + tw[None, :]
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    zs = torch.where(z > NEAR_PLANE, z, torch.ones_like(z))   # keep culled lanes finite
    fx, fy = float(view.fx), float(view.fy)
    zero = torch.zeros_like(zs)
    J = torch.stack([
        torch.stack([fx / zs, zero, -fx * x / (zs * zs)], -1),
        torch.stack([zero, fy / zs, -fy * y / (zs * zs)], -1),
    ], -2)
    T = J @ Rw
    Sp = T @ S_c @ T.transpose(-1, -2) + DILATION * torch.eye(2, dtype=F64)
    mean2d = torch.stack([fx * x / zs + float(view.cx), fy * y / zs + float(view.cy)], -1)
    return mean2d, Sp, z


def conic(Sp: torch.Tensor, det: torch.Tensor):
    """The conic A = Sigma'^-1 of a 2x2 covariance, as (a, b, c) with
    r = a dx^2 + 2 b dx dy + c dy^2 the squared Mahalanobis distance
    (Section 3, equation r).  ``det`` is det Sigma' (any nonzero value for a
    culled splat)."""
    return Sp[:, 1, 1] / det, -Sp[:, 0, 1] / det, Sp[:, 0, 0] / det


# --------------------------------------------------------------------------
# full per-primitive step: parameters -> screen-space records
# --------------------------------------------------------------------------
REC_FIELDS = ("mx", "my", "a", "b", "c", "rho", "o", "beta", "r", "g", "bl", "depth")


def preprocess(params: torch.Tensor, dim: int, rot: int, view,
               q_override: Optional[torch.Tensor] = None,
               variant: tuple = ()) -> Dict[str, torch.Tensor]:
    """Records for every primitive in one view (differentiable in params).

    params: float64 [F][n].  Returns a dict with ``rec`` [n,12] (the fields of
    REC_FIELDS), ``valid`` [n] bool and intermediates for tests.
    Culling (Reading): p_z <= 0.2, Sigma' not positive definite, or
    o(q) < 1/255.  rho = 1 - (255 o(q))^(-1/beta_x) is the largest r with
    o(q) (1 - r)^beta_x >= 1/255 (Section 3 Beta kernel, support r < 1).
    variant: any of NO_BETA_CONDITION, NO_BETA_OPACITY (Sec. 5.3 ablations).
    """
    sl = field_slices(dim, rot)
    C = dim - 3
    f = {k: params[s] for k, s in sl.items() if k != "_F"}
    n = params.shape[1]
    L = lower_factor(f, dim, rot)
    Sigma = covariance(L)
    mu_x = f["mu_x"].T
    q = query(f["mu_x"], view, C) if q_override is None else q_override
    v = q - f["mu_q"].T if C > 0 else torch.zeros(n, 0, dtype=F64)
    b_q = f["b_q"].T
    o = f["o"][0]
    if NO_BETA_OPACITY in variant:
        o_q = gaussian_opacity(o, Sigma[:, 3:, 3:], v)
    else:
        o_q = modulated_opacity(o, Sigma[:, 3:, 3:], v, b_q)
    mu_c, S_c = condition(mu_x, Sigma, v, b_q, beta_modulated=NO_BETA_CONDITION not in variant)
    mean2d, Sp, depth = project(mu_c, S_c, view)
    det = Sp[:, 0, 0] * Sp[:, 1, 1] - Sp[:, 0, 1] * Sp[:, 1, 0]
    valid = (depth > NEAR_PLANE) & (det > 0) & (Sp[:, 0, 0] > 0) & (Sp[:, 1, 1] > 0) \
        & (o_q >= ALPHA_MIN)
    a, b, c = conic(Sp, torch.where(valid, det, torch.ones_like(det)))
    beta_x = beta_of_b(f["b_x"][0])
    o_qs = torch.where(valid, o_q, torch.ones_like(o_q))
    rho = 1.0 - (255.0 * o_qs) ** (-1.0 / beta_x)
    rgb = f["rgb"].T
    rec = torch.stack([mean2d[:, 0], mean2d[:, 1], a, b, c, rho, o_q, beta_x,
                       rgb[:, 0], rgb[:, 1], rgb[:, 2], depth], -1)
    zero = torch.zeros_like(rec)
    rec = torch.where(valid[:, None], rec, zero)
    return {"rec": rec, "valid": valid, "Sigma": Sigma, "L": L, "q": q, "v": v,
            "o_q": o_q, "mu_c": mu_c, "S_c": S_c, "Sp": Sp, "depth": depth,
            "mean2d": mean2d, "beta_x": beta_x}
