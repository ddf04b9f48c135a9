"""Seeded scene, camera and target generators.

Every array here is drawn from ``numpy.random.default_rng(seed)`` in a fixed
order, so the product path and the oracle see bit-identical inputs.  Nothing
in this module evaluates the rendering method; it only draws numbers and
places them in the input formats documented in ``include/ubs.h``.

Primitive parameter format (float32, component-major ``[F][n]``), rows in
this order, with ``C = dim - 3`` query dimensions:

====================  ===========  =========================================
field                 rows         notes
====================  ===========  =========================================
``mu_x``              3            spatial mean (world units)
``mu_q``              C            query mean; 7-D order is ``[t, d0, d1, d2]``,
                                   N > 7 appends the view's extra query values
``rot``               4 or 3       quaternion ``(w, x, y, z)`` or skew ``w``
``log_s_x``           3            log of the spatial scales
``L_qx``              3*C          C x 3 block, row-major
``L_q``               C*(C+1)/2    lower triangle, row-major, diagonal as log
``b_x``               1            spatial Beta shape
``b_q``               C            per-query-dimension Beta shapes
``o``                 1            opacity in [0, 1] (already activated)
``rgb``               3            colour in [0, 1]
====================  ===========  =========================================

Workload recipes (the paper's datasets are not available, so these seeded
scenes stand in for them, at the paper's primitive counts):

* ``cfg0``: 2,000 static 3-D primitives, 128x128, camera at z = -4.
* ``cfg1``: 500,000 6-D primitives, 1264x832, forward only.
* ``dim10``: 1,000,000 10-D primitives (the 7-D query plus three values
  given by the view), 1920x1080, forward and backward.
* ``cfg2``: 1,000,000 6-D primitives, 1920x1080, forward and backward.
* ``headline``: 1,000,000 7-D primitives, 1920x1080, t = 0.5, fwd+bwd.
* ``cfg3``: 2,000,000 7-D primitives, 8 views of 1352x1014 on a circle.
* ``cfg4``: 4 scenes (100k / 500k / 1.5M / 3M, 7-D), 32 views of uneven
  resolution.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

ROT_QUAT = 0
ROT_SKEW = 1


def _rot_rows(rot: int) -> int:
    return 4 if rot == ROT_QUAT else 3


def param_count(dim: int, rot: int = ROT_QUAT) -> int:
    """Rows of the parameter array for a ``dim``-D scene (see module doc)."""
    c = dim - 3
    return 3 + c + _rot_rows(rot) + 3 + 3 * c + c * (c + 1) // 2 + 1 + c + 1 + 3


@dataclasses.dataclass
class SceneSpec:
    dim: int
    rot: int
    params: np.ndarray  # float32 [F][n]

    @property
    def n(self) -> int:
        return int(self.params.shape[1])


@dataclasses.dataclass
class ViewSpec:
    scene: int
    width: int
    height: int
    R: np.ndarray  # float32 [3][3] world -> camera rotation, OpenCV axes
    t: np.ndarray  # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    time: float = 0.0
    query: tuple = (0.0, 0.0, 0.0)   # query values beyond [t, d] (N > 7)


def look_at_view(center, width: int, height: int, *, scene: int = 0,
                 fov_deg: float = 60.0, time: float = 0.0) -> ViewSpec:
    """Pinhole camera at ``center`` looking at the world origin.

    OpenCV axes (x right, y down, z forward), world "down" = +y, horizontal
    field of view ``fov_deg``, principal point at the image centre.
    """
    c = np.asarray(center, dtype=np.float64)
    f = -c / np.linalg.norm(c)
    down = np.array([0.0, 1.0, 0.0])
    right = np.cross(down, f)
    right /= np.linalg.norm(right)
    dn = np.cross(f, right)
    R = np.stack([right, dn, f], axis=0)
    t = -R @ c
    focal = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return ViewSpec(scene=scene, width=int(width), height=int(height),
                    R=R.astype(np.float32), t=t.astype(np.float32),
                    fx=float(np.float32(focal)), fy=float(np.float32(focal)),
                    cx=width / 2.0, cy=height / 2.0, time=float(time))


def make_view(width: int, height: int, *, scene: int = 0, time: float = 0.0) -> ViewSpec:
    """The single-view camera of the static configs: at (0, 0, -4)."""
    return look_at_view((0.0, 0.0, -4.0), width, height, scene=scene, time=time)


def _normalize_rows(x: np.ndarray) -> np.ndarray:
    return x / np.linalg.norm(x, axis=0, keepdims=True)


def make_scene(dim: int, n: int, seed: int, *, dist: str = "cfg0",
               rot: int = ROT_QUAT) -> SceneSpec:
    """Draw ``n`` primitives of dimension ``dim`` with the named distribution.

    ``dist`` is one of ``cfg0`` (centres in [-1, 1]^3), ``cfg1`` (centres
    N(0, 1.5^2), angular block) or ``cfg3`` (``cfg1`` plus a temporal block).
    Draws are made field by field in the layout order.
    """
    if dim < 3:
        raise ValueError("dim must be >= 3")
    c = dim - 3
    rng = np.random.default_rng(seed)
    rows: List[np.ndarray] = []
    # mu_x
    if dist == "cfg0":
        rows.append(rng.uniform(-1.0, 1.0, size=(3, n)))
    else:
        rows.append(rng.normal(0.0, 1.5, size=(3, n)))
    # mu_q: [t, d] for 7-D, d for 6-D, [t, d, extra U(0, 1)] beyond 7-D,
    # generic U(0, 1) otherwise
    if c > 0:
        mq = np.empty((c, n))
        k = 0
        if c >= 4:
            mq[0] = rng.uniform(0.0, 1.0, size=n)
            k = 1
        if c - k == 3:
            mq[k:] = _normalize_rows(rng.normal(0.0, 1.0, size=(3, n)))
        elif c > 4:
            mq[1:4] = _normalize_rows(rng.normal(0.0, 1.0, size=(3, n)))
            mq[4:] = rng.uniform(0.0, 1.0, size=(c - 4, n))
        else:
            mq[k:] = rng.uniform(0.0, 1.0, size=(c - k, n))
        rows.append(mq)
    # rotation
    if rot == ROT_QUAT:
        rows.append(_normalize_rows(rng.normal(0.0, 1.0, size=(4, n))))
    else:
        rows.append(rng.normal(0.0, 0.3, size=(3, n)))
    # log spatial scales
    rows.append(rng.normal(-3.0, 0.3, size=(3, n)))
    if c > 0:
        # L_qx (C x 3, row-major)
        rows.append(rng.normal(0.0, 0.3, size=(3 * c, n)))
        # L_q lower triangle, row-major, diagonal stored as log scale
        lq = np.empty((c * (c + 1) // 2, n))
        k = 0
        for i in range(c):
            for j in range(i + 1):
                if i == j:
                    if c >= 4 and i == 0:
                        lq[k] = np.log(rng.uniform(0.02, 0.5, size=n))
                    else:
                        lq[k] = np.log(rng.uniform(0.2, 2.0, size=n))
                else:
                    lq[k] = rng.normal(0.0, 0.1, size=n)
                k += 1
        rows.append(lq)
    # b_x, b_q
    rows.append(rng.uniform(-1.0, 1.0, size=(1, n)))
    if c > 0:
        rows.append(rng.uniform(-1.0, 1.0, size=(c, n)))
    # opacity (activated) and colour
    rows.append(1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, size=(1, n)))))
    rows.append(rng.uniform(0.0, 1.0, size=(3, n)))
    params = np.ascontiguousarray(np.concatenate(rows, axis=0).astype(np.float32))
    assert params.shape[0] == param_count(dim, rot)
    return SceneSpec(dim=dim, rot=rot, params=params)


def make_target(height: int, width: int, seed: int = 1) -> np.ndarray:
    """Random U(0, 1) target image, float32 [H][W][3]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(height, width, 3)).astype(np.float32)


CONFIG_NAMES = ("cfg0", "cfg1", "cfg2", "headline", "cfg3", "cfg4", "dim10")


def make_config(name: str, *, n: Optional[int] = None, width: Optional[int] = None,
                height: Optional[int] = None, rot: int = ROT_QUAT,
                n_views: Optional[int] = None, scene_sizes=None) -> dict:
    """Build a named workload: scenes, views, per-view targets, mode.

    The keyword overrides shrink a workload for tests while keeping its
    distributions (``n`` primitives, ``width`` x ``height`` pixels).
    """
    if name == "cfg0":
        sc = make_scene(3, n or 2000, 0, dist="cfg0", rot=rot)
        W, H = width or 128, height or 128
        views = [make_view(W, H)]
        mode = "fwdbwd"
        scenes = [sc]
    elif name == "cfg1":
        sc = make_scene(6, n or 500_000, 0, dist="cfg1", rot=rot)
        W, H = width or 1264, height or 832
        views = [make_view(W, H)]
        mode = "fwd"
        scenes = [sc]
    elif name == "cfg2":
        sc = make_scene(6, n or 1_000_000, 0, dist="cfg1", rot=rot)
        W, H = width or 1920, height or 1080
        views = [make_view(W, H)]
        mode = "fwdbwd"
        scenes = [sc]
    elif name == "headline":
        sc = make_scene(7, n or 1_000_000, 0, dist="cfg3", rot=rot)
        W, H = width or 1920, height or 1080
        views = [make_view(W, H, time=0.5)]
        mode = "fwdbwd"
        scenes = [sc]
    elif name == "dim10":
        # beyond 7-D: the headline's 1M primitives with three further query
        # dimensions whose values come with the view
        sc = make_scene(10, n or 1_000_000, 0, dist="cfg3", rot=rot)
        W, H = width or 1920, height or 1080
        v = make_view(W, H, time=0.5)
        v.query = (0.2, 0.7, 0.5)
        views = [v]
        mode = "fwdbwd"
        scenes = [sc]
    elif name == "cfg3":
        sc = make_scene(7, n or 2_000_000, 0, dist="cfg3", rot=rot)
        W, H = width or 1352, height or 1014
        nv = n_views or 8
        views = []
        for k in range(nv):
            th = 2.0 * math.pi * k / nv
            views.append(look_at_view((4.0 * math.sin(th), 0.0, -4.0 * math.cos(th)),
                                      W, H, time=k / max(nv - 1, 1)))
        mode = "fwdbwd"
        scenes = [sc]
    elif name == "cfg4":
        sizes = scene_sizes or (100_000, 500_000, 1_500_000, 3_000_000)
        scenes = [make_scene(7, int(sz), s, dist="cfg3", rot=rot) for s, sz in enumerate(sizes)]
        nv = n_views or 32
        choices = [(640, 480), (1280, 720), (1920, 1080)]
        pick = np.random.default_rng(4).integers(0, 3, size=nv)
        views = []
        for j in range(nv):
            w, h = choices[int(pick[j])]
            if width is not None:
                w, h = width, height
            th = 2.0 * math.pi * j / nv
            views.append(look_at_view((4.0 * math.sin(th), 0.0, -4.0 * math.cos(th)),
                                      w, h, scene=j % len(scenes), time=j / max(nv - 1, 1)))
        mode = "fwdbwd"
    else:
        raise KeyError(name)
    targets = [make_target(v.height, v.width, seed=1 + k) for k, v in enumerate(views)]
    return {"name": name, "scenes": scenes, "views": views, "targets": targets, "mode": mode}


def make_splat_records(n: int, width: int, height: int, seed: int,
                       *, cull_frac: float = 0.1, max_extent: float = 40.0) -> np.ndarray:
    """Random screen-space splat records, float32 [n][12].

    Record layout (``include/ubs.h``): mean x, mean y, conic a, conic b,
    conic c, support rho, opacity, beta, r, g, b, depth.  The conic is drawn
    directly as a positive-definite quadratic form; a ``cull_frac`` share of
    records gets rho = 0 (culled).
    """
    rng = np.random.default_rng(seed)
    rec = np.zeros((n, 12), dtype=np.float64)
    rec[:, 0] = rng.uniform(-0.1 * width, 1.1 * width, size=n)
    rec[:, 1] = rng.uniform(-0.1 * height, 1.1 * height, size=n)
    ex = np.exp(rng.uniform(math.log(0.6), math.log(max_extent), size=n))
    ey = np.exp(rng.uniform(math.log(0.6), math.log(max_extent), size=n))
    corr = rng.uniform(-0.95, 0.95, size=n)
    a = 1.0 / (ex * ex)
    c = 1.0 / (ey * ey)
    rec[:, 2] = a
    rec[:, 3] = corr * np.sqrt(a * c)
    rec[:, 4] = c
    rec[:, 5] = rng.uniform(0.05, 0.999, size=n)
    rec[:, 6] = rng.uniform(0.05, 1.0, size=n)
    rec[:, 7] = np.exp(rng.uniform(math.log(0.3), math.log(30.0), size=n))
    rec[:, 8:11] = rng.uniform(0.0, 1.0, size=(n, 3))
    rec[:, 11] = rng.uniform(0.3, 10.0, size=n)
    culled = rng.uniform(size=n) < cull_frac
    rec[culled, 5] = 0.0
    return rec.astype(np.float32)


def make_elongated_records(n: int, width: int, height: int, seed: int,
                           *, ratio=(1e4, 1e8), minor=(0.3, 4.0)) -> np.ndarray:
    """Screen-space records of very elongated splats, float32 [n][12] (the
    layout of ``make_splat_records``): the 2-D covariance has eigenvalues
    lam1 in ``minor`` (px^2) and lam1 * ratio, ratio log-uniform in
    ``ratio``, at a uniform angle (a fifth of them within 1e-3 rad of an
    axis); the conic is its inverse, rounded to float32 (for the largest
    ratios the rounded conic can lose positive definiteness)."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, math.pi, size=n)
    near_axis = rng.uniform(size=n) < 0.2
    th[near_axis] = (rng.integers(0, 4, size=int(near_axis.sum())) * (math.pi / 2)
                     + rng.uniform(-1e-3, 1e-3, size=int(near_axis.sum())))
    l1 = rng.uniform(minor[0], minor[1], size=n)
    l2 = l1 * np.exp(rng.uniform(math.log(ratio[0]), math.log(ratio[1]), size=n))
    cs, sn = np.cos(th), np.sin(th)
    rec = np.zeros((n, 12), dtype=np.float64)
    rec[:, 0] = rng.uniform(-0.2 * width, 1.2 * width, size=n)
    rec[:, 1] = rng.uniform(-0.2 * height, 1.2 * height, size=n)
    rec[:, 2] = cs * cs / l1 + sn * sn / l2
    rec[:, 3] = cs * sn * (1.0 / l1 - 1.0 / l2)
    rec[:, 4] = sn * sn / l1 + cs * cs / l2
    rec[:, 5] = rng.uniform(0.05, 0.999, size=n)
    rec[:, 6] = rng.uniform(0.05, 1.0, size=n)
    rec[:, 7] = np.exp(rng.uniform(math.log(0.3), math.log(30.0), size=n))
    rec[:, 8:11] = rng.uniform(0.0, 1.0, size=(n, 3))
    rec[:, 11] = rng.uniform(0.3, 10.0, size=n)
    return rec.astype(np.float32)
