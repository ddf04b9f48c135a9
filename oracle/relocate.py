"""Relocation of dead primitives (Sec. 4.5, "Densification"; the MCMC
primitive management the paper adopts from Deformable Beta Splatting).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): plain float64 numpy,
written from the paper, used to check the HIP kernels.

Steps, in the paper's terms:
  1. a primitive is dead when its opacity is below o_min; the others are
     live;
  2. every dead slot picks a live primitive with probability proportional to
     its opacity (the random numbers are inputs: uniform u_k in [0, 1) for
     the k-th dead slot in index order), by inverse-CDF sampling over the
     running sum of the live opacities (if u_k * total rounds to the total,
     the last live primitive);
  3. a live primitive picked by N - 1 dead slots becomes N identical copies
     (itself and the slots), each with opacity o' = 1 - (1 - o)^(1/N), so
     that the N copies composite to the original opacity (the paper's
     cloning rule); all other parameters are copied unchanged (the paper:
     adjusting the opacity alone keeps the density, whatever the kernel);
  4. the Adam moments of every primitive whose parameters changed (the
     copies and their source) are reset to zero.
Readings (the paper is silent): o_min defaults to 0.005; a primitive that
is not finite counts as dead; with no live primitive nothing moves.

The CDF is exact in float64: live opacities are float32 values >= o_min, so
every partial sum is a multiple of 2^-31 below 2^22 (for n < 2^22), and the
pick of slot k is the first index whose inclusive sum exceeds u_k * total
(that product rounded once, in float64).
"""
from __future__ import annotations

import numpy as np

from .preprocess import field_slices

O_MIN = 0.005


def cloned_opacity(o: np.ndarray, copies: np.ndarray) -> np.ndarray:
    """o' = 1 - (1 - o)^(1/N): N copies of o' composite to o."""
    return 1.0 - np.power(1.0 - np.asarray(o, dtype=np.float64), 1.0 / np.asarray(copies, dtype=np.float64))


def relocate(params: np.ndarray, m: np.ndarray, v: np.ndarray, uniforms: np.ndarray, dim: int,
             rot: int, o_min: float = O_MIN):
    """Returns (params, m, v, targets) with targets[k] the primitive the k-th
    dead slot copies (index order of the dead slots); inputs are not modified."""
    sl = field_slices(dim, rot)
    P = np.array(params, dtype=np.float64)
    M = np.array(m, dtype=np.float64)
    V = np.array(v, dtype=np.float64)
    o = P[sl["o"].start]
    finite = np.all(np.isfinite(P), axis=0)
    live = finite & (o >= o_min)
    dead = np.flatnonzero(~live)
    if dead.size == 0 or not live.any():
        return P, M, V, np.zeros(0, dtype=np.int64)
    w = np.where(live, o, 0.0)
    cdf = np.cumsum(w)
    total = cdf[-1]
    x = np.asarray(uniforms[:dead.size], dtype=np.float64) * total
    targets = np.searchsorted(cdf, x, side="right")
    # u within an ulp of 1 can round x up to the total: the last live one
    targets[targets >= cdf.size] = np.searchsorted(cdf, total, side="left")
    copies = 1 + np.bincount(targets, minlength=P.shape[1])
    picked = np.flatnonzero(copies > 1)
    o_new = cloned_opacity(o[picked], copies[picked])
    P[:, dead] = P[:, targets]
    P[sl["o"].start, picked] = o_new
    P[sl["o"].start, dead] = o_new[np.searchsorted(picked, targets)]
    for idx in (dead, picked):
        M[:, idx] = 0.0
        V[:, idx] = 0.0
    return P, M, V, targets
