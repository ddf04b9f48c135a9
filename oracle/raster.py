"""ctypes wrappers of the oracle's plain-C compositing, adjoint and binning.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build

_lib = None

# relative bands for the ambiguity flags (alpha/r thresholds, T stop, depth
# order, 0.99 clamp, o(q) against 1/255 of an ambiguous record); see raster.c.
# A float32 renderer evaluates sigma = o (1 - r)^beta to ~1e-6 relative
# (exp2/log2 of an exponent of magnitude up to ~8), T over tens of factors to
# a few 1e-6, o(q) to a few 1e-7, and rounds depths to float32 (6e-8):
# the bands are about ten times those.
DEFAULT_BANDS = (1e-5, 1e-5, 1e-6, 1e-5, 1e-5)

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I = ctypes.POINTER(ctypes.c_int)
_U = ctypes.POINTER(ctypes.c_uint)
_U8 = ctypes.POINTER(ctypes.c_ubyte)
_U64 = ctypes.POINTER(ctypes.c_uint64)
_U32 = ctypes.POINTER(ctypes.c_uint32)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = load(path)
    return _lib


def load(path: str):
    """Open a build of ``raster.c`` at ``path`` and declare its signatures."""
    L = ctypes.CDLL(path)
    L.oracle_render_fwd.argtypes = [ctypes.c_int, _D, _U8, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, _D, _D, _D, _I, _U]
    L.oracle_render_pixels.argtypes = [ctypes.c_int, _D, _U8, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _I, _I, _D, _D, _D, _I, _U]
    L.oracle_render_bwd.argtypes = [ctypes.c_int, _D, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, _D, _D, _D, _D]
    L.oracle_bin.restype = ctypes.c_int64
    L.oracle_bin.argtypes = [ctypes.c_int, _F, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                             _U64, _U32]
    L.oracle_tile_hit.argtypes = [ctypes.c_double] * 10
    L.oracle_tile_hit.restype = ctypes.c_int
    L.oracle_set_bin_prefilter.argtypes = [ctypes.c_int]
    L.oracle_set_bin_prefilter.restype = None
    return L


def _p(a, t):
    return a.ctypes.data_as(t)


def render_fwd(rec: np.ndarray, W: int, H: int, amb: Optional[np.ndarray] = None,
               rows=None, bands=DEFAULT_BANDS):
    """Composite float64 records [n,12].  Returns image [H,W,3], T_final,
    contributor counts and ambiguity flags (see raster.c)."""
    rec = np.ascontiguousarray(rec, dtype=np.float64)
    n = rec.shape[0]
    y0, y1 = (0, H) if rows is None else rows
    img = np.zeros((H, W, 3))
    tf = np.ones((H, W))
    nc = np.zeros((H, W), dtype=np.int32)
    fl = np.zeros((H, W), dtype=np.uint32)
    ambp = None
    if amb is not None:
        amb = np.ascontiguousarray(amb, dtype=np.uint8)
        ambp = _p(amb, _U8)
    bd = np.asarray(bands, dtype=np.float64)
    lib().oracle_render_fwd(n, _p(rec, _D), ambp, W, H, y0, y1, _p(bd, _D), _p(img, _D),
                            _p(tf, _D), _p(nc, _I), _p(fl, _U))
    return img, tf, nc, fl


def render_pixels(rec: np.ndarray, W: int, H: int, xs, ys, amb=None, bands=DEFAULT_BANDS):
    """Composite only the listed pixels; returns colour [m,3], T, counts, flags."""
    rec = np.ascontiguousarray(rec, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    m = xs.shape[0]
    col = np.zeros((m, 3))
    tf = np.ones(m)
    nc = np.zeros(m, dtype=np.int32)
    fl = np.zeros(m, dtype=np.uint32)
    ambp = None
    if amb is not None:
        amb = np.ascontiguousarray(amb, dtype=np.uint8)
        ambp = _p(amb, _U8)
    bd = np.asarray(bands, dtype=np.float64)
    lib().oracle_render_pixels(rec.shape[0], _p(rec, _D), ambp, W, H, m, _p(xs, _I), _p(ys, _I),
                               _p(bd, _D), _p(col, _D), _p(tf, _D), _p(nc, _I), _p(fl, _U))
    return col, tf, nc, fl


def render_bwd(rec: np.ndarray, W: int, H: int, d_image: np.ndarray,
               d_tfinal: Optional[np.ndarray] = None, with_abs: bool = False, rows=None):
    """Adjoint of the compositing: d_rec [n,10] = (d mx, d my, d a, d b, d c,
    d o, d beta, d r, d g, d bl).  With ``with_abs`` also returns the sums of
    the absolute per-pixel terms (the scale of float32 summation error)."""
    rec = np.ascontiguousarray(rec, dtype=np.float64)
    gi = np.ascontiguousarray(d_image, dtype=np.float64)
    gt = None if d_tfinal is None else np.ascontiguousarray(d_tfinal, dtype=np.float64)
    out = np.zeros((rec.shape[0], 10))
    ab = np.zeros((rec.shape[0], 10)) if with_abs else None
    y0, y1 = (0, H) if rows is None else rows
    lib().oracle_render_bwd(rec.shape[0], _p(rec, _D), W, H, y0, y1, _p(gi, _D),
                            None if gt is None else _p(gt, _D), _p(out, _D),
                            None if ab is None else _p(ab, _D))
    return (out, ab) if with_abs else out


def tile_hit(mx, my, a, b, c, rho, x0, x1, y0, y1) -> bool:
    return bool(lib().oracle_tile_hit(mx, my, a, b, c, rho, x0, x1, y0, y1))


def bin_view(rec32: np.ndarray, W: int, H: int, tile_w: int = 16, tile_h: int = 16,
             tile_base: int = 0, rec_base: int = 0, full_scan: bool = False):
    """Binning reference for one view: keys (uint64) and values (uint32) in
    emission order (record index, then tiles row-major).  Each record's
    tiles are tested inside a float64 bounding window of its ellipse; with
    ``full_scan`` every tile of the view is tested (same result, slower)."""
    rec32 = np.ascontiguousarray(rec32, dtype=np.float32)
    n = rec32.shape[0]
    L = lib()
    L.oracle_set_bin_prefilter(0 if full_scan else 1)
    try:
        total = L.oracle_bin(n, _p(rec32, _F), W, H, tile_w, tile_h, tile_base, rec_base, 0,
                             None, None)
        keys = np.zeros(max(total, 1), dtype=np.uint64)
        vals = np.zeros(max(total, 1), dtype=np.uint32)
        L.oracle_bin(n, _p(rec32, _F), W, H, tile_w, tile_h, tile_base, rec_base, total,
                     _p(keys, _U64), _p(vals, _U32))
    finally:
        L.oracle_set_bin_prefilter(1)
    return keys[:total], vals[:total]


def sort_and_ranges(keys: np.ndarray, vals: np.ndarray, n_tiles: int):
    """Stable sort by key (numpy), then per-tile [start, end) ranges; empty
    tiles get (0, 0)."""
    order = np.argsort(keys, kind="stable")
    sk, sv = keys[order], vals[order]
    ranges = np.zeros((n_tiles, 2), dtype=np.uint32)
    if sk.size:
        tiles = (sk >> np.uint64(32)).astype(np.int64)
        starts = np.flatnonzero(np.r_[True, tiles[1:] != tiles[:-1]])
        ends = np.r_[starts[1:], sk.size]
        ranges[tiles[starts], 0] = starts
        ranges[tiles[starts], 1] = ends
    return sk, sv, ranges
