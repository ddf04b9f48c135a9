"""The binning's candidate-tile box (``csrc/tile_box.hpp``), compiled for the
host, against the oracle's exact tile test: every tile the oracle's binning
reference emits for a record lies inside the record's box.  Records are
very elongated splats (covariance axis ratios 1e4 to 1e8, including float32
conics that are no longer positive definite), where a float32 determinant
cancels; plus the ordinary synthetic records."""
import os
import subprocess

import numpy as np
import pytest

from oracle import raster as oraster
from paper_2510_03312_amd import build as hip_build
from synth import make_elongated_records, make_splat_records

HARNESS = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "tile_box.hpp"
int main(int argc, char** argv) {
  int W = atoi(argv[3]), H = atoi(argv[4]), tw = atoi(argv[5]), th = atoi(argv[6]);
  FILE* f = fopen(argv[1], "rb");
  std::vector<float> r;
  float x;
  while (fread(&x, 4, 1, f) == 1) r.push_back(x);
  fclose(f);
  const size_t n = r.size() / 12;
  std::vector<int> out(4 * n);
  for (size_t i = 0; i < n; ++i) {
    const float* p = &r[12 * i];
    ubs::TileBox b = ubs::tile_box_of(p[0], p[1], p[2], p[3], p[4], p[5], W, H, tw, th);
    out[4 * i] = b.tx0; out[4 * i + 1] = b.tx1; out[4 * i + 2] = b.ty0; out[4 * i + 3] = b.ty1;
  }
  FILE* g = fopen(argv[2], "wb");
  fwrite(out.data(), 4, out.size(), g);
  fclose(g);
  return 0;
}
'''


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(hip_build.HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("tilebox")
    src = d / "box.hip"
    src.write_text(HARNESS)
    exe = d / "box"
    flags = [f for f in hip_build.FLAGS if f not in ("-fPIC",)]
    subprocess.run([hip_build.HIPCC, *flags, str(src), "-o", str(exe)], check=True,
                   capture_output=True)
    return str(exe), d


def _boxes(harness, rec, W, H, tw, th):
    exe, d = harness
    fin, fout = d / "rec.bin", d / "box.bin"
    np.ascontiguousarray(rec, dtype=np.float32).tofile(fin)
    subprocess.run([exe, str(fin), str(fout), str(W), str(H), str(tw), str(th)], check=True)
    return np.fromfile(fout, dtype=np.int32).reshape(-1, 4)


def _check(harness, rec, W, H, tw=16, th=16):
    box = _boxes(harness, rec, W, H, tw, th)
    keys, vals = oraster.bin_view(rec, W, H, tw, th)
    tiles_x = (W + tw - 1) // tw
    tile = (keys >> np.uint64(32)).astype(np.int64)
    tx, ty = tile % tiles_x, tile // tiles_x
    b = box[vals.astype(np.int64)]
    inside = (tx >= b[:, 0]) & (tx <= b[:, 1]) & (ty >= b[:, 2]) & (ty <= b[:, 3])
    assert inside.all(), (np.flatnonzero(~inside)[:5], vals[~inside][:5])
    return keys.size, box


@pytest.mark.parametrize("ratio", [(1e4, 1e5), (1e5, 1e6), (1e6, 1e7), (1e7, 1e8)])
def test_box_holds_every_tile_of_elongated_splats(harness, ratio):
    W, H = 256, 208
    rec = make_elongated_records(6000, W, H, seed=int(np.log10(ratio[0])), ratio=ratio)
    a, b, c = (rec[:, k].astype(np.float64) for k in (2, 3, 4))
    n_indef = int((a * c - b * b <= 0).sum())
    pairs, box = _check(harness, rec, W, H)
    assert pairs > 1000
    if ratio[0] >= 1e7:
        assert n_indef > 0                      # the float32 conic lost definiteness


def test_box_of_an_indefinite_conic_is_the_whole_view(harness):
    rec = make_splat_records(4, 100, 60, seed=1, cull_frac=0.0)
    rec[:, 2], rec[:, 3], rec[:, 4] = 1.0, 1.0, 1.0        # det = 0 exactly
    rec[1, 3] = 2.0                                        # det < 0
    box = _boxes(harness, rec[:2], 100, 60, 16, 16)
    np.testing.assert_array_equal(box, [[0, 6, 0, 3], [0, 6, 0, 3]])
    _check(harness, rec[:2], 100, 60)


def test_box_holds_every_tile_of_ordinary_records(harness):
    for seed, (W, H, tw, th) in enumerate([(200, 150, 16, 16), (37, 23, 8, 8), (300, 90, 32, 16)]):
        rec = make_splat_records(3000, W, H, seed=seed, max_extent=min(60.0, W / 3))
        _check(harness, rec, W, H, tw, th)


def test_culled_and_non_finite_records_get_empty_boxes(harness):
    rec = make_splat_records(5, 64, 64, seed=2, cull_frac=0.0)
    rec[0, 5] = 0.0
    rec[1, 0] = np.nan
    rec[2, 2] = -1.0
    rec[3, 0] = 1e9
    box = _boxes(harness, rec, 64, 64, 16, 16)
    assert (box[:4, 0] > box[:4, 1]).all()
    assert box[4, 0] <= box[4, 1]
