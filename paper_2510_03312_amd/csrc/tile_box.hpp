// Candidate tiles of a screen-space record for the binning: the tile
// rectangle holding every pixel centre where r(p) = a dx^2 + 2 b dx dy +
// c dy^2 can reach rho (1 + 2^-10), the threshold of the exact overlap test.
//
// The extents are taken in float64.  The conic entries are float32, so the
// products a c and b b are exact in float64 and det = a c - b b carries a
// single rounding however elongated the ellipse (a float32 det cancels and,
// for axis ratios beyond ~1e3, can shrink the box below what the exact test
// accepts, or round to zero).  The half-widths sqrt(rb c / det),
// sqrt(rb a / det) are then within a few ulps; the box uses the threshold
// rho (1 + 2^-9) and a 2-pixel pad on top.  A conic that is not positive
// definite (det <= 0 exactly) has an unbounded sublevel set: its box is the
// whole view.  Records with rho <= 0 (culled) or a non-positive diagonal
// entry get an empty box.
//
// Host and device compile this identically (float64, no contraction), so a
// host program can check the box against the exact tile test.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace ubs {

struct TileBox {
  int tx0, tx1, ty0, ty1;  // inclusive; empty if tx0 > tx1
};

#pragma clang fp contract(off)
__host__ __device__ inline TileBox tile_box_of(float mx, float my, float a, float b, float c,
                                               float rho, int W, int H, int tile_w, int tile_h) {
  TileBox bx{1, 0, 1, 0};
  if (!(rho > 0.0f) || !(a > 0.0f) || !(c > 0.0f)) return bx;
  const int tiles_x = (W + tile_w - 1) / tile_w, tiles_y = (H + tile_h - 1) / tile_h;
  const double da = a, db = b, dc = c;
  const double det = da * dc - db * db;
  if (!(det > 0.0)) {
    bx.tx0 = 0;
    bx.tx1 = tiles_x - 1;
    bx.ty0 = 0;
    bx.ty1 = tiles_y - 1;
    return bx;
  }
  const double rb = double(rho) * (1.0 + 0x1p-9);
  const double ex = sqrt(rb * dc / det), ey = sqrt(rb * da / det);
  const double xl = (double(mx) - ex) - 2.0, xh = (double(mx) + ex) + 2.0;
  const double yl = (double(my) - ey) - 2.0, yh = (double(my) + ey) + 2.0;
  if (!(xh >= 0.0) || !(yh >= 0.0) || !(xl <= double(W)) || !(yl <= double(H))) return bx;
  bx.tx0 = int(floor(fmax(xl, 0.0) / double(tile_w)));
  bx.tx1 = int(floor(fmin(xh, double(W)) / double(tile_w)));
  bx.ty0 = int(floor(fmax(yl, 0.0) / double(tile_h)));
  bx.ty1 = int(floor(fmin(yh, double(H)) / double(tile_h)));
  if (bx.tx1 > tiles_x - 1) bx.tx1 = tiles_x - 1;
  if (bx.ty1 > tiles_y - 1) bx.ty1 = tiles_y - 1;
  return bx;
}
#pragma clang fp contract(on)

}  // namespace ubs
