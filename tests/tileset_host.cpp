// Host driver for the tile-list rule of the HIP library (tileset.hpp), built
// with the host compiler by test_tile_rule.py: reads one ellipse per line
// (mx my a b c Q W H sh as hexadecimal floats / integers) and prints, per
// ellipse, its tile box and the run of every row of the box.
#include <cstdio>

#include "tileset.hpp"

int main() {
  double mx, my, a, b, c, Q;
  int W, H, sh;
  while (std::scanf("%la %la %la %la %la %la %d %d %d", &mx, &my, &a, &b, &c, &Q, &W, &H, &sh) ==
         9) {
    r4d::TileBox bx;
    if (!r4d::tile_box(mx, my, a, b, c, Q, W, H, sh, bx)) {
      std::printf("none\n");
      continue;
    }
    const r4d::SpanGeom g = r4d::span_geom(mx, my, a, b, c, Q, W, H, sh, bx.x0, bx.x1);
    std::printf("box %d %d %d %d", bx.x0, bx.y0, bx.x1, bx.y1);
    for (int ty = bx.y0; ty < bx.y1; ++ty) {
      int x0, x1;
      r4d::row_span(g, ty, x0, x1);
      std::printf(" %d %d", x0, x1);
    }
    std::printf("\n");
  }
  return 0;
}
