// Host check of the fused tiling rules: the finest level takes 64-plane tiles
// where 2048 of them remain, else 32 planes halved until 512 tiles remain;
// coarse fused levels take the deepest of 16, 8 and 4 planes that leaves 512
// tiles; the fused iteration's SpMV runs on the fused tiles of a problem
// with 2048 of them.  Prints one line per case and exits with the number of
// mismatches.
#include <cstdio>

#include "fld.h"
#include "fld_engine.h"

using namespace fld;

int main() {
  struct Case {
    int n, l, tz, tiles;
    bool spf;
  };
  // n^3 grid, level l (0 finest): expected tile depth and tile count;
  // spf: whether the finest level's SpMV runs on the fused tiles
  const Case cases[] = {
      {640, 0, 64, 10 * 40 * 10, true},  {640, 1, 16, 5 * 20 * 20, true},
      {640, 2, 8, 3 * 10 * 20, true},    {256, 0, 32, 4 * 16 * 8, false},
      {256, 1, 4, 2 * 8 * 32, false},    {512, 0, 64, 8 * 32 * 8, true},
      {128, 0, 4, 2 * 8 * 32, false},    {64, 0, 2, 1 * 4 * 32, false},
  };
  fld_params p;
  fld_default_params(&p, 3e10, 1.0);
  int bad = 0;
  for (const Case &c : cases) {
    const int n = c.n >> c.l;
    int tx, ty, tz;
    fused_shape(p, c.l, n, n, n, tx, ty, tz);
    const int tiles = count_fused_tiles(p, c.l, n, n, n);
    fld_grid g{};
    g.nx = g.ny = g.nz = c.n;
    g.dx = g.dy = g.dz = 1.0;
    const bool spf = spmv_on_fused(make_hier(g, p));
    const bool ok = tz == c.tz && tiles == c.tiles && spf == c.spf && tx == (n < 64 ? n : 64) &&
                    ty == (n < 16 ? n : 16);
    printf("%d^3 level %d: tile %dx%dx%d, %d tiles, fused-tile SpMV %d %s\n", c.n, c.l, tx, ty,
           tz, tiles, spf, ok ? "ok" : "MISMATCH");
    bad += !ok;
  }
  printf("%d mismatches\n", bad);
  return bad;
}
