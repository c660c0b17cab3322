// Prints the launch shapes the stencil rules choose (test driver for
// tests/test_launch_rules.py; host arithmetic only).
//   launch_rules_cli pair <nx> <ny> <nz> <esz> <cus> <per_cu_narrow> <per_cu_wide>
//     -> "<tile_x> <tile_y> <zchunk> <groups> <pairs>" of the two-step kernel (FP32
//        3D compares the 64 x 16 and 128 x 16 tiles; FP64 takes 64 x 16; pairs = 1
//        where FP32 runs over pairs of x-adjacent points, tile in points)
//   launch_rules_cli step <nx> <ny> <nz> <esz>
//     -> "<tile_x> <tile_y> <zchunk>" of the one-step kernel (about 2048 groups)
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "launch_rules.h"

int main(int argc, char **argv)
{
  if (argc >= 6 && !strcmp(argv[1], "step")) {
    const int nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]), esz = atoi(argv[5]);
    const int by = 4 * ffpat::step_ry(ny, esz, 0);
    const long xy = (long)((nx + 63) / 64) * ((ny + by - 1) / by);
    printf("64 %d %d\n", by, ffpat::step_zchunk(nz, xy, 2048, 0));
    return 0;
  }
  if (argc >= 9 && !strcmp(argv[1], "pair")) {
    const int nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]), esz = atoi(argv[5]);
    const int cus = atoi(argv[6]), pn = atoi(argv[7]), pw = atoi(argv[8]);
    const bool f64 = esz == 8;
    ffpat::PairShape p = ffpat::pair_shape_for(nx, ny, nz, 64, 16, pn, cus, f64, 0);
    int pairs = 0;
    if (!f64) {
      const ffpat::PairShape w = ffpat::pair_shape_for(nx, ny, nz, 128, 16, pw, cus, false, 0);
      const bool wide = ffpat::pair_wide_better(p, w);
      if (wide) p = w;
      if (ffpat::pair_x_pairs(wide, nx)) {   // one group per unit, as the FP64 kernel
        p = ffpat::pair_shape_for(nx / 2, ny, nz, 64, 16, 1, cus, true, 0);
        p.bx = 128;
        pairs = 1;
      }
    }
    printf("%d %d %d %d %d\n", p.bx, p.by, p.zchunk, p.n_tiles, pairs);
    return 0;
  }
  fprintf(stderr, "usage: launch_rules_cli pair nx ny nz esz cus per_cu_narrow per_cu_wide | step nx ny nz esz\n");
  return 2;
}
