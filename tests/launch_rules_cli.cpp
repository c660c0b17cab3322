// Prints the launch shapes the stencil rules choose (test driver for
// tests/test_launch_rules.py; host arithmetic only).
//   launch_rules_cli pair <nx> <ny> <nz> <esz> <cus> <per_cu_narrow> <per_cu_wide>
//     -> "<tile_x> <tile_y> <zchunk> <groups> <pairs>" of the two-step kernel (FP32
//        3D compares the 64 x 16 and 128 x 16 tiles; FP64 takes 64 x 16; pairs = 1
//        where FP32 runs over pairs of x-adjacent points, tile in points)
//   launch_rules_cli step <nx> <ny> <nz> <esz>
//     -> "<tile_x> <tile_y> <zchunk>" of the one-step kernel (about 2048 groups)
//   launch_rules_cli wide3
//     -> checks the slot layout of the 1024-thread three-step kernel against every
//        LDS access it makes; prints "ok <interior> <ring2> <ring1> <outer>" (the
//        distinct points of each kind) or the first violation
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "launch_rules.h"

// Every LDS access of wave_step3_wide for one thread: base (wide3_bases) + the
// immediate offset the kernel adds (plane slot, 2 rows, the neighbour's shift) must
// stay inside its array and address the intended element: the point's plane slot,
// its row and column shifted by the neighbour, inside that array's plane.
static const char *check_access(int base, int off, int pad, int len, int slot, int pitch, int rows, int x, int y,
                                int dx, int dy)
{
  if (base < 0 || base >= len) return "base outside its array";
  if (off < 0 || off * 8 >= 65536) return "offset beyond an instruction's immediate";
  const int idx = base + off;
  if (idx < 0 || idx >= len) return "access outside its array";
  if (x + dx < 0 || x + dx >= pitch || y + dy < 0 || y + dy >= rows) return "neighbour outside the array's plane";
  if (idx - pad != slot + (y + dy) * pitch + (x + dx)) return "access at the wrong element";
  return nullptr;
}

static int wide3_check()
{
  using L = ffpat::Wide3;
  static int kind[L::KY][L::KX];               // 0 unset, 1 interior, 2 + role: ring of that role
  const char *err = nullptr;
  int count[5] = {0, 0, 0, 0, 0};
  for (int tid = 0; tid < L::NTH && !err; ++tid) {
    const int role = ffpat::wide3_role(tid / 64);
    const ffpat::PlanePoint i = ffpat::wide3_interior(tid), r = ffpat::wide3_ring(tid);
    const ffpat::Wide3Bases b = ffpat::wide3_bases(tid);
    // kinds of points, each plane point of one kind only
    const bool in_tile = i.lx >= L::XH && i.lx < L::XH + L::BX && i.ly >= 6 && i.ly < 6 + L::BY;
    if (!in_tile) err = "interior point outside the tile";
    else if (kind[i.ly][i.lx] != 0) err = "interior point taken twice";
    else kind[i.ly][i.lx] = 1, ++count[1];
    if (err) break;
    // ring point: inside the region of its role, outside the next inner region
    const int ins = role, inw[3] = {L::AX, L::CX, L::BX}, inh[3] = {L::AY, L::CY, L::BY};
    const int ow[3] = {L::KX, L::AX, L::CX}, oh[3] = {L::KY, L::AY, L::CY};
    const int ox = ins * L::E, oy = 2 * ins;
    const bool in_outer = r.lx >= ox && r.lx < ox + ow[role] && r.ly >= oy && r.ly < oy + oh[role];
    const int ix = ox + L::E, iy = oy + 2;
    const bool in_inner = r.lx >= ix && r.lx < ix + inw[role] && r.ly >= iy && r.ly < iy + inh[role];
    if (!in_outer || in_inner) { err = "ring point outside its ring"; break; }
    int &kr = kind[r.ly][r.lx];
    if (kr == 0) kr = 2 + role, ++count[2 + role];
    else if (kr != 2 + role) { err = "ring point of two kinds"; break; }
    // LDS accesses
    const int kd[6][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {0, -2}, {0, 2}};
    for (int B = 0; B < 2 && !err; ++B) {
      const int ks = B * L::KP;
      err = check_access(b.kI, ks + 2 * L::KX, L::KPAD, L::LK, ks, L::KX, L::KY, i.lx, i.ly, 0, 0);
      if (!err) err = check_access(b.kR, ks + 2 * L::KX, L::KPAD, L::LK, ks, L::KX, L::KY, r.lx, r.ly, 0, 0);
      for (int n = 0; n < 6 && !err; ++n) {
        const int off = ks + 2 * L::KX + kd[n][0] + kd[n][1] * L::KX;
        err = check_access(b.kI, off, L::KPAD, L::LK, ks, L::KX, L::KY, i.lx, i.ly, kd[n][0], kd[n][1]);
        if (!err && role >= 1)
          err = check_access(b.kR, off, L::KPAD, L::LK, ks, L::KX, L::KY, r.lx, r.ly, kd[n][0], kd[n][1]);
      }
    }
    const int nd[7][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}, {0, -2}, {0, 2}};
    for (int S = 0; S < 5 && !err; ++S) {
      const int qs = S * L::QP, rs = S * L::RP;
      // q in stage 1's region (origin (E, 2)), r in stage 2's (origin (2E, 4))
      const int qix = i.lx - L::E, qiy = i.ly - 2, qrx = r.lx - L::E, qry = r.ly - 2;
      const int rix = i.lx - 2 * L::E, riy = i.ly - 4, rrx = r.lx - 2 * L::E, rry = r.ly - 4;
      err = check_access(b.qI, qs + 2 * L::AX, L::QPAD, L::LQ, qs, L::AX, L::AY, qix, qiy, 0, 0);
      if (!err && role >= 1)
        err = check_access(b.qR, qs + 2 * L::AX, L::QPAD, L::LQ, qs, L::AX, L::AY, qrx, qry, 0, 0);
      if (!err) err = check_access(b.rI, rs + 2 * L::CX, 0, L::LR, rs, L::CX, L::CY, rix, riy, 0, 0);
      if (!err && role == 2) err = check_access(b.rR, rs, 0, L::LR, rs, L::CX, L::CY, rrx, rry, 0, 0);
      for (int n = 0; n < 7 && !err; ++n) {
        const int qo = qs + 2 * L::AX + nd[n][0] + nd[n][1] * L::AX;
        const int ro = rs + 2 * L::CX + nd[n][0] + nd[n][1] * L::CX;
        err = check_access(b.qI, qo, L::QPAD, L::LQ, qs, L::AX, L::AY, qix, qiy, nd[n][0], nd[n][1]);
        if (!err && role == 2)
          err = check_access(b.qR, qo, L::QPAD, L::LQ, qs, L::AX, L::AY, qrx, qry, nd[n][0], nd[n][1]);
        if (!err) err = check_access(b.rI, ro, 0, L::LR, rs, L::CX, L::CY, rix, riy, nd[n][0], nd[n][1]);
      }
    }
  }
  if (!err) {
    for (int y = 0; y < L::KY && !err; ++y)
      for (int x = 0; x < L::KX && !err; ++x)
        if (kind[y][x] == 0) err = "plane point without a slot";
  }
  if (!err && (count[1] != L::BX * L::BY || count[4] != L::N2 || count[3] != L::N1 || count[2] != L::NR))
    err = "point counts differ from the rings' sizes";
  // ring stages per plane on each SIMD (wave w on SIMD w % 4): 4, 4, 4, 3
  for (int simd = 0; simd < 4 && !err; ++simd) {
    int stages = 0;
    for (int w = simd; w < 16; w += 4) stages += ffpat::wide3_role(w);
    if (stages != (simd < 3 ? 4 : 3)) err = "ring stages unbalanced over the SIMDs";
  }
  if (err) {
    printf("FAIL %s\n", err);
    return 1;
  }
  printf("ok %d %d %d %d\n", count[1], count[4], count[3], count[2]);
  return 0;
}

int main(int argc, char **argv)
{
  if (argc >= 2 && !strcmp(argv[1], "wide3")) return wide3_check();
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
  if (argc >= 6 && !strcmp(argv[1], "triple")) {
    // FP32 three-step pass over pairs of points: tile width in points, height, chunk,
    // groups, and whether the grid takes it where the two-step rule keeps 64 points
    const int nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]), cus = atoi(argv[5]);
    const ffpat::PairShape p = ffpat::pair_shape_for(nx / 2, ny, nz, 64, 16, 1, cus, true, 0, ffpat::kTripleZmin);
    printf("%d %d %d %d %d\n", 2 * p.bx, p.by, p.zchunk, p.n_tiles, ffpat::wide3_grid_ok(nx, ny, nz) ? 1 : 0);
    return 0;
  }
  fprintf(stderr, "usage: launch_rules_cli pair nx ny nz esz cus per_cu_narrow per_cu_wide | step nx ny nz esz | "
                  "triple nx ny nz cus | wide3\n");
  return 2;
}
