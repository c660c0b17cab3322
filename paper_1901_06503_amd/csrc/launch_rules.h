// Launch-shape rules of the leapfrog stencil kernels: tile height and z-chunk of
// the one-step kernel, z-chunk and tile width of the two-step kernel, and the slot
// layout of the 1024-thread three-step kernel.  Plain host
// arithmetic on the grid, the element size, the device's compute units and the
// work-groups a unit holds at once (the callers query those from the runtime);
// nothing here touches the device, so the rules are testable on any host.
#pragma once

namespace ffpat {

// ---------------------------------------------------------------- one step per pass

// Tile height / 4 of the one-step kernel (measured on MI355X): tiles of 8 rows up to
// 256-row grids, 16 rows beyond (fewer halo re-reads once the fields no longer fit
// in the 256 MB MALL); FP64 16 rows from 128 rows on (8 below: more work-groups for
// small grids).  ry > 0 overrides.
inline int step_ry(int ny, int esz, int ry)
{
  if (ry > 0) return ry;
  return (ny > 256 || (esz == 8 && ny >= 128)) ? 4 : 2;
}

// Planes per work-group of the one-step kernel: about `groups` work-groups (the
// planes rounded to nearest), 1..16 planes per group.  Longer chunks lose
// parallelism, shorter ones re-read more z halo; below 128^3 parallelism wins.
// Measured on MI355X, us per step (this rule / the earlier floor of 4 planes):
// FP32 48^3 4.1 / 7.3, 64^3 4.5 / 8.0, 80^3 6.8 / 8.6, 96^3 8.2 / 9.2, 112^3 9.3 /
// 10.6; FP64 (tile height 8 below 128 rows) 64^3 4.9 / 11.2, 96^3 9.6 / 12.8.
// zchunk > 0 overrides (clamped to nz).
inline int step_zchunk(int nz, long xy, int groups, int zchunk)
{
  if (zchunk <= 0) {
    const long zc = ((long)nz * xy + groups / 2) / groups;
    zchunk = (int)(zc < 1 ? 1 : (zc > 16 ? 16 : zc));
  }
  return zchunk > nz ? nz : zchunk;
}

// --------------------------------------------------------------- two steps per pass

// z-planes a two-step work-group recomputes beyond its chunk (the stage-1 planes on
// either side), in the launch-time estimates below.
constexpr int kPairHalo = 4;

inline long pair_rounds(long groups, long resident)
{
  return (groups + resident - 1) / resident;
}

// Planes per work-group of the two-step kernel.  Its groups are long (a whole
// z-chunk each) and all of a launch's groups take about the same time, so a launch
// runs in rounds of `resident` groups and a last round that is only partly filled
// costs as much as a full one.  Where every chunk fits in one round at zmax planes
// or fewer, take as many chunks per x-y tile as fit (8 planes at least).
// Otherwise, with one group per compute unit, take the chunk that minimises
// rounds x (planes + halo), the longest on ties; with two per unit (whose short
// last round runs its groups alone on their units, faster), zmax.
// Measured on MI355X, us per leapfrog step (this rule / a fixed target of 512 FP32
// or 256 FP64 groups, which overshot one round by 5-12% at these sizes): FP32
// 160^3 14.1 / 18.9, 192^3 17.4 / 24.0, 224^3 27.6 (28 planes) / 36.8; FP64 160^3
// 22.7 / 37.1, 192^3 36.4 / 58.5, 224^3 64.3 / 101.4.  Beyond one round the
// estimate ranks the chunks as measured (one group per unit, 20..32 planes FP32
// 128-wide and 40..64 FP64, at 320^3..512^3); its picks, e.g. 128-wide FP32 384^3
// 28 planes 152.1 us (32: 163.1), FP64 384^3 55 planes 274.2 (64: 296.6), 448^3 50
// planes 446.0 (64: 455.4); 64 at 320^3 and 512^3.
inline int pair_zchunk(int nz, long xy, long resident, int per_cu, int zmax, int zmin = 8)
{
  if (xy < 1) xy = 1;
  const int zlo = nz < zmin ? nz : zmin, zhi = nz < zmax ? nz : zmax;
  const long fit = resident / xy;
  if (fit >= 1) {
    const long zc = (nz + fit - 1) / fit;
    if (zc <= zhi) return (int)(zc < zlo ? zlo : zc);
  }
  if (per_cu > 1) return zhi;
  int best = zhi;
  long best_cost = 0;
  for (int zc = zhi; zc >= zlo; --zc) {
    const int n_zc = (nz + zc - 1) / zc;
    const int bal = (nz + n_zc - 1) / n_zc;   // the same chunk count with balanced chunks
    const long cost = pair_rounds(xy * n_zc, resident) * (bal + kPairHalo);
    if (zc == zhi || cost < best_cost) {
      best = bal;
      best_cost = cost;
    }
  }
  return best;
}

// Longest z-chunk the rule may pick: 64 planes where a compute unit holds one group
// (FP64, and the FP32 128 x 16 tile), whose groups run in rounds; 32 where it holds
// two (the FP32 64 x 16 tile, which takes the longest chunk).  Measured on MI355X,
// 128 x 16 FP32 at 384^3, us per leapfrog step: 28 planes (the longest up to 32
// by the estimate) 149.0, 40 147.7, 48 150.4, 55 134.2, 64 143.6; the estimate
// ranks 55 first (7 chunks x 72 tiles: two nearly full rounds).
inline int pair_zmax(bool f64, int per_cu)
{
  return (f64 || per_cu == 1) ? 64 : 32;
}

// Launch shape of the two-step kernel with a bx x by tile on a grid.
struct PairShape {
  int bx, by;              // tile
  int tiles_x, tiles_y;
  int zchunk, n_tiles;     // planes per group, groups
  int per_cu, cus;         // groups a compute unit holds at once, compute units
};

// zchunk > 0 overrides the chunk rule (clamped to nz).
inline PairShape pair_shape_for(int nx, int ny, int nz, int bx, int by, int per_cu, int cus, bool f64, int zchunk,
                                int zmin = 8)
{
  PairShape p;
  p.bx = bx;
  p.by = by;
  p.tiles_x = (nx + bx - 1) / bx;
  p.tiles_y = (ny + by - 1) / by;
  p.per_cu = per_cu;
  p.cus = cus;
  if (zchunk <= 0)
    zchunk = pair_zchunk(nz, (long)p.tiles_x * p.tiles_y, (long)cus * per_cu, per_cu, pair_zmax(f64, per_cu), zmin);
  if (zchunk > nz) zchunk = nz;
  p.zchunk = zchunk;
  p.n_tiles = p.tiles_x * p.tiles_y * ((nz + zchunk - 1) / zchunk);
  return p;
}

// Estimated duration of a launch: rounds of resident groups times the planes a
// group computes, in units of one plane of a group.  t_shared: a group's plane time
// while its compute unit is full; t_alone: in a last round that leaves at most one
// group per unit.
inline double pair_cost(const PairShape &p, double t_shared, double t_alone)
{
  const long resident = (long)p.cus * p.per_cu;
  const long full = p.n_tiles / resident, rem = p.n_tiles % resident;
  double t = (double)full * t_shared;
  if (rem > 0) t += (rem <= p.cus && p.per_cu > 1) ? t_alone : t_shared;
  return t * (p.zchunk + kPairHalo);
}

// FP32 3D: whether the 128 x 16 tile (1024 threads, one group per compute unit) is
// faster than 64 x 16 (512 threads, two per unit).  The wide tile reads fewer bytes
// (a 64-wide tile's 2-point x halo costs a whole 128-byte line on each side: at
// 256^3 the wide tile's L2 fetches are 23% lower) but pads nx to a multiple of 128
// and halves the group count.  Plane times of a group measured on MI355X, relative
// to a 64-wide group sharing its unit: 128-wide 0.9, 64-wide alone 0.55.  With them
// the estimate picks the faster tile at all twelve cubes measured from 128^3 to
// 640^3 (us per step, wide / narrow: 224^3 24.8 / 26.4, 256^3 42.3 / 47.0, 288^3
// 74.8 / 78.3, 384^3 152.1 / 160.5 (28 planes per group), 512^3 347 / 391, 640^3
// 690 / 746; narrow / wide where narrow is kept: 128^3 9.8 / 11.3, 192^3 18.4 /
// 20.5, 320^3 91.4 / 101.9, 448^3 248 / 254; these with chunks of at most 32 planes).
// With up to 64 planes for the wide tile (pair_zmax) the estimate also takes it at
// 448^3 (50 planes): 236.8 us per step with one point per lane against 233.9 for the
// narrow tile, 228.4 with pairs of points per lane (even nx, pair_x_pairs).  A 64 x 32 tile with 1024 threads was
// 3-6% faster at 160^3 and 192^3 but 4-6% slower at 224^3 and 448^3 and is not a
// candidate.
inline bool pair_wide_better(const PairShape &narrow, const PairShape &wide)
{
  return pair_cost(wide, 0.9, 0.9) < pair_cost(narrow, 1.0, 0.55);
}

// FP32 3D: whether the two-step kernel runs over pairs of x-adjacent points, each
// pair one 8-byte element: the FP64 kernel's shape (64 x 16 elements = the 128 x 16
// tile in points, 512 threads, one group per compute unit, the p(k) plane
// double-buffered for one barrier per plane) with half the memory and LDS
// instructions per byte of the one-point form.  Wherever the 128 x 16 tile is chosen
// and nx is even (the elements then end at the grid's edge).  Measured on MI355X, us
// per leapfrog step (pairs / one point per lane, both with the chunk rule above):
// 224^3 26.4 / 26.5, 256^3 41.3 / 42.3, 288^3 72.1 / 74.0, 384^3 131.6 / 134.3,
// 448^3 228.4 / 236.8 (the 64 x 16 tile: 233.9), 512^3 314.9 / 319.0, 640^3
// 612.1 / 624.9.  Where the 64 x 16 tile is chosen it is slower (128^3 11.9 / 9.5,
// 192^3 21.3 / 19.6, 320^3 91.4 / 85.4).
inline bool pair_x_pairs(bool wide, int nx)
{
  return wide && nx % 2 == 0;
}

// ------------------------------------------- three steps per pass, 1024 threads

// FP32 grids that take three steps per pass over pairs of points (the 128 x 16 point
// tile) also where the two-step rule keeps the 64-point tile or one step per pass:
// even nx of at least 96 points whose pairs fill at least 60% of the tiles' width, ny
// of at least 64, at least 96^3 points.  Measured on MI355X, cubes, us per leapfrog
// step, the previous rule / three steps per pass: 96^3 8.15 (one step) / 6.76, 112^3
// 9.27 (one step) / 7.10, 128^3 9.48 / 8.05, 160^3 14.56 / 14.19, 192^3 18.98 / 18.55,
// 320^3 85.6 / 76.2; 64^3 4.45 (one step) / 5.7 at best, so smaller grids keep theirs.
inline bool wide3_grid_ok(int nx, int ny, int nz)
{
  if (nx % 2 != 0 || nx < 96 || ny < 64) return false;
  if ((long long)nx * ny * nz < 96LL * 96 * 96) return false;
  const int pairs = nx / 2, tiles = (pairs + 63) / 64;
  return 5 * pairs >= 3 * 64 * tiles;
}

// Shortest z-chunk of the three-step kernel where one round of groups covers the grid
// (a group marches its chunk plus 8 planes).  Measured on MI355X, us per leapfrog step:
// 128^3 4 planes 8.05, 5 8.07, 6 8.30, 8 9.16 (half the compute units idle); 96^3 3
// planes 6.76, 4 7.24, 6 8.10; 112^3 4 planes 7.10, 6 7.98.
constexpr int kTripleZmin = 3;


// Slot layout of wave_step3_wide (pairs of FP32 points, one 8-byte element per pair:
// one leapfrog step reaches one element in x and two rows in y).  Coordinates are
// (lx, ly) in the tile's p(k) plane with its halo, KX x KY elements; stage 1 (q)
// covers AX x AY of it from (1, 2), stage 2 (r) CX x CY from (2, 4), stage 3 (o)
// the BX x BY tile from (3, 6).  Constant expressions shared by the kernel and the
// host-side check of the layout.
struct Wide3 {
  static constexpr int NTH = 1024, BX = 64, BY = 16, E = 1, XH = 3 * E;
  static constexpr int KX = BX + 2 * XH, KY = BY + 12;
  static constexpr int AX = BX + 4 * E, AY = BY + 8;
  static constexpr int CX = BX + 2 * E, CY = BY + 4;
  static constexpr int N2 = CX * CY - BX * BY;   // ring of stage 2 (296 points)
  static constexpr int N1 = AX * AY - CX * CY;   // ring of stage 1 (312)
  static constexpr int NR = KX * KY - AX * AY;   // outer ring of the p(k) plane (328)
  static constexpr int KP = KY * KX, QP = AY * AX, RP = CY * CX;
  // LDS arrays in elements: two p(k) planes and a 5-plane q ring, each with two rows of
  // headroom in front, and a 5-plane r ring
  static constexpr int KPAD = 2 * KX, QPAD = 2 * AX;
  static constexpr int LK = KPAD + 2 * KP, LQ = QPAD + 5 * QP, LR = 5 * RP;
};

// Ring role of wave w (16 waves): 2 the ring of stage 2 (stages 1 and 2), 1 the ring
// of stage 1 (stage 1), 0 the outer ring of the p(k) plane (loaded into LDS only).
// Five, five and six waves, ordered so that with wave w on SIMD w % 4 the SIMDs carry
// 4, 4, 4 and 3 ring stages per plane.
constexpr int wide3_role(int w)
{
  constexpr int r[16] = {2, 2, 2, 1, 2, 2, 1, 1, 0, 0, 1, 1, 0, 0, 0, 0};
  return r[w];
}

// Rank of wave w among the waves of its role.
constexpr int wide3_role_index(int w)
{
  int n = 0;
  for (int v = 0; v < w; ++v) n += wide3_role(v) == wide3_role(w);
  return n;
}

struct PlanePoint {
  int lx, ly;
};

// Thread tid's interior point: tile row tid / 64, element tid % 64.
constexpr PlanePoint wide3_interior(int tid)
{
  return {Wide3::XH + tid % 64, 6 + tid / 64};
}

// The ring point of lane `lane` of the rank-th wave of ring role `role`: point u =
// rank x 64 + lane of the ring of width E (x) and 2 rows (y) around the region of
// that role (rw x rh elements at (role E, 2 role)); lanes beyond the ring's count
// repeat a point of it.
constexpr PlanePoint wide3_ring_point(int role, int rank, int lane)
{
  const int rw = role == 2 ? Wide3::CX : (role == 1 ? Wide3::AX : Wide3::KX);
  const int rh = role == 2 ? Wide3::CY : (role == 1 ? Wide3::AY : Wide3::KY);
  const int n = role == 2 ? Wide3::N2 : (role == 1 ? Wide3::N1 : Wide3::NR);
  constexpr int E = Wide3::E;
  int u = rank * 64 + lane;
  u = u < n ? u : u - n;
  int sx = 0, sy = 0;
  if (u < 4 * rw) {                      // rows 0, 1, rh - 2, rh - 1, full width
    const int r = u / rw;
    sy = r < 2 ? r : rh - 4 + r;
    sx = u - r * rw;
  } else {                               // rows 2 .. rh - 3, the E columns on either side
    const int j = u - 4 * rw;
    sy = 2 + j / (2 * E);
    const int cc = j % (2 * E);
    sx = cc < E ? cc : rw - 2 * E + cc;
  }
  return {sx + role * E, sy + 2 * role};
}

// Thread tid's ring point.
constexpr PlanePoint wide3_ring(int tid)
{
  return wide3_ring_point(wide3_role(tid / 64), wide3_role_index(tid / 64), tid % 64);
}

// LDS element indices, from the start of each array, of thread tid's slot bases: each
// 2 rows above its point in the array's plane (the lowest row any stage reads; the
// kernel adds the plane's offset, 2 rows and the neighbour's shift as immediates).
// The headroom keeps this inside the arrays for the ring points near the top that only
// write there (the outer ring's p(k), stage 1's ring's q).  The ring point's q base
// serves rings with stage 1, its r base (at the point: it only writes r) the ring of
// stage 2; elsewhere they are 0 and unused.
struct Wide3Bases {
  int kI, qI, rI, kR, qR, rR;
};
constexpr Wide3Bases wide3_bases_of(PlanePoint i, PlanePoint r, int role)
{
  using L = Wide3;
  Wide3Bases b{};
  b.kI = L::KPAD + (i.ly - 2) * L::KX + i.lx;
  b.qI = L::QPAD + (i.ly - 4) * L::AX + (i.lx - L::E);
  b.rI = (i.ly - 6) * L::CX + (i.lx - 2 * L::E);
  b.kR = L::KPAD + (r.ly - 2) * L::KX + r.lx;
  b.qR = role >= 1 ? L::QPAD + (r.ly - 4) * L::AX + (r.lx - L::E) : 0;
  b.rR = role == 2 ? (r.ly - 4) * L::CX + (r.lx - 2 * L::E) : 0;
  return b;
}
constexpr Wide3Bases wide3_bases(int tid)
{
  return wide3_bases_of(wide3_interior(tid), wide3_ring(tid), wide3_role(tid / 64));
}

}  // namespace ffpat
