// Plane-wise X-ray transform X (eq. Radon, Sec. 2.1), its transpose (the
// backprojection of Sec. 3.1) and the ramp preconditioner Lambda (Sec. 3.1).
//
// X uses linear interpolation along the minor axis of each ray (Sec. 4.1
// names linear interpolation).  The projector walks the ray one grid line
// of the major axis at a time (Joseph's method); the backprojector gathers
// the same weights per voxel, so the two are exact transposes.
#include "kernels.h"

#include <cstdlib>

namespace ffpat {

// ---------------------------------------------------------------------------
// Projector: one thread per detector bin j of angle a in ZP consecutive planes
// (the ray's crossings do not depend on z; the launch uses ZP = 1), coalesced
// writes along s.
// Rays march over rows (|cos| >= |sin|) or columns (|sin| > |cos|); for the
// latter the plane is read from its transposed copy, so in both cases the two
// taps of a lane sit in one contiguous line and neighbouring bins read
// neighbouring addresses.  Lines carry 3 zeros on each side: every crossing
// u of the marched range lies in [-2, nm + 1], so no tap needs a bounds check.
// Work order: angles fastest, then plane groups; each XCD owns a contiguous
// range of planes, so a plane (and its transpose) is fetched into one L2 and
// reused by every angle.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
pad_planes_kernel(const T *__restrict__ v, T *__restrict__ padN, T *__restrict__ padT, int nx, int ny, int need_n,
                  int need_t)
{
  __shared__ T tile[32][33];
  const int z = blockIdx.z;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  const T *src = v + (size_t)z * nx * ny;
  const int LPx = nx + kLinePadL + kLinePadR, LPy = ny + kLinePadL + kLinePadR;
  T *dn = padN + (size_t)z * ny * LPx + kLinePadL;
  T *dt = padT + (size_t)z * nx * LPy + kLinePadL;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int y = y0 + r, x = x0 + tx;
    if (x < nx && y < ny) {
      const T val = src[(size_t)y * nx + x];
      tile[r][tx] = val;
      if (need_n) dn[(size_t)y * LPx + x] = val;
    }
  }
  if (!need_t) return;
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int x = x0 + r, y = y0 + tx;
    if (x < nx && y < ny) dt[(size_t)x * LPy + y] = tile[tx][r];
  }
}

template <typename T, int ZP, int UNR>
__global__ void __launch_bounds__(256)
project_kernel(const T *__restrict__ padN, const T *__restrict__ padT, T *__restrict__ g,
               const AngleParams *__restrict__ ap, int nx, int ny, int nz, int ns, int n_angles, int n_work)
{
  const int b = blockIdx.x;
  const int per_xcd = (n_work + 7) / 8;
  const int t = (b % 8) * per_xcd + b / 8;
  if (t >= n_work) return;
  const int nzg = (nz + ZP - 1) / ZP;
  const int a = t % n_angles;
  const int rest = t / n_angles;
  const int z0 = (rest % nzg) * ZP;
  const int jb = rest / nzg;
  const int j = jb * 256 + threadIdx.x;
  if (j >= ns) return;

  const AngleParams P = ap[a];
  // padded plane (index 0 = first pad) of the marched orientation; block-uniform
  int nr, nm;
  const char *plane0;
  size_t pstride;   // bytes between consecutive planes of that copy
  if (P.major_x) {  // march over columns x_r (rows of the transpose), interpolate along y
    nr = nx; nm = ny;
    pstride = (size_t)nx * (ny + kLinePadL + kLinePadR) * sizeof(T);
    plane0 = reinterpret_cast<const char *>(padT);
  } else {          // march over rows y_r, interpolate along x
    nr = ny; nm = nx;
    pstride = (size_t)ny * (nx + kLinePadL + kLinePadR) * sizeof(T);
    plane0 = reinterpret_cast<const char *>(padN);
  }
  // the ZP planes of this group (past the last plane: the last plane again, never stored)
  const char *pl[ZP];
#pragma unroll
  for (int q = 0; q < ZP; ++q) pl[q] = plane0 + (size_t)min(z0 + q, nz - 1) * pstride;
  const unsigned LPB = (unsigned)((nm + kLinePadL + kLinePadR) * sizeof(T));   // line pitch in bytes
  const double A = P.u0 + (double)j * P.uj;
  // marched lines whose crossing lies in (-1, nm) (where a tap is inside), widened
  // by one line on each side; |ur| <= 1 keeps the crossings within [-2, nm + 1]
  double lo = 0.0, hi = (double)(nr - 1);
  if (P.ur != 0.0) {
    double r_a = (-1.0 - A) / P.ur, r_b = ((double)nm - A) / P.ur;
    if (r_a > r_b) { double tt = r_a; r_a = r_b; r_b = tt; }
    lo = fmin(fmax(lo, floor(r_a)), (double)nr);   // clamped before any int conversion
    hi = fmax(fmin(hi, ceil(r_b)), -1.0);
  } else if (!(A > -1.0 && A < (double)nm)) {
    hi = -1.0;
  }
  const int r0 = (int)lo, r1 = (int)hi;
  // The crossing (offset and interpolation weight) of a marched line is the same
  // in every plane: it is computed once and serves the ZP planes, whose loads
  // share one 32-bit byte offset from their uniform plane bases.
  unsigned rowb = (unsigned)r0 * LPB;
  T acc[ZP];
#pragma unroll
  for (int q = 0; q < ZP; ++q) acc[q] = T(0);
  if (sizeof(T) == 4) {
    // exact fixed-point stepping: u(r) = U / 2^32, U += ur_fix per line
    long long U = llrint(fma((double)r0, P.ur, A) * 4294967296.0);
    const long long UR = P.ur_fix;
#pragma unroll UNR
    for (int r = r0; r <= r1; ++r) {
      const unsigned off = rowb + (unsigned)(((int)(U >> 32) + kLinePadL) * (int)sizeof(T));
      const T f = (T)(unsigned)(U & 0xffffffffLL) * T(2.3283064365386963e-10);
      const T e = T(1) - f;
#pragma unroll
      for (int q = 0; q < ZP; ++q) {
        const T v0 = *reinterpret_cast<const T *>(pl[q] + off);
        const T v1 = *reinterpret_cast<const T *>(pl[q] + off + sizeof(T));
        acc[q] = fma(f, v1, fma(e, v0, acc[q]));   // linear interpolation, two FMAs per plane
      }
      U += UR;
      rowb += LPB;
    }
  } else {
#pragma unroll(UNR > 4 ? 4 : UNR)
    for (int r = r0; r <= r1; ++r) {
      const double u = fma((double)r, P.ur, A);
      const double fl = floor(u);
      const unsigned off = rowb + (unsigned)(((int)fl + kLinePadL) * (int)sizeof(T));
      const T f = (T)(u - fl);
      const T e = T(1) - f;
#pragma unroll
      for (int q = 0; q < ZP; ++q) {
        const T v0 = *reinterpret_cast<const T *>(pl[q] + off);
        const T v1 = *reinterpret_cast<const T *>(pl[q] + off + sizeof(T));
        acc[q] = fma(f, v1, fma(e, v0, acc[q]));
      }
      rowb += LPB;
    }
  }
#pragma unroll
  for (int q = 0; q < ZP; ++q)
    if (z0 + q < nz) g[((size_t)a * nz + z0 + q) * ns + j] = acc[q] * (T)P.w;
}

// ---------------------------------------------------------------------------
// Projector with the planes staged in LDS.  A 1024-thread work-group owns ZP
// consecutive planes (the launch uses 8 in FP32, 4 in FP64), one orientation (rays marching rows
// read the padded planes, rays marching columns the padded transposes), 32
// angles of that orientation and 256 detector bins; thread (bin j, quarter s) marches the rays
// of angles 8s..8s+7.  The marched lines are staged chunk by chunk into LDS
// with the ZP planes interleaved ([line][position] of ZP-vectors, in 16-byte
// slices: FP64 as two arrays of 2-vectors), so the two taps of a crossing in all
// ZP planes are a few vector LDS reads and the
// crossing's position and weights serve ZP planes.  Every ray visits every
// line: the tap index is clamped into the three zero pads on each side, where
// both taps are zero exactly when the crossing misses the line (the same sums
// as marching only the crossed lines).  Positions: exact 32.32 fixed point in
// FP32, double arithmetic in FP64 (as in project_kernel).
// ---------------------------------------------------------------------------
template <typename T, int ZP>
struct alignas(ZP * sizeof(T) >= 16 ? 16 : ZP * sizeof(T)) VecZ {
  T v[ZP];
};

constexpr int kLdsBytes = 139264;   // 136 KiB per work-group (one work-group per compute unit)

// LDS layout of ZP interleaved planes in 16-byte slices: the planes
// s*SW .. s*SW+SW-1 of position e sit in slice array s (element s*NP + e).  A
// lane's 16-byte read at position e and its neighbours' at e+1, e+2, ... then
// fall in consecutive bank groups; one 32-byte vector per position would use
// every other group and conflict two ways (measured: FP64 projection 13% and
// FP32 backprojection of 8 planes 17% faster at 256^3 / 256 angles).
template <typename T, int ZP>
struct Sliced {
  static constexpr int SW = ZP * (int)sizeof(T) > 16 ? 16 / (int)sizeof(T) : ZP;   // planes per slice
  static constexpr int NS = ZP / SW;                                                 // slices
  using Slice = VecZ<T, SW>;
  static constexpr int NP = kLdsBytes / (NS * (int)sizeof(Slice));                  // positions
};
constexpr int kProjAngles = 32, kProjAnglesPerThread = 8;

template <typename T, int ZP>
__global__ void __launch_bounds__(1024)
project_lds_kernel(const T *__restrict__ padN, const T *__restrict__ padT, T *__restrict__ g,
                   const AngleParams *__restrict__ ap, const int *__restrict__ aorder, int n_row_angles,
                   int n_angles, int nx, int ny, int nz, int ns, int n_groups_rows, int n_groups, int n_work)
{
  using S = Sliced<T, ZP>;
  constexpr int NV = S::NP, SW = S::SW, NS = S::NS;
  __shared__ typename S::Slice lds[NS * NV];
  const int b = blockIdx.x;
  const int per_xcd = (n_work + 7) / 8;
  const int t = (b % 8) * per_xcd + b / 8;
  if (t >= n_work) return;                  // whole group exits together
  const int nzg = (nz + ZP - 1) / ZP;
  const int grp = t % n_groups;
  const int rest = t / n_groups;
  const int z0 = (rest % nzg) * ZP;
  const int jb = rest / nzg;
  const bool rows = grp < n_groups_rows;
  const int gi = rows ? grp : grp - n_groups_rows;
  const int a_begin = rows ? 0 : n_row_angles;
  const int a_count = rows ? n_row_angles : n_angles - n_row_angles;
  const int nr = rows ? ny : nx, nm = rows ? nx : ny;
  const int LP = nm + kLinePadL + kLinePadR;
  const T *src = rows ? padN : padT;       // [nz][nr][LP]
  const int j = jb * 256 + (threadIdx.x & 255);
  const int quarter = threadIdx.x >> 8;     // uniform per wave
  const bool jin = j < ns;

  // per lane: the rays' positions at line 0 (FP32: fixed point; FP64: A = u0 + j uj)
  long long U[kProjAnglesPerThread];
  double A[kProjAnglesPerThread];
  T acc[kProjAnglesPerThread][ZP];
#pragma unroll
  for (int m = 0; m < kProjAnglesPerThread; ++m) {
    const int ia = gi * kProjAngles + quarter * kProjAnglesPerThread + m;
    U[m] = 0;
    A[m] = 0.0;
    if (ia < a_count) {
      const AngleParams &P = ap[aorder[a_begin + ia]];
      A[m] = P.u0 + (double)j * P.uj;
      if (sizeof(T) == 4) U[m] = llrint(A[m] * 4294967296.0);
    }
#pragma unroll
    for (int q = 0; q < ZP; ++q) acc[m][q] = T(0);
  }
  const size_t pl = (size_t)nr * LP;
  const T *sp[ZP];   // the group's planes (past the last plane: the last plane again, never stored)
#pragma unroll
  for (int q = 0; q < ZP; ++q) sp[q] = src + (size_t)min(z0 + q, nz - 1) * pl;
  const int R = min(nr, NV / LP);           // lines per chunk
  for (int c0 = 0; c0 < nr; c0 += R) {
    const int rc = min(R, nr - c0);
    __syncthreads();                        // the previous chunk has been read
    const int n_el = rc * LP;
    const size_t off0 = (size_t)c0 * LP;
    for (int e = threadIdx.x; e < n_el; e += 1024) {
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        typename S::Slice v;
#pragma unroll
        for (int q = 0; q < SW; ++q) v.v[q] = sp[sl * SW + q][off0 + e];
        lds[sl * NV + e] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kProjAnglesPerThread; ++m) {
      const int ia = gi * kProjAngles + quarter * kProjAnglesPerThread + m;
      if (ia >= a_count) break;             // uniform per wave
      if (sizeof(T) == 4) {
        const long long UR = ap[aorder[a_begin + ia]].ur_fix;
        long long u = U[m];
#pragma unroll 4
        for (int r = 0; r < rc; ++r) {
          const int i0 = min(max((int)(u >> 32), -3), nm + 1) + kLinePadL;
          const T f = (T)(unsigned)(u & 0xffffffffLL) * T(2.3283064365386963e-10);
          const T e = T(1) - f;
#pragma unroll
          for (int sl = 0; sl < NS; ++sl) {
            const typename S::Slice v0 = lds[sl * NV + r * LP + i0], v1 = lds[sl * NV + r * LP + i0 + 1];
#pragma unroll
            for (int q = 0; q < SW; ++q)
              acc[m][sl * SW + q] = fma(f, v1.v[q], fma(e, v0.v[q], acc[m][sl * SW + q]));
          }
          u += UR;
        }
        U[m] = u;
      } else {
        const double ur = ap[aorder[a_begin + ia]].ur;
#pragma unroll 2
        for (int r = 0; r < rc; ++r) {
          const double u = fma((double)(c0 + r), ur, A[m]);
          const double fl = floor(u);
          const int i0 = (int)fmin(fmax(fl, -3.0), (double)(nm + 1)) + kLinePadL;
          const T f = (T)(u - fl);
          const T e = T(1) - f;
#pragma unroll
          for (int sl = 0; sl < NS; ++sl) {
            const typename S::Slice v0 = lds[sl * NV + r * LP + i0], v1 = lds[sl * NV + r * LP + i0 + 1];
#pragma unroll
            for (int q = 0; q < SW; ++q)
              acc[m][sl * SW + q] = fma(f, v1.v[q], fma(e, v0.v[q], acc[m][sl * SW + q]));
          }
        }
      }
    }
  }
  if (!jin) return;
#pragma unroll
  for (int m = 0; m < kProjAnglesPerThread; ++m) {
    const int ia = gi * kProjAngles + quarter * kProjAnglesPerThread + m;
    if (ia >= a_count) break;
    const int a = aorder[a_begin + ia];
    const T w = sizeof(T) == 4 ? (T)ap[a].w_f : (T)ap[a].w;
#pragma unroll
    for (int q = 0; q < ZP; ++q)
      if (z0 + q < nz) g[((size_t)a * nz + z0 + q) * ns + j] = acc[m][q] * w;
  }
}

static bool xray_lds_enabled()
{
  static const bool on = [] {
    const char *e = getenv("FFPAT_XRAY_LDS");
    return e ? atoi(e) != 0 : true;
  }();
  return on;
}

// planes per work-group of the staged backprojector (0: use the L2-gather
// kernel): in FP32 16 where that still gives at least 256 work-groups (64 x 64
// voxel tiles), 8 from 8 planes on (the bin position and weights serve the planes:
// 8 are 3% faster than 4 at 256^3 / 256 angles, 16 another 6%, 588.7 -> 554.4 us),
// else 4 (FP64: 8 planes of accumulators would not fit the register budget);
// FFPAT_XRAY_LDS_ZP = 4, 8 or 16 overrides for FP32
static int xray_lds_planes(const Dims &d, size_t esz)
{
  static const int env = [] {
    const char *e = getenv("FFPAT_XRAY_LDS_ZP");
    const int v = e ? atoi(e) : 0;
    return (v == 4 || v == 8 || v == 16) ? v : 0;
  }();
  const int nz = d.nz;
  if (nz < 4) return 0;
  if (esz == 8) return 4;
  if (env) return nz >= env ? env : 4;
  const long tiles = (long)((d.nx + 63) / 64) * ((d.ny + 63) / 64);
  if (nz >= 16 && tiles * ((nz + 15) / 16) >= 256) return 16;
  return nz >= 8 ? 8 : 4;
}

// planes per thread of the backprojector (FFPAT_XRAY_ZP = 1, 4 or 8 overrides):
// one for fewer than four planes, else 4
static int xray_planes(int nz)
{
  static const int env = [] {
    const char *e = getenv("FFPAT_XRAY_ZP");
    const int v = e ? atoi(e) : 0;
    return (v == 1 || v == 4 || v == 8) ? v : 0;
  }();
  if (nz < 4) return 1;
  return env ? env : 4;
}

template <typename T, int ZP, int UNR>
static hipError_t project_dispatch(const Dims &d, int n_angles, int ns, const AngleParams *ap, const T *padN,
                                   const T *padT, T *g, hipStream_t s)
{
  const int jblocks = (ns + 255) / 256;
  const long n_work = (long)jblocks * ((d.nz + ZP - 1) / ZP) * n_angles;
  const long grid = (n_work + 7) / 8 * 8;
  const int tb = ns >= 256 ? 256 : ((ns + 63) / 64) * 64;
  project_kernel<T, ZP, UNR><<<(unsigned)grid, tb, 0, s>>>(padN, padT, g, ap, d.nx, d.ny, d.nz, ns, n_angles,
                                                            (int)n_work);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_project(const Dims &d, int n_angles, int ns, const AngleParams *ap, const int *aorder,
                          int n_row_angles, const T *vol, T *padN, T *padT, bool need_n, bool need_t, T *g,
                          hipStream_t s)
{
  dim3 pgrid((d.nx + 31) / 32, (d.ny + 31) / 32, d.nz);
  pad_planes_kernel<T><<<pgrid, 256, 0, s>>>(vol, padN, padT, d.nx, d.ny, need_n ? 1 : 0, need_t ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int lp_max = (d.nx > d.ny ? d.nx : d.ny) + kLinePadL + kLinePadR;
  // planes per work-group: eight in FP32 from 8 planes on (the crossing's position
  // and weights serve 8 planes; with the planes in 16-byte LDS slices 5% faster than
  // four at 256^3 / 256 angles, where one 32-byte vector per position was 14%
  // slower), else four (FP64: 8 planes of accumulators would not fit the registers)
  const int zp = (sizeof(T) == 4 && d.nz >= 8 && lp_max <= kLdsBytes / (int)(8 * sizeof(T))) ? 8 : 4;
  if (d.nz >= 4 && lp_max <= kLdsBytes / (int)(zp * sizeof(T)) && xray_lds_enabled()) {
    const int gr = (n_row_angles + kProjAngles - 1) / kProjAngles;
    const int gc = (n_angles - n_row_angles + kProjAngles - 1) / kProjAngles;
    const long n_work = (long)(gr + gc) * ((d.nz + zp - 1) / zp) * ((ns + 255) / 256);
    const long grid = (n_work + 7) / 8 * 8;
    if constexpr (sizeof(T) == 4) {
      if (zp == 8) {
        project_lds_kernel<T, 8><<<(unsigned)grid, 1024, 0, s>>>(padN, padT, g, ap, aorder, n_row_angles,
                                                                 n_angles, d.nx, d.ny, d.nz, ns, gr, gr + gc,
                                                                 (int)n_work);
        return hipGetLastError();
      }
    }
    project_lds_kernel<T, 4><<<(unsigned)grid, 1024, 0, s>>>(padN, padT, g, ap, aorder, n_row_angles, n_angles,
                                                             d.nx, d.ny, d.nz, ns, gr, gr + gc, (int)n_work);
    return hipGetLastError();
  }
  // one plane per thread, eight lines unrolled: measured at 256^3 / 256 angles,
  // sharing the crossings over 2 or 4 planes per thread was no faster (2x8) or
  // 16% slower (4x4; more planes in flight per compute unit, fewer cache hits)
  return project_dispatch<T, 1, 8>(d, n_angles, ns, ap, padN, padT, g, s);
}

// ---------------------------------------------------------------------------
// Backprojector: one thread per voxel column position (i, k) of a 64 x 4 tile
// in ZP consecutive planes, loop over angles, reading detector rows in the
// padded layout.  The bin position of (i, k) and its weights do not depend on
// z: they are computed once per angle and serve the ZP planes, whose rows are
// uniform bases with one shared 32-bit lane offset.
// With ds >= m dx for every angle (e.g. ds = dx) the footprint covers at most
// the bins floor(t) and floor(t) + 1: FP32 steps t in 32.32 fixed point and
// clamps the bin to [-2, ns + 1], where the pads (zeros) absorb voxels that
// project off the detector; FP64 evaluates t in double.  Otherwise every bin
// within the half-width is visited.  Tiles of one plane group are consecutive
// on one XCD so its detector rows stay in L2.
// ---------------------------------------------------------------------------
template <typename T, bool TWO_TAP, int ZP>
__global__ void __launch_bounds__(256)
backproject_kernel(const T *__restrict__ gpad, T *__restrict__ vol, const AngleParams *__restrict__ ap, int n_angles,
                   int nx, int ny, int nz, int ns, const T *__restrict__ kap, int tiles_x, int tiles_y, int n_work)
{
  const int b = blockIdx.x;
  const int per_xcd = (n_work + 7) / 8;
  const int tw = (b % 8) * per_xcd + b / 8;
  if (tw >= n_work) return;
  const int bx = tw % tiles_x;
  const int rest = tw / tiles_x;
  const int by = rest % tiles_y;
  const int z0 = (rest / tiles_y) * ZP;
  const int i = bx * 64 + (threadIdx.x & 63);
  const int k = by * 4 + (threadIdx.x >> 6);
  if (i >= nx || k >= ny) return;

  const int RS = ns + kRowPadL + kRowPadR;
  T acc[ZP];
#pragma unroll
  for (int q = 0; q < ZP; ++q) acc[q] = T(0);
  // detector rows (a, z0 + q): uniform bases; past the last plane, the last plane's row (never stored)
  const char *gz[ZP];
#pragma unroll
  for (int q = 0; q < ZP; ++q) gz[q] = reinterpret_cast<const char *>(gpad + (size_t)min(z0 + q, nz - 1) * RS);
  const size_t astride = (size_t)nz * RS * sizeof(T);
#pragma unroll 2
  for (int a = 0; a < n_angles; ++a) {
    const AngleParams &P = ap[a];
    const size_t aoff = (size_t)a * astride;
    if (TWO_TAP) {
      unsigned off;
      T w0, w1;
      if (sizeof(T) == 4) {
        const long long Tf = P.b0_fix + (long long)i * P.bi_fix + (long long)k * P.bk_fix;
        const int j0 = min(max((int)(Tf >> 32), -2), ns + 1);
        off = (unsigned)((j0 + kRowPadL) * (int)sizeof(T));
        const T f = (T)(unsigned)(Tf & 0xffffffffLL) * T(2.3283064365386963e-10);
        const T ih = P.inv_hw_f, wa = P.w_f;
        w0 = wa * fmax(T(1) - f * ih, T(0));
        w1 = wa * fmax(T(1) - (T(1) - f) * ih, T(0));
      } else {
        const double t = P.b0 + (double)i * P.bi + (double)k * P.bk;
        const double fl = fmin(fmax(floor(t), -2.0), (double)(ns + 1));
        off = (unsigned)(((int)fl + kRowPadL) * (int)sizeof(T));
        const T f = (T)(t - fl);
        const T ih = (T)P.inv_hw, wa = (T)P.w;
        // a clamped bin reads two pads, so the weights do not matter there
        w0 = wa * fmax(T(1) - f * ih, T(0));
        w1 = wa * fmax(T(1) - (T(1) - f) * ih, T(0));
      }
#pragma unroll
      for (int q = 0; q < ZP; ++q) {
        const char *row = gz[q] + aoff;
        const T v0 = *reinterpret_cast<const T *>(row + off);
        const T v1 = *reinterpret_cast<const T *>(row + off + sizeof(T));
        acc[q] = fma(w1, v1, fma(w0, v0, acc[q]));
      }
    } else {
      const double t = P.b0 + (double)i * P.bi + (double)k * P.bk;
      const int jlo = (int)fmin(fmax(ceil(t - P.hw), 0.0), (double)ns);
      const int jhi = (int)fmax(fmin(floor(t + P.hw), (double)(ns - 1)), -1.0);
      for (int j = jlo; j <= jhi; ++j) {
        const double wt = 1.0 - fabs((double)j - t) * P.inv_hw;
        if (wt > 0.0) {
          const T wj = (T)wt * (T)P.w;
#pragma unroll
          for (int q = 0; q < ZP; ++q)
            acc[q] += wj * reinterpret_cast<const T *>(gz[q] + aoff)[kRowPadL + j];
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < ZP; ++q) {
    if (z0 + q < nz) {
      const size_t idx = ((size_t)(z0 + q) * ny + k) * nx + i;
      vol[idx] = kap ? acc[q] * kap[idx] : acc[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Two-tap backprojector with the detector rows staged in LDS.  A 1024-thread
// work-group owns a 64 x 64 voxel tile in ZP consecutive planes (8 in FP32, 4
// in FP64); thread (i, kk) accumulates voxels (i, kk + 16 v), v = 0..3, in the
// ZP planes.  Chunks of angles are staged into LDS with the planes' rows interleaved
// ([angle][padded bin] of ZP-vectors in 16-byte slices: FP32 8 planes as two
// arrays of 4-vectors, 17% faster at 256^3 / 256 angles than one 32-byte vector
// per bin, whose reads conflict two ways; FP64 likewise 5%), so the two taps of a
// voxel in all ZP planes are a few vector LDS reads; the bin position and weights are computed
// once per voxel and angle.  Same arithmetic and order as backproject_kernel
// (angles in order, two FMAs per plane).
// ---------------------------------------------------------------------------
template <typename T, int ZP>
__global__ void __launch_bounds__(1024)
backproject_lds_kernel(const T *__restrict__ gpad, T *__restrict__ vol, const AngleParams *__restrict__ ap,
                       int n_angles, int nx, int ny, int nz, int ns, const T *__restrict__ kap, int tiles_x,
                       int tiles_y, int n_work)
{
  using S = Sliced<T, ZP>;
  constexpr int NV = S::NP, SW = S::SW, NS = S::NS;
  __shared__ typename S::Slice lds[NS * NV];
  const int b = blockIdx.x;
  const int per_xcd = (n_work + 7) / 8;
  const int tw = (b % 8) * per_xcd + b / 8;
  if (tw >= n_work) return;                 // whole group exits together
  const int bx = tw % tiles_x;
  const int rest = tw / tiles_x;
  const int by = rest % tiles_y;
  const int z0 = (rest / tiles_y) * ZP;
  const int i = bx * 64 + (threadIdx.x & 63);
  const int k0 = by * 64 + (threadIdx.x >> 6);
  const int RS = ns + kRowPadL + kRowPadR;
  const int AC = NV / RS;                   // angles per chunk

  T acc[4][ZP];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int q = 0; q < ZP; ++q) acc[v][q] = T(0);
  int zc[ZP];   // the group's planes (past the last plane: the last plane again, never stored)
#pragma unroll
  for (int q = 0; q < ZP; ++q) zc[q] = min(z0 + q, nz - 1);
  for (int a0 = 0; a0 < n_angles; a0 += AC) {
    const int ac = min(AC, n_angles - a0);
    __syncthreads();                        // the previous chunk has been read
    for (int e = threadIdx.x; e < ac * RS; e += 1024) {
      const int al = e / RS, jj = e - al * RS;
      const size_t row = (size_t)(a0 + al) * nz;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        typename S::Slice v;
#pragma unroll
        for (int q = 0; q < SW; ++q) v.v[q] = gpad[(row + zc[sl * SW + q]) * RS + jj];
        lds[sl * NV + e] = v;
      }
    }
    __syncthreads();
    for (int al = 0; al < ac; ++al) {
      const AngleParams &P = ap[a0 + al];
      const typename S::Slice *L = lds + al * RS;
      if (sizeof(T) == 4) {
        const long long T0 = P.b0_fix + (long long)i * P.bi_fix + (long long)k0 * P.bk_fix;
        const long long BK16 = 16 * P.bk_fix;
        const T ih = P.inv_hw_f, wa = P.w_f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const long long Tv = T0 + (long long)v * BK16;
          const int j0 = min(max((int)(Tv >> 32), -2), ns + 1) + kRowPadL;
          const T f = (T)(unsigned)(Tv & 0xffffffffLL) * T(2.3283064365386963e-10);
          const T w0 = wa * fmax(T(1) - f * ih, T(0));
          const T w1 = wa * fmax(T(1) - (T(1) - f) * ih, T(0));
#pragma unroll
          for (int sl = 0; sl < NS; ++sl) {
            const typename S::Slice v0 = L[sl * NV + j0], v1 = L[sl * NV + j0 + 1];
#pragma unroll
            for (int q = 0; q < SW; ++q)
              acc[v][sl * SW + q] = fma(w1, v1.v[q], fma(w0, v0.v[q], acc[v][sl * SW + q]));
          }
        }
      } else {
        const T ih = (T)P.inv_hw, wa = (T)P.w;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double t = P.b0 + (double)i * P.bi + (double)(k0 + 16 * v) * P.bk;
          const double fl = fmin(fmax(floor(t), -2.0), (double)(ns + 1));
          const int j0 = (int)fl + kRowPadL;
          const T f = (T)(t - fl);
          // a clamped bin reads two pads, so the weights do not matter there
          const T w0 = wa * fmax(T(1) - f * ih, T(0));
          const T w1 = wa * fmax(T(1) - (T(1) - f) * ih, T(0));
#pragma unroll
          for (int sl = 0; sl < NS; ++sl) {
            const typename S::Slice v0 = L[sl * NV + j0], v1 = L[sl * NV + j0 + 1];
#pragma unroll
            for (int q = 0; q < SW; ++q)
              acc[v][sl * SW + q] = fma(w1, v1.v[q], fma(w0, v0.v[q], acc[v][sl * SW + q]));
          }
        }
      }
    }
  }
  if (i >= nx) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int k = k0 + 16 * v;
    if (k >= ny) continue;
#pragma unroll
    for (int q = 0; q < ZP; ++q) {
      if (z0 + q >= nz) continue;
      const size_t idx = ((size_t)(z0 + q) * ny + k) * nx + i;
      vol[idx] = kap ? acc[v][q] * kap[idx] : acc[v][q];
    }
  }
}

template <typename T, int ZP>
static hipError_t backproject_dispatch(const Dims &d, int n_angles, int ns, const AngleParams *ap, bool two_tap,
                                       const T *gpad, T *vol, const T *kap, hipStream_t s)
{
  const int tiles_x = (d.nx + 63) / 64, tiles_y = (d.ny + 3) / 4;
  const long n_work = (long)tiles_x * tiles_y * ((d.nz + ZP - 1) / ZP);
  const long grid = (n_work + 7) / 8 * 8;
  if (two_tap)
    backproject_kernel<T, true, ZP><<<(unsigned)grid, 256, 0, s>>>(gpad, vol, ap, n_angles, d.nx, d.ny, d.nz, ns,
                                                                    kap, tiles_x, tiles_y, (int)n_work);
  else
    backproject_kernel<T, false, ZP><<<(unsigned)grid, 256, 0, s>>>(gpad, vol, ap, n_angles, d.nx, d.ny, d.nz, ns,
                                                                     kap, tiles_x, tiles_y, (int)n_work);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_backproject(const Dims &d, int n_angles, int ns, const AngleParams *ap, bool two_tap,
                              const T *gpad, T *vol, const T *kap, hipStream_t s)
{
  int zp = xray_lds_planes(d, sizeof(T));
  if (zp == 16 && ns + kRowPadL + kRowPadR > kLdsBytes / (int)(16 * sizeof(T))) zp = 8;   // long rows
  if (two_tap && zp > 0 && ns + kRowPadL + kRowPadR <= kLdsBytes / (int)(zp * sizeof(T)) && xray_lds_enabled()) {
    const int tiles_x = (d.nx + 63) / 64, tiles_y = (d.ny + 63) / 64;
    const long n_work = (long)tiles_x * tiles_y * ((d.nz + zp - 1) / zp);
    const long grid = (n_work + 7) / 8 * 8;
    if constexpr (sizeof(T) == 4) {
      if (zp == 16) {
        backproject_lds_kernel<T, 16><<<(unsigned)grid, 1024, 0, s>>>(gpad, vol, ap, n_angles, d.nx, d.ny, d.nz, ns,
                                                                      kap, tiles_x, tiles_y, (int)n_work);
        return hipGetLastError();
      }
      if (zp == 8) {
        backproject_lds_kernel<T, 8><<<(unsigned)grid, 1024, 0, s>>>(gpad, vol, ap, n_angles, d.nx, d.ny, d.nz, ns,
                                                                     kap, tiles_x, tiles_y, (int)n_work);
        return hipGetLastError();
      }
    }
    backproject_lds_kernel<T, 4><<<(unsigned)grid, 1024, 0, s>>>(gpad, vol, ap, n_angles, d.nx, d.ny, d.nz, ns,
                                                                 kap, tiles_x, tiles_y, (int)n_work);
    return hipGetLastError();
  }
  switch (xray_planes(d.nz)) {
    case 8: return backproject_dispatch<T, 8>(d, n_angles, ns, ap, two_tap, gpad, vol, kap, s);
    case 4: return backproject_dispatch<T, 4>(d, n_angles, ns, ap, two_tap, gpad, vol, kap, s);
    default: return backproject_dispatch<T, 1>(d, n_angles, ns, ap, two_tap, gpad, vol, kap, s);
  }
}

template <typename T>
__global__ void pad_rows_kernel(const T *__restrict__ g, T *__restrict__ gpad, int ns, size_t n)
{
  const int RS = ns + kRowPadL + kRowPadR;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t row = e / ns, j = e - row * ns;
    gpad[row * RS + kRowPadL + j] = g[e];
  }
}

template <typename T>
hipError_t launch_pad_rows(int rows, int ns, const T *g, T *gpad, hipStream_t s)
{
  pad_rows_kernel<T><<<2048, 256, 0, s>>>(g, gpad, ns, (size_t)rows * ns);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residual + ramp filter: one work-group per detector row (a, z).
//   r = mask (g - G);  y = mask (taps * r)  (Toeplitz, taps[n] = C h_n);
//   row_partials[row] = sum_j r_j y_j  (FP64, fixed-order tree).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
residual_ramp_kernel(const T *g, const T *__restrict__ G, const uint8_t *__restrict__ mask,
                     const T *__restrict__ taps, T *y, int ns, int y_stride, int y_off, double *row_partials)
{
  extern __shared__ unsigned char smem_raw[];
  T *r = reinterpret_cast<T *>(smem_raw);
  __shared__ double red[256];
  const size_t row = blockIdx.x;
  const size_t base = row * (size_t)ns;
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    T v = g[base + j];
    if (G) v -= G[base + j];
    if (mask && !mask[base + j]) v = T(0);
    r[j] = v;
  }
  __syncthreads();
  double part = 0.0;
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    T acc;
    if (taps) {
      acc = taps[0] * r[j];
      for (int n = 1; n < ns; n += 2) {
        T pair = T(0);
        if (j - n >= 0) pair += r[j - n];
        if (j + n < ns) pair += r[j + n];
        acc += taps[n] * pair;
      }
    } else {
      acc = r[j];
    }
    if (mask && !mask[base + j]) acc = T(0);
    y[row * (size_t)y_stride + y_off + j] = acc;
    part += (double)r[j] * (double)acc;
  }
  if (row_partials) {
    red[threadIdx.x] = part;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) row_partials[row] = red[0];
  }
}

// Rows of up to 2048 bins, register windows: thread t of a row computes the 8
// adjacent outputs j = 8t..8t+7.  For the odd taps n = 1, 3, ... the values
// r_{j-n} and r_{j+n} of its 8 outputs form two windows of 8 that move by two
// positions per tap, so each tap loads 4 new values (ring slots fixed by the tap
// modulo 4) instead of 16.  The row sits in LDS with a zero pad of P (a multiple
// of 8, at least ns + 8) on both sides and one spare word after every 8 positions
// (position e at word e + e/8), so that the lanes' reads, 8 positions apart, fall
// in distinct banks.  Each output's sum runs over the taps in order (centre tap,
// then n = 1, 3, ... with the left value added to the right), as in
// residual_ramp_kernel, with the same residual and mask; the row's FP64
// partial is summed in bin order.  At 256^3 / 256 angles: 0.14 ms FP32, 0.31 ms
// FP64, against 0.29 / 0.56 ms for 8 outputs per thread strided across the row
// (16 LDS reads per tap).
template <typename T>
__global__ void __launch_bounds__(256)
residual_ramp_win_kernel(const T *g, const T *__restrict__ G, const uint8_t *__restrict__ mask,
                         const T *__restrict__ taps, T *y, int ns, int rows, int y_stride, int y_off,
                         double *row_partials)
{
  extern __shared__ unsigned char smem_raw[];
  T *lr = reinterpret_cast<T *>(smem_raw);
  __shared__ double red[256];
  const int tpr = (ns + 7) / 8;              // threads per row
  const int rpb = 256 / tpr;                 // rows per work-group
  const int P = ((ns + 8) + 7) / 8 * 8;      // zeros on each side, a multiple of 8
  const int W = 2 * P + ns;                  // positions of a row
  const int WP = W + W / 8 + 1;              // words of a row
  const int rl = threadIdx.x / tpr, jt = threadIdx.x - rl * tpr;
  const bool in_group = rl < rpb;
  const size_t row = (size_t)blockIdx.x * rpb + (in_group ? rl : 0);
  const bool act = in_group && row < (size_t)rows;
  T *R = lr + (in_group ? rl : 0) * WP;
  if (in_group) {
    const size_t base = row * (size_t)ns;
    for (int e = jt; e < W; e += tpr) {
      const int j = e - P;
      T v = T(0);
      if (act && j >= 0 && j < ns) {
        v = g[base + j];
        if (G) v -= G[base + j];
        if (mask && !mask[base + j]) v = T(0);
      }
      R[e + (e >> 3)] = v;
    }
  }
  __syncthreads();
  // word of position P + 8 jt + d for d in [-16, 24): 9 (P/8 + jt) + d + floor(d / 8)
  const T *cb = R + 9 * (P / 8 + jt);
  T acc[8], cc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) cc[k] = cb[k];
  if (taps) {
    const T t0 = taps[0];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = t0 * cc[k];
    // ring slots: left value at position P + 8 jt + d (d = k - n) in Lr[d mod 8],
    // right value at P + 8 jt + d (d = k + n) in Rr[d mod 8]
    T Lr[8], Rr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dl = k - 1, dr = k + 1;      // the windows of n = 1
      Lr[(dl + 8) % 8] = cb[dl + (dl < 0 ? -1 : 0)];
      Rr[dr % 8] = cb[dr + (dr >= 8 ? 1 : 0)];
    }
    const T *lp = cb, *rp = cb;              // move by -9 / +9 words every 4 taps
    const int nt = ns / 2;                   // odd taps n = 1, 3, ..., < ns
    int s = 0;
    auto tap = [&](auto phase) {
      constexpr int I = decltype(phase)::value;   // s mod 4
      const T tn = taps[2 * s + 1];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int dl = k - (2 * I + 1), dr = k + (2 * I + 1);
        acc[k] = fma(tn, Lr[((dl % 8) + 8) % 8] + Rr[((dr % 8) + 8) % 8], acc[k]);
      }
      // next tap's new values: left d = -(2 I + 3), -(2 I + 2); right d = 2 I + 9, 2 I + 10
      // (relative to the pointers, which move by one block of 8 every 4 taps)
      constexpr int dl0 = -(2 * I + 3), dl1 = -(2 * I + 2), dr0 = 2 * I + 9, dr1 = 2 * I + 10;
      constexpr int wl0 = dl0 + (dl0 >= 0 ? dl0 / 8 : -((-dl0 + 7) / 8));
      constexpr int wl1 = dl1 + (dl1 >= 0 ? dl1 / 8 : -((-dl1 + 7) / 8));
      constexpr int wr0 = dr0 + dr0 / 8, wr1 = dr1 + dr1 / 8;
      Lr[((dl0 % 8) + 8) % 8] = lp[wl0];
      Lr[((dl1 % 8) + 8) % 8] = lp[wl1];
      Rr[dr0 % 8] = rp[wr0];
      Rr[dr1 % 8] = rp[wr1];
      ++s;
    };
    for (; s + 4 <= nt;) {
      tap(std::integral_constant<int, 0>{});
      tap(std::integral_constant<int, 1>{});
      tap(std::integral_constant<int, 2>{});
      tap(std::integral_constant<int, 3>{});
      lp -= 9;
      rp += 9;
    }
    if (s < nt) tap(std::integral_constant<int, 0>{});
    if (s < nt) tap(std::integral_constant<int, 1>{});
    if (s < nt) tap(std::integral_constant<int, 2>{});
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = cc[k];
  }
  double part = 0.0;
  if (act) {
    const size_t base = row * (size_t)ns;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = 8 * jt + k;
      if (j >= ns) break;
      T a = acc[k];
      if (mask && !mask[base + j]) a = T(0);
      y[row * (size_t)y_stride + y_off + j] = a;
      part += (double)cc[k] * (double)a;
    }
  }
  if (!row_partials) return;
  red[threadIdx.x] = part;
  __syncthreads();
  if (act && jt == 0) {
    double sum = 0.0;
    for (int q = 0; q < tpr; ++q) sum += red[threadIdx.x + q];
    row_partials[row] = sum;
  }
}

template <typename T>
hipError_t launch_residual_ramp(int rows, int ns, const T *g, const T *G, const uint8_t *mask, const T *taps, T *y,
                                int y_stride, int y_off, double *row_partials, hipStream_t s)
{
  if (ns <= 2048) {
    const int tpr = (ns + 7) / 8, rpb = 256 / tpr;
    const unsigned grid = (unsigned)((rows + rpb - 1) / rpb);
    const int P = ((ns + 8) + 7) / 8 * 8, W = 2 * P + ns;
    const size_t shmem = (size_t)rpb * (W + W / 8 + 1) * sizeof(T);
    residual_ramp_win_kernel<T><<<grid, 256, shmem, s>>>(g, G, mask, taps, y, ns, rows, y_stride, y_off,
                                                         row_partials);
    return hipGetLastError();
  }
  const size_t shmem = (size_t)ns * sizeof(T);
  residual_ramp_kernel<T><<<rows, 256, shmem, s>>>(g, G, mask, taps, y, ns, y_stride, y_off, row_partials);
  return hipGetLastError();
}

#define FFPAT_INST(T)                                                                                         \
  template hipError_t launch_project<T>(const Dims &, int, int, const AngleParams *, const int *, int, const T *, \
                                        T *, T *, bool, bool, T *, hipStream_t);                             \
  template hipError_t launch_backproject<T>(const Dims &, int, int, const AngleParams *, bool, const T *, T *, \
                                            const T *, hipStream_t);                                         \
  template hipError_t launch_pad_rows<T>(int, int, const T *, T *, hipStream_t);                             \
  template hipError_t launch_residual_ramp<T>(int, int, const T *, const T *, const uint8_t *, const T *, T *, \
                                              int, int, double *, hipStream_t);
FFPAT_INST(float)
FFPAT_INST(double)
#undef FFPAT_INST

}  // namespace ffpat
