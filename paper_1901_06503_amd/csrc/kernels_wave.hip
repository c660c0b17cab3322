// Leapfrog time stepping of the variable-speed wave equation (Sec. 2.1,
// eq. wave1/wave2), fourth-order in space, on gfx950.
//
//   S(p)   = sum over axes of (-p[-2] + 16 p[-1] - 30 p[0] + 16 p[+1] - p[+2]),
//            zero outside the grid (integer coefficients; 1/(12 dx^2) and
//            (c dt)^2 are folded into k' = (c dt)^2 / (12 dx^2)).
//   first  p1      = p0 + 1/2 k' S(p0)         (zero initial velocity)
//   leap   p(k+1)  = 2 p(k) - p(k-1) + k' S(p(k))
//
// The step is HBM-bound (16 B per point update in FP32: read p(k), p(k-1),
// k', write p(k+1)).  Two kernels:
//   * wave_step_naive: one thread per point, 13 global loads (cache-reliant).
//   * wave_step_blocked: 2.5D blocking.  A work-group owns a TX x TY tile of
//     x-y columns and marches along z; the plane under update sits in LDS
//     with a 2-point halo, the four z-neighbours of each column stay in
//     registers, so every p(k) value is fetched from HBM about once.
#include "kernels.h"
#include "launch_rules.h"

#include <type_traits>

#include <atomic>
#include <cfloat>
#include <cstdint>
#include <cstdlib>

namespace ffpat {

template <typename T, int NDIM, int MODE>
__global__ void __launch_bounds__(256)
wave_step_naive(const T *__restrict__ p, const T *prev, T *out, const T *__restrict__ kap, int nx, int ny, int nz)
{
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  const size_t idx = (size_t)z * sz + (size_t)y * sy + x;

  const T c0 = p[idx];
  T s1 = T(0), s2 = T(0);
  if (x >= 1) s1 += p[idx - 1];
  if (x + 1 < nx) s1 += p[idx + 1];
  if (x >= 2) s2 += p[idx - 2];
  if (x + 2 < nx) s2 += p[idx + 2];
  if (y >= 1) s1 += p[idx - sy];
  if (y + 1 < ny) s1 += p[idx + sy];
  if (y >= 2) s2 += p[idx - 2 * sy];
  if (y + 2 < ny) s2 += p[idx + 2 * sy];
  if (NDIM == 3) {
    if (z >= 1) s1 += p[idx - sz];
    if (z + 1 < nz) s1 += p[idx + sz];
    if (z >= 2) s2 += p[idx - 2 * sz];
    if (z + 2 < nz) s2 += p[idx + 2 * sz];
  }
  const T S = T(16) * s1 - s2 - T(NDIM == 3 ? 90 : 60) * c0;
  const T k = kap[idx];
  T v;
  if (MODE == STEP_FIRST || MODE == STEP_FIRST_DIV) v = c0 + T(0.5) * k * S;
  else v = T(2) * c0 - prev[idx] + k * S;
  if (MODE == STEP_FIRST_DIV || MODE == STEP_LEAP_DIV) v = v / k;
  out[idx] = v;
}

template <typename T, int NDIM>
static hipError_t naive_dispatch(StepMode mode, const Dims &d, const T *p, const T *prev, T *out, const T *kap,
                                 hipStream_t s)
{
  dim3 block(64, 4, 1);
  dim3 grid((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz);
  switch (mode) {
    case STEP_FIRST: wave_step_naive<T, NDIM, STEP_FIRST><<<grid, block, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz); break;
    case STEP_LEAP: wave_step_naive<T, NDIM, STEP_LEAP><<<grid, block, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz); break;
    case STEP_FIRST_DIV: wave_step_naive<T, NDIM, STEP_FIRST_DIV><<<grid, block, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz); break;
    case STEP_LEAP_DIV: wave_step_naive<T, NDIM, STEP_LEAP_DIV><<<grid, block, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 2.5D-blocked step.  Work-group = 256 threads = 4 wavefronts; tile = 64 x BY
// columns (BY = 4 RY), each wavefront owns whole 64-wide rows (coalesced).
// The group marches z over [zbeg, zbeg + zchunk): plane z of p(k) sits in LDS
// with a 2-point x/y halo (double-buffered, one barrier per plane); the
// values at z-2..z+2 of the thread's RY columns stay in registers; p(k) at
// z+3, p(k-1) and k' are fetched ahead of use.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T ld3(const T *__restrict__ p, int x, int y, int z, int nx, int ny, int nz)
{
  return (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) ? p[((size_t)z * ny + y) * nx + x] : T(0);
}

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p, bool nt)
{
  return nt ? __builtin_nontemporal_load(p) : *p;
}

template <typename T, int NDIM, int MODE, int RY, bool NT>
__global__ void __launch_bounds__(256)
wave_step_blocked(const T *__restrict__ p, const T *prev, T *out, const T *__restrict__ kap, int nx, int ny, int nz,
                  int zchunk, int tiles_x, int tiles_y, int n_tiles, int xy_fastest)
{
  constexpr int BX = 64, TYN = 4, BY = TYN * RY;
  constexpr int LW = BX + 4, LH = BY + 4;
  __shared__ T lds[2][LH * LW];

  // XCD-aware tile order: consecutive work-groups are dealt round-robin to
  // the 8 XCDs; give each XCD a contiguous range of tiles (x-y tiles or
  // z-chunks fastest within it) so that neighbouring tiles share that XCD's L2.
  const int b = blockIdx.x;
  const int per_xcd = (n_tiles + 7) / 8;
  const int t = (b % 8) * per_xcd + b / 8;
  if (t >= n_tiles) return;                      // whole group exits together
  const int n_zc = (nz + zchunk - 1) / zchunk;
  int zc, txy;
  if (xy_fastest) {
    const int n_xy = tiles_x * tiles_y;
    txy = t % n_xy;
    zc = t / n_xy;
  } else {
    zc = t % n_zc;
    txy = t / n_zc;
  }
  const int bxi = txy % tiles_x, byi = txy / tiles_x;

  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int x0 = bxi * BX, y0 = byi * BY;
  const int x = x0 + tx;
  const int zbeg = zc * zchunk;
  const int zend = min(nz, zbeg + zchunk);
  const size_t plane = (size_t)nx * ny;

  T w[RY][5];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = y0 + ty + TYN * r;
#pragma unroll
    for (int q = 0; q < 5; ++q)
      w[r][q] = (NDIM == 3 || q == 2) ? ld3(p, x, y, zbeg - 2 + q, nx, ny, nz) : T(0);
  }

  int buf = 0;
  for (int z = zbeg; z < zend; ++z, buf ^= 1) {
    T *L = lds[buf];
    // interior of plane z from registers
#pragma unroll
    for (int r = 0; r < RY; ++r) L[(ty + TYN * r + 2) * LW + tx + 2] = w[r][2];
    // halo of plane z: rows y0-2, y0-1, y0+BY, y0+BY+1 (full width), then
    // columns x0-2, x0-1, x0+BX, x0+BX+1 of the interior rows
    for (int e = threadIdx.x; e < 4 * LW + 4 * BY; e += 256) {
      int lr, lc;
      if (e < 4 * LW) {
        const int hr = e / LW;
        lr = hr < 2 ? hr : BY + hr;
        lc = e - hr * LW;
      } else {
        const int e2 = e - 4 * LW;
        const int hc = e2 / BY;
        lc = hc < 2 ? hc : BX + hc;
        lr = 2 + (e2 - hc * BY);
      }
      L[lr * LW + lc] = ld3(p, x0 + lc - 2, y0 + lr - 2, z, nx, ny, nz);
    }
    // values needed later in this step and by the next plane
    T nxt[RY], pv[RY], kv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int y = y0 + ty + TYN * r;
      const bool in = x < nx && y < ny;
      const size_t idx = (size_t)z * plane + (size_t)y * nx + x;
      // 3D: plane z+3 enters the window; 2D: the next centre plane z+1
      nxt[r] = ld3(p, x, y, NDIM == 3 ? z + 3 : z + 1, nx, ny, nz);
      kv[r] = in ? ld_stream(kap + idx, NT) : T(1);
      pv[r] = (in && (MODE == STEP_LEAP || MODE == STEP_LEAP_DIV)) ? ld_stream(prev + idx, NT) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int y = y0 + ty + TYN * r;
      const T *c = &L[(ty + TYN * r + 2) * LW + tx + 2];
      T s1 = (c[-1] + c[1]) + (c[-LW] + c[LW]);
      T s2 = (c[-2] + c[2]) + (c[-2 * LW] + c[2 * LW]);
      if (NDIM == 3) {
        s1 += w[r][1] + w[r][3];
        s2 += w[r][0] + w[r][4];
      }
      const T c0 = w[r][2];
      const T S = T(16) * s1 - s2 - T(NDIM == 3 ? 90 : 60) * c0;
      T v;
      if (MODE == STEP_FIRST || MODE == STEP_FIRST_DIV) v = c0 + T(0.5) * kv[r] * S;
      else v = T(2) * c0 - pv[r] + kv[r] * S;
      if (MODE == STEP_FIRST_DIV || MODE == STEP_LEAP_DIV) v = v / kv[r];
      if (x < nx && y < ny) {
        T *o = out + (size_t)z * plane + (size_t)y * nx + x;
        if (NT) __builtin_nontemporal_store(v, o);
        else *o = v;
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (NDIM == 3) {
        w[r][0] = w[r][1];
        w[r][1] = w[r][2];
        w[r][2] = w[r][3];
        w[r][3] = w[r][4];
        w[r][4] = nxt[r];
      } else {
        w[r][2] = nxt[r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Two leapfrog steps per pass (temporal blocking):
//   q = p(k+1) = 2 p(k) - p(k-1) + k' S(p(k))   on the tile plus a 2-point halo
//   o = p(k+2) = 2 q    - p(k)   + k' S(q)      on the tile
// One pass reads p(k-1), p(k), k' and writes p(k+1), p(k+2): 20 B per two point
// updates in FP32 instead of 32 B, the halo re-reads served by L2.
// A work-group owns a BX x BY tile (BX 64, or 128 in FP32) and a z-chunk.  It
// marches the stage-1 plane zs from zbeg - 2 to zend + 1; stage 2 follows two
// planes behind (z = zs - 2).
// Every thread owns up to PPT slots of rows 0..BY+3 of the p(k) plane's LDS
// region, BX + 8 wide: the extended tile (BX + 4) x (BY + 4) plus the two outer
// columns on each side, and keeps, per slot, p(k) at zs-2..zs+2 and, per
// extended-tile point, q at zs-4..zs and k' at zs-2..zs in registers (the outer
// columns then arrive in the same coalesced row loads; only the two outer rows
// above and below are loaded apart: 2.5-5.6% faster at 224^3..512^3 than loading
// the outer columns point by point, one cache line each).  LDS holds p(k) of plane
// zs with a 4-point halo (stage-1 x-y neighbours) and q of the last five planes
// with a 2-point halo (stage-2 x-y neighbours).  Every window slot is a plane
// index modulo 5 and the z loop is unrolled ten times, so the slots are fixed registers and LDS offsets (no
// copies when the window moves).  The loads of plane zs + 2 are issued during
// plane zs (two buffer sets, alternating), unconditionally (clamped in-grid
// addresses, values masked where used), so they stay in flight across the
// barriers (two per plane in FP32, one in FP64); loads and stores address a
// uniform plane base plus the lane's 32-bit byte offset (measured faster here
// than buffer-resource addressing, which saves the 64-bit adds).  q is zero
// outside the grid.
// Inputs and outputs are four distinct buffers (neighbouring groups read the
// inputs in their halos while this group writes).  Requires plane bytes < 2^31.
// ---------------------------------------------------------------------------
// Two adjacent FP32 points along x as one 8-byte element (the two-step kernel's FP32
// form for even nx): loads, stores and LDS accesses move 8 bytes per lane.
typedef float f32x2 __attribute__((ext_vector_type(2)));

// x-direction terms of the stencil at element c: s1 = p(x-1) + p(x+1), s2 = p(x-2) +
// p(x+2).  One point per element: the neighbouring elements.  Two points per element
// (x = 2j, 2j+1): the neighbours lie in elements j-1, j and j+1.
template <typename T>
struct StencilX {
  static __device__ __forceinline__ void terms(const T *c, T &s1, T &s2)
  {
    s1 = c[-1] + c[1];
    s2 = c[-2] + c[2];
  }
};
template <>
struct StencilX<f32x2> {
  static __device__ __forceinline__ void terms(const f32x2 *c, f32x2 &s1, f32x2 &s2)
  {
    const f32x2 l = c[-1], m = c[0], r = c[1];
    s1 = f32x2{l.y + m.y, m.x + r.x};
    s2 = f32x2{l.x + r.x, l.y + r.y};
  }
};

template <typename T>
__device__ __forceinline__ T ldb(const T *base, unsigned boff)
{
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff);
}

template <typename T>
__device__ __forceinline__ void stb(T *base, unsigned boff, T v)
{
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff) = v;
}

template <typename T, int NDIM, int RY, int NTH, int BX>
// FP32 with 512 threads: at most 128 VGPRs, so two work-groups share a compute unit
// (1024 threads allow no more than 128 in any case)
__global__ void __launch_bounds__(NTH, (sizeof(T) == 4 && NTH >= 512) ? 4 : 1)
wave_step2_blocked(const T *__restrict__ pm1, const T *__restrict__ pk, T *__restrict__ q_out,
                   T *__restrict__ o_out, const T *__restrict__ kap, int nx, int ny, int nz, int zchunk, int tiles_x,
                   int tiles_y, int n_tiles, int xy_fastest)
{
  constexpr int BY = 4 * RY;
  constexpr int EX = BX + 4, EY = BY + 4;   // extended tile: stage-1 output region
  constexpr int KX = BX + 8, KY = BY + 8;   // p(k) plane in LDS: stage-1 input region
  // threads walk rows 0..EY-1 of the LDS region, all KX columns, so consecutive
  // lanes address consecutive LDS words and consecutive grid points
  constexpr int NES = KX * EY;
  constexpr int PPT = (NES + NTH - 1) / NTH;
  constexpr int NRING = 4 * KX;              // rows 0, 1, KY-2, KY-1 of the p(k) plane
  constexpr int RPT = (NRING + NTH - 1) / NTH;
  // FP64: the p(k) plane double-buffered by plane parity, so that the next plane's
  // write cannot race this plane's stage-1 reads and one barrier per plane suffices
  // (stage 2 reads only q planes written two planes earlier and its own registers):
  // 0.5-3% faster in FP64; neutral to 1% slower in FP32, which keeps two barriers.
  constexpr int NLK = sizeof(T) == 8 ? 2 : 1;
  // FP32 64-wide: the lane offsets are made opaque each plane, so that every load
  // and store takes a scalar base plus the 32-bit offset instead of a 64-bit
  // address kept in registers (the compiler hoists base + offset out of the z loop
  // and then spills one such address): no spill, 0.6-5.7% faster at 160^3..448^3.
  // The 128-wide FP32 kernel (1-2% slower with it) and FP64 keep the hoisted form.
  constexpr bool SADDR = sizeof(T) == 4 && BX == 64;
  __shared__ T lk[NLK][KY * KX];
  __shared__ T lq[5][EY * KX];   // q planes, row pitch KX

  const int b = blockIdx.x;
  const int per_xcd = (n_tiles + 7) / 8;
  const int t = (b % 8) * per_xcd + b / 8;
  if (t >= n_tiles) return;                 // whole group exits together
  const int n_zc = (nz + zchunk - 1) / zchunk;
  int zc, txy;
  if (xy_fastest) {
    const int n_xy = tiles_x * tiles_y;
    txy = t % n_xy;
    zc = t / n_xy;
  } else {
    zc = t % n_zc;
    txy = t / n_zc;
  }
  const int x0 = (txy % tiles_x) * BX, y0 = (txy / tiles_x) * BY;
  const int zbeg = zc * zchunk;
  const int zend = min(nz, zbeg + zchunk);
  const size_t plane = (size_t)nx * ny;
  const int zstart = zbeg - 2;              // first stage-1 plane; ring slot of plane p: (p - zstart) mod 5

  // Per slot: its LDS column and extended-tile row, flags, and the byte offset of
  // its position within a plane, clamped into the grid so that every load is in
  // bounds (a point outside reads a neighbour's value and its flag zeroes it).
  int ex[PPT], ey[PPT];
  unsigned boff[PPT];
  bool win[PPT], ev[PPT], ingw[PPT], ing[PPT], inter[PPT];
  T w[PPT][5], r1[PPT][5], kr[PPT][5];
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    const int e = threadIdx.x + NTH * m;
    // ex: column of the p(k) plane in LDS (0..KX-1); every slot of rows 0..EY-1
    // keeps a p(k) window (the two outer columns on each side only feed the plane),
    // and the stage-1 points are columns 2..EX+1
    ey[m] = e < NES ? e / KX : 0;
    ex[m] = e < NES ? e - ey[m] * KX : 0;
    win[m] = e < NES;
    ev[m] = win[m] && ex[m] >= 2 && ex[m] < EX + 2;
    const int gx = x0 - 4 + ex[m], gy = y0 - 2 + ey[m];
    ingw[m] = win[m] && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    ing[m] = ev[m] && ingw[m];
    inter[m] = ing[m] && ex[m] >= 4 && ex[m] < EX && ey[m] >= 2 && ey[m] < EY - 2;
    boff[m] = (unsigned)((min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1)) * sizeof(T));
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      w[m][q] = T(0);
      r1[m][q] = T(0);
      kr[m][q] = T(0);
    }
    // 3D: p(k) at zstart-2..zstart+1 in slots 3, 4, 0, 1 (zstart + 2 arrives with the first plane)
#pragma unroll
    for (int d = -2; d <= 1; ++d) {
      const int zq = zstart + d;
      if (NDIM == 3 && zq >= 0 && zq < nz) {
        const T v = ldb(pk + (size_t)zq * plane, boff[m]);
        w[m][(d + 5) % 5] = ingw[m] ? v : T(0);
      }
    }
  }

  // ring elements of the p(k) plane owned by this thread (fixed positions)
  int rl[RPT];
  unsigned roff[RPT];
  bool rin[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int e = threadIdx.x + NTH * j;
    const bool rv = e < NRING;
    int lr = 0, lc = 0;
    if (rv) {
      const int hr = e / KX;
      lr = hr < 2 ? hr : KY - 4 + hr;
      lc = e - hr * KX;
    }
    rl[j] = rv ? lr * KX + lc : -1;
    const int gx = x0 - 4 + lc, gy = y0 - 4 + lr;
    rin[j] = rv && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    roff[j] = (unsigned)((min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1)) * sizeof(T));
  }

  // software pipeline: the loads of plane zs + 2 are issued during plane zs, into
  // the buffer set that plane zs has just been consumed from (sets alternate)
  T nw[2][PPT], npv[2][PPT], nkv[2][PPT], nring[2][RPT];
  auto fetch = [&](auto buf, int zf) {
    constexpr int B = decltype(buf)::value;
    const int zw = min(max(NDIM == 3 ? zf + 2 : zf, 0), nz - 1);   // p(k) plane entering the window
    const int zc2 = min(max(zf, 0), nz - 1);
    const T *bw = pk + (size_t)zw * plane, *bp = pm1 + (size_t)zc2 * plane, *bk = kap + (size_t)zc2 * plane;
    const T *br = pk + (size_t)zc2 * plane;
    if constexpr (SADDR) {
#pragma unroll
      for (int m = 0; m < PPT; ++m) asm volatile("" : "+v"(boff[m]));
#pragma unroll
      for (int j = 0; j < RPT; ++j) asm volatile("" : "+v"(roff[j]));
    }
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      nw[B][m] = ldb(bw, boff[m]);
      npv[B][m] = ldb(bp, boff[m]);
      nkv[B][m] = ldb(bk, boff[m]);
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) nring[B][j] = ldb(br, roff[j]);
  };
  fetch(std::integral_constant<int, 0>{}, zstart);
  fetch(std::integral_constant<int, 1>{}, zstart + 1);

  // one stage-1 plane zs with phase Q = (zs - zstart) mod 10: window slot of plane zs + d is
  // (P + d) mod 5 with P = Q mod 5, the plane's loads sit in buffer set Q mod 2
  auto step = [&](auto phase, int zs) {
    constexpr int Q = decltype(phase)::value;
    constexpr int P = Q % 5, B = Q % 2;
    constexpr int Sm2 = (P + 3) % 5, Sm1 = (P + 4) % 5, S0 = P, Sp1 = (P + 1) % 5, Sp2 = (P + 2) % 5;
    constexpr int Sm3 = (P + 2) % 5, Sm4 = (P + 1) % 5;
    const int z = zs - 2;
    const bool zs_in = zs >= 0 && zs < nz;
    const int zw = NDIM == 3 ? zs + 2 : zs;
    const bool zw_in = zw >= 0 && zw < nz;
    // stage-1 inputs of plane zs (fetched one plane ahead)
    T pv[PPT], kv[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      const T v = (ingw[m] && zw_in) ? nw[B][m] : T(0);
      if (NDIM == 3) w[m][Sp2] = v;
      else w[m][S0] = v;
      pv[m] = npv[B][m];   // used only where the point and plane zs are inside the grid
      kv[m] = nkv[B][m];
      if (win[m]) lk[B % NLK][(ey[m] + 2) * KX + ex[m]] = w[m][S0];
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j)
      if (rl[j] >= 0) lk[B % NLK][rl[j]] = (rin[j] && zs_in) ? nring[B][j] : T(0);
    fetch(std::integral_constant<int, B>{}, zs + 2);   // clamped: past the last plane it re-reads valid memory, unused
    __syncthreads();
    // stage 1: q(zs) on the extended tile
    T *q_pl = q_out + (size_t)min(max(zs, 0), nz - 1) * plane;
    const bool zs_own = zs >= zbeg && zs < zend;
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      if (!ev[m]) continue;
      const T *c = &lk[B % NLK][(ey[m] + 2) * KX + ex[m]];
      T s1, s2;
      StencilX<T>::terms(c, s1, s2);
      s1 = s1 + (c[-KX] + c[KX]);
      s2 = s2 + (c[-2 * KX] + c[2 * KX]);
      if (NDIM == 3) {
        s1 += w[m][Sm1] + w[m][Sp1];
        s2 += w[m][Sm2] + w[m][Sp2];
      }
      const T c0 = w[m][S0];
      const T S = T(16) * s1 - s2 - T(NDIM == 3 ? 90 : 60) * c0;
      const T q = (ing[m] && zs_in) ? T(2) * c0 - pv[m] + kv[m] * S : T(0);
      lq[S0][ey[m] * KX + ex[m]] = q;
      r1[m][S0] = q;
      kr[m][S0] = kv[m];
      if (inter[m] && zs_own) {   // the point's own plane in its own chunk
        if constexpr (SADDR) asm volatile("" : "+v"(boff[m]));
        stb(q_pl, boff[m], q);
      }
    }
    if constexpr (NLK == 1) __syncthreads();   // the p(k) plane is rewritten next
    // stage 2: o(z) on the tile, z = zs - 2: q(z) x-y neighbours from LDS, z neighbours
    // (planes z-2..z+2 = zs-4..zs) from registers
    if (z >= zbeg) {
      T *o_pl = o_out + (size_t)z * plane;
#pragma unroll
      for (int m = 0; m < PPT; ++m) {
        if (!inter[m]) continue;
        const T *c = &lq[Sm2][ey[m] * KX + ex[m]];
        T s1, s2;
        StencilX<T>::terms(c, s1, s2);
        s1 = s1 + (c[-KX] + c[KX]);
        s2 = s2 + (c[-2 * KX] + c[2 * KX]);
        if (NDIM == 3) {
          s1 += r1[m][Sm3] + r1[m][Sm1];
          s2 += r1[m][Sm4] + r1[m][S0];
        }
        const T c0 = r1[m][Sm2];
        const T S = T(16) * s1 - s2 - T(NDIM == 3 ? 90 : 60) * c0;
        if constexpr (SADDR) asm volatile("" : "+v"(boff[m]));
        stb(o_pl, boff[m], T(2) * c0 - w[m][Sm2] + kr[m][Sm2] * S);
      }
    }
  };

  const int zlast = zend + 1;               // last stage-1 plane
  for (int zb = zstart; zb <= zlast; zb += 10) {
    step(std::integral_constant<int, 0>{}, zb);
    if (zb + 1 > zlast) break;
    step(std::integral_constant<int, 1>{}, zb + 1);
    if (zb + 2 > zlast) break;
    step(std::integral_constant<int, 2>{}, zb + 2);
    if (zb + 3 > zlast) break;
    step(std::integral_constant<int, 3>{}, zb + 3);
    if (zb + 4 > zlast) break;
    step(std::integral_constant<int, 4>{}, zb + 4);
    if (zb + 5 > zlast) break;
    step(std::integral_constant<int, 5>{}, zb + 5);
    if (zb + 6 > zlast) break;
    step(std::integral_constant<int, 6>{}, zb + 6);
    if (zb + 7 > zlast) break;
    step(std::integral_constant<int, 7>{}, zb + 7);
    if (zb + 8 > zlast) break;
    step(std::integral_constant<int, 8>{}, zb + 8);
    if (zb + 9 > zlast) break;
    step(std::integral_constant<int, 9>{}, zb + 9);
  }
}

// ---------------------------------------------------------------------------
// Two leapfrog steps per pass, 3D, 8-byte elements (FP64, or FP32 as pairs of
// x-adjacent points), 64 x 16 element tile, 512 threads: the arithmetic of
// wave_step2_blocked (every sum in the same order, so the results are the same
// bits) with points assigned to threads so that no lane-dependent branch sits
// between the LDS reads of different points:
//   slots 0 and 1: the tile's 1024 interior points, one 64-wide row per
//     wavefront and slot (coalesced); they run stage 1 and stage 2 and keep the
//     q and k' z-windows;
//   slot 2: the other points of the LDS region's rows 2..21 (the extended tile's
//     2-point halo and the two outer points on each side; 416 elements in FP64,
//     336 pairs), stage 1 only, so no q or k' windows;
//   ring: rows 0, 1, 22, 23 of the p(k) plane (288 elements, 272 pairs).
// The x halos are counted in elements: pairs of points need half the elements
// (and stage 1 half the halo columns) that single points do.
// Stage 1 issues the LDS reads of all three slots before any arithmetic and
// stage 2 those of both interior slots, so each stage waits for LDS once per
// plane.  Stage 1 runs on every slot unconditionally; a point off the grid or
// plane yields q = 0 by a select, the outer columns' values land in q columns
// that stage 2 never reads, and threads without a halo point write theirs to a
// spare LDS word and to q column 0.  The results are pinned in registers before
// the global stores, so the compiler cannot sink a slot's LDS reads into them.
// The stores are buffer stores whose range check drops the lanes off the grid and,
// for planes outside the group's chunk, all lanes (a zero-size range): every plane
// issues the same memory instructions on every path, so the compiler's wait
// counts stay exact and the loads of plane zs + 2 remain in flight across the
// barriers of planes zs and zs + 1 instead of being waited for together with the
// stores that a branch may or may not have issued.  Prefetch and windows as in
// wave_step2_blocked.
// ---------------------------------------------------------------------------
template <typename T>
struct NbrX;   // x neighbours read from LDS (the centre comes from registers)
template <>
struct NbrX<double> {
  static constexpr int N = 4;   // c[-2], c[-1], c[1], c[2]
  template <typename P>
  static __device__ __forceinline__ void load(P c, double *v)
  {
    v[0] = c[-2];
    v[1] = c[-1];
    v[2] = c[1];
    v[3] = c[2];
  }
  static __device__ __forceinline__ void terms(const double *v, double, double &s1, double &s2)
  {
    s1 = v[1] + v[2];
    s2 = v[0] + v[3];
  }
};
template <>
struct NbrX<f32x2> {
  static constexpr int N = 2;   // elements j-1 and j+1 (points 2j-2, 2j-1 and 2j+2, 2j+3)
  template <typename P>
  static __device__ __forceinline__ void load(P c, f32x2 *v)
  {
    v[0] = c[-1];
    v[1] = c[1];
  }
  static __device__ __forceinline__ void terms(const f32x2 *v, f32x2 m, f32x2 &s1, f32x2 &s2)
  {
    const f32x2 l = v[0], r = v[1];
    s1 = f32x2{l.y + m.y, m.x + r.x};
    s2 = f32x2{l.x + r.x, l.y + r.y};
  }
};

// An empty asm statement that passes N register values through at once: the loads
// that produce them are all issued before it, the wait for them comes once, at it,
// and the arithmetic on them after it.
template <typename T, int N>
struct LdsFence;
template <typename T>
struct LdsFence<T, 18> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
                 "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]));
  }
};
template <typename T>
struct LdsFence<T, 24> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
                 "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]), "+v"(v[18]), "+v"(v[19]), "+v"(v[20]),
                 "+v"(v[21]), "+v"(v[22]), "+v"(v[23]));
  }
};

// 8-byte store through a buffer resource of `bytes` bytes at `base`: lanes whose byte
// offset is out of range (and all lanes when bytes = 0) write nothing.
template <typename T>
__device__ __forceinline__ void st_ranged(T *base, unsigned bytes, unsigned boff, T v)
{
  static_assert(sizeof(T) == 8, "8-byte elements");
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, boff, 0, 0);
}

// 8-byte load through a buffer resource of `bytes` bytes at `base`: lanes whose byte
// offset is out of range (and all lanes when bytes = 0) read zeros.
template <typename T>
__device__ __forceinline__ T ld_ranged(const T *base, unsigned bytes, unsigned boff)
{
  static_assert(sizeof(T) == 8, "8-byte elements");
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(base), (short)0, (int)bytes, 0x00020000);
  return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}

// RESTRICT: the inputs and outputs are declared non-aliasing.  Without it (FP32
// pairs) the compiler must keep each plane's prefetch loads ahead of the plane's
// stores, i.e. where they are written; with it, it sinks them past the z loop's
// exit tests to the next plane, which halves the prefetch distance: the FP32 pairs
// kernel is 1% faster without, the FP64 kernel 7% faster with (without, it spills).
// DIV: the second step is the adjoint solve's last one, divided by k' (the
// single-step kernel's STEP_LEAP_DIV, the same expression).  FIRSTSTEP: the pass
// starts a solve from pk = p(0) with zero initial velocity (its first step is the
// single-step kernel's STEP_FIRST expression; pm1 is not read) and yields p(1), p(2).
template <typename T, bool RESTRICT, bool DIV = false, bool FIRSTSTEP = false>
__global__ void __launch_bounds__(512, 1)
wave_step2_split(std::conditional_t<RESTRICT, const T *__restrict__, const T *> pm1,
                 std::conditional_t<RESTRICT, const T *__restrict__, const T *> pk,
                 std::conditional_t<RESTRICT, T *__restrict__, T *> q_out,
                 std::conditional_t<RESTRICT, T *__restrict__, T *> o_out,
                 std::conditional_t<RESTRICT, const T *__restrict__, const T *> kap, int nx, int ny, int nz,
                 int zchunk, int tiles_x, int tiles_y, int n_tiles, int xy_fastest)
{
  constexpr int NTH = 512, BX = 64, BY = 16;
  // x halos in elements: the p(k) plane needs 4 points on each side, stage 1 runs on
  // 2 more points on each side than the tile: 4 and 2 elements in FP64, 2 and 1 for
  // pairs of points
  constexpr int XH = NbrX<T>::N == 2 ? 2 : 4, SH = XH / 2;
  constexpr int EY = BY + 4;                 // stage-1 rows
  constexpr int KX = BX + 2 * XH, KY = BY + 8;   // p(k) plane in LDS (FP64 72 x 24, pairs 68 x 24)
  constexpr int NIN = BX * BY / NTH;         // interior slots per thread (2)
  constexpr int NHALO = KX * EY - BX * BY;   // other points of LDS rows 2..KY-3 (FP64 416, pairs 336)
  constexpr int NRING = 4 * KX;              // LDS rows 0, 1, KY-2, KY-1 (FP64 288, pairs 272)
  constexpr int PPT = NIN + 1;
  constexpr int NB = NbrX<T>::N + 4;         // LDS reads per point and stage
  static_assert(BX * BY == NIN * NTH && NHALO <= NTH && NRING <= NTH, "slot layout");
  __shared__ T lk[2][KY * KX + 1];           // p(k) plane, double-buffered by plane parity (+ a spare word)
  __shared__ T lq[5][EY * KX];               // q planes, row pitch KX

  const int b = blockIdx.x;
  const int per_xcd = (n_tiles + 7) / 8;
  const int t = (b % 8) * per_xcd + b / 8;
  if (t >= n_tiles) return;                  // whole group exits together
  const int n_zc = (nz + zchunk - 1) / zchunk;
  int zc, txy;
  if (xy_fastest) {
    const int n_xy = tiles_x * tiles_y;
    txy = t % n_xy;
    zc = t / n_xy;
  } else {
    zc = t % n_zc;
    txy = t / n_zc;
  }
  const int x0 = (txy % tiles_x) * BX, y0 = (txy / tiles_x) * BY;
  const int zbeg = zc * zchunk;
  const int zend = min(nz, zbeg + zchunk);
  const size_t plane = (size_t)nx * ny;
  const int zstart = zbeg - 2;
  const int tid = threadIdx.x;

  // per slot: LDS index in the p(k) plane and in a q plane, in-grid flags, byte
  // offset of the (clamped) grid position within a plane
  int lofs[PPT], lwr[PPT], qofs[PPT];   // LDS read centre, write index, q-plane index
  unsigned boff[PPT], soff[NIN];          // load offset (clamped); store offset (out of range off the grid)
  bool ingw[PPT], ing[PPT];
  const unsigned plane_bytes = (unsigned)(plane * sizeof(T));
  T w[PPT][5], r1[NIN][5], kr[NIN][5];
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    int ex, ey;
    bool has = true;
    if (m < NIN) {
      const int i = tid + NTH * m;
      ey = 2 + i / BX;
      ex = XH + i % BX;
    } else if (tid < 4 * KX) {             // extended rows 0, 1, EY-2, EY-1, full width
      const int r = tid / KX;
      ey = r < 2 ? r : EY - 4 + r;
      ex = tid - r * KX;
    } else if (tid < NHALO) {              // rows 2..EY-3, columns 0..XH-1 and KX-XH..KX-1
      const int j = tid - 4 * KX;
      ey = 2 + j / (2 * XH);
      const int cc = j % (2 * XH);
      ex = cc < XH ? cc : KX - 2 * XH + cc;
    } else {                               // no halo point: reads around an interior position
      has = false;
      ey = 2;
      ex = XH;
    }
    lofs[m] = (ey + 2) * KX + ex;
    lwr[m] = has ? lofs[m] : KY * KX;      // the spare word
    qofs[m] = has ? ey * KX + ex : 0;      // q column 0: never read
    const int gx = x0 - XH + ex, gy = y0 - 2 + ey;
    ingw[m] = has && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    ing[m] = ingw[m] && ex >= XH - SH && ex < XH + BX + SH;   // a stage-1 point of the grid
    boff[m] = (unsigned)((min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1)) * sizeof(T));
    if (m < NIN) soff[m] = ing[m] ? boff[m] : 0xFFFFFFF0u;
#pragma unroll
    for (int q = 0; q < 5; ++q) w[m][q] = T(0);
#pragma unroll
    for (int d = -2; d <= 1; ++d) {
      const int zq = zstart + d;
      if (zq >= 0 && zq < nz) {
        const T v = ldb(pk + (size_t)zq * plane, boff[m]);
        w[m][(d + 5) % 5] = ingw[m] ? v : T(0);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < NIN; ++m)
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      r1[m][q] = T(0);
      kr[m][q] = T(0);
    }

  // ring element of the p(k) plane owned by this thread
  const bool has_ring = tid < NRING;
  int rl;
  unsigned roff;
  bool rin;
  {
    const int hr = has_ring ? tid / KX : 0;
    const int lr = hr < 2 ? hr : KY - 4 + hr;
    const int lc = has_ring ? tid - hr * KX : 0;
    rl = lr * KX + lc;
    const int gx = x0 - XH + lc, gy = y0 - 4 + lr;
    rin = has_ring && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    roff = (unsigned)((min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1)) * sizeof(T));
  }

  T nw[2][PPT], npv[2][PPT], nkv[2][PPT], nring[2];
  auto fetch = [&](auto buf, int zf) {
    constexpr int B = decltype(buf)::value;
    const int zw = min(max(zf + 2, 0), nz - 1);   // p(k) plane entering the window
    const int zc2 = min(max(zf, 0), nz - 1);
    const T *bw = pk + (size_t)zw * plane, *bp = pm1 + (size_t)zc2 * plane, *bk = kap + (size_t)zc2 * plane;
    const T *br = pk + (size_t)zc2 * plane;
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      nw[B][m] = ldb(bw, boff[m]);
      npv[B][m] = FIRSTSTEP ? T(0) : ldb(bp, boff[m]);
      nkv[B][m] = ldb(bk, boff[m]);
    }
    nring[B] = ldb(br, roff);
  };
  fetch(std::integral_constant<int, 0>{}, zstart);
  fetch(std::integral_constant<int, 1>{}, zstart + 1);

  // STAGE2: whether the plane's stage 2 is needed (not on the group's first four
  // planes, whose o, two planes behind, lies before the chunk)
  auto step = [&](auto phase, auto stage2, int zs) {
    constexpr int Q = decltype(phase)::value;
    constexpr bool STAGE2 = decltype(stage2)::value;
    constexpr int P = Q % 5, B = Q % 2;
    constexpr int Sm2 = (P + 3) % 5, Sm1 = (P + 4) % 5, S0 = P, Sp1 = (P + 1) % 5, Sp2 = (P + 2) % 5;
    constexpr int Sm3 = (P + 2) % 5, Sm4 = (P + 1) % 5;
    const int z = zs - 2;
    const bool zs_in = zs >= 0 && zs < nz;
    const bool zw_in = zs + 2 >= 0 && zs + 2 < nz;
    T pv[PPT], kv[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      w[m][Sp2] = (ingw[m] && zw_in) ? nw[B][m] : T(0);
      pv[m] = npv[B][m];
      kv[m] = nkv[B][m];
    }
#pragma unroll
    for (int m = 0; m < PPT; ++m) lk[B][lwr[m]] = w[m][S0];
    if (has_ring) lk[B][rl] = (rin && zs_in) ? nring[B] : T(0);
    fetch(std::integral_constant<int, B>{}, zs + 2);
    __syncthreads();
    // stage 1: q(zs) on every slot; all LDS reads first
    T nb[PPT][NB];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      const T *c = &lk[B][lofs[m]];
      NbrX<T>::load(c, nb[m]);
      nb[m][NB - 4] = c[-KX];
      nb[m][NB - 3] = c[KX];
      nb[m][NB - 2] = c[-2 * KX];
      nb[m][NB - 1] = c[2 * KX];
    }
    LdsFence<T, PPT * NB>::all(&nb[0][0]);   // every read issued before the first wait
    T qv[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      const T c0 = w[m][S0];
      T s1, s2;
      NbrX<T>::terms(nb[m], c0, s1, s2);
      s1 = s1 + (nb[m][NB - 4] + nb[m][NB - 3]);
      s2 = s2 + (nb[m][NB - 2] + nb[m][NB - 1]);
      s1 += w[m][Sm1] + w[m][Sp1];
      s2 += w[m][Sm2] + w[m][Sp2];
      const T S = T(16) * s1 - s2 - T(90) * c0;
      const T qn = FIRSTSTEP ? c0 + T(0.5) * kv[m] * S : T(2) * c0 - pv[m] + kv[m] * S;
      qv[m] = (ing[m] && zs_in) ? qn : T(0);
    }
#pragma unroll
    for (int m = 0; m < PPT; ++m) lq[S0][qofs[m]] = qv[m];
#pragma unroll
    for (int m = 0; m < NIN; ++m) {
      r1[m][S0] = qv[m];
      kr[m][S0] = kv[m];
      asm volatile("" : : "v"(qv[m]));
    }
    {                                        // q(zs) where the plane belongs to this group's chunk
      const bool own = zs >= zbeg && zs < zend;
      T *q_pl = q_out + (size_t)min(max(zs, 0), nz - 1) * plane;
#pragma unroll
      for (int m = 0; m < NIN; ++m) st_ranged(q_pl, own ? plane_bytes : 0u, soff[m], qv[m]);
    }
    if constexpr (!STAGE2) return;
    // stage 2: o(z) on the interior slots, z = zs - 2 >= zbeg
    {
      T nq[NIN][NB];
#pragma unroll
      for (int m = 0; m < NIN; ++m) {
        const T *c = &lq[Sm2][qofs[m]];
        NbrX<T>::load(c, nq[m]);
        nq[m][NB - 4] = c[-KX];
        nq[m][NB - 3] = c[KX];
        nq[m][NB - 2] = c[-2 * KX];
        nq[m][NB - 1] = c[2 * KX];
      }
      T *o_pl = o_out + (size_t)z * plane;
      T ov[NIN];
#pragma unroll
      for (int m = 0; m < NIN; ++m) {
        const T c0 = r1[m][Sm2];
        T s1, s2;
        NbrX<T>::terms(nq[m], c0, s1, s2);
        s1 = s1 + (nq[m][NB - 4] + nq[m][NB - 3]);
        s2 = s2 + (nq[m][NB - 2] + nq[m][NB - 1]);
        s1 += r1[m][Sm3] + r1[m][Sm1];
        s2 += r1[m][Sm4] + r1[m][S0];
        const T S = T(16) * s1 - s2 - T(90) * c0;
        T v = T(2) * c0 - w[m][Sm2] + kr[m][Sm2] * S;
        if constexpr (DIV) v = v / kr[m][Sm2];
        ov[m] = v;
        asm volatile("" : : "v"(ov[m]));
      }
#pragma unroll
      for (int m = 0; m < NIN; ++m) st_ranged(o_pl, plane_bytes, soff[m], ov[m]);
    }
  };

  const int zlast = zend + 1;                // last stage-1 plane
  using No2 = std::false_type;
  using With2 = std::true_type;
  step(std::integral_constant<int, 0>{}, No2{}, zstart);       // o planes zbeg-4 .. zbeg-1
  step(std::integral_constant<int, 1>{}, No2{}, zstart + 1);
  step(std::integral_constant<int, 2>{}, No2{}, zstart + 2);
  step(std::integral_constant<int, 3>{}, No2{}, zstart + 3);
  for (int zb = zbeg + 2; zb <= zlast; zb += 10) {             // o planes zbeg .. zend-1
    step(std::integral_constant<int, 4>{}, With2{}, zb);
    if (zb + 1 > zlast) break;
    step(std::integral_constant<int, 5>{}, With2{}, zb + 1);
    if (zb + 2 > zlast) break;
    step(std::integral_constant<int, 6>{}, With2{}, zb + 2);
    if (zb + 3 > zlast) break;
    step(std::integral_constant<int, 7>{}, With2{}, zb + 3);
    if (zb + 4 > zlast) break;
    step(std::integral_constant<int, 8>{}, With2{}, zb + 4);
    if (zb + 5 > zlast) break;
    step(std::integral_constant<int, 9>{}, With2{}, zb + 5);
    if (zb + 6 > zlast) break;
    step(std::integral_constant<int, 10>{}, With2{}, zb + 6);
    if (zb + 7 > zlast) break;
    step(std::integral_constant<int, 11>{}, With2{}, zb + 7);
    if (zb + 8 > zlast) break;
    step(std::integral_constant<int, 12>{}, With2{}, zb + 8);
    if (zb + 9 > zlast) break;
    step(std::integral_constant<int, 13>{}, With2{}, zb + 9);
  }
}

template <typename T>
struct LdsFence<T, 14> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]));
  }
};
template <typename T>
struct LdsFence<T, 26> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
                 "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]), "+v"(v[18]), "+v"(v[19]), "+v"(v[20]),
                 "+v"(v[21]), "+v"(v[22]), "+v"(v[23]), "+v"(v[24]), "+v"(v[25]));
  }
};
template <typename T>
struct LdsFence<T, 30> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
                 "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]), "+v"(v[18]), "+v"(v[19]), "+v"(v[20]),
                 "+v"(v[21]), "+v"(v[22]), "+v"(v[23]), "+v"(v[24]), "+v"(v[25]), "+v"(v[26]), "+v"(v[27]),
                 "+v"(v[28]), "+v"(v[29]));
  }
};
template <typename T>
struct LdsFence<T, 32> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
                 "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]), "+v"(v[18]), "+v"(v[19]), "+v"(v[20]),
                 "+v"(v[21]), "+v"(v[22]), "+v"(v[23]), "+v"(v[24]), "+v"(v[25]), "+v"(v[26]), "+v"(v[27]),
                 "+v"(v[28]), "+v"(v[29]), "+v"(v[30]), "+v"(v[31]));
  }
};
template <typename T>
struct LdsFence<T, 36> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
                 "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]), "+v"(v[18]), "+v"(v[19]), "+v"(v[20]),
                 "+v"(v[21]), "+v"(v[22]), "+v"(v[23]), "+v"(v[24]), "+v"(v[25]), "+v"(v[26]), "+v"(v[27]),
                 "+v"(v[28]), "+v"(v[29]), "+v"(v[30]), "+v"(v[31]), "+v"(v[32]), "+v"(v[33]), "+v"(v[34]),
                 "+v"(v[35]));
  }
};

// Three leapfrog steps per pass (eq. wave1), FP64: from p(k-1), p(k) and k' the
// kernel computes q = p(k+1), r = p(k+2) and o = p(k+3) and writes r and o, the two
// levels the next pass starts from: five words per voxel for three steps (the
// two-step kernel moves five for two).  Same tile (64 x 16 elements, 512 threads, one
// group per compute unit), same arithmetic, in the same order, as wave_step2_split,
// so the results equal those of two- and one-step passes bit for bit.  (FP32, as
// pairs of points, runs the same stages in wave_step3_wide.)
//
// Regions of the tile, in elements (E = one step's x reach: 2 in FP64, 1 for pairs of
// points; two rows in y):
//   p(k) plane in LDS: tile + 3E in x, 6 rows in y        (KX x KY)
//   stage 1, q:        tile + 2E, 4 rows                  (AX x AY)
//   stage 2, r:        tile + E, 2 rows                   (CX x CY)
//   stage 3, o:        the tile
// Thread slots: 0 and 1 interior (all three stages), 2 the ring of stage 2 around
// the tile (stages 1 and 2), 3 the ring of stage 1 around that (stage 1 only), and
// one point of the outer ring of the p(k) plane, which only enters LDS.  Threads
// beyond a ring's point count repeat a point of the same ring: they load, compute
// and write the same values as its owner.  Points off the grid load zeros (loads
// through buffer resources with the plane's byte range), so their q and r are
// exactly zero, as the zero values outside the grid require, without a mask.
// Per plane zs (stage 1), in one barrier interval: stage 1 at zs, stage 2 at zs - 2,
// stage 3 at zs - 4.  The q and r planes live in 5-plane LDS rings; stage 2 reads
// q's x-y neighbours, centre and z-neighbours there, stage 3 r's.  The value a thread
// has just computed for its own column is taken from its register.  A ring slot is
// rewritten five planes after it was written, after the barrier that follows its
// last read.  Loads run one plane ahead.
// Measured on MI355X, us per leapfrog step (two-step kernel / this one): 256^3 70.0 /
// 69.2, 384^3 254.6 / 250.0 (FP64 plans keep two steps per pass unless
// FFPAT_PLAN_THREE_STEP asks otherwise).  The same kernel over pairs of FP32 points,
// with r's z-column in registers, ran 36.3 us per step at 256^3 (two-step 39.9);
// there q's z-column in registers too spilled (51.3), k' of stages 2 and 3 loaded
// again instead of kept took 43.2, loads two planes ahead 42.5.
// FIRSTSTEP: the pass starts the solve: stage 1 is the first step from p(0) with zero
// initial velocity (the single-step kernel's STEP_FIRST, the same expression; pm1 is
// not read), so the pass yields p(2) and p(3).
template <typename T, bool RESTRICT, bool FIRSTSTEP = false>
__global__ void __launch_bounds__(512, 1)
wave_step3_split(std::conditional_t<RESTRICT, const T *__restrict__, const T *> pm1,
                 std::conditional_t<RESTRICT, const T *__restrict__, const T *> pk,
                 std::conditional_t<RESTRICT, T *__restrict__, T *> r_out,
                 std::conditional_t<RESTRICT, T *__restrict__, T *> o_out,
                 std::conditional_t<RESTRICT, const T *__restrict__, const T *> kap, int nx, int ny, int nz,
                 int zchunk, int tiles_x, int tiles_y, int n_tiles, int xy_fastest)
{
  constexpr int NTH = 512, BX = 64, BY = 16;
  constexpr int NX = NbrX<T>::N;              // x-neighbour reads per point (pairs 2, FP64 4)
  constexpr int E = NX / 2;
  constexpr int XH = 3 * E;
  constexpr int KX = BX + 2 * XH, KY = BY + 12;
  constexpr int AX = BX + 4 * E, AY = BY + 8;
  constexpr int CX = BX + 2 * E, CY = BY + 4;
  constexpr int NIN = BX * BY / NTH;          // interior slots per thread (2)
  constexpr int N2 = CX * CY - BX * BY;       // ring of stage 2 (pairs 296, FP64 336)
  constexpr int N1 = AX * AY - CX * CY;       // ring of stage 1 (pairs 312, FP64 368)
  constexpr int NR = KX * KY - AX * AY;       // outer ring of the p(k) plane (pairs 328, FP64 400)
  constexpr int PPT = NIN + 2;
  static_assert(std::is_same_v<T, double>, "pairs of FP32 points run wave_step3_wide");
  constexpr int NB = NX + 4;                  // LDS reads per point: x-y neighbours
  constexpr int NB2 = NB + 4;                 // stage 2: and q's centre and three z-neighbours
  static_assert(NIN == 2 && N2 <= NTH && N1 <= NTH && NR <= NTH && 2 * N2 >= NTH && 2 * N1 >= NTH &&
                    2 * NR >= NTH,
                "slot layout");
  constexpr int KP = KY * KX, QP = AY * AX, RP = CY * CX;   // plane sizes in elements
  __shared__ T lk[2][KP];                     // p(k) plane, double-buffered by plane parity
  __shared__ T lq[5][QP];                     // q ring
  __shared__ T lr[5][RP];                     // r ring

  const int b = blockIdx.x;
  const int per_xcd = (n_tiles + 7) / 8;
  const int t = (b % 8) * per_xcd + b / 8;
  if (t >= n_tiles) return;                   // whole group exits together
  const int n_zc = (nz + zchunk - 1) / zchunk;
  int zc, txy;
  if (xy_fastest) {
    const int n_xy = tiles_x * tiles_y;
    txy = t % n_xy;
    zc = t / n_xy;
  } else {
    zc = t % n_zc;
    txy = t / n_zc;
  }
  const int x0 = (txy % tiles_x) * BX, y0 = (txy / tiles_x) * BY;
  const int zbeg = zc * zchunk;
  const int zend = min(nz, zbeg + zchunk);
  const size_t plane = (size_t)nx * ny;
  const int zstart = zbeg - 4;                // first stage-1 plane
  const int tid = threadIdx.x;

  // per slot: LDS index of the point in the p(k) plane, in the q ring and in the r
  // ring; byte offset of the point in a plane, out of range off the grid (its
  // loads read zeros, its stores write nothing).  The second interior slot lies
  // 8 rows below the first.
  int lofs[PPT], qrd[PPT], rrd[PPT - 1];
  unsigned boff[PPT];
  const unsigned plane_bytes = (unsigned)(plane * sizeof(T));
  auto plane_range = [&](int z) { return (z >= 0 && z < nz) ? plane_bytes : 0u; };
  auto plane_at = [&](const T *f, int z) { return f + (size_t)min(max(z, 0), nz - 1) * plane; };
  T w[PPT][5];        // p(k) z-window of every slot
  T kw[PPT - 1][5];   // k' of the slots of stage 2, planes zs-4..zs
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    int lx, ly;
    if (m < NIN) {
      ly = 6 + tid / BX + m * (NTH / BX);
      lx = XH + tid % BX;
    } else {
      // ring of width E (x) and 2 rows (y) just outside a region of rw x rh elements
      const int rwid = m == 2 ? CX : AX, rh = m == 2 ? CY : AY, n = m == 2 ? N2 : N1;
      const int u = tid < n ? tid : tid - n;  // n > NTH / 2: every thread gets a point
      int sx, sy;
      if (u < 4 * rwid) {                     // rows 0, 1, rh-2, rh-1, full width
        const int r = u / rwid;
        sy = r < 2 ? r : rh - 4 + r;
        sx = u - r * rwid;
      } else {                                // rows 2..rh-3, columns 0..E-1 and rwid-E..rwid-1
        const int j = u - 4 * rwid;
        sy = 2 + j / (2 * E);
        const int cc = j % (2 * E);
        sx = cc < E ? cc : rwid - 2 * E + cc;
      }
      const int inset = m == 2 ? 2 : 1;       // region origin in the p(k) plane: (inset E, 2 inset)
      lx = sx + inset * E;
      ly = sy + 2 * inset;
    }
    lofs[m] = ly * KX + lx;
    qrd[m] = (ly - 2) * AX + (lx - E);
    if (m < PPT - 1) rrd[m] = (ly - 4) * CX + (lx - 2 * E);
    const int gx = x0 - XH + lx, gy = y0 - 6 + ly;
    const bool ing = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    boff[m] = ing ? (unsigned)((gy * nx + gx) * sizeof(T)) : 0xFFFFFFF0u;
#pragma unroll
    for (int d = -2; d <= 1; ++d) {
      const int zq = zstart + d;
      w[m][(d + 5) % 5] = ld_ranged(plane_at(pk, zq), plane_range(zq), boff[m]);
    }
    w[m][2] = T(0);
  }
#pragma unroll
  for (int m = 0; m < PPT - 1; ++m)
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      kw[m][q] = T(0);
    }

  // LDS base of each slot in each array, at its lowest read (slots that only write
  // an array: at the point), kept in a register the compiler cannot see through:
  // every access is then that base plus an immediate offset (the arrays span 149 KB,
  // beyond an instruction's 64 KB offset)
  using LP = __attribute__((address_space(3))) T *;
  auto opaque = [](T *p) {
    LP q = (LP)p;
    asm volatile("" : "+v"(q));
    return q;
  };
  LP kb[PPT], qb[PPT], rb[PPT - 1];
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    kb[m] = opaque(&lk[0][lofs[m] - 2 * KX]);
    qb[m] = opaque(&lq[0][qrd[m] - (m < PPT - 1 ? 2 * AX : 0)]);
    if (m < PPT - 1) rb[m] = opaque(&lr[0][rrd[m] - (m < NIN ? 2 * CX : 0)]);
  }

  // outer-ring element of the p(k) plane (NR > NTH / 2: every thread has one)
  unsigned roff;
  LP ringb;
  {
    const int u = tid < NR ? tid : tid - NR;
    int lx, ly;
    if (u < 4 * KX) {                         // rows 0, 1, KY-2, KY-1
      const int r = u / KX;
      ly = r < 2 ? r : KY - 4 + r;
      lx = u - r * KX;
    } else {                                  // rows 2..KY-3, columns 0..E-1 and KX-E..KX-1
      const int j = u - 4 * KX;
      ly = 2 + j / (2 * E);
      const int cc = j % (2 * E);
      lx = cc < E ? cc : KX - 2 * E + cc;
    }
    const int gx = x0 - XH + lx, gy = y0 - 6 + ly;
    const bool rin = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    roff = rin ? (unsigned)((gy * nx + gx) * sizeof(T)) : 0xFFFFFFF0u;
    ringb = opaque(&lk[0][ly * KX + lx]);
  }

  // loads for stage-1 plane zf, issued one plane ahead: p(k) plane zf + 2 (entering
  // the window), p(k-1) and k' of plane zf, p(k) plane zf for the outer ring
  T nw[PPT], npv[PPT], nkv[PPT], nring;
  auto fetch = [&](int zf) {
    const unsigned bw = plane_range(zf + 2), bc = plane_range(zf);
    const T *pw = plane_at(pk, zf + 2), *pp = FIRSTSTEP ? pk : plane_at(pm1, zf);
    const T *pkap = plane_at(kap, zf), *pr = plane_at(pk, zf);
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      nw[m] = ld_ranged(pw, bw, boff[m]);
      if constexpr (!FIRSTSTEP) npv[m] = ld_ranged(pp, bc, boff[m]);
      nkv[m] = ld_ranged(pkap, bc, boff[m]);
    }
    nring = ld_ranged(pr, bc, roff);
  };
  fetch(zstart);

  // NS: the stages a plane needs (the first four planes of a group only feed stage 1's
  // q to later planes, the next four have no o of the chunk yet)
  auto step = [&](auto phase, auto nstages, int zs) {
    constexpr int Q = decltype(phase)::value, NS = decltype(nstages)::value;
    constexpr int P = Q % 5, B = Q % 2;
    // ring and window slot of plane zs + d
    constexpr int Sm6 = (P + 4) % 5, Sm5 = P, Sm4 = (P + 1) % 5, Sm3 = (P + 2) % 5, Sm2 = (P + 3) % 5;
    constexpr int Sm1 = (P + 4) % 5, S0 = P, Sp1 = (P + 1) % 5, Sp2 = (P + 2) % 5;
    const int z1 = zs - 2, z2 = zs - 4;
    T pv[PPT], kv[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      w[m][Sp2] = nw[m];
      if constexpr (FIRSTSTEP) pv[m] = T(0);
      else pv[m] = npv[m];
      kv[m] = nkv[m];
    }
#pragma unroll
    for (int m = 0; m < PPT - 1; ++m) kw[m][S0] = kv[m];
#pragma unroll
    for (int m = 0; m < PPT; ++m) kb[m][B * KP + 2 * KX] = w[m][S0];
    ringb[B * KP] = nring;
    fetch(zs + 1);
    __syncthreads();

    // stage 1: q(zs) on every slot
    T qv[PPT];
    {
      T nb[PPT][NB];
#pragma unroll
      for (int m = 0; m < PPT; ++m) {
        const LP c = kb[m] + (B * KP + 2 * KX);
        NbrX<T>::load(c, nb[m]);
        nb[m][NX + 0] = c[-KX];
        nb[m][NX + 1] = c[KX];
        nb[m][NX + 2] = c[-2 * KX];
        nb[m][NX + 3] = c[2 * KX];
      }
      LdsFence<T, PPT * NB>::all(&nb[0][0]);   // every read issued before the first wait
#pragma unroll
      for (int m = 0; m < PPT; ++m) {
        const T c0 = w[m][S0];
        T s1, s2;
        NbrX<T>::terms(nb[m], c0, s1, s2);
        s1 = s1 + (nb[m][NX + 0] + nb[m][NX + 1]);
        s2 = s2 + (nb[m][NX + 2] + nb[m][NX + 3]);
        s1 += w[m][Sm1] + w[m][Sp1];
        s2 += w[m][Sm2] + w[m][Sp2];
        const T S = T(16) * s1 - s2 - T(90) * c0;
        if constexpr (FIRSTSTEP) qv[m] = c0 + T(0.5) * kv[m] * S;
        else qv[m] = T(2) * c0 - pv[m] + kv[m] * S;
      }
#pragma unroll
      for (int m = 0; m < PPT; ++m) qb[m][S0 * QP + (m < PPT - 1 ? 2 * AX : 0)] = qv[m];
    }

    if constexpr (NS == 1) return;

    // stage 2: r(z1) on slots 0..2, from z1 = zbeg - 2 on
    T rv[PPT - 1];
    {
      T nq[PPT - 1][NB2];
#pragma unroll
      for (int m = 0; m < PPT - 1; ++m) {
        const LP c = qb[m] + (Sm2 * QP + 2 * AX);
        T *v = nq[m];
        NbrX<T>::load(c, v);
        v[NX + 0] = c[-AX];
        v[NX + 1] = c[AX];
        v[NX + 2] = c[-2 * AX];
        v[NX + 3] = c[2 * AX];
        v[NB + 0] = c[0];
        v[NB + 1] = qb[m][Sm3 * QP + 2 * AX];
        v[NB + 2] = qb[m][Sm1 * QP + 2 * AX];
        v[NB + 3] = qb[m][Sm4 * QP + 2 * AX];
      }
      LdsFence<T, (PPT - 1) * NB2>::all(&nq[0][0]);
#pragma unroll
      for (int m = 0; m < PPT - 1; ++m) {
        const T *v = nq[m];
        const T c0 = v[NB + 0];
        T s1, s2;
        NbrX<T>::terms(v, c0, s1, s2);
        s1 = s1 + (v[NX + 0] + v[NX + 1]);
        s2 = s2 + (v[NX + 2] + v[NX + 3]);
        s1 += v[NB + 1] + v[NB + 2];
        s2 += v[NB + 3] + qv[m];
        const T S = T(16) * s1 - s2 - T(90) * c0;
        rv[m] = T(2) * c0 - w[m][Sm2] + kw[m][Sm2] * S;
      }
#pragma unroll
      for (int m = 0; m < PPT - 1; ++m) rb[m][Sm2 * RP + (m < NIN ? 2 * CX : 0)] = rv[m];
#pragma unroll
      for (int m = 0; m < NIN; ++m) asm volatile("" : : "v"(rv[m]));
      const bool own = z1 >= zbeg && z1 < zend;
      T *r_pl = r_out + (size_t)min(max(z1, 0), nz - 1) * plane;
#pragma unroll
      for (int m = 0; m < NIN; ++m) st_ranged(r_pl, own ? plane_bytes : 0u, boff[m], rv[m]);
    }

    if constexpr (NS == 2) return;

    // stage 3: o(z2) on the interior slots, from z2 = zbeg on
    {
      constexpr int N3 = NB + 5;   // LDS reads per slot
      T nr[NIN][N3];
#pragma unroll
      for (int m = 0; m < NIN; ++m) {
        const LP c = rb[m] + (Sm4 * RP + 2 * CX);
        T *v = nr[m];
        NbrX<T>::load(c, v);
        v[NX + 0] = c[-CX];
        v[NX + 1] = c[CX];
        v[NX + 2] = c[-2 * CX];
        v[NX + 3] = c[2 * CX];
        v[NB] = qb[m][Sm4 * QP + 2 * AX];   // q(z2)
        v[NB + 1] = c[0];
        v[NB + 2] = rb[m][Sm5 * RP + 2 * CX];
        v[NB + 3] = rb[m][Sm3 * RP + 2 * CX];
        v[NB + 4] = rb[m][Sm6 * RP + 2 * CX];
      }
      LdsFence<T, NIN * N3>::all(&nr[0][0]);
      T ov[NIN];
#pragma unroll
      for (int m = 0; m < NIN; ++m) {
        const T *v = nr[m];
        const T c0 = v[NB + 1];
        const T zm1 = v[NB + 2], zp1 = v[NB + 3];
        const T zm2 = v[NB + 4];
        T s1, s2;
        NbrX<T>::terms(v, c0, s1, s2);
        s1 = s1 + (v[NX + 0] + v[NX + 1]);
        s2 = s2 + (v[NX + 2] + v[NX + 3]);
        s1 += zm1 + zp1;
        s2 += zm2 + rv[m];
        const T S = T(16) * s1 - s2 - T(90) * c0;
        ov[m] = T(2) * c0 - v[NB] + kw[m][Sm4] * S;
        asm volatile("" : : "v"(ov[m]));
      }
      T *o_pl = o_out + (size_t)z2 * plane;
#pragma unroll
      for (int m = 0; m < NIN; ++m) st_ranged(o_pl, plane_bytes, boff[m], ov[m]);
    }
  };

  const int zlast = zend + 3;                 // last stage-1 plane
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  using S3 = std::integral_constant<int, 3>;
  step(std::integral_constant<int, 0>{}, S1{}, zstart);       // r planes zbeg-6 .. zbeg-3, o zbeg-8 ..
  step(std::integral_constant<int, 1>{}, S1{}, zstart + 1);
  step(std::integral_constant<int, 2>{}, S1{}, zstart + 2);
  step(std::integral_constant<int, 3>{}, S1{}, zstart + 3);
  step(std::integral_constant<int, 4>{}, S2{}, zbeg);         // r planes zbeg-2 .. zbeg+1, o zbeg-4 ..
  step(std::integral_constant<int, 5>{}, S2{}, zbeg + 1);
  step(std::integral_constant<int, 6>{}, S2{}, zbeg + 2);
  step(std::integral_constant<int, 7>{}, S2{}, zbeg + 3);
  for (int zb = zbeg + 4; zb <= zlast; zb += 10) {            // o planes zbeg .. zend-1
    step(std::integral_constant<int, 8>{}, S3{}, zb);
    if (zb + 1 > zlast) break;
    step(std::integral_constant<int, 9>{}, S3{}, zb + 1);
    if (zb + 2 > zlast) break;
    step(std::integral_constant<int, 10>{}, S3{}, zb + 2);
    if (zb + 3 > zlast) break;
    step(std::integral_constant<int, 11>{}, S3{}, zb + 3);
    if (zb + 4 > zlast) break;
    step(std::integral_constant<int, 12>{}, S3{}, zb + 4);
    if (zb + 5 > zlast) break;
    step(std::integral_constant<int, 13>{}, S3{}, zb + 5);
    if (zb + 6 > zlast) break;
    step(std::integral_constant<int, 14>{}, S3{}, zb + 6);
    if (zb + 7 > zlast) break;
    step(std::integral_constant<int, 15>{}, S3{}, zb + 7);
    if (zb + 8 > zlast) break;
    step(std::integral_constant<int, 16>{}, S3{}, zb + 8);
    if (zb + 9 > zlast) break;
    step(std::integral_constant<int, 17>{}, S3{}, zb + 9);
  }
}

template <typename T>
struct LdsFence<T, 6> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]));
  }
};
template <typename T>
struct LdsFence<T, 11> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]));
  }
};
template <typename T>
struct LdsFence<T, 10> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]));
  }
};
template <typename T>
struct LdsFence<T, 12> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]));
  }
};
template <typename T>
struct LdsFence<T, 20> {
  static __device__ __forceinline__ void all(T *v)
  {
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),
                 "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]),
                 "+v"(v[14]), "+v"(v[15]), "+v"(v[16]), "+v"(v[17]), "+v"(v[18]), "+v"(v[19]));
  }
};

// Three leapfrog steps per pass (eq. wave1) over pairs of FP32 points, with 1024
// threads: the tile (64 x 16 elements), the stages, the LDS rings and the arithmetic
// of wave_step3_split, but one interior point per thread (wave w takes tile row w) and
// one ring point, whose kind is the wave's: the ring of stage 2 (stages 1 and 2), the
// ring of stage 1 (stage 1) or the outer ring of the p(k) plane (loaded into LDS
// only).  The layout is wide3_interior, wide3_ring and wide3_role of launch_rules.h.
// Each wave computes its own slots only (with 512 threads and two interior points
// each, every thread also carries one point of each ring, repeated on the threads
// beyond a ring's count), and four waves per SIMD hide more of the per-plane chain
// (LDS reads, arithmetic, LDS writes, three times, and one barrier) than two.  With
// 128 VGPRs, r's z-column is read from the ring (in registers the kernel spills).
// The sums run in the same order as in the one- and two-step passes, whose results
// it equals bit for bit.
// Measured on MI355X, us per leapfrog step, 512 threads (two interior points per
// thread, r's z-column in registers) / this kernel: 224^3 24.75 / 22.54, 256^3 35.86 /
// 33.94, 288^3 67.52 / 63.42, 352^3 106.61 / 98.83, 384^3 123.85 / 121.33, 448^3
// 212.06 / 201.31, 512^3 272.69 / 264.87; the outer-ring waves then dropped their
// p(k-1) and k' loads: 33.5 at 256^3, 119.0 at 384^3.  Variants (256^3 / 384^3): the
// ring's stage-2 reads behind a wait of their own 34.6 at 256^3; roles grouped by kind
// (waves 0-4, 5-9, 10-15) 33.9 / 124.2; the outer-ring waves issuing all three stages'
// reads at once 34.6 / 123.3; k' of the ring's stage 2 loaded again instead of kept
// 35.8 / 128.3; stage 2's reads issued with stage 1's (spills) 42.0 / 151.1.
// The interior's reads are waited for after the ring branch, not in each arm of it:
// waits in both arms gave the interior values two definitions, joined by 8-byte
// register moves (34 per plane; with one wait after the branch, 4), 7% faster per
// step at 128^3 and 1.5% at 256^3.
template <bool FIRSTSTEP, bool DIV = false>
__global__ void __launch_bounds__(1024, 1)
wave_step3_wide(const f32x2 *pm1, const f32x2 *pk, f32x2 *r_out, f32x2 *o_out, const f32x2 *kap, int nx, int ny,
                int nz, int zchunk, int tiles_x, int tiles_y, int n_tiles, int xy_fastest, int raise_outer)
{
  using T = f32x2;
  using L = Wide3;
  constexpr int NTH = L::NTH, BX = L::BX, BY = L::BY;
  constexpr int NX = NbrX<T>::N;              // 2: the elements at x - 1 and x + 1
  constexpr int E = L::E, XH = L::XH;
  constexpr int KX = L::KX, AX = L::AX, CX = L::CX;
  constexpr int NB = NX + 4;
  constexpr int NB2 = NB + 4;
  static_assert(NX == 2 * E && BX * BY == NTH && L::N2 <= 5 * 64 && L::N1 <= 5 * 64 && L::NR <= 6 * 64,
                "slot layout");
  constexpr int KP = L::KP, QP = L::QP, RP = L::RP;
  __shared__ T lk[L::LK];                     // p(k) planes (double-buffered), with headroom
  __shared__ T lq[L::LQ];                     // q ring, with headroom
  __shared__ T lr[L::LR];                     // r ring

  const int b = blockIdx.x;
  const int per_xcd = (n_tiles + 7) / 8;
  const int t = (b % 8) * per_xcd + b / 8;
  if (t >= n_tiles) return;
  const int n_zc = (nz + zchunk - 1) / zchunk;
  int zc, txy;
  if (xy_fastest) {
    const int n_xy = tiles_x * tiles_y;
    txy = t % n_xy;
    zc = t / n_xy;
  } else {
    zc = t % n_zc;
    txy = t / n_zc;
  }
  const int x0 = (txy % tiles_x) * BX, y0 = (txy / tiles_x) * BY;
  const int zbeg = zc * zchunk;
  const int zend = min(nz, zbeg + zchunk);
  const size_t plane = (size_t)nx * ny;
  const int zstart = zbeg - 4;
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  // the wave's ring role and its rank among the waves of that role, from constants
  constexpr unsigned long long ROLES = [] {
    unsigned long long r = 0;
    for (int w = 0; w < 16; ++w) r |= (unsigned long long)wide3_role(w) << (4 * w);
    return r;
  }();
  constexpr unsigned long long RANKS = [] {
    unsigned long long r = 0;
    for (int w = 0; w < 16; ++w) r |= (unsigned long long)wide3_role_index(w) << (4 * w);
    return r;
  }();
  const int role = (int)((ROLES >> (4 * wv)) & 15), rank = (int)((RANKS >> (4 * wv)) & 15);
  const bool ring1 = role >= 1, ring2 = role == 2;   // the ring point computes stage 1 / stage 2
  // The outer-ring waves (p(k) loads and LDS writes only, besides their row of the tile)
  // issue ahead of the others on their SIMD: the plane's halo reaches LDS sooner and the
  // barrier opens earlier.  Measured on MI355X, us per leapfrog step, equal priorities /
  // outer ring raised: 128^3 7.62 / 7.28, 256^3 32.2 / 30.5, 384^3 115.2 / 107.7; raising
  // the waves of the stage-2 ring instead (the most work) gave nothing (31.9 at 256^3),
  // raising every wave around its loads and the barrier 32.0, the rings of stages 1 and 2
  // over the outer ring 31.2.  (Raising the halo- or ring-loading waves of the FP64
  // two-step kernel, whose threads all carry interior points, changed nothing: 69.2-70.0
  // us per step at 256^3 either way.)
  if (raise_outer && role == 0) __builtin_amdgcn_s_setprio(1);

  const unsigned plane_bytes = (unsigned)(plane * sizeof(T));
  auto plane_range = [&](int z) { return (z >= 0 && z < nz) ? plane_bytes : 0u; };
  auto plane_at = [&](const T *f, int z) { return f + (size_t)min(max(z, 0), nz - 1) * plane; };
  auto grid_off = [&](int lx, int ly) {
    const int gx = x0 - XH + lx, gy = y0 - 6 + ly;
    const bool ing = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    return ing ? (unsigned)((gy * nx + gx) * sizeof(T)) : 0xFFFFFFF0u;
  };

  // interior point (row wv of the tile, element lane) and ring point of the thread
  const PlanePoint ip = wide3_interior(tid), rp = wide3_ring_point(role, rank, tid & 63);
  const int ilx = ip.lx, ily = ip.ly, rlx = rp.lx, rly = rp.ly;
  const unsigned boffI = grid_off(ilx, ily), boffR = grid_off(rlx, rly);

  T wI[5], wR[5], kwI[5], kwR[5];
#pragma unroll
  for (int d = -2; d <= 1; ++d) {
    const int zq = zstart + d;
    wI[(d + 5) % 5] = ld_ranged(plane_at(pk, zq), plane_range(zq), boffI);
    wR[(d + 5) % 5] = ld_ranged(plane_at(pk, zq), plane_range(zq), boffR);
  }
  wI[2] = T(0);
  wR[2] = T(0);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    kwI[q] = T(0);
    kwR[q] = T(0);
  }

  // LDS bases (wide3_bases) kept opaque, so that every access is base + immediate
  // offset, as in wave_step3_split
  using LP = __attribute__((address_space(3))) T *;
  auto opaque = [](T *p) {
    LP q = (LP)p;
    asm volatile("" : "+v"(q));
    return q;
  };
  const Wide3Bases lb = wide3_bases_of(ip, rp, role);
  const LP kbI = opaque(&lk[lb.kI]), qbI = opaque(&lq[lb.qI]), rbI = opaque(&lr[lb.rI]);
  const LP kbR = opaque(&lk[lb.kR]), qbR = opaque(&lq[lb.qR]), rwrR = opaque(&lr[lb.rR]);

  T nwI, npvI, nkvI, nwR, npvR = T(0), nkvR = T(0);
  auto fetch = [&](int zf) {
    const unsigned bw = plane_range(zf + 2), bc = plane_range(zf);
    const T *pw = plane_at(pk, zf + 2), *pp = FIRSTSTEP ? pk : plane_at(pm1, zf);
    const T *pkap = plane_at(kap, zf);
    nwI = ld_ranged(pw, bw, boffI);
    if constexpr (!FIRSTSTEP) npvI = ld_ranged(pp, bc, boffI);
    nkvI = ld_ranged(pkap, bc, boffI);
    nwR = ld_ranged(pw, bw, boffR);
    if (ring1) {                              // outer-ring waves need neither
      if constexpr (!FIRSTSTEP) npvR = ld_ranged(pp, bc, boffR);
      nkvR = ld_ranged(pkap, bc, boffR);
    }
  };
  fetch(zstart);

  auto stencil = [](const T *nb, T c0, T zm1, T zp1, T zm2, T zp2) {
    T s1, s2;
    NbrX<T>::terms(nb, c0, s1, s2);
    s1 = s1 + (nb[NX + 0] + nb[NX + 1]);
    s2 = s2 + (nb[NX + 2] + nb[NX + 3]);
    s1 += zm1 + zp1;
    s2 += zm2 + zp2;
    return T(16) * s1 - s2 - T(90) * c0;
  };
  auto xy_reads = [](LP c, int pitch, T *v) {
    NbrX<T>::load(c, v);
    v[NX + 0] = c[-pitch];
    v[NX + 1] = c[pitch];
    v[NX + 2] = c[-2 * pitch];
    v[NX + 3] = c[2 * pitch];
  };

  auto step = [&](auto phase, auto nstages, int zs) {
    constexpr int Q = decltype(phase)::value, NS = decltype(nstages)::value;
    constexpr int P = Q % 5, B = Q % 2;
    constexpr int Sm6 = (P + 4) % 5, Sm5 = P, Sm4 = (P + 1) % 5, Sm3 = (P + 2) % 5, Sm2 = (P + 3) % 5;
    constexpr int Sm1 = (P + 4) % 5, S0 = P, Sp1 = (P + 1) % 5, Sp2 = (P + 2) % 5;
    const int z1 = zs - 2, z2 = zs - 4;
    wI[Sp2] = nwI;
    wR[Sp2] = nwR;
    T pvI = T(0), pvR = T(0);
    if constexpr (!FIRSTSTEP) {
      pvI = npvI;
      pvR = npvR;
    }
    const T kvI = nkvI, kvR = nkvR;
    kwI[S0] = kvI;
    kwR[S0] = kvR;
    kbI[B * KP + 2 * KX] = wI[S0];
    kbR[B * KP + 2 * KX] = wR[S0];
    fetch(zs + 1);
    __syncthreads();

    // stage 1: q(zs) on the interior point and on a ring point of stage 1 or 2
    T qI, qR = T(0);
    {
      T nbI[NB];
      xy_reads(kbI + (B * KP + 2 * KX), KX, nbI);
      if (ring1) {
        T nbR[NB];
        xy_reads(kbR + (B * KP + 2 * KX), KX, nbR);
        LdsFence<T, NB>::all(nbR);
        const T c0 = wR[S0];
        const T S = stencil(nbR, c0, wR[Sm1], wR[Sp1], wR[Sm2], wR[Sp2]);
        qR = FIRSTSTEP ? c0 + T(0.5) * kvR * S : T(2) * c0 - pvR + kvR * S;
        qbR[S0 * QP + 2 * AX] = qR;
      }
      LdsFence<T, NB>::all(nbI);
      const T c0 = wI[S0];
      const T S = stencil(nbI, c0, wI[Sm1], wI[Sp1], wI[Sm2], wI[Sp2]);
      qI = FIRSTSTEP ? c0 + T(0.5) * kvI * S : T(2) * c0 - pvI + kvI * S;
      qbI[S0 * QP + 2 * AX] = qI;
    }
    if constexpr (NS == 1) return;

    // stage 2: r(z1) on the interior point and on a ring point of stage 2; q's centre
    // and z-neighbours from the ring, q(zs) of the thread's own column from stage 1
    T rI;
    {
      auto reads = [&](LP qb, T *v) {
        xy_reads(qb + (Sm2 * QP + 2 * AX), AX, v);
        v[NB + 0] = qb[Sm2 * QP + 2 * AX];
        v[NB + 1] = qb[Sm3 * QP + 2 * AX];
        v[NB + 2] = qb[Sm1 * QP + 2 * AX];
        v[NB + 3] = qb[Sm4 * QP + 2 * AX];
      };
      T nqI[NB2];
      reads(qbI, nqI);
      if (ring2) {
        T nqR[NB2];
        reads(qbR, nqR);
        LdsFence<T, NB2>::all(nqR);
        const T *v = nqR;
        const T S = stencil(v, v[NB], v[NB + 1], v[NB + 2], v[NB + 3], qR);
        const T rR = T(2) * v[NB] - wR[Sm2] + kwR[Sm2] * S;
        rwrR[Sm2 * RP] = rR;
      }
      LdsFence<T, NB2>::all(nqI);
      const T *v = nqI;
      const T S = stencil(v, v[NB], v[NB + 1], v[NB + 2], v[NB + 3], qI);
      rI = T(2) * v[NB] - wI[Sm2] + kwI[Sm2] * S;
      rbI[Sm2 * RP + 2 * CX] = rI;
      asm volatile("" : : "v"(rI));
      const bool own = z1 >= zbeg && z1 < zend;
      st_ranged(r_out + (size_t)min(max(z1, 0), nz - 1) * plane, own ? plane_bytes : 0u, boffI, rI);
    }
    if constexpr (NS == 2) return;

    // stage 3: o(z2) on the interior point; r's centre and z-neighbours from the ring
    // as well (with them in registers the kernel exceeds 128 VGPRs), r(zs - 2) of the
    // thread's own column from stage 2
    {
      T nr[NB + 5];
      xy_reads(rbI + (Sm4 * RP + 2 * CX), CX, nr);
      nr[NB] = qbI[Sm4 * QP + 2 * AX];   // q(z2)
      nr[NB + 1] = rbI[Sm4 * RP + 2 * CX];
      nr[NB + 2] = rbI[Sm5 * RP + 2 * CX];
      nr[NB + 3] = rbI[Sm3 * RP + 2 * CX];
      nr[NB + 4] = rbI[Sm6 * RP + 2 * CX];
      LdsFence<T, NB + 5>::all(nr);
      const T S = stencil(nr, nr[NB + 1], nr[NB + 2], nr[NB + 3], nr[NB + 4], rI);
      T o = T(2) * nr[NB + 1] - nr[NB] + kwI[Sm4] * S;
      if constexpr (DIV) o = o / kwI[Sm4];     // the adjoint solve's last step
      asm volatile("" : : "v"(o));
      st_ranged(o_out + (size_t)z2 * plane, plane_bytes, boffI, o);
    }
  };

  const int zlast = zend + 3;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  using S3 = std::integral_constant<int, 3>;
  step(std::integral_constant<int, 0>{}, S1{}, zstart);
  step(std::integral_constant<int, 1>{}, S1{}, zstart + 1);
  step(std::integral_constant<int, 2>{}, S1{}, zstart + 2);
  step(std::integral_constant<int, 3>{}, S1{}, zstart + 3);
  step(std::integral_constant<int, 4>{}, S2{}, zbeg);
  step(std::integral_constant<int, 5>{}, S2{}, zbeg + 1);
  step(std::integral_constant<int, 6>{}, S2{}, zbeg + 2);
  step(std::integral_constant<int, 7>{}, S2{}, zbeg + 3);
  for (int zb = zbeg + 4; zb <= zlast; zb += 10) {
    step(std::integral_constant<int, 8>{}, S3{}, zb);
    if (zb + 1 > zlast) break;
    step(std::integral_constant<int, 9>{}, S3{}, zb + 1);
    if (zb + 2 > zlast) break;
    step(std::integral_constant<int, 10>{}, S3{}, zb + 2);
    if (zb + 3 > zlast) break;
    step(std::integral_constant<int, 11>{}, S3{}, zb + 3);
    if (zb + 4 > zlast) break;
    step(std::integral_constant<int, 12>{}, S3{}, zb + 4);
    if (zb + 5 > zlast) break;
    step(std::integral_constant<int, 13>{}, S3{}, zb + 5);
    if (zb + 6 > zlast) break;
    step(std::integral_constant<int, 14>{}, S3{}, zb + 6);
    if (zb + 7 > zlast) break;
    step(std::integral_constant<int, 15>{}, S3{}, zb + 7);
    if (zb + 8 > zlast) break;
    step(std::integral_constant<int, 16>{}, S3{}, zb + 8);
    if (zb + 9 > zlast) break;
    step(std::integral_constant<int, 17>{}, S3{}, zb + 9);
  }
}

// Tunables of the blocked kernel (set once per process from the environment
// for sweeps; the defaults are the measured best on MI355X).
struct BlockedConfig {
  int ry = 2;        // rows per thread: tile height 4 * ry
  int zchunk = 0;    // planes per work-group; 0 = choose from the grid size
  int order = 1;     // 1: x-y tiles fastest within an XCD's range; 0: z-chunks fastest
  int groups = 2048; // target work-group count when zchunk = 0
  int nt = 0;        // non-temporal loads of p(k-1), k' and stores of p(k+1)
  int ry2 = 0;       // two-step kernel: tile height / 4 (0: default 4)
  int zchunk2 = 0;   // two-step kernel: planes per work-group (0: from the grid size)
  int threads2 = 512; // two-step kernel: work-group size (256, 512 or 1024)
  int bx2 = 0;       // two-step kernel: tile width (0: chosen per grid; 64, or 128 in FP32 3D)
  int x2 = -1;       // two-step kernel, FP32 3D, even nx: pairs of x-adjacent points per lane (-1: by the rule)
  int split = 1;     // two-step kernel, 8-byte elements, 64 x 16 tile, 512 threads: wave_step2_split (0: blocked)
  int triple = -1;   // three steps per pass (wave_step3_split): -1 by the rule, 0 never, 1 wherever it applies
  int zchunk3 = 0;   // three-step kernel: planes per work-group (0: from the grid size)
  int prio3 = 1;     // three-step kernel: outer-ring waves at a raised priority (0: all equal)
};

static BlockedConfig blocked_config(const Dims &d, size_t esz)
{
  // default tile height (measured on MI355X): 8 rows up to 256-row grids, 16 rows
  // beyond (fewer halo re-reads once the fields no longer fit in the 256 MB MALL);
  // FP64 16 rows from 128 rows on (8 below: more work-groups for small grids)
  static BlockedConfig env = [] {
    BlockedConfig c;
    c.ry = 0;
    if (const char *e = getenv("FFPAT_STENCIL_RY")) c.ry = atoi(e);
    if (const char *e = getenv("FFPAT_STENCIL_ZCHUNK")) c.zchunk = atoi(e);
    if (const char *e = getenv("FFPAT_STENCIL_ORDER")) c.order = atoi(e) ? 1 : 0;
    if (const char *e = getenv("FFPAT_STENCIL_GROUPS")) c.groups = atoi(e) > 0 ? atoi(e) : 2048;
    if (const char *e = getenv("FFPAT_STENCIL_NT")) c.nt = atoi(e) ? 1 : 0;
    if (const char *e = getenv("FFPAT_STENCIL2_RY")) c.ry2 = atoi(e);
    if (const char *e = getenv("FFPAT_STENCIL2_ZCHUNK")) c.zchunk2 = atoi(e);
    if (const char *e = getenv("FFPAT_STENCIL2_BX")) c.bx2 = atoi(e) == 128 ? 128 : (atoi(e) == 64 ? 64 : 0);
    if (const char *e = getenv("FFPAT_STENCIL2_X2")) c.x2 = atoi(e) ? 1 : 0;
    if (const char *e = getenv("FFPAT_STENCIL2_SPLIT")) c.split = atoi(e) ? 1 : 0;
    if (const char *e = getenv("FFPAT_STENCIL3")) c.triple = atoi(e) ? 1 : 0;
    if (const char *e = getenv("FFPAT_STENCIL3_ZCHUNK")) c.zchunk3 = atoi(e);
    if (const char *e = getenv("FFPAT_STENCIL3_PRIO")) c.prio3 = atoi(e) ? 1 : 0;
    if (const char *e = getenv("FFPAT_STENCIL2_THREADS")) {
      const int v = atoi(e);
      c.threads2 = v == 1024 ? 1024 : (v == 256 ? 256 : 512);
    }
    if (c.ry != 0 && c.ry != 1 && c.ry != 2 && c.ry != 4 && c.ry != 8) c.ry = 0;
    if (c.zchunk < 0) c.zchunk = 0;
    return c;
  }();
  BlockedConfig cfg = env;
  cfg.ry = step_ry(d.ny, (int)esz, cfg.ry);
  return cfg;
}

static int step_zchunk(const Dims &d, const BlockedConfig &cfg, int tiles_x, int tiles_y)
{
  return ffpat::step_zchunk(d.nz, (long)tiles_x * tiles_y, cfg.groups, cfg.zchunk);
}

void wave_step_shape(const Dims &d, size_t esz, int *tile_x, int *tile_y, int *zchunk)
{
  const BlockedConfig cfg = blocked_config(d, esz);
  const int by = 4 * cfg.ry;
  *tile_x = 64;
  *tile_y = by;
  *zchunk = step_zchunk(d, cfg, (d.nx + 63) / 64, (d.ny + by - 1) / by);
}

template <typename T, int NDIM, int RY>
static hipError_t blocked_dispatch(StepMode mode, const Dims &d, const T *p, const T *prev, T *out, const T *kap,
                                   const BlockedConfig &cfg, hipStream_t s)
{
  constexpr int BY = 4 * RY;
  const int tiles_x = (d.nx + 63) / 64, tiles_y = (d.ny + BY - 1) / BY;
  const int zchunk = step_zchunk(d, cfg, tiles_x, tiles_y);
  const int xyf = cfg.order;
  const int n_zc = (d.nz + zchunk - 1) / zchunk;
  const int n_tiles = tiles_x * tiles_y * n_zc;
  const int grid = ((n_tiles + 7) / 8) * 8;
  if (cfg.nt) {
    switch (mode) {
      case STEP_FIRST: wave_step_blocked<T, NDIM, STEP_FIRST, RY, true><<<grid, 256, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz, zchunk, tiles_x, tiles_y, n_tiles, xyf); break;
      case STEP_LEAP: wave_step_blocked<T, NDIM, STEP_LEAP, RY, true><<<grid, 256, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz, zchunk, tiles_x, tiles_y, n_tiles, xyf); break;
      case STEP_FIRST_DIV: wave_step_blocked<T, NDIM, STEP_FIRST_DIV, RY, true><<<grid, 256, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz, zchunk, tiles_x, tiles_y, n_tiles, xyf); break;
      case STEP_LEAP_DIV: wave_step_blocked<T, NDIM, STEP_LEAP_DIV, RY, true><<<grid, 256, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz, zchunk, tiles_x, tiles_y, n_tiles, xyf); break;
    }
  } else {
    switch (mode) {
      case STEP_FIRST: wave_step_blocked<T, NDIM, STEP_FIRST, RY, false><<<grid, 256, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz, zchunk, tiles_x, tiles_y, n_tiles, xyf); break;
      case STEP_LEAP: wave_step_blocked<T, NDIM, STEP_LEAP, RY, false><<<grid, 256, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz, zchunk, tiles_x, tiles_y, n_tiles, xyf); break;
      case STEP_FIRST_DIV: wave_step_blocked<T, NDIM, STEP_FIRST_DIV, RY, false><<<grid, 256, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz, zchunk, tiles_x, tiles_y, n_tiles, xyf); break;
      case STEP_LEAP_DIV: wave_step_blocked<T, NDIM, STEP_LEAP_DIV, RY, false><<<grid, 256, 0, s>>>(p, prev, out, kap, d.nx, d.ny, d.nz, zchunk, tiles_x, tiles_y, n_tiles, xyf); break;
    }
  }
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t blocked_select(StepMode mode, const Dims &d, const T *p, const T *prev, T *out, const T *kap,
                                 hipStream_t s)
{
  const BlockedConfig cfg = blocked_config(d, sizeof(T));
  switch (cfg.ry) {
    case 1: return blocked_dispatch<T, NDIM, 1>(mode, d, p, prev, out, kap, cfg, s);
    case 4: return blocked_dispatch<T, NDIM, 4>(mode, d, p, prev, out, kap, cfg, s);
    case 8: return blocked_dispatch<T, NDIM, 8>(mode, d, p, prev, out, kap, cfg, s);
    default: return blocked_dispatch<T, NDIM, 2>(mode, d, p, prev, out, kap, cfg, s);
  }
}

// Compute units of the current device (0 if the runtime cannot say), cached per
// device: launches ask for it several times.
static int device_cus()
{
  constexpr int kMaxDevices = 64;
  static std::atomic<int> cache[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (dev >= 0 && dev < kMaxDevices) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 0;
  if (dev >= 0 && dev < kMaxDevices) cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

// Launch shape of wave_step2_split (the 64 x 16 tile of 8-byte elements, 512 threads).
template <typename T>
static PairShape pair_shape_split(const Dims &d, const BlockedConfig &cfg)
{
  static const int occ = [] {
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wave_step2_split<T, std::is_same_v<T, double>>,
                                                        512, 0) == hipSuccess ? n : 0;
  }();
  const int cus = device_cus();
  return pair_shape_for(d.nx, d.ny, d.nz, 64, 16, occ > 0 ? occ : 1, cus > 0 ? cus : 256, true, cfg.zchunk2);
}

template <typename T, int NDIM, int RY, int NTH, int BX>
static PairShape pair_shape(const Dims &d, const BlockedConfig &cfg)
{
  static const int occ = [] {
    int n = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wave_step2_blocked<T, NDIM, RY, NTH, BX>, NTH, 0) ==
                   hipSuccess ? n : 0;
  }();
  const bool f64 = sizeof(T) == 8;
  // if the runtime cannot say: FP32 with up to 512 threads two groups per unit, else one
  const int per_cu = occ > 0 ? occ : ((!f64 && NTH <= 512) ? 2 : 1);
  const int cus = device_cus();
  return pair_shape_for(d.nx, d.ny, d.nz, BX, 4 * RY, per_cu, cus > 0 ? cus : 256, f64, cfg.zchunk2);
}

// The instantiations of the two-step kernel: <NDIM, RY (tile height / 4), threads, tile width>.
enum PairVariant {
  PAIR_2D_RY4, PAIR_2D_RY2,                                  // 256 threads, 64 wide
  PAIR_WIDE,                                                 // FP32 3D: 128 x 16, 1024 threads
  PAIR_RY8_T1024, PAIR_RY4_T1024, PAIR_RY8_T512, PAIR_RY4_T512, PAIR_RY2_T512, PAIR_RY4_T256, PAIR_RY2_T256,
};

// FP32 3D with the default work-group (512 threads, tile 64 x 16): whether the
// 128 x 16 tile (1024 threads) is used; FFPAT_STENCIL2_BX=64 or 128 forces the width.
template <typename T>
static bool pair_wide_preferred(const Dims &d, const BlockedConfig &cfg)
{
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    if (d.ndim != 3 || cfg.bx2 == 64) return false;
    if (cfg.bx2 == 128) return true;
    if (cfg.threads2 != 512 || (cfg.ry2 > 0 && cfg.ry2 != 4)) return false;
    return pair_wide_better(pair_shape<T, 3, 4, 512, 64>(d, cfg), pair_shape<T, 3, 4, 1024, 128>(d, cfg));
  }
}

template <typename T>
static PairVariant pair_variant(const Dims &d, const BlockedConfig &cfg)
{
  const int ry = cfg.ry2 > 0 ? cfg.ry2 : 4;
  if (d.ndim == 2) return ry == 4 ? PAIR_2D_RY4 : PAIR_2D_RY2;
  if (pair_wide_preferred<T>(d, cfg)) return PAIR_WIDE;
  if (cfg.threads2 == 1024) return ry == 8 ? PAIR_RY8_T1024 : PAIR_RY4_T1024;
  if (cfg.threads2 == 512) return ry == 8 ? PAIR_RY8_T512 : (ry == 4 ? PAIR_RY4_T512 : PAIR_RY2_T512);
  return ry == 4 ? PAIR_RY4_T256 : PAIR_RY2_T256;
}

// Calls f with the kernel instantiation of variant v (as a null pointer of its type
// tag) so that the shape and the launch are taken from the same list.
template <int NDIM, int RY, int NTH, int BX>
struct PairTag {
  static constexpr int ndim = NDIM, ry = RY, nth = NTH, bx = BX;
};

template <typename T, typename F>
static auto visit_pair(PairVariant v, F &&f)
{
  switch (v) {
    case PAIR_2D_RY4: return f(PairTag<2, 4, 256, 64>{});
    case PAIR_2D_RY2: return f(PairTag<2, 2, 256, 64>{});
    case PAIR_WIDE:
      if constexpr (sizeof(T) == 4) return f(PairTag<3, 4, 1024, 128>{});
      else return f(PairTag<3, 4, 512, 64>{});   // never chosen in FP64
    case PAIR_RY8_T1024: return f(PairTag<3, 8, 1024, 64>{});
    case PAIR_RY4_T1024: return f(PairTag<3, 4, 1024, 64>{});
    case PAIR_RY8_T512: return f(PairTag<3, 8, 512, 64>{});
    case PAIR_RY4_T512: return f(PairTag<3, 4, 512, 64>{});
    case PAIR_RY2_T512: return f(PairTag<3, 2, 512, 64>{});
    case PAIR_RY4_T256: return f(PairTag<3, 4, 256, 64>{});
    default: return f(PairTag<3, 2, 256, 64>{});
  }
}

// FP32 3D with even nx, where the 128 x 16 tile is chosen: the two-step kernel over
// pairs of x-adjacent points, each pair one 8-byte element (the FP64 kernel's shape:
// 64 x 16 elements, 512 threads, the p(k) plane double-buffered for one barrier per
// plane).  The grid it sees has nx / 2 columns.  FFPAT_STENCIL2_X2 = 0 or 1 forces
// the choice (1: every even nx).
using PairX2 = PairTag<3, 4, 512, 64>;

template <typename T>
static bool pair_x2(const Dims &d, const BlockedConfig &cfg)
{
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    if (d.ndim != 3 || d.nx % 2 != 0 || cfg.x2 == 0) return false;
    return cfg.x2 == 1 || pair_x_pairs(pair_wide_preferred<T>(d, cfg), d.nx);
  }
}

static Dims x2_dims(const Dims &d)
{
  Dims e = d;
  e.nx = d.nx / 2;
  return e;
}

template <typename T>
hipError_t launch_wave_pair(const Dims &d, const T *pm1, const T *pk, T *q_out, T *o_out, const T *kap,
                            hipStream_t s)
{
  const BlockedConfig cfg = blocked_config(d, sizeof(T));
  if constexpr (sizeof(T) == 4) {
    // 8-byte elements need 8-byte aligned fields (a caller's buffer may start at any
    // float); otherwise one point per lane, with the same tile and chunk
    const bool aligned = ((reinterpret_cast<uintptr_t>(pm1) | reinterpret_cast<uintptr_t>(pk) |
                           reinterpret_cast<uintptr_t>(q_out) | reinterpret_cast<uintptr_t>(o_out) |
                           reinterpret_cast<uintptr_t>(kap)) & 7) == 0;
    if (aligned && pair_x2<T>(d, cfg)) {
      const Dims e = x2_dims(d);
      if (cfg.split) {
        const PairShape p = pair_shape_split<f32x2>(e, cfg);
        const int grid = ((p.n_tiles + 7) / 8) * 8;
        wave_step2_split<f32x2, false><<<grid, 512, 0, s>>>(
            reinterpret_cast<const f32x2 *>(pm1), reinterpret_cast<const f32x2 *>(pk),
            reinterpret_cast<f32x2 *>(q_out), reinterpret_cast<f32x2 *>(o_out), reinterpret_cast<const f32x2 *>(kap),
            e.nx, e.ny, e.nz, p.zchunk, p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
        return hipGetLastError();
      }
      const PairShape p = pair_shape<f32x2, PairX2::ndim, PairX2::ry, PairX2::nth, PairX2::bx>(e, cfg);
      const int grid = ((p.n_tiles + 7) / 8) * 8;
      wave_step2_blocked<f32x2, PairX2::ndim, PairX2::ry, PairX2::nth, PairX2::bx><<<grid, PairX2::nth, 0, s>>>(
          reinterpret_cast<const f32x2 *>(pm1), reinterpret_cast<const f32x2 *>(pk),
          reinterpret_cast<f32x2 *>(q_out), reinterpret_cast<f32x2 *>(o_out), reinterpret_cast<const f32x2 *>(kap),
          e.nx, e.ny, e.nz, p.zchunk, p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
      return hipGetLastError();
    }
  }
  if constexpr (sizeof(T) == 8) {
    if (cfg.split && pair_variant<T>(d, cfg) == PAIR_RY4_T512) {
      const PairShape p = pair_shape_split<T>(d, cfg);
      const int grid = ((p.n_tiles + 7) / 8) * 8;
      wave_step2_split<T, true><<<grid, 512, 0, s>>>(pm1, pk, q_out, o_out, kap, d.nx, d.ny, d.nz, p.zchunk,
                                                     p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
      return hipGetLastError();
    }
  }
  return visit_pair<T>(pair_variant<T>(d, cfg), [&](auto tag) {
    using Tag = decltype(tag);
    const PairShape p = pair_shape<T, Tag::ndim, Tag::ry, Tag::nth, Tag::bx>(d, cfg);
    const int grid = ((p.n_tiles + 7) / 8) * 8;
    wave_step2_blocked<T, Tag::ndim, Tag::ry, Tag::nth, Tag::bx><<<grid, Tag::nth, 0, s>>>(
        pm1, pk, q_out, o_out, kap, d.nx, d.ny, d.nz, p.zchunk, p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
    return hipGetLastError();
  });
}


// Launch shape of wave_step3_split: the two-step kernel's rule on the same tile.
template <typename T>
static PairShape triple_shape(const Dims &d, const BlockedConfig &cfg)
{
  static const int occ = [] {
    int n = 0;
    hipError_t e;
    if constexpr (std::is_same_v<T, f32x2>)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wave_step3_wide<false>, 1024, 0);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wave_step3_split<T, true>, 512, 0);
    return e == hipSuccess ? n : 0;
  }();
  const int cus = device_cus();
  return pair_shape_for(d.nx, d.ny, d.nz, 64, 16, occ > 0 ? occ : 1, cus > 0 ? cus : 256, true, cfg.zchunk3,
                        kTripleZmin);
}

// Where three steps per pass run: wherever the two-step pass would take
// wave_step2_split (FP32 as pairs of points, FP64 with the 64 x 16 tile), and in FP32
// also on the grids of wide3_grid_ok where the two-step rule keeps the 64-point tile
// (unless pairs or the 128-point tile are switched off).
template <typename T>
static bool triple_applies(const Dims &d, const BlockedConfig &cfg, bool aligned)
{
  if (!cfg.split || cfg.triple == 0 || d.ndim != 3) return false;
  if constexpr (sizeof(T) == 4)
    return aligned && (pair_x2<T>(d, cfg) || (cfg.x2 != 0 && cfg.bx2 != 64 && wide3_grid_ok(d.nx, d.ny, d.nz)));
  else return pair_variant<T>(d, cfg) == PAIR_RY4_T512;
}

template <typename T>
hipError_t launch_wave_triple(const Dims &d, const T *pm1, const T *pk, T *r_out, T *o_out, const T *kap,
                              hipStream_t s, bool first, bool *taken)
{
  const BlockedConfig cfg = blocked_config(d, sizeof(T));
  const bool aligned = (((first ? 0 : reinterpret_cast<uintptr_t>(pm1)) | reinterpret_cast<uintptr_t>(pk) |
                         reinterpret_cast<uintptr_t>(r_out) | reinterpret_cast<uintptr_t>(o_out) |
                         reinterpret_cast<uintptr_t>(kap)) & 7) == 0;
  *taken = triple_applies<T>(d, cfg, aligned);
  if (!*taken) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    const Dims e = x2_dims(d);
    const PairShape p = triple_shape<f32x2>(e, cfg);
    const int grid = ((p.n_tiles + 7) / 8) * 8;
    const f32x2 *a = reinterpret_cast<const f32x2 *>(first ? pk : pm1), *b = reinterpret_cast<const f32x2 *>(pk);
    f32x2 *r2 = reinterpret_cast<f32x2 *>(r_out), *o2 = reinterpret_cast<f32x2 *>(o_out);
    const f32x2 *k2 = reinterpret_cast<const f32x2 *>(kap);
    if (first)
      wave_step3_wide<true><<<grid, 1024, 0, s>>>(a, b, r2, o2, k2, e.nx, e.ny, e.nz, p.zchunk, p.tiles_x, p.tiles_y,
                                                  p.n_tiles, cfg.order, cfg.prio3);
    else
      wave_step3_wide<false><<<grid, 1024, 0, s>>>(a, b, r2, o2, k2, e.nx, e.ny, e.nz, p.zchunk, p.tiles_x, p.tiles_y,
                                                   p.n_tiles, cfg.order, cfg.prio3);
  } else {
    const PairShape p = triple_shape<T>(d, cfg);
    const int grid = ((p.n_tiles + 7) / 8) * 8;
    if (first)
      wave_step3_split<T, true, true><<<grid, 512, 0, s>>>(pk, pk, r_out, o_out, kap, d.nx, d.ny, d.nz, p.zchunk,
                                                           p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
    else
      wave_step3_split<T, true, false><<<grid, 512, 0, s>>>(pm1, pk, r_out, o_out, kap, d.nx, d.ny, d.nz, p.zchunk,
                                                            p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wave_triple_div(const Dims &d, const T *pm1, const T *pk, T *r_out, T *o_out, const T *kap,
                                  hipStream_t s, bool *taken)
{
  *taken = false;
  if constexpr (sizeof(T) == 4) {
    const BlockedConfig cfg = blocked_config(d, sizeof(T));
    const bool aligned = ((reinterpret_cast<uintptr_t>(pm1) | reinterpret_cast<uintptr_t>(pk) |
                           reinterpret_cast<uintptr_t>(r_out) | reinterpret_cast<uintptr_t>(o_out) |
                           reinterpret_cast<uintptr_t>(kap)) & 7) == 0;
    if (!triple_applies<T>(d, cfg, aligned)) return hipSuccess;
    const Dims e = x2_dims(d);
    const PairShape p = triple_shape<f32x2>(e, cfg);
    const int grid = ((p.n_tiles + 7) / 8) * 8;
    wave_step3_wide<false, true><<<grid, 1024, 0, s>>>(
        reinterpret_cast<const f32x2 *>(pm1), reinterpret_cast<const f32x2 *>(pk), reinterpret_cast<f32x2 *>(r_out),
        reinterpret_cast<f32x2 *>(o_out), reinterpret_cast<const f32x2 *>(kap), e.nx, e.ny, e.nz, p.zchunk, p.tiles_x,
        p.tiles_y, p.n_tiles, cfg.order, cfg.prio3);
    *taken = true;
    return hipGetLastError();
  } else {
    (void)d, (void)pm1, (void)pk, (void)r_out, (void)o_out, (void)kap, (void)s;
    return hipSuccess;
  }
}

template <typename T>
hipError_t launch_wave_pair_first(const Dims &d, const T *pk, T *q_out, T *o_out, const T *kap, hipStream_t s,
                                  bool *taken)
{
  const BlockedConfig cfg = blocked_config(d, sizeof(T));
  *taken = false;
  if (!cfg.split || d.ndim != 3) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    const bool aligned = ((reinterpret_cast<uintptr_t>(pk) | reinterpret_cast<uintptr_t>(q_out) |
                           reinterpret_cast<uintptr_t>(o_out) | reinterpret_cast<uintptr_t>(kap)) & 7) == 0;
    if (!aligned || !pair_x2<T>(d, cfg)) return hipSuccess;
    const Dims e = x2_dims(d);
    const PairShape p = pair_shape_split<f32x2>(e, cfg);
    const int grid = ((p.n_tiles + 7) / 8) * 8;
    const f32x2 *b = reinterpret_cast<const f32x2 *>(pk);
    wave_step2_split<f32x2, false, false, true><<<grid, 512, 0, s>>>(
        b, b, reinterpret_cast<f32x2 *>(q_out), reinterpret_cast<f32x2 *>(o_out),
        reinterpret_cast<const f32x2 *>(kap), e.nx, e.ny, e.nz, p.zchunk, p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
  } else {
    if (pair_variant<T>(d, cfg) != PAIR_RY4_T512) return hipSuccess;
    const PairShape p = pair_shape_split<T>(d, cfg);
    const int grid = ((p.n_tiles + 7) / 8) * 8;
    wave_step2_split<T, true, false, true><<<grid, 512, 0, s>>>(pk, pk, q_out, o_out, kap, d.nx, d.ny, d.nz,
                                                                p.zchunk, p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
  }
  *taken = true;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wave_pair_div(const Dims &d, const T *pm1, const T *pk, T *q_out, T *o_out, const T *kap,
                                hipStream_t s, bool *taken)
{
  const BlockedConfig cfg = blocked_config(d, sizeof(T));
  *taken = false;
  if (!cfg.split || d.ndim != 3) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    const bool aligned = ((reinterpret_cast<uintptr_t>(pm1) | reinterpret_cast<uintptr_t>(pk) |
                           reinterpret_cast<uintptr_t>(q_out) | reinterpret_cast<uintptr_t>(o_out) |
                           reinterpret_cast<uintptr_t>(kap)) & 7) == 0;
    if (!aligned || !pair_x2<T>(d, cfg)) return hipSuccess;
    const Dims e = x2_dims(d);
    const PairShape p = pair_shape_split<f32x2>(e, cfg);
    const int grid = ((p.n_tiles + 7) / 8) * 8;
    wave_step2_split<f32x2, false, true><<<grid, 512, 0, s>>>(
        reinterpret_cast<const f32x2 *>(pm1), reinterpret_cast<const f32x2 *>(pk), reinterpret_cast<f32x2 *>(q_out),
        reinterpret_cast<f32x2 *>(o_out), reinterpret_cast<const f32x2 *>(kap), e.nx, e.ny, e.nz, p.zchunk, p.tiles_x,
        p.tiles_y, p.n_tiles, cfg.order);
  } else {
    if (pair_variant<T>(d, cfg) != PAIR_RY4_T512) return hipSuccess;
    const PairShape p = pair_shape_split<T>(d, cfg);
    const int grid = ((p.n_tiles + 7) / 8) * 8;
    wave_step2_split<T, true, true><<<grid, 512, 0, s>>>(pm1, pk, q_out, o_out, kap, d.nx, d.ny, d.nz, p.zchunk,
                                                         p.tiles_x, p.tiles_y, p.n_tiles, cfg.order);
  }
  *taken = true;
  return hipGetLastError();
}

template <typename T>
bool wave_triple_shape(const Dims &d, int *tile_x, int *tile_y, int *zchunk)
{
  const BlockedConfig cfg = blocked_config(d, sizeof(T));
  if (!triple_applies<T>(d, cfg, true)) return false;
  if constexpr (sizeof(T) == 4) {
    const PairShape p = triple_shape<f32x2>(x2_dims(d), cfg);
    *tile_x = 2 * p.bx;
    *tile_y = p.by;
    *zchunk = p.zchunk;
  } else {
    const PairShape p = triple_shape<T>(d, cfg);
    *tile_x = p.bx;
    *tile_y = p.by;
    *zchunk = p.zchunk;
  }
  return true;
}

template <typename T>
void wave_pair_shape(const Dims &d, int *tile_x, int *tile_y, int *zchunk)
{
  const BlockedConfig cfg = blocked_config(d, sizeof(T));
  if constexpr (sizeof(T) == 4) {
    if (pair_x2<T>(d, cfg)) {
      const PairShape p = cfg.split ? pair_shape_split<f32x2>(x2_dims(d), cfg)
                                    : pair_shape<f32x2, PairX2::ndim, PairX2::ry, PairX2::nth, PairX2::bx>(x2_dims(d), cfg);
      *tile_x = 2 * p.bx;   // in points
      *tile_y = p.by;
      *zchunk = p.zchunk;
      return;
    }
  }
  PairShape p;
  if (sizeof(T) == 8 && cfg.split && pair_variant<T>(d, cfg) == PAIR_RY4_T512) {
    p = pair_shape_split<double>(d, cfg);
  } else {
    p = visit_pair<T>(pair_variant<T>(d, cfg), [&](auto tag) {
      using Tag = decltype(tag);
      return pair_shape<T, Tag::ndim, Tag::ry, Tag::nth, Tag::bx>(d, cfg);
    });
  }
  *tile_x = p.bx;
  *tile_y = p.by;
  *zchunk = p.zchunk;
}

bool wave_pairs_preferred(const Dims &d, size_t esz)
{
  static const int env = [] {
    const char *e = getenv("FFPAT_STENCIL_TB");
    return e ? (atoi(e) != 0 ? 1 : 0) : -1;
  }();
  if (env >= 0) return env == 1;
  // measured on MI355X, us per step one / two steps per pass: FP32 112^3 9.3 / 9.5,
  // 128^3 10.3 / 9.8, 256^3 49.6 / 42.4, 384^3 198 / 152; FP64 96^3 9.6 / 12.0,
  // 112^3 11.0 / 12.2, 128^3 13.9 / 13.3, 256^3 111 / 74.4, 384^3 391 / 271.
  // Smaller grids keep one step per pass.
  (void)esz;
  return d.nvox() >= (size_t)128 * 128 * 128;
}

template <typename T>
bool wave_triples_available(const Dims &d)
{
  return triple_applies<T>(d, blocked_config(d, sizeof(T)), true);
}

bool wave_triples_preferred(const Dims &d, size_t esz)
{
  static const bool single = [] {      // FFPAT_STENCIL_TB=0: one step per pass throughout
    const char *e = getenv("FFPAT_STENCIL_TB");
    return e && atoi(e) == 0;
  }();
  if (single) return false;
  const BlockedConfig cfg = blocked_config(d, esz);
  if (cfg.triple >= 0) return cfg.triple == 1;
  // FP32 (pairs of points), measured on MI355X, us per leapfrog step two / three steps
  // per pass: 224^3 25.2 / 25.0, 256^3 39.9 / 36.3, 288^3 68.6 / 67.7, 352^3 112.4 /
  // 106.5, 448^3 219.7 / 212.4, 512^3 306.0 / 272.9.  FP64: 1-2% at 256^3 and 384^3,
  // slower where short z-chunks make its 8-plane halo costly; kept at two.
  return esz == 4;
}

bool wave_pairs_fit(const Dims &d, size_t esz)
{
  return (size_t)d.nx * d.ny * esz < ((size_t)1 << 31);
}

template <typename T>
hipError_t launch_wave_step(StencilKind kind, StepMode mode, const Dims &d, const T *p, const T *prev, T *out,
                            const T *kap, hipStream_t s)
{
  if (kind == STENCIL_NAIVE) {
    if (d.ndim == 2) return naive_dispatch<T, 2>(mode, d, p, prev, out, kap, s);
    return naive_dispatch<T, 3>(mode, d, p, prev, out, kap, s);
  }
  if (d.ndim == 2) return blocked_select<T, 2>(mode, d, p, prev, out, kap, s);
  return blocked_select<T, 3>(mode, d, p, prev, out, kap, s);
}

// ---------------------------------------------------------------------------
// Plan set-up: k' from c, and the range / validity of c.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void make_kappa_kernel(const T *__restrict__ c, size_t n, double dt2_over_12dx2, T *__restrict__ kap)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double cv = (double)c[i];
    kap[i] = (T)(cv * cv * dt2_over_12dx2);
  }
}

template <typename T>
hipError_t launch_make_kappa(const Dims &d, const T *c, double dt, double dx, T *kap, hipStream_t s)
{
  make_kappa_kernel<T><<<1024, 256, 0, s>>>(c, d.nvox(), dt * dt / (12.0 * dx * dx), kap);
  return hipGetLastError();
}

// partials laid out as [3][nblocks]: min, max, bad count.
template <typename T>
__global__ void __launch_bounds__(256) c_stats_partial(const T *__restrict__ c, size_t n, double *partials, int nblocks)
{
  __shared__ double smin[256], smax[256], sbad[256];
  double mn = DBL_MAX, mx = -DBL_MAX, bad = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = (double)c[i];
    if (!(v > 0.0) || !isfinite(v)) bad += 1.0;
    else {
      mn = fmin(mn, v);
      mx = fmax(mx, v);
    }
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      sbad[threadIdx.x] += sbad[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = smin[0];
    partials[nblocks + blockIdx.x] = smax[0];
    partials[2 * nblocks + blockIdx.x] = sbad[0];
  }
}

__global__ void __launch_bounds__(256) c_stats_final(const double *partials, int nblocks, double *stats)
{
  __shared__ double smin[256], smax[256], sbad[256];
  double mn = DBL_MAX, mx = -DBL_MAX, bad = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
    mn = fmin(mn, partials[i]);
    mx = fmax(mx, partials[nblocks + i]);
    bad += partials[2 * nblocks + i];
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      sbad[threadIdx.x] += sbad[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = smin[0];
    stats[1] = smax[0];
    stats[2] = sbad[0];
  }
}

template <typename T>
hipError_t launch_c_stats(const Dims &d, const T *c, double *partials, int nblocks, double *stats, hipStream_t s)
{
  c_stats_partial<T><<<nblocks, 256, 0, s>>>(c, d.nvox(), partials, nblocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  c_stats_final<<<1, 256, 0, s>>>(partials, nblocks, stats);
  return hipGetLastError();
}

#define FFPAT_INST(T)                                                                                        \
  template hipError_t launch_wave_pair<T>(const Dims &, const T *, const T *, T *, T *, const T *, hipStream_t); \
  template void wave_pair_shape<T>(const Dims &, int *, int *, int *);                                     \
  template hipError_t launch_wave_triple<T>(const Dims &, const T *, const T *, T *, T *, const T *, hipStream_t, \
                                            bool, bool *);                                                  \
  template hipError_t launch_wave_pair_div<T>(const Dims &, const T *, const T *, T *, T *, const T *,        \
                                              hipStream_t, bool *);                                         \
  template hipError_t launch_wave_triple_div<T>(const Dims &, const T *, const T *, T *, T *, const T *,      \
                                                hipStream_t, bool *);                                       \
  template hipError_t launch_wave_pair_first<T>(const Dims &, const T *, T *, T *, const T *, hipStream_t,    \
                                                bool *);                                                    \
  template bool wave_triple_shape<T>(const Dims &, int *, int *, int *);                                    \
  template bool wave_triples_available<T>(const Dims &);                                                   \
  template hipError_t launch_wave_step<T>(StencilKind, StepMode, const Dims &, const T *, const T *, T *,  \
                                          const T *, hipStream_t);                                          \
  template hipError_t launch_make_kappa<T>(const Dims &, const T *, double, double, T *, hipStream_t);     \
  template hipError_t launch_c_stats<T>(const Dims &, const T *, double *, int, double *, hipStream_t);
FFPAT_INST(float)
FFPAT_INST(double)
#undef FFPAT_INST

}  // namespace ffpat
