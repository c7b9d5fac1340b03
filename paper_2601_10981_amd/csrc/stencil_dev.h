// Device helpers shared by the fused RK4 stencils (steady flows in
// stencil.hip, forced flows in forced.hip): table access, descriptor lookup,
// the stencil at one column of an LDS stage plane and the ring order of a
// workgroup's columns. Internal.
#pragma once

#include "pr_internal.h"

namespace pr {

template <typename T>
__device__ __forceinline__ const T* tab_of(const Geom& g);
template <>
__device__ __forceinline__ const double* tab_of<double>(const Geom& g) { return g.tab64; }
template <>
__device__ __forceinline__ const float* tab_of<float>(const Geom& g) { return g.tab32; }

// Locate the descriptor owning global tile `t` (descriptors sorted by
// tile_begin): binary search over uniform data.
template <typename D>
__device__ __forceinline__ int find_desc(const D* d, int nd, long long t) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].tile_begin <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Fused RK4 step.

// L at one column of a stage plane, general velocity: x neighbours from
// registers, y and z neighbours from the LDS plane (row-major, RZ columns per
// row).
// Every multiply-add is an explicit fma and nothing else is contracted, so
// each value is bitwise the same in every instantiation and tiling.
template <typename T, int RZ>
__device__ __forceinline__ T lop(T xm, T c, T xp, const T* __restrict__ pl, int i, T clap,
                                 T vx, T vy, T vz) {
#pragma clang fp contract(off)
  const T ym = pl[i - RZ], yp = pl[i + RZ], zm = pl[i - 1], zp = pl[i + 1];
  const T lap = fma((T)-6, c, ((xp + xm) + (yp + ym)) + (zp + zm));
  const T adv = fma(vz, zp - zm, fma(vy, yp - ym, vx * (xp - xm)));
  return fma(clap, lap, -adv);
}

// L for a velocity with only an x component, regrouped per neighbour:
// (clap - v_x) u_{x+1} + (clap + v_x) u_{x-1} + clap (y and z neighbours)
// - 6 clap u, with a = clap - v_x, b = clap + v_x and e = -6 clap.
template <typename T, int RZ>
__device__ __forceinline__ T lop_x(T xm, T c, T xp, const T* __restrict__ pl, int i, T clap,
                                   T e, T a, T b) {
#pragma clang fp contract(off)
  const T ym = pl[i - RZ], yp = pl[i + RZ], zm = pl[i - 1], zp = pl[i + 1];
  const T syz = (yp + ym) + (zp + zm);
  return fma(a, xp, fma(b, xm, fma(clap, syz, e * c)));
}

__device__ __forceinline__ int wrapi(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Column p of a workgroup's (TY + 2H) x (TZ + 2H) region in ring order: the
// TY x TZ interior first (row-major), then the rings at distance 1, 2, ..., H
// from it (each row-major). Region coordinates (ry, rz) and ring level.
// Stage s of the fused step is needed on levels <= H - s, so with this order
// whole waves skip the stages none of their columns needs.
template <int TY, int TZ>
__device__ __forceinline__ void ring_col(int p, int& ry, int& rz, int& lev) {
  constexpr int H = kFusedHalo;
  if (p < TY * TZ) {
    ry = H + p / TZ;
    rz = H + p % TZ;
    lev = 0;
    return;
  }
  int start = TY * TZ;
#pragma unroll
  for (int L = 1; L <= H; ++L) {
    const int WY = TY + 2 * L, WZ = TZ + 2 * L;
    const int ring = WY * WZ - (WY - 2) * (WZ - 2);
    if (p < start + ring) {
      int q = p - start, by, bz;
      if (q < WZ) {
        by = 0;
        bz = q;
      } else if (q < WZ + 2 * (WY - 2)) {
        q -= WZ;
        by = 1 + q / 2;
        bz = (q & 1) ? WZ - 1 : 0;
      } else {
        by = WY - 1;
        bz = q - WZ - 2 * (WY - 2);
      }
      ry = by + H - L;
      rz = bz + H - L;
      lev = L;
      return;
    }
    start += ring;
  }
  ry = rz = 0;
  lev = 99;   // beyond the region (no column)
}

}  // namespace pr
