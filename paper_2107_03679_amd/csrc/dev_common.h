// Device helpers shared by the HIP kernels: complex64 arithmetic, float-float
// (double-float) arithmetic built from error-free transforms, wavefront and
// block reductions, and grid geometry of the vertex-centred levels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

#define HELM_WAVE 64

// ------------------------------------------------------- workgroup order
// gfx950 hands out the workgroups of a launch round-robin over its 8 XCDs,
// each with a private L2.  xcd_tile() maps the hardware workgroup id to a
// logical (right-hand side, tile).  g = 0 (the default) is the plain order,
// right-hand side fastest: the blocks of one tile for all right-hand sides
// are dispatched together, spread over the XCDs, and share the coefficient
// tile.  g >= 1 makes every XCD walk one contiguous stretch of the order
// "groups of g right-hand sides; tiles in raster order; the right-hand sides
// of a group fastest", so that neighbouring tiles of one field meet in one
// L2.  On MI355X the plain order measured 5.5% faster over the whole
// 512^2 x 60 solve than g = 1, 4 or 16 (same box, alternating runs), so the
// remap is kept only as an option.  Bijective on [0, B T) for any g >= 0.
#define HELM_XCDS 8u
struct TileId {
  int b, t;
};
__host__ __device__ __forceinline__ TileId xcd_tile(unsigned id, unsigned B, unsigned T, unsigned g) {
  if (g == 0) {  // plain order: right-hand side fastest, tiles in raster order
    TileId o;
    o.b = (int)(id % B);
    o.t = (int)(id / B);
    return o;
  }
  const unsigned G = B * T, q = G / HELM_XCDS, r = G % HELM_XCDS, x = id % HELM_XCDS;
  const unsigned l = x * q + (x < r ? x : r) + id / HELM_XCDS;
  const unsigned span = g * T, grp = l / span, rem = l - grp * span;
  const unsigned gs = B - grp * g < g ? B - grp * g : g;
  TileId o;
  o.b = (int)(grp * g + rem % gs);
  o.t = (int)(rem / gs);
  return o;
}
// The order of the up-legs (k_up_mv2w, k_up_col): workgroup id -> position l in one
// logical order such that every XCD walks one contiguous stretch of it, of equal length
// (+-1).  With "right-hand sides (or groups of them) fastest, then tiles in raster order"
// the workgroups sharing a coefficient tile and the neighbouring tiles sharing halo rows
// meet in one L2; for these two kernels it measured faster than the plain order.
// Bijective on [0, G).
__host__ __device__ __forceinline__ unsigned xcd_stretch(unsigned id, unsigned G) {
  const unsigned q = G / HELM_XCDS, r = G % HELM_XCDS, x = id % HELM_XCDS;
  return x * q + (x < r ? x : r) + id / HELM_XCDS;
}
// right-hand sides per group in xcd_tile() for the field kernels (0: the plain order)
#ifndef HELM_RHS_GROUP
#define HELM_RHS_GROUP 0u
#endif


// ---------------------------------------------------------------- complex64
__host__ __device__ __forceinline__ c32 cadd(c32 a, c32 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ c32 csub(c32 a, c32 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ c32 cscale(c32 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// conj(a) * b
__host__ __device__ __forceinline__ c32 cconjmul(c32 a, c32 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x));
}
// acc + a * b
__host__ __device__ __forceinline__ c32 cfma(c32 a, c32 b, c32 acc) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
// 1 / d via conj(d) / |d|^2
__host__ __device__ __forceinline__ c32 crcp(c32 d) {
  float inv = 1.0f / fmaf(d.x, d.x, d.y * d.y);
  return make_float2(d.x * inv, -d.y * inv);
}
__host__ __device__ __forceinline__ c32 cconj(c32 a) { return make_float2(a.x, -a.y); }

// ------------------------------------------------------------- float-float
// A value hi + lo with |lo| <= ulp(hi)/2.  TwoSum (Knuth) and TwoProd (FMA)
// are error-free; the compound operations follow the usual double-float
// algorithms (Dekker 1971; Hida, Li and Bailey 2001) with ~2^-44 relative
// error, far below what the residual test needs.
// Device code is compiled with FP contraction enabled and the AMDGPU backend
// fuses aggressively (a product feeding several adds becomes FMAs); that
// would break the error-free transforms, so contraction is switched off
// inside every float-float routine.
#define HELM_NO_CONTRACT _Pragma("clang fp contract(off)")

struct ff {
  float hi, lo;
};

__host__ __device__ __forceinline__ ff two_sum(float a, float b) {
  HELM_NO_CONTRACT
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__host__ __device__ __forceinline__ ff fast_two_sum(float a, float b) {
  HELM_NO_CONTRACT
  float s = a + b;
  float e = b - (s - a);
  return {s, e};
}
__host__ __device__ __forceinline__ ff two_prod(float a, float b) {
  HELM_NO_CONTRACT
  float p = a * b;
  float e = fmaf(a, b, -p);
  return {p, e};
}
__host__ __device__ __forceinline__ ff ff_add(ff a, ff b) {
  HELM_NO_CONTRACT
  ff s = two_sum(a.hi, b.hi);
  ff t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__host__ __device__ __forceinline__ ff ff_neg(ff a) {
  HELM_NO_CONTRACT return {-a.hi, -a.lo}; }
__host__ __device__ __forceinline__ ff ff_sub(ff a, ff b) {
  HELM_NO_CONTRACT return ff_add(a, ff_neg(b)); }
__host__ __device__ __forceinline__ ff ff_mul(ff a, ff b) {
  HELM_NO_CONTRACT
  ff p = two_prod(a.hi, b.hi);
  p.lo = fmaf(a.hi, b.lo, fmaf(a.lo, b.hi, p.lo));
  return fast_two_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ ff ff_from(float a) { return {a, 0.0f}; }

struct cff {
  ff re, im;
};
__host__ __device__ __forceinline__ cff cff_add(cff a, cff b) {
  HELM_NO_CONTRACT return {ff_add(a.re, b.re), ff_add(a.im, b.im)}; }
__host__ __device__ __forceinline__ cff cff_sub(cff a, cff b) {
  HELM_NO_CONTRACT return {ff_sub(a.re, b.re), ff_sub(a.im, b.im)}; }
__host__ __device__ __forceinline__ cff cff_mul(cff a, cff b) {
  HELM_NO_CONTRACT
  return {ff_sub(ff_mul(a.re, b.re), ff_mul(a.im, b.im)), ff_add(ff_mul(a.re, b.im), ff_mul(a.im, b.re))};
}
__host__ __device__ __forceinline__ cff cff_make(c32 hi, c32 lo) { return {{hi.x, lo.x}, {hi.y, lo.y}}; }

// ------------------------------------------------------------ reductions
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = HELM_WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, HELM_WAVE);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = HELM_WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, HELM_WAVE);
  return v;
}

// -------------------------------------------------------------- geometry
// Number of Sommerfeld ghost neighbours of point (x, y[, z]) on an n^d grid.
__host__ __device__ __forceinline__ int ghosts2(int x, int y, int n) {
  return (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1);
}
__host__ __device__ __forceinline__ int ghosts3(int x, int y, int z, int n) {
  return (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1) + (z == 0) + (z == n - 1);
}

// Element at a byte offset from a base: a wavefront-uniform base and a 32-bit
// per-lane offset let the loads and stores use the scalar-base address form.
__device__ __forceinline__ const c32& at_byte(const c32* base, unsigned off) {
  return *reinterpret_cast<const c32*>(reinterpret_cast<const char*>(base) + off);
}
__device__ __forceinline__ c32& at_byte(c32* base, unsigned off) {
  return *reinterpret_cast<c32*>(reinterpret_cast<char*>(base) + off);
}

__device__ __forceinline__ float scale_of(ScaleSet s, int b) { return s.p ? s.p[(long long)b * s.stride] : 1.0f; }

// diagonal of the level operator: 2d - coef - g * #ghosts
__device__ __forceinline__ c32 diag_at(const LevelArgs& lv, long long p, int ng, int dim) {
  c32 c = lv.coef[p];
  return make_float2(2.0f * dim - c.x - ng * lv.ghost.x, -c.y - ng * lv.ghost.y);
}

struct Coord {
  int x, y, z;
};
// Coordinates of flat index p (< 2^31) on an n^dim grid, 32-bit arithmetic.
__host__ __device__ __forceinline__ Coord coord_of32(unsigned p, unsigned n, int dim) {
  Coord c;
  const unsigned q = p / n;
  c.x = (int)(p - q * n);
  if (dim == 2) {
    c.y = (int)q;
    c.z = 0;
  } else {
    const unsigned r = q / n;
    c.y = (int)(q - r * n);
    c.z = (int)r;
  }
  return c;
}
// Advance coordinates by `step` points along the flat index (step >= 0).
__host__ __device__ __forceinline__ void coord_advance(Coord& c, int step, int n, int dim) {
  c.x += step;
  while (c.x >= n) {
    c.x -= n;
    if (++c.y == n && dim == 3) {
      c.y = 0;
      ++c.z;
    }
  }
}
// A' v at point p with branch-free, always in-bounds neighbour loads:
// out-of-grid neighbours load v[p] and are multiplied by 0.
__host__ __device__ __forceinline__ c32 stencil_point(const c32* v, long long p, const Coord& c, int n, int dim,
                                                      c32 D) {
  const long long n2 = (long long)n * n;
  const int xm = c.x > 0, xp = c.x < n - 1, ym = c.y > 0, yp = c.y < n - 1;
  const c32 vc = v[p];
  const c32 a = v[p - xm], b = v[p + xp], cc = v[p - (long long)ym * n], d = v[p + (long long)yp * n];
  c32 nb = make_float2(xm * a.x + xp * b.x + ym * cc.x + yp * d.x, xm * a.y + xp * b.y + ym * cc.y + yp * d.y);
  if (dim == 3) {
    const int zm = c.z > 0, zp = c.z < n - 1;
    const c32 e = v[p - zm * n2], f = v[p + zp * n2];
    nb.x += zm * e.x + zp * f.x;
    nb.y += zm * e.y + zp * f.y;
  }
  return csub(cmul(D, vc), nb);
}
__host__ __device__ __forceinline__ int ghosts_of(const Coord& c, int n, int dim) {
  return dim == 2 ? ghosts2(c.x, c.y, n) : ghosts3(c.x, c.y, c.z, n);
}
// sum of the in-grid neighbours of point p
__device__ __forceinline__ c32 neighbour_sum(const c32* v, long long p, const Coord& c, int n, int dim) {
  c32 s = make_float2(0.f, 0.f);
  if (c.x > 0) s = cadd(s, v[p - 1]);
  if (c.x < n - 1) s = cadd(s, v[p + 1]);
  if (c.y > 0) s = cadd(s, v[p - n]);
  if (c.y < n - 1) s = cadd(s, v[p + n]);
  if (dim == 3) {
    const long long n2 = (long long)n * n;
    if (c.z > 0) s = cadd(s, v[p - n2]);
    if (c.z < n - 1) s = cadd(s, v[p + n2]);
  }
  return s;
}

