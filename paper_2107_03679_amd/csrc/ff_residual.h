// Per-point float-float residual r = h^2 b - A'(x_hi + x_lo), shared by the
// GPU kernel and host-side verification builds (all arithmetic is FP32
// error-free transforms; no FP64).
#pragma once

#include "dev_common.h"

struct FFArgs {
  const c32* rhs;
  long long rhs_stride;
  int conj_rhs;
  const c32* x_hi;
  const c32* x_lo;
  int x_zero;
  const c32* d_hi;  // diagonal of A' (2d - c - #ghosts (1 + j k_b h)), float-float
  const c32* d_lo;
  float h2_hi, h2_lo;
  c32* r_out;
  long long r_stride;
  float out_scale;
};

__host__ __device__ __forceinline__ cff ff_load_x(const c32* xh, const c32* xl, long long p) {
  return cff_make(xh[p], xl ? xl[p] : make_float2(0.f, 0.f));
}

// h^2 b (conjugated for the adjoint) as a float-float pair
__host__ __device__ __forceinline__ cff ff_scaled_rhs(const FFArgs& a, c32 bv) {
  const ff h2 = {a.h2_hi, a.h2_lo};
  if (a.conj_rhs) bv.y = -bv.y;
  return cff{ff_mul(ff_from(bv.x), h2), ff_mul(ff_from(bv.y), h2)};
}

__host__ __device__ __forceinline__ c32 ff_round(const cff& r) {
  return make_float2(r.re.hi + r.re.lo, r.im.hi + r.im.lo);
}

// rb, xh, xl point at this right-hand side's vectors (xh == NULL: x = 0).
__host__ __device__ inline c32 ff_residual_point(const FFArgs& a, const c32* rb, const c32* xh, const c32* xl,
                                                 long long p, const Coord& c, int n, int dim) {
  cff r = ff_scaled_rhs(a, rb[p]);
  if (xh) {
    const cff D = cff_make(a.d_hi[p], a.d_lo[p]);
    cff ax = cff_mul(D, ff_load_x(xh, xl, p));
    cff nb = {ff_from(0.f), ff_from(0.f)};
    if (c.x > 0) nb = cff_add(nb, ff_load_x(xh, xl, p - 1));
    if (c.x < n - 1) nb = cff_add(nb, ff_load_x(xh, xl, p + 1));
    if (c.y > 0) nb = cff_add(nb, ff_load_x(xh, xl, p - n));
    if (c.y < n - 1) nb = cff_add(nb, ff_load_x(xh, xl, p + n));
    if (dim == 3) {
      const long long n2 = (long long)n * n;
      if (c.z > 0) nb = cff_add(nb, ff_load_x(xh, xl, p - n2));
      if (c.z < n - 1) nb = cff_add(nb, ff_load_x(xh, xl, p + n2));
    }
    ax = cff_sub(ax, nb);
    r = cff_sub(r, ax);
  }
  return ff_round(r);
}
