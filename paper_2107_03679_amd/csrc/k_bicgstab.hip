// Batched multigrid-preconditioned Bi-CGSTAB (Alg. 3 of the paper) for all
// right-hand sides of a scan, with the float-float solution of the GMRES
// path.  One iteration for right-hand side q (M = multigrid cycle):
//   p = r + beta (p - sigma v)                    k_bicg_dir
//   y = M p;  v = A y;  <r^, v>                   multigrid, k_bicg_apply
//   alpha = rho / <r^, v>                         k_bicg_alpha
//   s = r - alpha v                               k_bicg_s
//   z = M s;  t = A z;  <t, s>, <t, t>            multigrid, k_bicg_apply
//   sigma = <t, s> / <t, t>                       k_bicg_sigma
//   x += alpha y + sigma z;  r = s - sigma t;  <r^, r>, ||r||^2
//                                                 k_bicg_update
//   beta = (rho' / rho)(alpha / sigma), stop test k_bicg_rho
// <a, b> = a^H b.  Scalars are FP64 (complex), reductions deterministic
// (per-block FP32 partials, FP64 over blocks in a fixed order).  When the
// recursive residual meets the tolerance the right-hand side stops; the
// float-float true residual then decides, and a failed check restarts the
// recurrence from the true residual (r^ = r, p = r).
//
// Slots: V[q][0] = r (and s), V[q][1] = r^, V[q][2] = p, V[q][3] = v,
// V[q][4] = t;  Z[q][0] = y, Z[q][1] = z;  g[q][0..3] = rho, alpha, sigma,
// beta.  jcount[q] = -1 marks a restart.
#include "dev_common.h"
#include "kernels.h"

namespace {

constexpr int NT = 256;
constexpr int PPT = 8;
constexpr int CH = NT * PPT;
constexpr int NWAVE = NT / HELM_WAVE;

enum { S_R = 0, S_RHAT = 1, S_P = 2, S_V = 3, S_T = 4 };

__device__ __forceinline__ c32* vslot(const KrylovArgs& k, int b, int i) {
  return k.V + ((long long)b * (k.m + 1) + i) * k.N;
}
__device__ __forceinline__ c32* zslot(const KrylovArgs& k, int b, int i) {
  return k.Z + ((long long)b * k.m + i) * k.N;
}
__device__ __forceinline__ double2* scal(const KrylovArgs& k, int b) { return k.g + (long long)b * (k.m + 1); }
__device__ __forceinline__ c32 to_c32(double2 v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ bool zfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// block sum of (one complex, one real) value per thread -> partial slots of block blk
__device__ __forceinline__ void block_partials(const KrylovArgs& k, int b, int blk, int slot, c32 cv, float rv,
                                               bool with_real) {
  __shared__ float red[3][NWAVE];
  cv.x = wave_sum(cv.x);
  cv.y = wave_sum(cv.y);
  if (with_real) rv = wave_sum(rv);
  const int lane = threadIdx.x % HELM_WAVE, wave = threadIdx.x / HELM_WAVE;
  if (lane == 0) {
    red[0][wave] = cv.x;
    red[1][wave] = cv.y;
    red[2][wave] = rv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float sx = 0.f, sy = 0.f, sr = 0.f;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) {
      sx += red[0][q];
      sy += red[1][q];
      sr += red[2][q];
    }
    k.P1[((long long)b * k.nblk + blk) * (k.m + 1) + slot] = make_float2(sx, sy);
    if (with_real) k.P2[(long long)b * k.nblk + blk] = sr;
  }
}

// FP64 sum over the blocks of partial slot `slot` (one wavefront)
__device__ __forceinline__ double2 reduce_c(const KrylovArgs& k, int b, int slot) {
  double sx = 0.0, sy = 0.0;
  for (int blk = threadIdx.x; blk < k.nblk; blk += HELM_WAVE) {
    const c32 v = k.P1[((long long)b * k.nblk + blk) * (k.m + 1) + slot];
    sx += v.x;
    sy += v.y;
  }
  return make_double2(wave_sum_d(sx), wave_sum_d(sy));
}
__device__ __forceinline__ double reduce_r(const KrylovArgs& k, int b) {
  double s = 0.0;
  for (int blk = threadIdx.x; blk < k.nblk; blk += HELM_WAVE) s += k.P2[(long long)b * k.nblk + blk];
  return wave_sum_d(s);
}

// FP64 sum of the true residual's partial squared norms (k.nres of them)
__device__ __forceinline__ double reduce_res(const KrylovArgs& k, int b) {
  double s = 0.0;
  for (int blk = threadIdx.x; blk < k.nres; blk += HELM_WAVE) s += k.P2[(long long)b * k.nres + blk];
  return wave_sum_d(s);
}

__device__ __forceinline__ void breakdown(const KrylovArgs& k, int b) {
  k.status[b] = HELM_STATUS_BREAKDOWN_DEV;
  k.active[b] = 0;
}

// p = r + beta (p - sigma v); on a restart r^ = r and p = r
__global__ __launch_bounds__(NT) void k_bicg_dir(KrylovArgs k) {
  const int b = blockIdx.y;
  if (!k.active[b]) return;
  const long long p0 = (long long)blockIdx.x * CH + threadIdx.x;
  const c32* r = vslot(k, b, S_R);
  c32* pv = vslot(k, b, S_P);
  if (k.jcount[b] < 0) {
    c32* rh = vslot(k, b, S_RHAT);
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const long long p = p0 + (long long)t * NT;
      if (p < k.N) {
        const c32 rv = r[p];
        rh[p] = rv;
        pv[p] = rv;
      }
    }
    return;
  }
  const double2* sc = scal(k, b);
  const c32 beta = to_c32(sc[3]), sigma = to_c32(sc[2]);
  const c32* v = vslot(k, b, S_V);
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    if (p < k.N) pv[p] = cfma(beta, csub(pv[p], cmul(sigma, v[p])), r[p]);
  }
}

// out = A in (in = Z slot zs, out = V slot vs); partial dots:
// second = 0: <r^, out> in partial slot 0;  second = 1: <out, s> in slot 1 and ||out||^2
__global__ __launch_bounds__(NT) void k_bicg_apply(int nrhs, KrylovArgs k, int zs, int vs, LevelArgs fine,
                                                   int second) {
  const TileId id = xcd_tile(blockIdx.x, nrhs, k.nblk, HELM_RHS_GROUP);
  const int b = id.b, blk = id.t;
  if (!k.active[b]) return;
  const long long p0 = (long long)blk * CH + threadIdx.x;
  const c32* z = zslot(k, b, zs);
  c32* w = vslot(k, b, vs);
  const c32* o = vslot(k, b, second ? S_R : S_RHAT);
  c32 d = make_float2(0.f, 0.f);
  float nn = 0.f;
  Coord c = coord_of32((unsigned)p0, (unsigned)fine.n, k.dim);
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    if (p < k.N) {
      const c32 wv = stencil_point(z, p, c, fine.n, k.dim, diag_at(fine, p, ghosts_of(c, fine.n, k.dim), k.dim));
      w[p] = wv;
      const c32 ov = o[p];
      if (second) {
        d = cadd(d, cconjmul(wv, ov));  // <t, s>
        nn = fmaf(wv.x, wv.x, fmaf(wv.y, wv.y, nn));
      } else {
        d = cadd(d, cconjmul(ov, wv));  // <r^, v>
      }
    }
    coord_advance(c, NT, fine.n, k.dim);
  }
  block_partials(k, b, blk, second ? 1 : 0, d, nn, second != 0);
}

// alpha = rho / <r^, v>
__global__ __launch_bounds__(HELM_WAVE) void k_bicg_alpha(KrylovArgs k) {
  const int b = blockIdx.x;
  if (!k.active[b]) return;
  const double2 den = reduce_c(k, b, 0);
  if (threadIdx.x != 0) return;
  k.jcount[b] = 0;
  double2* sc = scal(k, b);
  if (!zfinite(den) || (den.x == 0.0 && den.y == 0.0)) {
    breakdown(k, b);
    return;
  }
  sc[1] = zdiv(sc[0], den);
}

// s = r - alpha v (in place over r)
__global__ __launch_bounds__(NT) void k_bicg_s(KrylovArgs k) {
  const int b = blockIdx.y;
  if (!k.active[b]) return;
  const long long p0 = (long long)blockIdx.x * CH + threadIdx.x;
  const c32 na = to_c32(scal(k, b)[1]);
  const c32 nalpha = make_float2(-na.x, -na.y);
  c32* r = vslot(k, b, S_R);
  const c32* v = vslot(k, b, S_V);
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    if (p < k.N) r[p] = cfma(nalpha, v[p], r[p]);
  }
}

// sigma = <t, s> / <t, t>  (0 when t = 0: then s = 0 and the step is complete)
__global__ __launch_bounds__(HELM_WAVE) void k_bicg_sigma(KrylovArgs k) {
  const int b = blockIdx.x;
  if (!k.active[b]) return;
  const double2 ts = reduce_c(k, b, 1);
  const double tt = reduce_r(k, b);
  if (threadIdx.x != 0) return;
  if (!zfinite(ts) || !isfinite(tt)) {
    breakdown(k, b);
    return;
  }
  scal(k, b)[2] = tt > 0.0 ? make_double2(ts.x / tt, ts.y / tt) : make_double2(0.0, 0.0);
}

// x += alpha y + sigma z (float-float);  r = s - sigma t;  partials <r^, r>, ||r||^2
__global__ __launch_bounds__(NT) void k_bicg_update(int nrhs, KrylovArgs k, c32* x_hi, c32* x_lo) {
  const TileId id = xcd_tile(blockIdx.x, nrhs, k.nblk, HELM_RHS_GROUP);
  const int b = id.b, blk = id.t;
  if (!k.active[b]) return;
  const long long p0 = (long long)blk * CH + threadIdx.x;
  const double2* sc = scal(k, b);
  const c32 alpha = to_c32(sc[1]), sigma = to_c32(sc[2]);
  const c32 nsigma = make_float2(-sigma.x, -sigma.y);
  const c32 *y = zslot(k, b, 0), *z = zslot(k, b, 1), *tv = vslot(k, b, S_T), *rh = vslot(k, b, S_RHAT);
  c32* r = vslot(k, b, S_R);
  c32* xh = x_hi + (long long)b * k.N;
  c32* xl = x_lo + (long long)b * k.N;
  c32 d = make_float2(0.f, 0.f);
  float nn = 0.f;
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    if (p < k.N) {
      const c32 dx = cfma(sigma, z[p], cmul(alpha, y[p]));
      const c32 h = xh[p], l = xl[p];
      const ff re = ff_add({h.x, l.x}, ff_from(dx.x));
      const ff im = ff_add({h.y, l.y}, ff_from(dx.y));
      xh[p] = make_float2(re.hi, im.hi);
      xl[p] = make_float2(re.lo, im.lo);
      const c32 rv = cfma(nsigma, tv[p], r[p]);
      r[p] = rv;
      d = cadd(d, cconjmul(rh[p], rv));
      nn = fmaf(rv.x, rv.x, fmaf(rv.y, rv.y, nn));
    }
  }
  block_partials(k, b, blk, 2, d, nn, true);
}

// rho' = <r^, r>, beta = (rho' / rho)(alpha / sigma); stop when ||r|| <= tol or at the iteration cap
__global__ __launch_bounds__(HELM_WAVE) void k_bicg_rho(KrylovArgs k) {
  const int b = blockIdx.x;
  if (!k.active[b]) return;
  const double2 rho1 = reduce_c(k, b, 2);
  const double rr = reduce_r(k, b);
  if (threadIdx.x != 0) return;
  double2* sc = scal(k, b);
  const int it = (k.iters[b] += 2);
  if (!zfinite(rho1) || !isfinite(rr)) {
    breakdown(k, b);
    return;
  }
  const double2 sigma = sc[2];
  if (sqrt(rr) <= k.tol[b] || it >= k.max_iters) {
    k.active[b] = 0;  // the true residual decides
    return;
  }
  if ((sigma.x == 0.0 && sigma.y == 0.0) || (sc[0].x == 0.0 && sc[0].y == 0.0)) {
    k.active[b] = 0;  // the recurrence cannot continue: check and restart from the true residual
    return;
  }
  sc[3] = zmul(zdiv(rho1, sc[0]), zdiv(sc[1], sigma));
  sc[0] = rho1;
}

// After a true residual of the right-hand sides that stopped iterating: converged,
// capped, or a restart from the true residual (rho = ||r||^2, r^ = r).
__global__ __launch_bounds__(HELM_WAVE) void k_bicg_finalize(KrylovArgs k, int first) {
  const int b = blockIdx.x;
  if (k.status[b] != HELM_RUNNING || k.active[b]) return;
  const double s = reduce_res(k, b);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(s);
  if (first) {
    k.bnorm[b] = rn;
    k.tol[b] = k.rtol * k.inner_factor * rn;
  }
  const double bn = k.bnorm[b];
  if (!isfinite(rn) || !isfinite(bn)) {
    k.status[b] = HELM_STATUS_BREAKDOWN_DEV;
    k.relres[b] = rn / bn;
    return;
  }
  const double rel = bn > 0.0 ? rn / bn : 0.0;
  k.relres[b] = rel;
  if (rel <= k.rtol) {
    k.status[b] = HELM_STATUS_CONVERGED_DEV;
    return;
  }
  if (k.iters[b] >= k.max_iters) {
    k.status[b] = HELM_STATUS_NOT_CONVERGED_DEV;
    return;
  }
  k.active[b] = 1;
  k.jcount[b] = -1;
  double2* sc = scal(k, b);
  sc[0] = make_double2(s, 0.0);
  sc[1] = make_double2(1.0, 0.0);
  sc[2] = make_double2(1.0, 0.0);
  sc[3] = make_double2(0.0, 0.0);
}

}  // namespace

void launch_bicg_dir(hipStream_t s, int B, const KrylovArgs& k) {
  hipLaunchKernelGGL(k_bicg_dir, dim3(k.nblk, B), dim3(NT), 0, s, k);
}
void launch_bicg_apply(hipStream_t s, int B, const KrylovArgs& k, int zs, int vs, const LevelArgs& fine,
                       int second) {
  hipLaunchKernelGGL(k_bicg_apply, dim3(B * k.nblk), dim3(NT), 0, s, B, k, zs, vs, fine, second);
}
void launch_bicg_alpha(hipStream_t s, int B, const KrylovArgs& k) {
  hipLaunchKernelGGL(k_bicg_alpha, dim3(B), dim3(HELM_WAVE), 0, s, k);
}
void launch_bicg_s(hipStream_t s, int B, const KrylovArgs& k) {
  hipLaunchKernelGGL(k_bicg_s, dim3(k.nblk, B), dim3(NT), 0, s, k);
}
void launch_bicg_sigma(hipStream_t s, int B, const KrylovArgs& k) {
  hipLaunchKernelGGL(k_bicg_sigma, dim3(B), dim3(HELM_WAVE), 0, s, k);
}
void launch_bicg_update(hipStream_t s, int B, const KrylovArgs& k, c32* x_hi, c32* x_lo) {
  hipLaunchKernelGGL(k_bicg_update, dim3(B * k.nblk), dim3(NT), 0, s, B, k, x_hi, x_lo);
}
void launch_bicg_rho(hipStream_t s, int B, const KrylovArgs& k) {
  hipLaunchKernelGGL(k_bicg_rho, dim3(B), dim3(HELM_WAVE), 0, s, k);
}
void launch_bicg_finalize(hipStream_t s, int B, const KrylovArgs& k, int first) {
  hipLaunchKernelGGL(k_bicg_finalize, dim3(B), dim3(HELM_WAVE), 0, s, k, first);
}
