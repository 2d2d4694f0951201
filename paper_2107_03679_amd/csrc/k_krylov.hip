// Batched restarted FGMRES kernels (right preconditioning) with a float-float
// outer iterate.  Every kernel takes all B right-hand sides of a scan; a
// per-RHS `active` flag makes converged systems skip their work.
//
// One Arnoldi step j for right-hand side q:
//   z_j = M(v_j)                       (multigrid kernels)
//   w   = A z_j,  d_i = <V_i, w>       (k_arnoldi_dots, fused matvec + dots)
//   h_i = vs_i d_i                     (k_arnoldi_reduce, FP64)
//   w  -= sum_i h_i v_i, ||w||^2       (k_arnoldi_update)
//   Givens update of column j, residual estimate, v_{j+1} = w / h_{j+1,j}
//                                      (k_givens, FP64, one wavefront per RHS)
// The basis is stored unnormalised with a scale per vector (v_i = vs_i V_i),
// which saves the normalisation pass.  <a, b> = a^H b.
#include "dev_common.h"
#include "ff_residual.h"
#include "kernels.h"

namespace {

constexpr int NT = 256;       // threads per block of the flat kernels
constexpr int PPT = 8;        // points per thread
constexpr int CH = NT * PPT;  // points per block
constexpr int NWAVE = NT / HELM_WAVE;
constexpr int MAXM = 64;
constexpr int SSTEP_MAXM = 12;  // longest s-step cycle (the Gram matrix lives in registers)
constexpr int VCH = 4;        // basis vectors streamed together by k_x_update

__device__ __forceinline__ long long vidx(const KrylovArgs& k, int b, int i) {
  return ((long long)b * (k.m + 1) + i) * k.N;
}
__device__ __forceinline__ long long zidx(const KrylovArgs& k, int b, int i) {
  return ((long long)b * k.m + i) * k.N;
}


__global__ __launch_bounds__(NT) void k_arnoldi_dots(int nrhs, KrylovArgs k, int j, LevelArgs fine,
                                                    int with_matvec) {
  __shared__ c32 red[NWAVE][MAXM + 1];
  // consecutive chunks of one field share stencil rows, one chunk of a group shares the coefficient
  const TileId id = xcd_tile(blockIdx.x, nrhs, k.nblk, HELM_RHS_GROUP);
  const int b = id.b, blk = id.t;
  if (!k.active[b]) return;
  const long long p0 = (long long)blk * CH + threadIdx.x;
  c32* w_out = k.V + vidx(k, b, j + 1);
  c32 w[PPT];
  if (with_matvec) {
    const c32* z = k.Z + zidx(k, b, j);
    Coord c = coord_of32((unsigned)p0, (unsigned)fine.n, k.dim);
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const long long p = p0 + (long long)t * NT;
      w[t] = make_float2(0.f, 0.f);
      if (p < k.N) {
        const c32 D = diag_at(fine, p, ghosts_of(c, fine.n, k.dim), k.dim);
        w[t] = stencil_point(z, p, c, fine.n, k.dim, D);
        w_out[p] = w[t];
      }
      coord_advance(c, NT, fine.n, k.dim);
    }
  } else {
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const long long p = p0 + (long long)t * NT;
      w[t] = p < k.N ? w_out[p] : make_float2(0.f, 0.f);
    }
  }
  const int lane = threadIdx.x % HELM_WAVE, wave = threadIdx.x / HELM_WAVE;
  // one basis vector ahead: the next vector's points (from the nearest valid point, so that
  // no load waits behind the guard of its product) are in flight while the current one's
  // dot product is formed
  auto ldv = [&](int i, c32* o) {
    const c32* vi = k.V + vidx(k, b, i);
#pragma unroll
    for (int t = 0; t < PPT; ++t) o[t] = vi[min(p0 + (long long)t * NT, k.N - 1)];
  };
  c32 vc[PPT], vn[PPT];
  ldv(0, vc);
  for (int i = 0; i <= j; ++i) {
    if (i + 1 <= j) ldv(i + 1, vn);
    c32 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const long long p = p0 + (long long)t * NT;
      if (p < k.N) acc = cadd(acc, cconjmul(vc[t], w[t]));
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    if (lane == 0) red[wave][i] = acc;
#pragma unroll
    for (int t = 0; t < PPT; ++t) vc[t] = vn[t];
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += NT) {
    c32 s = red[0][i];
#pragma unroll
    for (int q = 1; q < NWAVE; ++q) s = cadd(s, red[q][i]);
    k.P1[((long long)b * k.nblk + blk) * (k.m + 1) + i] = s;
  }
}

// h_i = vs_i * sum over blocks of the partial dots (FP64, fixed order: deterministic)
__global__ __launch_bounds__(NT) void k_arnoldi_reduce(KrylovArgs k, int j, int accumulate) {
  const int b = blockIdx.x;
  if (!k.active[b]) return;
  const int lane = threadIdx.x % HELM_WAVE, wave = threadIdx.x / HELM_WAVE;
  for (int i = wave; i <= j; i += NWAVE) {
    double sx = 0.0, sy = 0.0;
    for (int blk = lane; blk < k.nblk; blk += HELM_WAVE) {
      const c32 v = k.P1[((long long)b * k.nblk + blk) * (k.m + 1) + i];
      sx += v.x;
      sy += v.y;
    }
    sx = wave_sum_d(sx);
    sy = wave_sum_d(sy);
    if (lane == 0) {
      const double vsi = k.vs[b * (k.m + 1) + i];
      const double hx = sx * vsi, hy = sy * vsi;
      double2* hij = &k.H[((long long)b * (k.m + 1) + i) * k.m + j];
      if (accumulate) {
        hij->x += hx;
        hij->y += hy;
      } else {
        *hij = make_double2(hx, hy);
      }
      k.coef[b * (k.m + 1) + i] = make_float2((float)(hx * vsi), (float)(hy * vsi));
    }
  }
}

// w -= sum_i coef_i V_i; partial ||w||^2
__global__ __launch_bounds__(NT) void k_arnoldi_update(KrylovArgs k, int j) {
  __shared__ float red[NWAVE];
  const int b = blockIdx.y;
  if (!k.active[b]) return;
  const long long p0 = (long long)blockIdx.x * CH + threadIdx.x;
  c32* wv = k.V + vidx(k, b, j + 1);
  c32 w[PPT];
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    w[t] = p < k.N ? wv[p] : make_float2(0.f, 0.f);
  }
  // one basis vector ahead: the next vector's points (from the nearest valid point, so that
  // no load waits behind a guard) are in flight while the current one is subtracted, in the
  // order of i; w past N is never stored or summed
  auto ldv = [&](int i, c32* o) {
    const c32* vi = k.V + vidx(k, b, i);
#pragma unroll
    for (int t = 0; t < PPT; ++t) o[t] = vi[min(p0 + (long long)t * NT, k.N - 1)];
  };
  c32 vc[PPT], vn[PPT];
  ldv(0, vc);
  for (int i = 0; i <= j; ++i) {
    if (i + 1 <= j) ldv(i + 1, vn);
    const c32 ci = k.coef[b * (k.m + 1) + i];
    const c32 nci = make_float2(-ci.x, -ci.y);
#pragma unroll
    for (int t = 0; t < PPT; ++t) w[t] = cfma(nci, vc[t], w[t]);
#pragma unroll
    for (int t = 0; t < PPT; ++t) vc[t] = vn[t];
  }
  float nrm = 0.f;
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    if (p < k.N) {
      wv[p] = w[t];
      nrm = fmaf(w[t].x, w[t].x, fmaf(w[t].y, w[t].y, nrm));
    }
  }
  nrm = wave_sum(nrm);
  const int lane = threadIdx.x % HELM_WAVE, wave = threadIdx.x / HELM_WAVE;
  if (lane == 0) red[wave] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) s += red[q];
    k.P2[(long long)b * k.nblk + blockIdx.x] = s;
  }
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double zabs(double2 a) { return hypot(a.x, a.y); }

// Back-substitution y = H(0:kk, 0:kk)^-1 g(0:kk) for right-hand side b (FP64, one thread;
// yd: kk FP64 slots in LDS, where a per-thread array indexed at run time would spill).
// y of the kk-column triangular system H y = g (H row stride m), written to k.y
__device__ void back_substitute(const KrylovArgs& k, int b, int kk, double2* yd, const double2* H, const double2* g) {
  for (int i = kk - 1; i >= 0; --i) {
    double2 s = g[i];
    for (int l = i + 1; l < kk; ++l) {
      const double2 t = zmul(H[i * k.m + l], yd[l]);
      s.x -= t.x;
      s.y -= t.y;
    }
    const double2 d = H[i * k.m + i];
    const double den = d.x * d.x + d.y * d.y;
    yd[i] = make_double2((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den);
  }
  for (int i = 0; i < k.m; ++i)
    k.y[b * k.m + i] = i < kk ? make_float2((float)yd[i].x, (float)yd[i].y) : make_float2(0.f, 0.f);
}

// Givens update of column j (FP64), residual estimate, stop decision, least squares at cycle end.
__global__ __launch_bounds__(HELM_WAVE) void k_givens(KrylovArgs k, int j) {
  __shared__ double2 yd[MAXM];
  const int b = blockIdx.x;
  if (!k.active[b]) return;
  double s = 0.0;
  for (int blk = threadIdx.x; blk < k.nblk; blk += HELM_WAVE) s += k.P2[(long long)b * k.nblk + blk];
  s = wave_sum_d(s);
  if (threadIdx.x != 0) return;
  const int m = k.m;
  double2* H = k.H + (long long)b * (m + 1) * m;
  double* cs = k.cs + (long long)b * m;
  double2* sn = k.sn + (long long)b * m;
  double2* g = k.g + (long long)b * (m + 1);
  const double hj1 = sqrt(s);
  // previous rotations G_i = [[c, s], [-conj(s), c]] on rows i, i+1
  for (int i = 0; i < j; ++i) {
    const double2 a = H[i * m + j], c2 = H[(i + 1) * m + j];
    const double2 t1 = zmul(sn[i], c2);
    const double2 t2 = zmul(zconj(sn[i]), a);
    H[i * m + j] = make_double2(cs[i] * a.x + t1.x, cs[i] * a.y + t1.y);
    H[(i + 1) * m + j] = make_double2(cs[i] * c2.x - t2.x, cs[i] * c2.y - t2.y);
  }
  const double2 a = H[j * m + j];
  const double aa = zabs(a);
  double c;
  double2 sv;
  if (hj1 == 0.0) {
    c = 1.0;
    sv = make_double2(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    sv = make_double2(1.0, 0.0);
  } else {
    const double rho = hypot(aa, hj1);
    c = aa / rho;
    sv = make_double2(a.x / aa * hj1 / rho, a.y / aa * hj1 / rho);  // (a/|a|) conj(hj1) / rho, hj1 real
  }
  cs[j] = c;
  sn[j] = sv;
  H[j * m + j] = make_double2(c * a.x + sv.x * hj1, c * a.y + sv.y * hj1);
  H[(j + 1) * m + j] = make_double2(0.0, 0.0);
  const double2 gj = g[j];
  const double2 t = zmul(zconj(sv), gj);
  g[j + 1] = make_double2(-t.x, -t.y);
  g[j] = make_double2(c * gj.x, c * gj.y);
  const double est = zabs(g[j + 1]);
  const int it = ++k.iters[b];
  k.jcount[b] = j + 1;
  if (!isfinite(est) || !isfinite(hj1) || !isfinite(zabs(H[j * m + j]))) {
    // discard this step: the last good least-squares solution is the previous column set
    k.status[b] = HELM_STATUS_BREAKDOWN_DEV;
    k.active[b] = 0;
    k.jcount[b] = 0;
    return;
  }
  k.vs[b * (m + 1) + j + 1] = hj1 > 0.0 ? (float)(1.0 / hj1) : 0.0f;
  const bool stop = est <= k.tol[b] || hj1 == 0.0 || it >= k.max_iters;
  if (stop) k.active[b] = 0;
  if (stop || j == m - 1) back_substitute(k, b, j + 1, yd, H, g);
}

// x += sum_{i < jcount} y_i Z_i, accumulated into the float-float pair (x_hi, x_lo)
__global__ __launch_bounds__(NT) void k_x_update(KrylovArgs k, c32* x_hi, c32* x_lo) {
  const int b = blockIdx.y;
  const int kk = k.jcount[b];
  if (kk == 0) return;
  const long long p0 = (long long)blockIdx.x * CH + threadIdx.x;
  c32 d[PPT];
#pragma unroll
  for (int t = 0; t < PPT; ++t) d[t] = make_float2(0.f, 0.f);
  for (int i0 = 0; i0 < kk; i0 += VCH) {
#pragma unroll
    for (int q = 0; q < VCH; ++q) {
      if (i0 + q < kk) {
        const c32 yi = k.y[b * k.m + i0 + q];
        const c32* zi = k.Z + zidx(k, b, i0 + q);
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
          const long long p = p0 + (long long)t * NT;
          if (p < k.N) d[t] = cfma(yi, zi[p], d[t]);
        }
      }
    }
  }
  c32* xh = x_hi + (long long)b * k.N;
  c32* xl = x_lo + (long long)b * k.N;
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    if (p < k.N) {
      const c32 h = xh[p], l = xl[p];
      ff re = ff_add({h.x, l.x}, ff_from(d[t].x));
      ff im = ff_add({h.y, l.y}, ff_from(d[t].y));
      xh[p] = make_float2(re.hi, im.hi);
      xl[p] = make_float2(re.lo, im.lo);
    }
  }
}

__global__ __launch_bounds__(NT) void k_residual_ff(int nrhs, KrylovArgs k, FFArgs a) {
  __shared__ float red[NWAVE];
  const TileId id = xcd_tile(blockIdx.x, nrhs, k.nblk, HELM_RHS_GROUP);
  const int b = id.b, blk = id.t;
  if (k.status && (k.status[b] != HELM_RUNNING || (k.bicg && k.active[b]))) return;
  const long long p0 = (long long)blk * CH + threadIdx.x;
  const int n = k.n, dim = k.dim;
  const c32* rb = a.rhs + (long long)b * a.rhs_stride;
  const c32* xh = a.x_zero ? nullptr : a.x_hi + (long long)b * k.N;
  const c32* xl = (a.x_zero || !a.x_lo) ? nullptr : a.x_lo + (long long)b * k.N;
  c32* ro = a.r_out + (long long)b * a.r_stride;
  float nrm = 0.f;
  Coord c = coord_of32((unsigned)p0, (unsigned)n, dim);
#pragma unroll 2
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    const Coord ct = c;
    coord_advance(c, NT, n, dim);
    if (p >= k.N) continue;
    const c32 rv = ff_residual_point(a, rb, xh, xl, p, ct, n, dim);
    ro[p] = cscale(rv, a.out_scale);
    nrm = fmaf(rv.x, rv.x, fmaf(rv.y, rv.y, nrm));
  }
  if (!k.P2) return;
  nrm = wave_sum(nrm);
  const int lane = threadIdx.x % HELM_WAVE, wave = threadIdx.x / HELM_WAVE;
  if (lane == 0) red[wave] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) s += red[q];
    k.P2[(long long)b * k.nblk + blk] = s;
  }
}

// The end of a restart cycle on a 2D grid in one pass: x += sum_{i < jcount}
// y_i Z_i (as k_x_update) and the true residual of the new x (as
// k_residual_ff), on a 62 x TY tile with a one-point ring, one column per
// lane.  The new float-float x of the region is kept in LDS for the stencil,
// so x is not read a second time; Z is read on the region (the ring adds
// 64 (TY + 2) / (62 TY) - 1 of it).  Every tile reads x on its ring, which
// neighbouring tiles own, so the new x goes to the other buffer of the pair
// (x0, x1): right-hand side b reads buffer xpar[b] and writes 1 - xpar[b],
// and k_finalize flips xpar[b] after the pass.  Same arithmetic per point as
// the two kernels; one partial squared norm per tile, k.P2[b][tile].
template <int TY>
__global__ __launch_bounds__(NT) void k_x_update_residual2(int nrhs, KrylovArgs k, FFArgs a, XPair x0, XPair x1) {
  constexpr int TX = 62, VY = TY + 2, RPI = NT / HELM_WAVE, IV = VY / RPI;
  static_assert(VY % RPI == 0, "whole row groups");
  __shared__ c32 sH[VY][HELM_WAVE];
  __shared__ c32 sL[VY][HELM_WAVE];
  __shared__ float red[NWAVE];
  const int n = k.n;
  const int tiles_x = (n + TX - 1) / TX;
  const unsigned tiles = (unsigned)(tiles_x * ((n + TY - 1) / TY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (k.status[b] != HELM_RUNNING) return;
  const int kk = k.jcount[b];
  const int fx0 = (id.t % tiles_x) * TX, fy0 = (id.t / tiles_x) * TY;
  const int lx = threadIdx.x % HELM_WAVE, r0 = threadIdx.x / HELM_WAVE;
  const int gx = fx0 - 1 + lx;
  const bool inx = gx >= 0 && gx < n;
  const bool tcol = lx >= 1 && lx <= TX && gx < n;
  const XPair src = k.xpar[b] ? x1 : x0, dst = k.xpar[b] ? x0 : x1;
  const c32* xh = src.hi + (long long)b * k.N;
  const c32* xl = src.lo + (long long)b * k.N;
  c32* oh = dst.hi + (long long)b * k.N;
  c32* ol = dst.lo + (long long)b * k.N;
  const c32* rb = a.rhs + (long long)b * a.rhs_stride;
  c32 hv[IV], lv[IV], d[IV], bv[IV], dh[IV], dl[IV];
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 - 1 + ly;
    const bool ok = inx && gy >= 0 && gy < n;
    const bool tp = ok && tcol && ly >= 1 && ly <= TY;
    const long long p = ok ? (long long)gy * n + gx : 0;
    hv[it] = ok ? xh[p] : make_float2(0.f, 0.f);
    lv[it] = ok ? xl[p] : make_float2(0.f, 0.f);
    bv[it] = tp ? rb[p] : make_float2(0.f, 0.f);
    dh[it] = tp ? a.d_hi[p] : make_float2(0.f, 0.f);
    dl[it] = tp ? a.d_lo[p] : make_float2(0.f, 0.f);
    d[it] = make_float2(0.f, 0.f);
  }
  // the sum in the order of i, as k_x_update; the rows of XG basis vectors are loaded
  // together (nearest in-grid column, no lane predicate: d of a lane outside the grid is
  // never used), then added in order
  constexpr int XG = 4;
  const unsigned ob = (unsigned)min(max(gx, 0), n - 1) * (unsigned)sizeof(c32);
  const int r0u = __builtin_amdgcn_readfirstlane(r0);  // uniform rows: scalar row bases
  for (int i0 = 0; i0 < kk; i0 += XG) {
    c32 zv[XG][IV];
#pragma unroll
    for (int u = 0; u < XG; ++u) {
      if (i0 + u >= kk) break;
      const c32* zi = k.Z + zidx(k, b, i0 + u);
#pragma unroll
      for (int it = 0; it < IV; ++it) {
        const int gy = fy0 - 1 + r0u + RPI * it;
        if (gy >= 0 && gy < n) zv[u][it] = at_byte(zi + (long long)gy * n, ob);
      }
    }
#pragma unroll
    for (int u = 0; u < XG; ++u) {
      if (i0 + u >= kk) break;
      const c32 yi = k.y[b * k.m + i0 + u];
#pragma unroll
      for (int it = 0; it < IV; ++it) {
        const int gy = fy0 - 1 + r0u + RPI * it;
        if (gy >= 0 && gy < n) d[it] = cfma(yi, zv[u][it], d[it]);
      }
    }
  }
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 - 1 + ly;
    if (!inx || gy < 0 || gy >= n) {
      sH[ly][lx] = make_float2(0.f, 0.f);
      sL[ly][lx] = make_float2(0.f, 0.f);
      continue;
    }
    if (kk > 0) {
      const ff re = ff_add({hv[it].x, lv[it].x}, ff_from(d[it].x));
      const ff im = ff_add({hv[it].y, lv[it].y}, ff_from(d[it].y));
      hv[it] = make_float2(re.hi, im.hi);
      lv[it] = make_float2(re.lo, im.lo);
    }
    if (tcol && ly >= 1 && ly <= TY) {  // the tile's points, updated or not, go to the other buffer
      const long long p = (long long)gy * n + gx;
      oh[p] = hv[it];
      ol[p] = lv[it];
    }
    sH[ly][lx] = hv[it];
    sL[ly][lx] = lv[it];
  }
  __syncthreads();
  c32* ro = a.r_out + (long long)b * a.r_stride;
  float nrm = 0.f;
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 - 1 + ly;
    if (!tcol || ly < 1 || ly > TY || gy >= n) continue;
    cff r = ff_scaled_rhs(a, bv[it]);
    cff ax = cff_mul(cff_make(dh[it], dl[it]), cff_make(sH[ly][lx], sL[ly][lx]));
    cff nb = {ff_from(0.f), ff_from(0.f)};  // the in-grid neighbours in the order of ff_residual_point
    if (gx > 0) nb = cff_add(nb, cff_make(sH[ly][lx - 1], sL[ly][lx - 1]));
    if (gx < n - 1) nb = cff_add(nb, cff_make(sH[ly][lx + 1], sL[ly][lx + 1]));
    if (gy > 0) nb = cff_add(nb, cff_make(sH[ly - 1][lx], sL[ly - 1][lx]));
    if (gy < n - 1) nb = cff_add(nb, cff_make(sH[ly + 1][lx], sL[ly + 1][lx]));
    ax = cff_sub(ax, nb);
    r = cff_sub(r, ax);
    const c32 rv = ff_round(r);
    ro[(long long)gy * n + gx] = cscale(rv, a.out_scale);
    nrm = fmaf(rv.x, rv.x, fmaf(rv.y, rv.y, nrm));
  }
  nrm = wave_sum(nrm);
  if (lx == 0) red[r0] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) s += red[q];
    k.P2[(long long)b * tiles + id.t] = s;
  }
}
// tile rows of the fused update and residual
#ifndef HELM_XRES_TY
#define HELM_XRES_TY 10
#endif
constexpr int XRES_TX = 62, XRES_TY = HELM_XRES_TY;

// Acceptance test of a learned preconditioner output z_j: partial sums of
// |v_j - A' z_j|^2 (v_j = vs_j V_j has unit norm); the residual itself is
// stored in resid[b] when resid is non-null.
__global__ __launch_bounds__(NT) void k_accept_partials(KrylovArgs k, int j, LevelArgs fine, VecSet resid) {
  __shared__ float red[NWAVE];
  const int b = blockIdx.x, blk = blockIdx.y;
  if (!k.active[b]) return;
  const long long p0 = (long long)blk * CH + threadIdx.x;
  const c32* z = k.Z + zidx(k, b, j);
  const c32* v = k.V + vidx(k, b, j);
  const float vsj = k.vs[b * (k.m + 1) + j];
  Coord c = coord_of32((unsigned)p0, (unsigned)fine.n, k.dim);
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    if (p < k.N) {
      const c32 D = diag_at(fine, p, ghosts_of(c, fine.n, k.dim), k.dim);
      const c32 d = csub(cscale(v[p], vsj), stencil_point(z, p, c, fine.n, k.dim, D));
      if (resid.p) resid.p[(long long)b * resid.stride + p] = d;
      s = fmaf(d.x, d.x, fmaf(d.y, d.y, s));
    }
    coord_advance(c, NT, fine.n, k.dim);
  }
  s = wave_sum(s);
  const int lane = threadIdx.x % HELM_WAVE, wave = threadIdx.x / HELM_WAVE;
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) t += red[q];
    k.P2[(long long)b * k.nblk + blk] = t;
  }
}

// mg_mask[b] = 1 where the learned output is rejected (||v - A z|| > tol or not finite)
__global__ __launch_bounds__(HELM_WAVE) void k_accept_decide(KrylovArgs k, double tol, int* mg_mask, int* fallbacks) {
  const int b = blockIdx.x;
  if (!k.active[b]) {
    if (threadIdx.x == 0) mg_mask[b] = 0;
    return;
  }
  double s = 0.0;
  for (int blk = threadIdx.x; blk < k.nblk; blk += HELM_WAVE) s += k.P2[(long long)b * k.nblk + blk];
  s = wave_sum_d(s);
  if (threadIdx.x != 0) return;
  const double ratio = sqrt(s);
  const int reject = !(ratio <= tol);
  mg_mask[b] = reject;
  fallbacks[b] += reject;
}

// Where the learned output was rejected: z_j = 0 and resid = v_j, so that the
// multigrid correction that follows is the plain cycle of v_j.
__global__ void k_reject_reset(KrylovArgs k, int j, const int* mg_mask, VecSet resid) {
  const int b = blockIdx.x;
  if (!k.active[b] || !mg_mask[b]) return;
  const float vsj = k.vs[b * (k.m + 1) + j];
  for (long long p = (long long)blockIdx.y * blockDim.x + threadIdx.x; p < k.N;
       p += (long long)gridDim.y * blockDim.x) {
    k.Z[zidx(k, b, j) + p] = make_float2(0.f, 0.f);
    resid.p[(long long)b * resid.stride + p] = cscale(k.V[vidx(k, b, j) + p], vsj);
  }
}

// After a true residual: decide convergence, else restart the cycle from r.
__global__ __launch_bounds__(HELM_WAVE) void k_finalize(KrylovArgs k, int first) {
  const int b = blockIdx.x;
  if (k.status[b] != HELM_RUNNING) return;
  double s = 0.0;
  for (int blk = threadIdx.x; blk < k.nres; blk += HELM_WAVE) s += k.P2[(long long)b * k.nres + blk];
  s = wave_sum_d(s);
  if (threadIdx.x != 0) return;
  if (k.flip_x) k.xpar[b] ^= 1;  // the pass wrote the new iterate to the other buffer
  const double rn = sqrt(s);
  k.jcount[b] = 0;
  k.active[b] = 0;
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
  k.vs[b * (k.m + 1)] = (float)(1.0 / rn);
  // the s-step basis W_1..W_m is used unscaled (the Arnoldi steps overwrite these)
  for (int i = 1; i <= k.m; ++i) k.vs[b * (k.m + 1) + i] = 1.0f;
  double2* g = k.g + (long long)b * (k.m + 1);
  g[0] = make_double2(rn, 0.0);
  for (int i = 1; i <= k.m; ++i) g[i] = make_double2(0.0, 0.0);
}

// ------------------------------------------------------------ s-step GMRES
// GMRES(m) with the same right preconditioner, written in s-step form: the
// basis of the Krylov space of A M is built without orthogonalisation,
//   W_0 = r / ||r||,  Z_j = M(W_j),  W_{j+1} = A Z_j   (j = 0 .. m-1),
// then the Gram matrix G = W^H W (one pass) gives W = Q R by Cholesky
// (G = R^H R) and the least-squares problem min ||r - sum_j y_j A Z_j|| becomes
// min || ||r|| R_00 e_0 - R[:, 1:] y || with R[:, 1:] upper Hessenberg, solved
// by the same Givens rotations as the Arnoldi form.  In exact arithmetic the
// iterates are those of GMRES(m); the basis is never orthogonalised, so a
// step costs one matvec (16 B per point) instead of two passes over the basis.

// W_{j+1} = A Z_j
__global__ __launch_bounds__(NT) void k_sstep_matvec(int nrhs, KrylovArgs k, int j, LevelArgs fine) {
  const TileId id = xcd_tile(blockIdx.x, nrhs, k.nblk, HELM_RHS_GROUP);
  const int b = id.b, blk = id.t;
  if (!k.active[b]) return;
  const long long p0 = (long long)blk * CH + threadIdx.x;
  const c32* z = k.Z + zidx(k, b, j);
  c32* w = k.V + vidx(k, b, j + 1);
  Coord c = coord_of32((unsigned)p0, (unsigned)fine.n, k.dim);
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const long long p = p0 + (long long)t * NT;
    if (p < k.N) w[p] = stencil_point(z, p, c, fine.n, k.dim, diag_at(fine, p, ghosts_of(c, fine.n, k.dim), k.dim));
    coord_advance(c, NT, fine.n, k.dim);
  }
}

// Block partials of the Gram matrix of (s_0 W_0, W_1, .., W_{M-1}, A Z_{M-1}):
// the last basis vector is formed in registers and never stored.  Entry
// (i, j), i <= j, in packed upper order, is sum conj(w_i) w_j, accumulated in
// FP64 from the first product: the basis is far from orthogonal (condition
// numbers up to ~1e6 at m = 12) and the Cholesky factor of G loses the
// square of that, so G must be the Gram matrix of the stored vectors to
// FP64 accuracy.
// Entry e of the packed upper triangle of an nv x nv matrix is (packed_row,
// packed_col); the loops fold to constants where e does.
__host__ __device__ constexpr int packed_row(int e, int nv) {
  int i = 0;
  while (e >= nv - i) e -= nv - i++;
  return i;
}
__host__ __device__ constexpr int packed_col(int e, int nv) {
  int i = 0;
  while (e >= nv - i) e -= nv - i++;
  return i + e;
}

constexpr int GP = 256;  // points staged per step (measured: 64 slower, 128 ~5% slower)

// acc[U] += conj(w_i) w_j for the entry e = G + U NWAVE = (i, j) and the ones after it
template <int NV, int G, int U>
__device__ __forceinline__ void gram_entries(double2* acc, const double2* wd) {
  constexpr int NE = NV * (NV + 1) / 2, e = G + U * NWAVE;
  if constexpr (e < NE) {
    constexpr int i = packed_row(e, NV), j = packed_col(e, NV);
    acc[U].x = fma(wd[i].x, wd[j].x, fma(wd[i].y, wd[j].y, acc[U].x));
    acc[U].y = fma(wd[i].x, wd[j].y, fma(-wd[i].y, wd[j].x, acc[U].y));
    gram_entries<NV, G, U + 1>(acc, wd);
  }
}

// Wave G of the block accumulates the entries e = G, G + NWAVE, ... of the
// packed triangle over the staged points (lanes q and q + 64).
template <int M, int G>
__device__ __forceinline__ void gram_accumulate(double2* acc, const c32 (*buf)[GP], int lane) {
  constexpr int NV = M + 1;
#pragma unroll 1
  for (int h = 0; h < GP / HELM_WAVE; ++h) {
    const int q = lane + h * HELM_WAVE;
    double2 wd[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const c32 w = buf[v][q];
      wd[v] = make_double2((double)w.x, (double)w.y);
    }
    gram_entries<NV, G, 0>(acc, wd);
  }
}

// Block partials of the Gram matrix of (s_0 W_0, W_1, .., W_{M-1}, A Z_{M-1}):
// the last basis vector is formed in registers and never stored.  Entry
// (i, j), i <= j, in packed upper order, is sum conj(w_i) w_j, accumulated in
// FP64 from the first product: the basis is far from orthogonal (condition
// numbers up to ~1e6 at m = 12) and the Cholesky factor of G loses the
// square of that, so G must be the Gram matrix of the stored vectors to
// FP64 accuracy.  The block stages GP points of all M + 1 vectors in LDS
// (the next step's loads in flight meanwhile); each wave keeps a quarter of
// the entries, so the FP64 accumulators fit with several waves per SIMD.
template <int M>
__global__ __launch_bounds__(NT) void k_sstep_gram(int nrhs, KrylovArgs k, LevelArgs fine, double2* part) {
  constexpr int NV = M + 1, NE = NV * (NV + 1) / 2, NU = (NE + NWAVE - 1) / NWAVE;
  constexpr int STEPS = CH / GP;
  static_assert(CH % GP == 0 && GP % HELM_WAVE == 0, "staging shape");
  __shared__ c32 buf[2][NV][GP];
  const TileId id = xcd_tile(blockIdx.x, nrhs, k.nblk, HELM_RHS_GROUP);
  const int b = id.b, blk = id.t;
  if (!k.active[b]) return;
  const float s0 = k.vs[b * (k.m + 1)];
  const long long p0 = (long long)blk * CH;
  const c32* z = k.Z + zidx(k, b, M - 1);
  const c32* vb = k.V + vidx(k, b, 0);
  // Item v of this thread is point q = threadIdx.x of basis vector v (NT == GP).  The
  // prefetch of the next step only loads: the vectors at the nearest valid point and, for
  // the last vector, Z's stencil values and the coefficient; the stencil, the zeros past N
  // and the scale of W_0 are applied when the step is stored to LDS, after the current
  // step's accumulation, so that no arithmetic waits on the loads in flight.
  static_assert(NT == GP, "one point per thread and vector");
  constexpr int NS = 7;  // stencil values of the last vector: centre, x-, x+, y-, y+, z-, z+
  struct Pre {
    c32 w[M];
    c32 st[NS];
    c32 coef;
    long long p;
  };
  const int dim = k.dim, nf = fine.n;
  const long long nf2 = (long long)nf * nf;
  auto load = [&](int step, Pre& o) {
    const long long p = p0 + (long long)step * GP + threadIdx.x;
    const long long pc = p < k.N ? p : k.N - 1;  // nearest valid point
    o.p = p;
#pragma unroll
    for (int v = 0; v < M; ++v) o.w[v] = vb[(long long)v * k.N + pc];
    const Coord c = coord_of32((unsigned)pc, (unsigned)nf, dim);
    const int xm = c.x > 0, xp = c.x < nf - 1, ym = c.y > 0, yp = c.y < nf - 1;
    o.st[0] = z[pc];
    o.st[1] = z[pc - xm];
    o.st[2] = z[pc + xp];
    o.st[3] = z[pc - (long long)ym * nf];
    o.st[4] = z[pc + (long long)yp * nf];
    if (dim == 3) {
      const int zm = c.z > 0, zp = c.z < nf - 1;
      o.st[5] = z[pc - zm * nf2];
      o.st[6] = z[pc + zp * nf2];
    }
    o.coef = fine.coef[pc];
  };
  auto store = [&](int slot, const Pre& o) {
    const bool ok = o.p < k.N;
    const long long pc = ok ? o.p : k.N - 1;
#pragma unroll
    for (int v = 0; v < M; ++v) {
      c32 w = ok ? o.w[v] : make_float2(0.f, 0.f);
      if (v == 0) w = cscale(w, s0);
      buf[slot][v][threadIdx.x] = w;
    }
    // the last basis vector A Z_{M-1} at the point: the arithmetic of stencil_point and
    // diag_at on the values loaded above
    const Coord c = coord_of32((unsigned)pc, (unsigned)nf, dim);
    const int ng = ghosts_of(c, nf, dim);
    const c32 D = make_float2(2.0f * dim - o.coef.x - ng * fine.ghost.x, -o.coef.y - ng * fine.ghost.y);
    const int xm = c.x > 0, xp = c.x < nf - 1, ym = c.y > 0, yp = c.y < nf - 1;
    const c32 a = o.st[1], bb = o.st[2], cc = o.st[3], d = o.st[4];
    c32 nb = make_float2(xm * a.x + xp * bb.x + ym * cc.x + yp * d.x, xm * a.y + xp * bb.y + ym * cc.y + yp * d.y);
    if (dim == 3) {
      const int zm = c.z > 0, zp = c.z < nf - 1;
      nb.x += zm * o.st[5].x + zp * o.st[6].x;
      nb.y += zm * o.st[5].y + zp * o.st[6].y;
    }
    buf[slot][M][threadIdx.x] = ok ? csub(cmul(D, o.st[0]), nb) : make_float2(0.f, 0.f);
  };
  double2 acc[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) acc[u] = make_double2(0.0, 0.0);
  const int lane = threadIdx.x % HELM_WAVE, wave = threadIdx.x / HELM_WAVE;
  const int steps = (int)min((long long)STEPS, (k.N - p0 + GP - 1) / GP);
  Pre pre;
  load(0, pre);
  for (int st = 0; st < steps; ++st) {
    store(st & 1, pre);
    if (st + 1 < steps) load(st + 1, pre);
    __syncthreads();
    const c32(*cur)[GP] = buf[st & 1];
    switch (wave) {
      case 0: gram_accumulate<M, 0>(acc, cur, lane); break;
      case 1: gram_accumulate<M, 1>(acc, cur, lane); break;
      case 2: gram_accumulate<M, 2>(acc, cur, lane); break;
      default: gram_accumulate<M, 3>(acc, cur, lane); break;
    }
  }
  static_assert(NWAVE == 4, "one entry group per wave");
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int e = wave + u * NWAVE;
    const double sx = wave_sum_d(acc[u].x), sy = wave_sum_d(acc[u].y);
    if (lane == 0 && e < NE) part[((long long)b * k.nblk + blk) * NE + e] = make_double2(sx, sy);
  }
}

// Per right-hand side (one wavefront): reduce the Gram partials (FP64, fixed
// order), Cholesky G = R^H R, Givens rotations of the Hessenberg R[:, 1:],
// the residual estimate of every leading size, and the least-squares solution
// for the smallest size that meets the inner tolerance (else all usable
// columns).  A column whose Cholesky pivot vanishes (the Krylov space is
// exhausted to working precision) ends the usable basis there.
template <int M>
__global__ __launch_bounds__(NT) void k_sstep_solve(KrylovArgs k, const double2* part) {
  constexpr int NV = M + 1, NE = NV * (NV + 1) / 2, S = NT / NE;
  static_assert(S >= 1, "one thread per entry at least");
  __shared__ double2 G[NE];
  __shared__ double2 red[S][NE];
  __shared__ double2 R[NV][NV];  // Cholesky factor (LDS: a per-thread array of this size would spill)
  __shared__ double2 yd[M];
  const int b = blockIdx.x;
  if (!k.active[b]) return;
  // thread (e, s) sums the partials of entry e over blocks s, s + S, ... (four loads in
  // flight), then the S sums of each entry are added in a fixed order
  if (threadIdx.x < NE * S) {
    const int e = threadIdx.x % NE, s0 = threadIdx.x / NE;
    const double2* pb = part + (long long)b * k.nblk * NE + e;
    double2 a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = make_double2(0.0, 0.0);
    int blk = s0;
    for (; blk + 3 * S < k.nblk; blk += 4 * S) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 v = pb[(long long)(blk + u * S) * NE];
        a[u].x += v.x;
        a[u].y += v.y;
      }
    }
    for (; blk < k.nblk; blk += S) {
      const double2 v = pb[(long long)blk * NE];
      a[0].x += v.x;
      a[0].y += v.y;
    }
    red[s0][e] = make_double2((a[0].x + a[1].x) + (a[2].x + a[3].x), (a[0].y + a[1].y) + (a[2].y + a[3].y));
  }
  __syncthreads();
  if (threadIdx.x < NE) {
    double2 g = red[0][threadIdx.x];
    for (int q = 1; q < S; ++q) g = make_double2(g.x + red[q][threadIdx.x].x, g.y + red[q][threadIdx.x].y);
    G[threadIdx.x] = g;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int m = k.m;
  // packed index of (i, j), i <= j
  auto gi = [](int i, int j) { return i * NV - i * (i - 1) / 2 + (j - i); };
  int keep = NV;  // usable leading columns of W
  bool finite = true;
  for (int j = 0; j < NV && keep == NV; ++j) {
    double d = G[gi(j, j)].x;
    const double gjj = d;
    for (int i = 0; i < j; ++i) d -= R[i][j].x * R[i][j].x + R[i][j].y * R[i][j].y;
    if (!isfinite(d) || !isfinite(gjj)) {
      finite = false;
      keep = j;
      break;
    }
    if (!(d > 1e-13 * gjj) || !(gjj > 0.0)) {
      keep = j;
      break;
    }
    const double rjj = sqrt(d);
    R[j][j] = make_double2(rjj, 0.0);
    for (int l = j + 1; l < NV; ++l) {
      double2 v = G[gi(j, l)];
      for (int i = 0; i < j; ++i) {
        const double2 t = zmul(zconj(R[i][j]), R[i][l]);
        v.x -= t.x;
        v.y -= t.y;
      }
      R[j][l] = make_double2(v.x / rjj, v.y / rjj);
    }
  }
  const int mm = keep - 1;  // usable preconditioned directions
  k.iters[b] += M;           // preconditioner applications performed
  if (!finite || mm < 1) {
    k.status[b] = HELM_STATUS_BREAKDOWN_DEV;
    k.jcount[b] = 0;
    k.active[b] = 0;
    return;
  }
  // the rotated Hessenberg, rotations and right-hand side stay in LDS (a single
  // thread's chain of dependent global accesses would dominate the kernel)
  __shared__ double2 H[(M + 1) * M];
  __shared__ double cs[M];
  __shared__ double2 sn[M];
  __shared__ double2 g[M + 1];
  const double rn = 1.0 / (double)k.vs[b * (m + 1)];
  for (int i = 0; i <= m; ++i) g[i] = make_double2(0.0, 0.0);
  g[0] = make_double2(rn * R[0][0].x, 0.0);
  int kstar = mm;
  for (int col = 0; col < mm; ++col) {
    // column col of the Hessenberg: R[0..col+1][col+1]
    for (int i = 0; i <= col + 1; ++i) H[i * m + col] = R[i][col + 1];
    for (int i = 0; i < col; ++i) {
      const double2 a = H[i * m + col], c2 = H[(i + 1) * m + col];
      const double2 t1 = zmul(sn[i], c2);
      const double2 t2 = zmul(zconj(sn[i]), a);
      H[i * m + col] = make_double2(cs[i] * a.x + t1.x, cs[i] * a.y + t1.y);
      H[(i + 1) * m + col] = make_double2(cs[i] * c2.x - t2.x, cs[i] * c2.y - t2.y);
    }
    const double2 a = H[col * m + col];
    const double2 hb = H[(col + 1) * m + col];
    const double aa = zabs(a), bb = zabs(hb);
    double cr;
    double2 sv;
    if (bb == 0.0) {
      cr = 1.0;
      sv = make_double2(0.0, 0.0);
    } else if (aa == 0.0) {
      cr = 0.0;
      sv = zconj(make_double2(hb.x / bb, hb.y / bb));
    } else {
      const double rho = hypot(aa, bb);
      cr = aa / rho;
      const double2 ph = make_double2(a.x / aa, a.y / aa);
      sv = zmul(ph, make_double2(hb.x / rho, -hb.y / rho));  // (a/|a|) conj(hb) / rho
    }
    cs[col] = cr;
    sn[col] = sv;
    const double2 t = zmul(sv, hb);
    H[col * m + col] = make_double2(cr * a.x + t.x, cr * a.y + t.y);
    H[(col + 1) * m + col] = make_double2(0.0, 0.0);
    const double2 gj = g[col];
    const double2 t2 = zmul(zconj(sv), gj);
    g[col + 1] = make_double2(-t2.x, -t2.y);
    g[col] = make_double2(cr * gj.x, cr * gj.y);
    if (zabs(g[col + 1]) <= k.tol[b]) {
      kstar = col + 1;
      break;
    }
  }
  k.jcount[b] = kstar;
  k.active[b] = 0;
  back_substitute(k, b, kstar, yd, H, g);
}

__global__ void k_status_init(KrylovArgs k, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  k.status[b] = HELM_RUNNING;
  k.active[b] = 0;
  k.jcount[b] = 0;
  k.iters[b] = 0;
  k.relres[b] = 0.0;
}

inline unsigned nblk_of(long long N) { return (unsigned)((N + CH - 1) / CH); }

}  // namespace

int krylov_blocks_per_rhs(long long N) { return (int)nblk_of(N); }
int krylov_max_restart() { return MAXM; }
int sstep_max_restart() { return SSTEP_MAXM; }
long long sstep_gram_entries(int m) { return (long long)(m + 1) * (m + 2) / 2; }

namespace {
// W_{j+1} = A Z_j in 3D, marching in z: a 64 x 8 column over MZ planes, two
// points per thread.  Each thread keeps its points' values of the planes
// below, at and above in registers (the next plane's loads in flight while
// the current one is formed); the in-plane neighbours come from an LDS copy
// of the plane and a one-point ring.  Each plane of Z_j is read once per
// column (the flat kernel's z-neighbours, a plane apart, mostly miss the L2).
constexpr int MX = 64, MY = 8, MZ = 16, MT = 256;
__global__ __launch_bounds__(MT) void k_matvec_march3(int nrhs, KrylovArgs k, int j, LevelArgs fine) {
  __shared__ c32 sP[MY + 2][MX + 2];
  const int n = fine.n;
  const int tx_n = (n + MX - 1) / MX, ty_n = (n + MY - 1) / MY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((n + MZ - 1) / MZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (!k.active[b]) return;
  const int x0 = (id.t % tx_n) * MX, y0 = ((id.t / tx_n) % ty_n) * MY, z0 = (id.t / (tx_n * ty_n)) * MZ;
  const int z1 = min(n, z0 + MZ);
  const c32* zv = k.Z + zidx(k, b, j);
  c32* wv = k.V + vidx(k, b, j + 1);
  const long long n2 = (long long)n * n;
  // own points (tx + 32 h, ty), h = 0, 1
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  bool own[2];
  long long o[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int gx = x0 + tx + 32 * h, gy = y0 + ty;
    own[h] = gx < n && gy < n;
    o[h] = own[h] ? (long long)gy * n + gx : 0;
  }
  // ring point of this thread (LDS coordinates), if any: 2 (MX + 2) + 2 MY of them
  int rx = -1, ry = -1;
  {
    const int t = threadIdx.x;
    if (t < MX + 2) rx = t, ry = 0;
    else if (t < 2 * (MX + 2)) rx = t - (MX + 2), ry = MY + 1;
    else if (t < 2 * (MX + 2) + MY) rx = 0, ry = t - 2 * (MX + 2) + 1;
    else if (t < 2 * (MX + 2) + 2 * MY) rx = MX + 1, ry = t - 2 * (MX + 2) - MY + 1;
  }
  const int rgx = x0 - 1 + rx, rgy = y0 - 1 + ry;
  const bool ring = rx >= 0 && rgx >= 0 && rgx < n && rgy >= 0 && rgy < n;
  const long long ro = ring ? (long long)rgy * n + rgx : 0;
  auto at = [&](bool ok, int z, long long off) {
    return ok && z >= 0 && z < n ? zv[z * n2 + off] : make_float2(0.f, 0.f);
  };
  c32 zm[2], zc[2], zp[2], kc[2];
  c32 zr = at(ring, z0, ro);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    zm[h] = at(own[h], z0 - 1, o[h]);
    zc[h] = at(own[h], z0, o[h]);
    zp[h] = at(own[h], z0 + 1, o[h]);
    kc[h] = own[h] ? fine.coef[z0 * n2 + o[h]] : make_float2(0.f, 0.f);
  }
  for (int z = z0; z < z1; ++z) {
#pragma unroll
    for (int h = 0; h < 2; ++h) sP[ty + 1][tx + 1 + 32 * h] = zc[h];
    if (rx >= 0) sP[ry][rx] = zr;
    // the next plane's loads
    c32 zn[2], kn[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      zn[h] = at(own[h], z + 2, o[h]);
      kn[h] = own[h] && z + 1 < n ? fine.coef[(z + 1) * n2 + o[h]] : make_float2(0.f, 0.f);
    }
    const c32 zrn = at(ring, z + 1, ro);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!own[h]) continue;
      const int lx = tx + 1 + 32 * h, ly = ty + 1;
      const int ng = ghosts3(x0 + tx + 32 * h, y0 + ty, z, n);
      const c32 D = make_float2(6.0f - kc[h].x - ng * fine.ghost.x, -kc[h].y - ng * fine.ghost.y);
      const c32 nb = cadd(cadd(cadd(sP[ly][lx - 1], sP[ly][lx + 1]), cadd(sP[ly - 1][lx], sP[ly + 1][lx])),
                          cadd(zm[h], zp[h]));
      wv[z * n2 + o[h]] = csub(cmul(D, zc[h]), nb);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      zm[h] = zc[h];
      zc[h] = zp[h];
      zp[h] = zn[h];
      kc[h] = kn[h];
    }
    zr = zrn;
  }
}

// The float-float true residual in 3D, marching in z (the layout of
// k_matvec_march3): x_hi and x_lo of the planes below, at and above in registers,
// the in-plane neighbours from LDS copies of the plane with a one-point ring.
// Same arithmetic per point as ff_residual_point (in-grid neighbours in the same
// order); one partial squared norm per column tile, k.P2[b][tile].
__global__ __launch_bounds__(MT) void k_residual_ff_march3(int nrhs, KrylovArgs k, FFArgs a) {
  __shared__ c32 sH[MY + 2][MX + 2];
  __shared__ c32 sL[MY + 2][MX + 2];
  __shared__ float red[NWAVE];
  const int n = k.n;
  const int tx_n = (n + MX - 1) / MX, ty_n = (n + MY - 1) / MY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((n + MZ - 1) / MZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (k.status && (k.status[b] != HELM_RUNNING || (k.bicg && k.active[b]))) return;
  const int x0 = (id.t % tx_n) * MX, y0 = ((id.t / tx_n) % ty_n) * MY, z0 = (id.t / (tx_n * ty_n)) * MZ;
  const int z1 = min(n, z0 + MZ);
  const c32* xh = a.x_hi + (long long)b * k.N;
  const c32* xl = a.x_lo ? a.x_lo + (long long)b * k.N : nullptr;
  const c32* rb = a.rhs + (long long)b * a.rhs_stride;
  c32* ro = a.r_out + (long long)b * a.r_stride;
  const long long n2 = (long long)n * n;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  bool own[2];
  long long o[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int gx = x0 + tx + 32 * h, gy = y0 + ty;
    own[h] = gx < n && gy < n;
    o[h] = own[h] ? (long long)gy * n + gx : 0;
  }
  int rx = -1, ry = -1;  // this thread's ring point (LDS coordinates), if any
  {
    const int t = threadIdx.x;
    if (t < MX + 2) rx = t, ry = 0;
    else if (t < 2 * (MX + 2)) rx = t - (MX + 2), ry = MY + 1;
    else if (t < 2 * (MX + 2) + MY) rx = 0, ry = t - 2 * (MX + 2) + 1;
    else if (t < 2 * (MX + 2) + 2 * MY) rx = MX + 1, ry = t - 2 * (MX + 2) - MY + 1;
  }
  const int rgx = x0 - 1 + rx, rgy = y0 - 1 + ry;
  const bool ring = rx >= 0 && rgx >= 0 && rgx < n && rgy >= 0 && rgy < n;
  const long long rof = ring ? (long long)rgy * n + rgx : 0;
  const c32 zero = make_float2(0.f, 0.f);
  auto hi = [&](bool ok, int z, long long off) { return ok && z >= 0 && z < n ? xh[z * n2 + off] : zero; };
  auto lo = [&](bool ok, int z, long long off) { return ok && xl && z >= 0 && z < n ? xl[z * n2 + off] : zero; };
  c32 hm[2], hc[2], hp[2], lm[2], lc[2], lp[2], dh[2], dl[2], bc[2];
  c32 rh = hi(ring, z0, rof), rl = lo(ring, z0, rof);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    hm[h] = hi(own[h], z0 - 1, o[h]);
    lm[h] = lo(own[h], z0 - 1, o[h]);
    hc[h] = hi(own[h], z0, o[h]);
    lc[h] = lo(own[h], z0, o[h]);
    hp[h] = hi(own[h], z0 + 1, o[h]);
    lp[h] = lo(own[h], z0 + 1, o[h]);
    const long long p = z0 * n2 + o[h];
    dh[h] = own[h] ? a.d_hi[p] : zero;
    dl[h] = own[h] ? a.d_lo[p] : zero;
    bc[h] = own[h] ? rb[p] : zero;
  }
  float nrm = 0.f;
  for (int z = z0; z < z1; ++z) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      sH[ty + 1][tx + 1 + 32 * h] = hc[h];
      sL[ty + 1][tx + 1 + 32 * h] = lc[h];
    }
    if (rx >= 0) {
      sH[ry][rx] = rh;
      sL[ry][rx] = rl;
    }
    // the next plane's loads
    c32 hn[2], ln[2], dhn[2], dln[2], bn[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      hn[h] = hi(own[h], z + 2, o[h]);
      ln[h] = lo(own[h], z + 2, o[h]);
      const bool nx = own[h] && z + 1 < n;
      const long long p = nx ? (z + 1) * n2 + o[h] : 0;
      dhn[h] = nx ? a.d_hi[p] : zero;
      dln[h] = nx ? a.d_lo[p] : zero;
      bn[h] = nx ? rb[p] : zero;
    }
    const c32 rhn = hi(ring, z + 1, rof), rln = lo(ring, z + 1, rof);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!own[h]) continue;
      const int lx = tx + 1 + 32 * h, ly = ty + 1, gx = x0 + tx + 32 * h, gy = y0 + ty;
      cff r = ff_scaled_rhs(a, bc[h]);
      cff ax = cff_mul(cff_make(dh[h], dl[h]), cff_make(hc[h], lc[h]));
      cff nb = {ff_from(0.f), ff_from(0.f)};  // the in-grid neighbours in the order of ff_residual_point
      if (gx > 0) nb = cff_add(nb, cff_make(sH[ly][lx - 1], sL[ly][lx - 1]));
      if (gx < n - 1) nb = cff_add(nb, cff_make(sH[ly][lx + 1], sL[ly][lx + 1]));
      if (gy > 0) nb = cff_add(nb, cff_make(sH[ly - 1][lx], sL[ly - 1][lx]));
      if (gy < n - 1) nb = cff_add(nb, cff_make(sH[ly + 1][lx], sL[ly + 1][lx]));
      if (z > 0) nb = cff_add(nb, cff_make(hm[h], lm[h]));
      if (z < n - 1) nb = cff_add(nb, cff_make(hp[h], lp[h]));
      ax = cff_sub(ax, nb);
      r = cff_sub(r, ax);
      const c32 rv = ff_round(r);
      ro[z * n2 + o[h]] = cscale(rv, a.out_scale);
      nrm = fmaf(rv.x, rv.x, fmaf(rv.y, rv.y, nrm));
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      hm[h] = hc[h];
      lm[h] = lc[h];
      hc[h] = hp[h];
      lc[h] = lp[h];
      hp[h] = hn[h];
      lp[h] = ln[h];
      dh[h] = dhn[h];
      dl[h] = dln[h];
      bc[h] = bn[h];
    }
    rh = rhn;
    rl = rln;
  }
  if (!k.P2) return;
  nrm = wave_sum(nrm);
  const int lane = threadIdx.x % HELM_WAVE, wave = threadIdx.x / HELM_WAVE;
  if (lane == 0) red[wave] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) s += red[q];
    k.P2[(long long)b * tiles + id.t] = s;
  }
}
}  // namespace

void launch_sstep_matvec(hipStream_t s, int B, const KrylovArgs& k, int j, const LevelArgs& fine) {
  if (k.dim == 3) {
    const int n = fine.n;
    const int tiles = ((n + MX - 1) / MX) * ((n + MY - 1) / MY) * ((n + MZ - 1) / MZ);
    hipLaunchKernelGGL(k_matvec_march3, dim3(B * tiles), dim3(MT), 0, s, B, k, j, fine);
    return;
  }
  hipLaunchKernelGGL(k_sstep_matvec, dim3(B * k.nblk), dim3(NT), 0, s, B, k, j, fine);
}

namespace {
template <int M>
void sstep_tail(hipStream_t s, int B, const KrylovArgs& k, const LevelArgs& fine, double2* part) {
  hipLaunchKernelGGL(k_sstep_gram<M>, dim3(B * k.nblk), dim3(NT), 0, s, B, k, fine, part);
  hipLaunchKernelGGL(k_sstep_solve<M>, dim3(B), dim3(NT), 0, s, k, (const double2*)part);
}
}  // namespace

void launch_sstep_gram_solve(hipStream_t s, int B, const KrylovArgs& k, const LevelArgs& fine, double2* part) {
  switch (k.m) {
    case 1: sstep_tail<1>(s, B, k, fine, part); break;
    case 2: sstep_tail<2>(s, B, k, fine, part); break;
    case 3: sstep_tail<3>(s, B, k, fine, part); break;
    case 4: sstep_tail<4>(s, B, k, fine, part); break;
    case 5: sstep_tail<5>(s, B, k, fine, part); break;
    case 6: sstep_tail<6>(s, B, k, fine, part); break;
    case 7: sstep_tail<7>(s, B, k, fine, part); break;
    case 8: sstep_tail<8>(s, B, k, fine, part); break;
    case 9: sstep_tail<9>(s, B, k, fine, part); break;
    case 10: sstep_tail<10>(s, B, k, fine, part); break;
    case 11: sstep_tail<11>(s, B, k, fine, part); break;
    default: sstep_tail<12>(s, B, k, fine, part); break;
  }
}

void launch_arnoldi_dots(hipStream_t s, int B, const KrylovArgs& k, int j, const LevelArgs* fine, int with_matvec) {
  LevelArgs lv = fine ? *fine : LevelArgs{};
  hipLaunchKernelGGL(k_arnoldi_dots, dim3(B * k.nblk), dim3(NT), 0, s, B, k, j, lv, with_matvec);
}
void launch_arnoldi_reduce(hipStream_t s, int B, const KrylovArgs& k, int j, int accumulate) {
  hipLaunchKernelGGL(k_arnoldi_reduce, dim3(B), dim3(NT), 0, s, k, j, accumulate);
}
void launch_arnoldi_update(hipStream_t s, int B, const KrylovArgs& k, int j) {
  hipLaunchKernelGGL(k_arnoldi_update, dim3(k.nblk, B), dim3(NT), 0, s, k, j);
}
void launch_givens(hipStream_t s, int B, const KrylovArgs& k, int j) {
  hipLaunchKernelGGL(k_givens, dim3(B), dim3(HELM_WAVE), 0, s, k, j);
}
void launch_x_update(hipStream_t s, int B, const KrylovArgs& k, c32* x_hi, c32* x_lo) {
  hipLaunchKernelGGL(k_x_update, dim3(k.nblk, B), dim3(NT), 0, s, k, x_hi, x_lo);
}
int krylov_residual_partials(const KrylovArgs& k, int x_zero) {
  if (k.dim != 3 || x_zero) return k.nblk;
  const int n = k.n;
  return ((n + MX - 1) / MX) * ((n + MY - 1) / MY) * ((n + MZ - 1) / MZ);
}
void launch_residual_ff(hipStream_t s, int B, const KrylovArgs& k, const c32* rhs, long long rhs_stride,
                        int conj_rhs, const c32* x_hi, const c32* x_lo, int x_zero, const c32* d_hi,
                        const c32* d_lo, float h2_hi, float h2_lo, c32* r_out, long long r_stride, float out_scale) {
  FFArgs a{rhs, rhs_stride, conj_rhs, x_hi, x_lo, x_zero, d_hi, d_lo, h2_hi, h2_lo, r_out, r_stride, out_scale};
  if (k.dim == 3 && !x_zero) {  // the stencil's z-neighbours through registers
    hipLaunchKernelGGL(k_residual_ff_march3, dim3(B * krylov_residual_partials(k, 0)), dim3(MT), 0, s, B, k, a);
    return;
  }
  hipLaunchKernelGGL(k_residual_ff, dim3(B * k.nblk), dim3(NT), 0, s, B, k, a);
}
int krylov_xres_tiles(int n) { return ((n + XRES_TX - 1) / XRES_TX) * ((n + XRES_TY - 1) / XRES_TY); }
void launch_x_update_residual(hipStream_t s, int B, const KrylovArgs& k, XPair x0, XPair x1, const c32* rhs,
                              long long rhs_stride, int conj_rhs, const c32* d_hi, const c32* d_lo, float h2_hi,
                              float h2_lo, c32* r_out, long long r_stride) {
  FFArgs a{rhs, rhs_stride, conj_rhs, nullptr, nullptr, 0, d_hi, d_lo, h2_hi, h2_lo, r_out, r_stride, 1.0f};
  hipLaunchKernelGGL(k_x_update_residual2<XRES_TY>, dim3(B * krylov_xres_tiles(k.n)), dim3(NT), 0, s, B, k, a, x0,
                     x1);
}
void launch_finalize(hipStream_t s, int B, const KrylovArgs& k, int first) {
  hipLaunchKernelGGL(k_finalize, dim3(B), dim3(HELM_WAVE), 0, s, k, first);
}
void launch_accept(hipStream_t s, int B, const KrylovArgs& k, int j, const LevelArgs& fine, double tol, int* mg_mask,
                   int* fallbacks, VecSet resid) {
  hipLaunchKernelGGL(k_accept_partials, dim3(B, k.nblk), dim3(NT), 0, s, k, j, fine, resid);
  hipLaunchKernelGGL(k_accept_decide, dim3(B), dim3(HELM_WAVE), 0, s, k, tol, mg_mask, fallbacks);
}
void launch_reject_reset(hipStream_t s, int B, const KrylovArgs& k, int j, const int* mg_mask, VecSet resid) {
  const long long nb = (k.N + 255) / 256;
  hipLaunchKernelGGL(k_reject_reset, dim3(B, (unsigned)(nb < 65535 ? nb : 65535)), dim3(256), 0, s, k, j, mg_mask, resid);
}
void launch_status_init(hipStream_t s, int B, const KrylovArgs& k) {
  hipLaunchKernelGGL(k_status_init, dim3((B + 63) / 64), dim3(64), 0, s, k, B);
}
