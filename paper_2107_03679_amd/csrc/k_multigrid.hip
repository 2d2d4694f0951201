// Multigrid kernels for the shifted operator K'_l = -Lap'_l - kappa c_l
// (h_l^2-scaled, Sec. IV-B/IV-C):
//  * fused 2D legs of a V-cycle started from a zero guess with one pre- and
//    one post-relaxation (the paper's nu1 = nu2 = 1, omega_S = 0.8):
//      down: v1 = w D^-1 r;  rc = 4 R (r - K v1)          (LDS tile, 2-cell halo)
//      up:   v2 = w D^-1 r + P e;  z = v2 + w D^-1 (r - K v2)
//    v1 is recomputed by the up-leg instead of being stored.
//  * generic kernels (any dimension, any nu, W-cycles): Jacobi sweeps
//    (eq. dampedJ), residual + full-weighting restriction, prolongation.
//  * the exact coarsest solve as a product with the explicit inverse.
// D = diag(K) includes the Sommerfeld ghost terms: D = 2d - coef - g * #ghosts.
#include "dev_common.h"
#include "kernels.h"

namespace {


// ------------------------------------------------------------ fused 2D legs
// Down-leg on a TCX x TCY tile of coarse points (fine footprint 2 TCX + 1 wide):
//   stage 1: r and v1 = W r on the (2 TCX + 3) x (2 TCY + 3) halo region, v1 -> LDS
//   stage 2: s = r - K v1 = (1 - w) r + sum of in-grid neighbours of v1 (D v1 = w r)
//            on the (2 TCX + 1) x (2 TCY + 1) interior, by the thread that holds r
//   stage 3: rc = 4 R s (scaled coarse right-hand side)
// With RES the leg starts a repeated visit of the level from the current
// solution e (Alg. 2 with a non-zero guess, written as e + MG(r - K e, 0)):
// its right-hand side is r - K e, formed on the halo region from e on a
// one-point wider ring, so that the residual is never stored.
template <int TCX, int TCY, bool RES>
__global__ __launch_bounds__(TCX* TCY) void k_down_fused2(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv,
                                                           float omega, VecSet rc, int nc, const int* active,
                                                           VecSet ev) {
  constexpr int RX = 2 * TCX + 3, RY = 2 * TCY + 3;
  constexpr int SX = 2 * TCX + 1, SY = 2 * TCY + 1;
  constexpr int NT = TCX * TCY, NR = RX * RY, IT = (NR + NT - 1) / NT;
  constexpr int EX = RES ? RX + 2 : 1, EY = RES ? RY + 2 : 1;
  __shared__ c32 sV[RY][RX];
  __shared__ c32 sS[SY][SX];
  __shared__ c32 sE[EY][EX];
  const int n = lv.n;
  const int tiles_x = (nc + TCX - 1) / TCX;
  const unsigned tiles = (unsigned)(tiles_x * ((nc + TCY - 1) / TCY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int cx0 = (id.t % tiles_x) * TCX;
  const int cy0 = (id.t / tiles_x) * TCY;
  const int fx0 = 2 * cx0 - 2, fy0 = 2 * cy0 - 2;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  c32 rv[IT], wv[IT], kv[RES ? IT : 1];
  if constexpr (RES) {
    const c32* eb = ev.p + (long long)b * ev.stride;
    for (int idx = threadIdx.x; idx < EX * EY; idx += NT) {
      const int gx = fx0 - 1 + idx % EX, gy = fy0 - 1 + idx / EX;
      const bool ok = gx >= 0 && gx < n && gy >= 0 && gy < n;
      sE[idx / EX][idx % EX] = ok ? eb[(long long)gy * n + gx] : make_float2(0.f, 0.f);
    }
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int gx = fx0 + idx % RX, gy = fy0 + idx / RX;
    const bool ok = idx < NR && gx >= 0 && gx < n && gy >= 0 && gy < n;
    const long long p = ok ? (long long)gy * n + gx : 0;
    rv[it] = ok ? rb[p] : make_float2(0.f, 0.f);
    wv[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    if constexpr (RES) kv[it] = ok ? lv.coef[p] : make_float2(0.f, 0.f);
  }
  if constexpr (RES) __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    rv[it] = cscale(rv[it], sc);
    if constexpr (RES) {
      // r - K e with K e = D e - (sum of in-grid neighbours); sE is zero outside the grid
      const int lx = idx % RX + 1, ly = idx / RX + 1;
      const int gx = fx0 + idx % RX, gy = fy0 + idx / RX;
      if (idx < NR && gx >= 0 && gx < n && gy >= 0 && gy < n) {
        const int ng = ghosts2(gx, gy, n);
        const c32 D = make_float2(4.0f - kv[it].x - ng * lv.ghost.x, -kv[it].y - ng * lv.ghost.y);
        const c32 nb = cadd(cadd(sE[ly][lx - 1], sE[ly][lx + 1]), cadd(sE[ly - 1][lx], sE[ly + 1][lx]));
        rv[it] = cadd(csub(rv[it], cmul(D, sE[ly][lx])), nb);
      }
    }
    if (idx < NR) sV[idx / RX][idx % RX] = cmul(rv[it], wv[it]);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int lx = idx % RX, ly = idx / RX;
    if (idx >= NR || lx == 0 || lx == RX - 1 || ly == 0 || ly == RY - 1) continue;
    const int gx = fx0 + lx, gy = fy0 + ly;
    c32 s = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const c32 nb = cadd(cadd(sV[ly][lx - 1], sV[ly][lx + 1]), cadd(sV[ly - 1][lx], sV[ly + 1][lx]));
      s = cadd(cscale(rv[it], 1.0f - omega), nb);
    }
    sS[ly - 1][lx - 1] = s;
  }
  __syncthreads();
  const int tx = threadIdx.x % TCX, ty = threadIdx.x / TCX;
  const int I = cx0 + tx, J = cy0 + ty;
  if (I < nc && J < nc) {
    const int sx = 2 * tx + 1, sy = 2 * ty + 1;
    c32 acc = cscale(sS[sy][sx], 4.0f);
    acc = cadd(acc, cscale(cadd(cadd(sS[sy][sx - 1], sS[sy][sx + 1]), cadd(sS[sy - 1][sx], sS[sy + 1][sx])), 2.0f));
    acc = cadd(acc, cadd(cadd(sS[sy - 1][sx - 1], sS[sy - 1][sx + 1]), cadd(sS[sy + 1][sx - 1], sS[sy + 1][sx + 1])));
    // scaled coarse right-hand side: 4 * (1/16) * stencil sum
    rc.p[(long long)b * rc.stride + (long long)J * nc + I] = cscale(acc, 0.25f);
  }
}

// bilinear prolongation at fine point (gx, gy) from the LDS coarse tile whose
// origin is coarse point (cxs, cys) (printed formula of Sec. IV-C)
template <int CX>
__device__ __forceinline__ c32 prolong_lds(const c32 (*sE)[CX], int gx, int gy, int cxs, int cys) {
  const int I = (gx >> 1) - cxs, J = (gy >> 1) - cys;
  const int ox = gx & 1, oy = gy & 1;
  c32 pe = sE[J][I];
  if (ox && oy) return cscale(cadd(cadd(pe, sE[J][I + 1]), cadd(sE[J + 1][I], sE[J + 1][I + 1])), 0.25f);
  if (ox) return cscale(cadd(pe, sE[J][I + 1]), 0.5f);
  if (oy) return cscale(cadd(pe, sE[J + 1][I]), 0.5f);
  return pe;
}

// Up-leg on a TX x TY tile of fine points; thread (tx, ty0..ty0+PY) owns a
// column segment and keeps r and W of its own points in registers:
//   v2 = W r + P e on the (TX + 2) x (TY + 2) halo region (own points + a ring) -> LDS
//   z  = v2 + W (r - K v2) = (1 - w) v2 + W (r + sum of in-grid neighbours of v2)
// With RES (see k_down_fused2) the right-hand side is r - K e, formed from e
// on a two-point ring, and the leg writes e + z: the result of the repeated
// visit.  z must not alias e (other tiles read e's halo).
template <int TX, int TY, int PY, bool RES>
__global__ __launch_bounds__(TX*(TY / PY)) void k_up_fused2(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv,
                                                             float omega, VecSet ec, int nc, VecSet z,
                                                             const int* active, VecSet ev) {
  constexpr int HX = TX + 2, HY = TY + 2;
  constexpr int CX = TX / 2 + 2, CY = TY / 2 + 2;
  constexpr int NT = TX * (TY / PY);
  constexpr int NRING = 2 * HX + 2 * TY;
  constexpr int FX = RES ? TX + 4 : 1, FY = RES ? TY + 4 : 1;
  static_assert(NRING <= NT, "one ring point per thread");
  __shared__ c32 sE[CY][CX];
  __shared__ c32 sV[HY][HX];
  __shared__ c32 sF[FY][FX];
  const int n = lv.n;
  const int tiles_x = (n + TX - 1) / TX;
  const unsigned tiles = (unsigned)(tiles_x * ((n + TY - 1) / TY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int fx0 = (id.t % tiles_x) * TX;
  const int fy0 = (id.t / tiles_x) * TY;
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const int tx = threadIdx.x % TX, ty0 = (threadIdx.x / TX) * PY;
  // ring point of this thread (halo-local coordinates), if any
  int rlx = -1, rly = -1;
  {
    const int t = threadIdx.x;
    if (t < HX) {
      rlx = t;
      rly = 0;
    } else if (t < 2 * HX) {
      rlx = t - HX;
      rly = HY - 1;
    } else if (t < 2 * HX + TY) {
      rlx = 0;
      rly = t - 2 * HX + 1;
    } else if (t < NRING) {
      rlx = HX - 1;
      rly = t - 2 * HX - TY + 1;
    }
  }
  // issue every global load first
  constexpr int NE = CX * CY, ITE = (NE + NT - 1) / NT;
  c32 ev_c[ITE], rv[PY + 1], wv[PY + 1];
#pragma unroll
  for (int it = 0; it < ITE; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int I = cxs + idx % CX, J = cys + idx / CX;
    const bool ok = idx < NE && I >= 0 && I < nc && J >= 0 && J < nc;
    ev_c[it] = ok ? eb[(long long)J * nc + I] : make_float2(0.f, 0.f);
  }
  c32 kv[RES ? PY + 1 : 1];
  if constexpr (RES) {
    const c32* fb = ev.p + (long long)b * ev.stride;
    for (int idx = threadIdx.x; idx < FX * FY; idx += NT) {
      const int gx = fx0 - 2 + idx % FX, gy = fy0 - 2 + idx / FX;
      const bool ok = gx >= 0 && gx < n && gy >= 0 && gy < n;
      sF[idx / FX][idx % FX] = ok ? fb[(long long)gy * n + gx] : make_float2(0.f, 0.f);
    }
  }
#pragma unroll
  for (int k = 0; k <= PY; ++k) {
    const int gx = k < PY ? fx0 + tx : fx0 - 1 + rlx;
    const int gy = k < PY ? fy0 + ty0 + k : fy0 - 1 + rly;
    const bool ok = (k < PY || rlx >= 0) && gx >= 0 && gx < n && gy >= 0 && gy < n;
    const long long p = ok ? (long long)gy * n + gx : 0;
    rv[k] = ok ? cscale(rb[p], sc) : make_float2(0.f, 0.f);
    wv[k] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    if constexpr (RES) kv[k] = ok ? lv.coef[p] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int it = 0; it < ITE; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx < NE) sE[idx / CX][idx % CX] = ev_c[it];
  }
  __syncthreads();
  if constexpr (RES) {
    // r - K e at the own and ring points (sF is zero outside the grid)
#pragma unroll
    for (int k = 0; k <= PY; ++k) {
      const int lx = k < PY ? tx + 1 : rlx, ly = k < PY ? ty0 + k + 1 : rly;
      const int gx = fx0 - 1 + lx, gy = fy0 - 1 + ly;
      if ((k < PY || rlx >= 0) && gx >= 0 && gx < n && gy >= 0 && gy < n) {
        const int ng = ghosts2(gx, gy, n);
        const c32 D = make_float2(4.0f - kv[k].x - ng * lv.ghost.x, -kv[k].y - ng * lv.ghost.y);
        const c32 nb = cadd(cadd(sF[ly + 1][lx], sF[ly + 1][lx + 2]), cadd(sF[ly][lx + 1], sF[ly + 2][lx + 1]));
        rv[k] = cadd(csub(rv[k], cmul(D, sF[ly + 1][lx + 1])), nb);
      }
    }
  }
  c32 v2own[PY];
#pragma unroll
  for (int k = 0; k <= PY; ++k) {
    const int lx = k < PY ? tx + 1 : rlx, ly = k < PY ? ty0 + k + 1 : rly;
    if (k == PY && rlx < 0) continue;
    const int gx = fx0 - 1 + lx, gy = fy0 - 1 + ly;
    c32 v2 = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) v2 = cadd(cmul(rv[k], wv[k]), prolong_lds<CX>(sE, gx, gy, cxs, cys));
    if (k < PY) v2own[k] = v2;
    sV[ly][lx] = v2;
  }
  __syncthreads();
  c32* zb = z.p + (long long)b * z.stride;
#pragma unroll
  for (int k = 0; k < PY; ++k) {
    const int lx = tx + 1, ly = ty0 + k + 1;
    const int gx = fx0 + tx, gy = fy0 + ty0 + k;
    if (gx < n && gy < n) {
      const c32 nb = cadd(cadd(sV[ly][lx - 1], sV[ly][lx + 1]), cadd(sV[ly - 1][lx], sV[ly + 1][lx]));
      c32 zv = cadd(cscale(v2own[k], 1.0f - omega), cmul(wv[k], cadd(rv[k], nb)));
      if constexpr (RES) zv = cadd(zv, sF[ly + 1][lx + 1]);
      zb[(long long)gy * n + gx] = zv;
    }
  }
}

// Up-leg of Z_j fused with the next basis vector W_{j+1} = A Z_j of the s-step
// form, on a TX x TY tile of fine points:
//   v2 = W r + P e on the tile and a two-point ring   -> LDS
//   z  = (1 - w) v2 + W (r + neighbours of v2) on the tile and a one-point ring -> LDS
//   Z_j = z and W_{j+1} = D_A z - (neighbours of z) on the tile
// (la is the operator A, lv the level's preconditioning operator).  Saves the
// separate matvec's pass over Z_j.
template <int TX, int TY>
__global__ __launch_bounds__(256) void k_up_mv2(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la,
                                                float omega, VecSet ec, int nc, VecSet z, VecSet w,
                                                const int* active) {
  constexpr int NT = 256;
  constexpr int VX = TX + 4, VY = TY + 4, ZX = TX + 2, ZY = TY + 2;
  constexpr int CX = TX / 2 + 3, CY = TY / 2 + 3;
  __shared__ c32 sE[CY][CX];
  __shared__ c32 sV[VY][VX];
  __shared__ c32 sZ[ZY][ZX];
  const int n = lv.n;
  const int tiles_x = (n + TX - 1) / TX;
  const unsigned tiles = (unsigned)(tiles_x * ((n + TY - 1) / TY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int fx0 = (id.t % tiles_x) * TX, fy0 = (id.t / tiles_x) * TY;
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const c32* rb = r.p + (long long)b * r.stride;
  const float sc = scale_of(rs, b);
  for (int idx = threadIdx.x; idx < CX * CY; idx += NT) {
    const int I = cxs + idx % CX, J = cys + idx / CX;
    const bool ok = I >= 0 && I < nc && J >= 0 && J < nc;
    sE[idx / CX][idx % CX] = ok ? eb[(long long)J * nc + I] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  constexpr int IV = (VX * VY + NT - 1) / NT, IZ = (ZX * ZY + NT - 1) / NT, IT = (TX * TY + NT - 1) / NT;
  {
    c32 rv[IV], wv[IV];
#pragma unroll
    for (int it = 0; it < IV; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int gx = fx0 - 2 + idx % VX, gy = fy0 - 2 + idx / VX;
      const bool ok = idx < VX * VY && gx >= 0 && gx < n && gy >= 0 && gy < n;
      const long long p = ok ? (long long)gy * n + gx : 0;
      rv[it] = ok ? rb[p] : make_float2(0.f, 0.f);
      wv[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < IV; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx >= VX * VY) continue;
      const int gx = fx0 - 2 + idx % VX, gy = fy0 - 2 + idx / VX;
      c32 v2 = make_float2(0.f, 0.f);
      if (gx >= 0 && gx < n && gy >= 0 && gy < n)
        v2 = cadd(cmul(cscale(rv[it], sc), wv[it]), prolong_lds<CX>(sE, gx, gy, cxs, cys));
      sV[idx / VX][idx % VX] = v2;
    }
  }
  // r and W on the one-point ring region (cached: the loads above fetched them)
  c32 rz[IZ], wz[IZ];
#pragma unroll
  for (int it = 0; it < IZ; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int gx = fx0 - 1 + idx % ZX, gy = fy0 - 1 + idx / ZX;
    const bool ok = idx < ZX * ZY && gx >= 0 && gx < n && gy >= 0 && gy < n;
    const long long p = ok ? (long long)gy * n + gx : 0;
    rz[it] = ok ? rb[p] : make_float2(0.f, 0.f);
    wz[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IZ; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= ZX * ZY) continue;
    const int lx = idx % ZX + 1, ly = idx / ZX + 1;  // sV coordinates
    const int gx = fx0 - 2 + lx, gy = fy0 - 2 + ly;
    c32 zv = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const c32 nb = cadd(cadd(sV[ly][lx - 1], sV[ly][lx + 1]), cadd(sV[ly - 1][lx], sV[ly + 1][lx]));
      zv = cadd(cscale(sV[ly][lx], 1.0f - omega), cmul(wz[it], cadd(cscale(rz[it], sc), nb)));
    }
    sZ[idx / ZX][idx % ZX] = zv;
  }
  // the operator's coefficient at the own points
  c32 kv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int gx = fx0 + idx % TX, gy = fy0 + idx / TX;
    const bool ok = idx < TX * TY && gx < n && gy < n;
    kv[it] = ok ? la.coef[(long long)gy * n + gx] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  c32* zb = z.p + (long long)b * z.stride;
  c32* wb = w.p + (long long)b * w.stride;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int lx = idx % TX + 1, ly = idx / TX + 1;  // sZ coordinates
    const int gx = fx0 + lx - 1, gy = fy0 + ly - 1;
    if (idx >= TX * TY || gx >= n || gy >= n) continue;
    const long long p = (long long)gy * n + gx;
    const c32 zc = sZ[ly][lx];
    const int ng = ghosts2(gx, gy, n);
    const c32 D = make_float2(4.0f - kv[it].x - ng * la.ghost.x, -kv[it].y - ng * la.ghost.y);
    const c32 nb = cadd(cadd(sZ[ly][lx - 1], sZ[ly][lx + 1]), cadd(sZ[ly - 1][lx], sZ[ly + 1][lx]));
    zb[p] = zc;
    wb[p] = csub(cmul(D, zc), nb);
  }
}

// The same fused up-leg and matvec with a wavefront-wide column layout: the
// region is 64 columns wide (a 60-column tile and a two-point ring), each
// thread owns one column (lane) and every fourth row, so that the v2, z and
// output stages are done by the thread that loaded the point's r, W and A
// coefficient (kept in registers, no reloads), and no index needs a division.
template <int TY>
__global__ __launch_bounds__(256) void k_up_mv2w(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la,
                                                 float omega, VecSet ec, int nc, VecSet z, VecSet w,
                                                 const int* active) {
  constexpr int TX = 60, VX = 64, VY = TY + 4, ZY = TY + 2, RPI = 4, IV = VY / RPI;
  static_assert(VY % RPI == 0, "whole row groups");
  constexpr int CX = TX / 2 + 3, CY = TY / 2 + 3;
  __shared__ c32 sE[CY][CX];
  __shared__ c32 sV[VY][VX];
  __shared__ c32 sZ[ZY][VX];  // z of region point (lx, ly) at sZ[ly - 1][lx]
  const int n = lv.n;
  const int tiles_x = (n + TX - 1) / TX;
  const unsigned tiles = (unsigned)(tiles_x * ((n + TY - 1) / TY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int fx0 = (id.t % tiles_x) * TX, fy0 = (id.t / tiles_x) * TY;
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const c32* rb = r.p + (long long)b * r.stride;
  const float sc = scale_of(rs, b);
  const int lx = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int gx = fx0 - 2 + lx;
  const bool inx = gx >= 0 && gx < n;
  const bool tcol = lx >= 2 && lx < TX + 2 && gx < n;  // a column of the tile
  // every global load first: the coarse tile, r, W and (tile points) the A coefficient
  constexpr int IE = (CX * CY + 255) / 256;
  c32 evc[IE];
#pragma unroll
  for (int it = 0; it < IE; ++it) {
    const int idx = threadIdx.x + it * 256;
    const int I = cxs + idx % CX, J = cys + idx / CX;
    const bool ok = idx < CX * CY && I >= 0 && I < nc && J >= 0 && J < nc;
    evc[it] = ok ? eb[(long long)J * nc + I] : make_float2(0.f, 0.f);
  }
  c32 rv[IV], wv[IV], kv[IV];
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 - 2 + ly;
    const bool ok = inx && gy >= 0 && gy < n;
    const long long p = ok ? (long long)gy * n + gx : 0;
    rv[it] = ok ? cscale(rb[p], sc) : make_float2(0.f, 0.f);
    wv[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    kv[it] = ok && tcol && ly >= 2 && ly < TY + 2 ? la.coef[p] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int it = 0; it < IE; ++it) {
    const int idx = threadIdx.x + it * 256;
    if (idx < CX * CY) sE[idx / CX][idx % CX] = evc[it];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // v2 = W r + P e (zero outside the grid)
    const int ly = r0 + RPI * it, gy = fy0 - 2 + ly;
    c32 v2 = make_float2(0.f, 0.f);
    if (inx && gy >= 0 && gy < n) {
      const int I = (gx >> 1) - cxs, J = (gy >> 1) - cys, ox = gx & 1, oy = gy & 1;
      const c32 a = sE[J][I], bb = sE[J][I + ox], c = sE[J + oy][I], d = sE[J + oy][I + ox];
      v2 = cadd(cmul(rv[it], wv[it]), cscale(cadd(cadd(a, bb), cadd(c, d)), 0.25f));
    }
    sV[ly][lx] = v2;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // z on the tile and a one-point ring (zero outside the grid)
    const int ly = r0 + RPI * it, gy = fy0 - 2 + ly;
    if (lx < 1 || lx > VX - 2 || ly < 1 || ly > VY - 2) continue;
    c32 zv = make_float2(0.f, 0.f);
    if (inx && gy >= 0 && gy < n) {
      const c32 nb = cadd(cadd(sV[ly][lx - 1], sV[ly][lx + 1]), cadd(sV[ly - 1][lx], sV[ly + 1][lx]));
      zv = cadd(cscale(sV[ly][lx], 1.0f - omega), cmul(wv[it], cadd(rv[it], nb)));
    }
    sZ[ly - 1][lx] = zv;
  }
  __syncthreads();
  c32* zb = z.p + (long long)b * z.stride;
  c32* wb = w.p + (long long)b * w.stride;
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // Z_j and W_{j+1} = A Z_j on the tile
    const int ly = r0 + RPI * it, gy = fy0 - 2 + ly;
    if (!tcol || ly < 2 || ly >= TY + 2 || gy >= n) continue;
    const long long p = (long long)gy * n + gx;
    const c32 zc = sZ[ly - 1][lx];
    const int ng = ghosts2(gx, gy, n);
    const c32 D = make_float2(4.0f - kv[it].x - ng * la.ghost.x, -kv[it].y - ng * la.ghost.y);
    const c32 nb = cadd(cadd(sZ[ly - 1][lx - 1], sZ[ly - 1][lx + 1]), cadd(sZ[ly - 2][lx], sZ[ly][lx]));
    zb[p] = zc;
    wb[p] = csub(cmul(D, zc), nb);
  }
}

// Column-layout legs (the autotuner's last variants): the fine region is one
// wavefront wide, each thread owns a column (lane) and every fourth row, so
// the stages need no division and reuse the registers of the loads.  Same
// arithmetic per point as k_down_fused2 / k_up_fused2 (bit-identical results).
// Down-leg: 30 x TCY coarse points, fine region 63 x (2 TCY + 3) at 2 c0 - 2.
// With RES the right-hand side is r - K e (a repeated visit, as in k_down_fused2),
// formed from e staged in LDS on the region and a one-point ring.
template <int TCY, bool RES>
__global__ __launch_bounds__(256) void k_down_col(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, float omega,
                                                  VecSet rc, int nc, const int* active, VecSet ev) {
  constexpr int TCX = 30, RXU = 2 * TCX + 3, RYU = 2 * TCY + 3, RPI = 4, VY = (RYU + RPI - 1) / RPI * RPI,
                IV = VY / RPI;
  constexpr int FX = RES ? RXU + 2 : 1, FY = RES ? RYU + 2 : 1;
  __shared__ c32 sV[VY][64];
  __shared__ c32 sS[VY][64];
  __shared__ c32 sF[FY][FX];
  const int n = lv.n;
  const int tiles_x = (nc + TCX - 1) / TCX;
  const unsigned tiles = (unsigned)(tiles_x * ((nc + TCY - 1) / TCY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int cx0 = (id.t % tiles_x) * TCX, cy0 = (id.t / tiles_x) * TCY;
  const int fx0 = 2 * cx0 - 2, fy0 = 2 * cy0 - 2;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const int lx = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int gx = fx0 + lx;
  const bool inx = lx < RXU && gx >= 0 && gx < n;
  if constexpr (RES) {
    const c32* fb = ev.p + (long long)b * ev.stride;
    for (int idx = threadIdx.x; idx < FX * FY; idx += 256) {
      const int fx = fx0 - 1 + idx % FX, fy = fy0 - 1 + idx / FX;
      const bool ok = fx >= 0 && fx < n && fy >= 0 && fy < n;
      sF[idx / FX][idx % FX] = ok ? fb[(long long)fy * n + fx] : make_float2(0.f, 0.f);
    }
  }
  c32 rv[IV], wv[IV], kv[RES ? IV : 1];
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 + ly;
    const bool ok = inx && ly < RYU && gy >= 0 && gy < n;
    const long long p = ok ? (long long)gy * n + gx : 0;
    rv[it] = ok ? rb[p] : make_float2(0.f, 0.f);
    wv[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    if constexpr (RES) kv[it] = ok ? lv.coef[p] : make_float2(0.f, 0.f);
  }
  if constexpr (RES) __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 + ly;
    rv[it] = cscale(rv[it], sc);
    if constexpr (RES) {
      // r - K e with K e = D e - (sum of in-grid neighbours); sF is zero outside the grid
      if (inx && ly < RYU && gy >= 0 && gy < n) {
        const int ng = ghosts2(gx, gy, n);
        const c32 D = make_float2(4.0f - kv[it].x - ng * lv.ghost.x, -kv[it].y - ng * lv.ghost.y);
        const int fx = lx + 1, fy = ly + 1;
        const c32 nb = cadd(cadd(sF[fy][fx - 1], sF[fy][fx + 1]), cadd(sF[fy - 1][fx], sF[fy + 1][fx]));
        rv[it] = cadd(csub(rv[it], cmul(D, sF[fy][fx])), nb);
      }
    }
    sV[ly][lx] = cmul(rv[it], wv[it]);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 + ly;
    if (lx < 1 || lx > RXU - 2 || ly < 1 || ly > RYU - 2) continue;
    c32 sv = make_float2(0.f, 0.f);
    if (inx && gy >= 0 && gy < n) {
      const c32 nb = cadd(cadd(sV[ly][lx - 1], sV[ly][lx + 1]), cadd(sV[ly - 1][lx], sV[ly + 1][lx]));
      sv = cadd(cscale(rv[it], 1.0f - omega), nb);
    }
    sS[ly][lx] = sv;
  }
  __syncthreads();
  if (threadIdx.x < TCX * TCY) {
    const int tx = threadIdx.x % TCX, ty = threadIdx.x / TCX;
    const int I = cx0 + tx, J = cy0 + ty;
    if (I < nc && J < nc) {
      const int sx = 2 * tx + 2, sy = 2 * ty + 2;
      c32 acc = cscale(sS[sy][sx], 4.0f);
      acc = cadd(acc, cscale(cadd(cadd(sS[sy][sx - 1], sS[sy][sx + 1]), cadd(sS[sy - 1][sx], sS[sy + 1][sx])), 2.0f));
      acc = cadd(acc, cadd(cadd(sS[sy - 1][sx - 1], sS[sy - 1][sx + 1]), cadd(sS[sy + 1][sx - 1], sS[sy + 1][sx + 1])));
      rc.p[(long long)b * rc.stride + (long long)J * nc + I] = cscale(acc, 0.25f);
    }
  }
}

// Up-leg: 62 x TY fine points, region (tile and a one-point ring) 64 x (TY + 2).
// With RES the right-hand side is r - K e, formed from e on the region and a
// one-point ring, and the leg writes e + z (as k_up_fused2).
template <int TY, bool RES>
__global__ __launch_bounds__(256) void k_up_col(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, float omega,
                                                VecSet ec, int nc, VecSet z, const int* active, VecSet ev) {
  constexpr int TX = 62, VY = TY + 2, RPI = 4, IV = VY / RPI;
  static_assert(VY % RPI == 0 && TY % 2 == 0, "whole row groups, even tile origin");
  constexpr int CX = TX / 2 + 2, CY = TY / 2 + 2;
  constexpr int FX = RES ? 66 : 1, FY = RES ? VY + 2 : 1;
  __shared__ c32 sE[CY][CX];
  __shared__ c32 sV[VY][64];
  __shared__ c32 sF[FY][FX];
  const int n = lv.n;
  const int tiles_x = (n + TX - 1) / TX;
  const unsigned tiles = (unsigned)(tiles_x * ((n + TY - 1) / TY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int fx0 = (id.t % tiles_x) * TX, fy0 = (id.t / tiles_x) * TY;
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const c32* rb = r.p + (long long)b * r.stride;
  const float sc = scale_of(rs, b);
  const int lx = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int gx = fx0 - 1 + lx;
  const bool inx = gx >= 0 && gx < n;
  constexpr int IE = (CX * CY + 255) / 256;
  c32 evc[IE];
#pragma unroll
  for (int it = 0; it < IE; ++it) {
    const int idx = threadIdx.x + it * 256;
    const int I = cxs + idx % CX, J = cys + idx / CX;
    const bool ok = idx < CX * CY && I >= 0 && I < nc && J >= 0 && J < nc;
    evc[it] = ok ? eb[(long long)J * nc + I] : make_float2(0.f, 0.f);
  }
  if constexpr (RES) {
    const c32* fb = ev.p + (long long)b * ev.stride;
    for (int idx = threadIdx.x; idx < FX * FY; idx += 256) {
      const int fx = fx0 - 2 + idx % FX, fy = fy0 - 2 + idx / FX;
      const bool ok = fx >= 0 && fx < n && fy >= 0 && fy < n;
      sF[idx / FX][idx % FX] = ok ? fb[(long long)fy * n + fx] : make_float2(0.f, 0.f);
    }
  }
  c32 rv[IV], wv[IV], kv[RES ? IV : 1];
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int gy = fy0 - 1 + r0 + RPI * it;
    const bool ok = inx && gy >= 0 && gy < n;
    const long long p = ok ? (long long)gy * n + gx : 0;
    rv[it] = ok ? rb[p] : make_float2(0.f, 0.f);
    wv[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    if constexpr (RES) kv[it] = ok ? lv.coef[p] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int it = 0; it < IE; ++it) {
    const int idx = threadIdx.x + it * 256;
    if (idx < CX * CY) sE[idx / CX][idx % CX] = evc[it];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // v2 = W r + P e on the region (zero outside the grid)
    const int ly = r0 + RPI * it, gy = fy0 - 1 + ly;
    rv[it] = cscale(rv[it], sc);
    if constexpr (RES) {
      if (inx && gy >= 0 && gy < n) {
        const int ng = ghosts2(gx, gy, n);
        const c32 D = make_float2(4.0f - kv[it].x - ng * lv.ghost.x, -kv[it].y - ng * lv.ghost.y);
        const int fx = lx + 1, fy = ly + 1;
        const c32 nb = cadd(cadd(sF[fy][fx - 1], sF[fy][fx + 1]), cadd(sF[fy - 1][fx], sF[fy + 1][fx]));
        rv[it] = cadd(csub(rv[it], cmul(D, sF[fy][fx])), nb);
      }
    }
    c32 v2 = make_float2(0.f, 0.f);
    if (inx && gy >= 0 && gy < n) {
      const int I = (gx >> 1) - cxs, J = (gy >> 1) - cys, ox = gx & 1, oy = gy & 1;
      const c32 a = sE[J][I], bb = sE[J][I + ox], c = sE[J + oy][I], d = sE[J + oy][I + ox];
      v2 = cadd(cmul(rv[it], wv[it]), cscale(cadd(cadd(a, bb), cadd(c, d)), 0.25f));
    }
    sV[ly][lx] = v2;
  }
  __syncthreads();
  c32* zb = z.p + (long long)b * z.stride;
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 - 1 + ly;
    if (lx < 1 || lx > TX || ly < 1 || ly > TY || gx >= n || gy >= n) continue;
    const c32 nb = cadd(cadd(sV[ly][lx - 1], sV[ly][lx + 1]), cadd(sV[ly - 1][lx], sV[ly + 1][lx]));
    c32 zv = cadd(cscale(sV[ly][lx], 1.0f - omega), cmul(wv[it], cadd(rv[it], nb)));
    if constexpr (RES) zv = cadd(zv, sF[ly + 1][lx + 1]);
    zb[(long long)gy * n + gx] = zv;
  }
}

// ------------------------------------------------------------ fused 3D legs
// The 2D legs' arithmetic with the 7-point operator, 27-point full weighting
// (weights (1/4, 1/2, 1/4) per axis) and trilinear prolongation.
// Down-leg on a TCX x TCY x TCZ tile of coarse points: r, W on the fine region
// with a two-point halo (origin 2 c0 - 2), v1 = W r -> LDS; s on the region's
// interior -> LDS; rc = 4 R s.
template <int TCX, int TCY, int TCZ>
__global__ __launch_bounds__(TCX* TCY* TCZ) void k_down_fused3(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv,
                                                                float omega, VecSet rc, int nc, const int* active) {
  constexpr int RX = 2 * TCX + 3, RY = 2 * TCY + 3, RZ = 2 * TCZ + 3;
  constexpr int SX = RX - 2, SY = RY - 2, SZ = RZ - 2;
  constexpr int NT = TCX * TCY * TCZ, NR = RX * RY * RZ, IT = (NR + NT - 1) / NT;
  __shared__ c32 sV[RZ][RY][RX];
  __shared__ c32 sS[SZ][SY][SX];
  const int n = lv.n;
  const int tx_n = (nc + TCX - 1) / TCX, ty_n = (nc + TCY - 1) / TCY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((nc + TCZ - 1) / TCZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int cx0 = (id.t % tx_n) * TCX, cy0 = ((id.t / tx_n) % ty_n) * TCY, cz0 = (id.t / (tx_n * ty_n)) * TCZ;
  const int fx0 = 2 * cx0 - 2, fy0 = 2 * cy0 - 2, fz0 = 2 * cz0 - 2;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const long long n2 = (long long)n * n;
  c32 rv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int lx = idx % RX, ly = (idx / RX) % RY, lz = idx / (RX * RY);
    const int gx = fx0 + lx, gy = fy0 + ly, gz = fz0 + lz;
    const bool ok = idx < NR && gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n;
    const long long p = ok ? gz * n2 + (long long)gy * n + gx : 0;
    rv[it] = ok ? cscale(rb[p], sc) : make_float2(0.f, 0.f);
    const c32 wv = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    if (idx < NR) sV[lz][ly][lx] = cmul(rv[it], wv);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= NR) continue;
    const int lx = idx % RX, ly = (idx / RX) % RY, lz = idx / (RX * RY);
    if (lx == 0 || lx == RX - 1 || ly == 0 || ly == RY - 1 || lz == 0 || lz == RZ - 1) continue;
    const int gx = fx0 + lx, gy = fy0 + ly, gz = fz0 + lz;
    c32 sv = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n) {
      const c32 nb = cadd(cadd(cadd(sV[lz][ly][lx - 1], sV[lz][ly][lx + 1]), cadd(sV[lz][ly - 1][lx], sV[lz][ly + 1][lx])),
                          cadd(sV[lz - 1][ly][lx], sV[lz + 1][ly][lx]));
      sv = cadd(cscale(rv[it], 1.0f - omega), nb);
    }
    sS[lz - 1][ly - 1][lx - 1] = sv;
  }
  __syncthreads();
  const int tx = threadIdx.x % TCX, ty = (threadIdx.x / TCX) % TCY, tz = threadIdx.x / (TCX * TCY);
  const int I = cx0 + tx, J = cy0 + ty, K = cz0 + tz;
  if (I < nc && J < nc && K < nc) {
    const float w1[3] = {0.25f, 0.5f, 0.25f};
    c32 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
          acc = cadd(acc, cscale(sS[2 * tz + dz][2 * ty + dy][2 * tx + dx], w1[dx] * w1[dy] * w1[dz]));
    rc.p[(long long)b * rc.stride + ((long long)K * nc + J) * nc + I] = cscale(acc, 4.0f);
  }
}

// Down-leg marching in z: a TCX x TCY column of coarse points, coarse planes
// [kz0, kz0 + KZ).  Per fine plane f (bottom to top): v1(f) = W r on the
// plane's (2 TCX + 3) x (2 TCY + 3) region -> one of three LDS planes; then
// s(f - 1) on the region's interior from v1(f - 2 .. f) -> LDS; then the
// plane's in-plane full weighting is added to the coarse plane(s) it belongs
// to (weight 1/2 for f - 1 = 2K, 1/4 to K - 1 and K for f - 1 = 2K - 1),
// accumulated in registers; a coarse plane is written once complete.
template <int TCX, int TCY, int KZ>
__global__ __launch_bounds__(256) void k_down_march3(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, float omega,
                                                     VecSet rc, int nc, const int* active) {
  constexpr int NT = 256;
  constexpr int RX = 2 * TCX + 3, RY = 2 * TCY + 3, SX = RX - 2, SY = RY - 2;
  constexpr int NR = RX * RY, IT = (NR + NT - 1) / NT;
  static_assert(TCX * TCY <= NT, "one coarse point per thread");
  __shared__ c32 sV[3][RY][RX];
  __shared__ c32 sS[SY][SX];
  const int n = lv.n;
  const int tx_n = (nc + TCX - 1) / TCX, ty_n = (nc + TCY - 1) / TCY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((nc + KZ - 1) / KZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int cx0 = (id.t % tx_n) * TCX, cy0 = ((id.t / tx_n) % ty_n) * TCY, kz0 = (id.t / (tx_n * ty_n)) * KZ;
  const int kz1 = min(nc, kz0 + KZ);
  const int fx0 = 2 * cx0 - 2, fy0 = 2 * cy0 - 2;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const long long n2 = (long long)n * n;
  // this thread's region points: in-plane offset and whether it lies in the grid
  long long off[IT];
  bool inxy[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int gx = fx0 + idx % RX, gy = fy0 + idx / RX;
    inxy[it] = idx < NR && gx >= 0 && gx < n && gy >= 0 && gy < n;
    off[it] = inxy[it] ? (long long)gy * n + gx : 0;
  }
  const int f0 = 2 * kz0 - 2, f1 = 2 * kz1;  // fine planes whose v1 is needed
  c32 rn[IT], wn[IT], rp[IT];
  auto fetch = [&](int f) {
    const bool inz = f >= 0 && f < n;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const bool ok = inz && inxy[it];
      const long long p = ok ? f * n2 + off[it] : 0;
      rn[it] = ok ? rb[p] : make_float2(0.f, 0.f);
      wn[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    }
  };
  fetch(f0);
  const int tx = threadIdx.x % TCX, ty = threadIdx.x / TCX;
  const bool coarse = threadIdx.x < TCX * TCY && cx0 + tx < nc && cy0 + ty < nc;
  c32 acc = make_float2(0.f, 0.f);
  for (int f = f0; f <= f1; ++f) {
    c32 rf[IT];
    const int slot = (f - f0) % 3;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      rf[it] = cscale(rn[it], sc);
      const int idx = threadIdx.x + it * NT;
      if (idx < NR) sV[slot][idx / RX][idx % RX] = cmul(rf[it], wn[it]);
    }
    if (f < f1) fetch(f + 1);
    __syncthreads();
    const int g = f - 1;  // the plane whose s is formed now
    if (g >= f0 + 1) {
      const int sm = (g - 1 - f0) % 3, s0 = (g - f0) % 3;
      const bool ing = g >= 0 && g < n;
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NT;
        const int lx = idx % RX, ly = idx / RX;
        if (idx >= NR || lx == 0 || lx == RX - 1 || ly == 0 || ly == RY - 1) continue;
        c32 sv = make_float2(0.f, 0.f);
        if (ing && inxy[it]) {
          const c32 nb = cadd(cadd(cadd(sV[s0][ly][lx - 1], sV[s0][ly][lx + 1]),
                                   cadd(sV[s0][ly - 1][lx], sV[s0][ly + 1][lx])),
                              cadd(sV[sm][ly][lx], sV[slot][ly][lx]));
          sv = cadd(cscale(rp[it], 1.0f - omega), nb);
        }
        sS[ly - 1][lx - 1] = sv;
      }
    }
    __syncthreads();
    if (g >= f0 + 1 && coarse) {
      const int sx = 2 * tx + 1, sy = 2 * ty + 1;
      c32 t = cscale(sS[sy][sx], 0.25f);
      t = cadd(t, cscale(cadd(cadd(sS[sy][sx - 1], sS[sy][sx + 1]), cadd(sS[sy - 1][sx], sS[sy + 1][sx])), 0.125f));
      t = cadd(t, cscale(cadd(cadd(sS[sy - 1][sx - 1], sS[sy - 1][sx + 1]), cadd(sS[sy + 1][sx - 1], sS[sy + 1][sx + 1])),
                         0.0625f));
      if (g & 1) {  // g = 2K + 1: closes K (unless g is the chunk's first plane), opens K + 1
        if (g > f0 + 1) {
          const int K = (g - 1) >> 1;
          acc = cadd(acc, cscale(t, 0.25f));
          rc.p[(long long)b * rc.stride + ((long long)K * nc + cy0 + ty) * nc + cx0 + tx] = cscale(acc, 4.0f);
        }
        acc = cscale(t, 0.25f);
      } else {
        acc = cadd(acc, cscale(t, 0.5f));
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) rp[it] = rf[it];
  }
}

// Up-leg on a TX x TY x TZ tile of fine points: v2 = W r + P e on the tile and a
// one-point ring -> LDS; z = (1 - w) v2 + W (r + sum of the 6 neighbours of v2).
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_up_fused3(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, float omega,
                                                    VecSet ec, int nc, VecSet z, const int* active) {
  constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
  constexpr int CX = TX / 2 + 2, CY = TY / 2 + 2, CZ = TZ / 2 + 2;
  constexpr int NT = 256, NH = HX * HY * HZ, IT = (NH + NT - 1) / NT;
  __shared__ c32 sE[CZ][CY][CX];
  __shared__ c32 sV[HZ][HY][HX];
  const int n = lv.n;
  const int tx_n = (n + TX - 1) / TX, ty_n = (n + TY - 1) / TY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((n + TZ - 1) / TZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int fx0 = (id.t % tx_n) * TX, fy0 = ((id.t / tx_n) % ty_n) * TY, fz0 = (id.t / (tx_n * ty_n)) * TZ;
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1, czs = fz0 / 2 - 1;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const long long n2 = (long long)n * n, nc2 = (long long)nc * nc;
  for (int idx = threadIdx.x; idx < CX * CY * CZ; idx += NT) {
    const int I = cxs + idx % CX, J = cys + (idx / CX) % CY, K = czs + idx / (CX * CY);
    const bool ok = I >= 0 && I < nc && J >= 0 && J < nc && K >= 0 && K < nc;
    sE[idx / (CX * CY)][(idx / CX) % CY][idx % CX] = ok ? eb[K * nc2 + (long long)J * nc + I] : make_float2(0.f, 0.f);
  }
  c32 rv[IT], wv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int gx = fx0 - 1 + idx % HX, gy = fy0 - 1 + (idx / HX) % HY, gz = fz0 - 1 + idx / (HX * HY);
    const bool ok = idx < NH && gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n;
    const long long p = ok ? gz * n2 + (long long)gy * n + gx : 0;
    rv[it] = ok ? cscale(rb[p], sc) : make_float2(0.f, 0.f);
    wv[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= NH) continue;
    const int lx = idx % HX, ly = (idx / HX) % HY, lz = idx / (HX * HY);
    const int gx = fx0 - 1 + lx, gy = fy0 - 1 + ly, gz = fz0 - 1 + lz;
    c32 v2 = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n && gz >= 0 && gz < n) {
      const int I = (gx >> 1) - cxs, J = (gy >> 1) - cys, K = (gz >> 1) - czs;
      const int ox = gx & 1, oy = gy & 1, oz = gz & 1;
      c32 pe = make_float2(0.f, 0.f);
      for (int kz = 0; kz <= oz; ++kz)
        for (int ky = 0; ky <= oy; ++ky)
          for (int kx = 0; kx <= ox; ++kx) pe = cadd(pe, sE[K + kz][J + ky][I + kx]);
      const float wgt = (ox ? 0.5f : 1.0f) * (oy ? 0.5f : 1.0f) * (oz ? 0.5f : 1.0f);
      v2 = cadd(cmul(rv[it], wv[it]), cscale(pe, wgt));
    }
    sV[lz][ly][lx] = v2;
  }
  __syncthreads();
  c32* zb = z.p + (long long)b * z.stride;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= NH) continue;
    const int lx = idx % HX, ly = (idx / HX) % HY, lz = idx / (HX * HY);
    if (lx == 0 || lx == HX - 1 || ly == 0 || ly == HY - 1 || lz == 0 || lz == HZ - 1) continue;
    const int gx = fx0 - 1 + lx, gy = fy0 - 1 + ly, gz = fz0 - 1 + lz;
    if (gx >= n || gy >= n || gz >= n) continue;
    const c32 nb = cadd(cadd(cadd(sV[lz][ly][lx - 1], sV[lz][ly][lx + 1]), cadd(sV[lz][ly - 1][lx], sV[lz][ly + 1][lx])),
                        cadd(sV[lz - 1][ly][lx], sV[lz + 1][ly][lx]));
    zb[gz * n2 + (long long)gy * n + gx] =
        cadd(cscale(sV[lz][ly][lx], 1.0f - omega), cmul(wv[it], cadd(rv[it], nb)));
  }
}

// Up-leg marching in z: a TX x TY column of fine points, output planes
// [fz0, fz0 + FZ).  Per fine plane f: v2(f) = W r + P e on the column and a
// one-point in-plane ring -> one of three LDS planes (the coarse planes that P
// reads are kept two at a time in LDS); then z(f - 1) on the column from
// v2(f - 2 .. f).
template <int TX, int TY, int FZ>
__global__ __launch_bounds__(256) void k_up_march3(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, float omega,
                                                   VecSet ec, int nc, VecSet z, const int* active) {
  constexpr int NT = 256, HX = TX + 2, HY = TY + 2, NH = HX * HY, IT = (NH + NT - 1) / NT;
  constexpr int CX = TX / 2 + 2, CY = TY / 2 + 2, NCP = CX * CY, ITC = (NCP + NT - 1) / NT;
  __shared__ c32 sE[2][CY][CX];
  __shared__ c32 sV[3][HY][HX];
  const int n = lv.n;
  const int tx_n = (n + TX - 1) / TX, ty_n = (n + TY - 1) / TY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((n + FZ - 1) / FZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int fx0 = (id.t % tx_n) * TX, fy0 = ((id.t / tx_n) % ty_n) * TY, fz0 = (id.t / (tx_n * ty_n)) * FZ;
  const int fz1 = min(n, fz0 + FZ);
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const long long n2 = (long long)n * n, nc2 = (long long)nc * nc;
  long long off[IT];
  bool inxy[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int gx = fx0 - 1 + idx % HX, gy = fy0 - 1 + idx / HX;
    inxy[it] = idx < NH && gx >= 0 && gx < n && gy >= 0 && gy < n;
    off[it] = inxy[it] ? (long long)gy * n + gx : 0;
  }
  long long coff[ITC];
  bool cin[ITC];
#pragma unroll
  for (int it = 0; it < ITC; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int I = cxs + idx % CX, J = cys + idx / CX;
    cin[it] = idx < NCP && I >= 0 && I < nc && J >= 0 && J < nc;
    coff[it] = cin[it] ? (long long)J * nc + I : 0;
  }
  c32 rn[IT], wn[IT], rp[IT], wp[IT], cn[ITC];
  auto fetch = [&](int f) {
    const bool inz = f >= 0 && f < n;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const bool ok = inz && inxy[it];
      const long long p = ok ? f * n2 + off[it] : 0;
      rn[it] = ok ? rb[p] : make_float2(0.f, 0.f);
      wn[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    }
  };
  auto fetch_coarse = [&](int K) {
    const bool inz = K >= 0 && K < nc;
#pragma unroll
    for (int it = 0; it < ITC; ++it) {
      const bool ok = inz && cin[it];
      cn[it] = ok ? eb[K * nc2 + coff[it]] : make_float2(0.f, 0.f);
    }
  };
  auto store_coarse = [&](int K) {
#pragma unroll
    for (int it = 0; it < ITC; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < NCP) sE[K & 1][idx / CX][idx % CX] = cn[it];
    }
  };
  const int fa = fz0 - 1, fb = fz1;  // planes whose v2 is needed
  int khi = (max(fa, 0) >> 1) + 1;   // highest coarse plane in LDS
  fetch_coarse(khi - 1);
  store_coarse(khi - 1);
  fetch_coarse(khi);
  store_coarse(khi);
  fetch(fa);
  for (int f = fa; f <= fb; ++f) {
    c32 rf[IT], wf[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      rf[it] = cscale(rn[it], sc);
      wf[it] = wn[it];
    }
    const int knext = (f + 2) >> 1;  // the higher coarse plane that v2(f + 1) reads
    if (f < fb) {
      fetch(f + 1);
      if (knext > khi) fetch_coarse(knext);
    }
    __syncthreads();
    {
      const int slot = (f - fa) % 3;
      const bool inz = f >= 0 && f < n;
      const int klo = f >> 1;
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NT;
        if (idx >= NH) continue;
        const int gx = fx0 - 1 + idx % HX, gy = fy0 - 1 + idx / HX;
        c32 v2 = make_float2(0.f, 0.f);
        if (inz && inxy[it]) {
          c32 pe = prolong_lds<CX>(sE[klo & 1], gx, gy, cxs, cys);
          if (f & 1) pe = cscale(cadd(pe, prolong_lds<CX>(sE[(klo + 1) & 1], gx, gy, cxs, cys)), 0.5f);
          v2 = cadd(cmul(rf[it], wf[it]), pe);
        }
        sV[slot][idx / HX][idx % HX] = v2;
      }
    }
    __syncthreads();
    if (f < fb && knext > khi) {  // the coarse plane that replaces one no longer read
      store_coarse(knext);
      khi = knext;
    }
    const int g = f - 1;  // output plane
    if (g >= fz0) {
      const int sm = (g - 1 - fa) % 3, s0 = (g - fa) % 3, sp = (f - fa) % 3;
      c32* zb = z.p + (long long)b * z.stride + g * n2;
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NT;
        const int lx = idx % HX, ly = idx / HX;
        if (idx >= NH || lx == 0 || lx == HX - 1 || ly == 0 || ly == HY - 1 || !inxy[it]) continue;
        const c32 nb = cadd(cadd(cadd(sV[s0][ly][lx - 1], sV[s0][ly][lx + 1]), cadd(sV[s0][ly - 1][lx], sV[s0][ly + 1][lx])),
                            cadd(sV[sm][ly][lx], sV[sp][ly][lx]));
        zb[off[it]] = cadd(cscale(sV[s0][ly][lx], 1.0f - omega), cmul(wp[it], cadd(rp[it], nb)));
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      rp[it] = rf[it];
      wp[it] = wf[it];
    }
  }
}

// ------------------------------------------------- fused finest-level step
// One kernel for the finest-level work between two coarse-grid visits of
// consecutive s-step basis vectors: the up-leg of step j, the basis matvec
// W_{j+1} = A Z_j, and the down-leg of step j+1:
//   v2 = W r + P e;  z = (1 - w) v2 + W (r + sum nb v2)          (Z_j, written)
//   w  = A z                                                     (W_{j+1}, written)
//   v1 = W w;  s = (1 - w) w + sum nb v1;  rc = 4 R s            (next coarse rhs, written)
// on a TCX x TCY tile of coarse points of the next down-leg.  Relative to the
// tile's first owned fine point, s is needed on [-1, 2T-1], v1 and w on
// [-2, 2T], z on [-3, 2T+1], v2 (and r, W) on [-4, 2T+2]: each thread keeps
// r, W and w of its points of that widest region in registers; v2/s and z/v1
// share two LDS planes.  Fine points [0, 2T) of the tile are owned (written).
// r = s_j W_j with its per-RHS scale; W_{j+1} is unscaled.
template <int TCX, int TCY>
__global__ __launch_bounds__(TCX* TCY) void k_step_fused2(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv,
                                                           LevelArgs la, float omega, VecSet ec, int nc, VecSet zout,
                                                           VecSet wout, VecSet rc, const int* active) {
  constexpr int RX = 2 * TCX + 7, RY = 2 * TCY + 7;  // widest region, origin (-4, -4)
  constexpr int NT = TCX * TCY, NR = RX * RY, IT = (NR + NT - 1) / NT;
  constexpr int CX = TCX + 4, CY = TCY + 4;          // coarse correction, origin (cx0 - 2, cy0 - 2)
  __shared__ c32 sA[RY][RX];  // v2, then s
  __shared__ c32 sB[RY][RX];  // z, then v1
  __shared__ c32 sE[CY][CX];
  const int n = lv.n;
  const int tiles_x = (nc + TCX - 1) / TCX;
  const unsigned tiles = (unsigned)(tiles_x * ((nc + TCY - 1) / TCY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int cx0 = (id.t % tiles_x) * TCX, cy0 = (id.t / tiles_x) * TCY;
  const int fx0 = 2 * cx0, fy0 = 2 * cy0;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const c32* eb = ec.p + (long long)b * ec.stride;
  // ---- loads: r and W on the widest region (registers), the coarse correction (LDS)
  c32 rv[IT], wv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int gx = fx0 - 4 + idx % RX, gy = fy0 - 4 + idx / RX;
    const bool ok = idx < NR && gx >= 0 && gx < n && gy >= 0 && gy < n;
    const long long p = ok ? (long long)gy * n + gx : 0;
    rv[it] = ok ? cscale(rb[p], sc) : make_float2(0.f, 0.f);
    wv[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
  }
  for (int idx = threadIdx.x; idx < CX * CY; idx += NT) {
    const int I = cx0 - 2 + idx % CX, J = cy0 - 2 + idx / CX;
    const bool ok = I >= 0 && I < nc && J >= 0 && J < nc;
    sE[idx / CX][idx % CX] = ok ? eb[(long long)J * nc + I] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  // ---- v2 = W r + P e on [-4, 2T+2]  (0 outside the grid)
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= NR) continue;
    const int lx = idx % RX, ly = idx / RX;
    const int gx = fx0 - 4 + lx, gy = fy0 - 4 + ly;
    c32 v2 = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const int I = (gx >> 1) - (cx0 - 2), J = (gy >> 1) - (cy0 - 2);
      const int ox = gx & 1, oy = gy & 1;
      c32 pe = sE[J][I];
      if (ox && oy) pe = cscale(cadd(cadd(pe, sE[J][I + 1]), cadd(sE[J + 1][I], sE[J + 1][I + 1])), 0.25f);
      else if (ox) pe = cscale(cadd(pe, sE[J][I + 1]), 0.5f);
      else if (oy) pe = cscale(cadd(pe, sE[J + 1][I]), 0.5f);
      v2 = cadd(cmul(rv[it], wv[it]), pe);
    }
    sA[ly][lx] = v2;
  }
  __syncthreads();
  // ---- z = (1 - w) v2 + W (r + sum nb v2) on [-3, 2T+1]; Z_j on the owned points
  c32* zb = zout.p + (long long)b * zout.stride;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= NR) continue;
    const int lx = idx % RX, ly = idx / RX;
    if (lx < 1 || lx > RX - 2 || ly < 1 || ly > RY - 2) continue;
    const int gx = fx0 - 4 + lx, gy = fy0 - 4 + ly;
    c32 z = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const c32 nb = cadd(cadd(sA[ly][lx - 1], sA[ly][lx + 1]), cadd(sA[ly - 1][lx], sA[ly + 1][lx]));
      z = cadd(cscale(sA[ly][lx], 1.0f - omega), cmul(wv[it], cadd(rv[it], nb)));
      if (lx >= 4 && lx < 4 + 2 * TCX && ly >= 4 && ly < 4 + 2 * TCY) zb[(long long)gy * n + gx] = z;
    }
    sB[ly][lx] = z;
  }
  __syncthreads();
  // ---- w = A z on [-2, 2T]; W_{j+1} on the owned points (w kept in registers)
  c32* wb = wout.p + (long long)b * wout.stride;
  c32 wa[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    wa[it] = make_float2(0.f, 0.f);
    if (idx >= NR) continue;
    const int lx = idx % RX, ly = idx / RX;
    if (lx < 2 || lx > RX - 3 || ly < 2 || ly > RY - 3) continue;
    const int gx = fx0 - 4 + lx, gy = fy0 - 4 + ly;
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const long long p = (long long)gy * n + gx;
      const c32 D = diag_at(la, p, ghosts2(gx, gy, n), 2);
      const c32 nb = cadd(cadd(sB[ly][lx - 1], sB[ly][lx + 1]), cadd(sB[ly - 1][lx], sB[ly + 1][lx]));
      wa[it] = csub(cmul(D, sB[ly][lx]), nb);
      if (lx >= 4 && lx < 4 + 2 * TCX && ly >= 4 && ly < 4 + 2 * TCY) wb[p] = wa[it];
    }
  }
  __syncthreads();
  // ---- v1 = W w on [-2, 2T] (into the z plane)
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= NR) continue;
    const int lx = idx % RX, ly = idx / RX;
    if (lx < 2 || lx > RX - 3 || ly < 2 || ly > RY - 3) continue;
    sB[ly][lx] = cmul(wv[it], wa[it]);
  }
  __syncthreads();
  // ---- s = (1 - w) w + sum nb v1 on [-1, 2T-1] (into the v2 plane; 0 outside the grid)
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= NR) continue;
    const int lx = idx % RX, ly = idx / RX;
    if (lx < 3 || lx > RX - 4 || ly < 3 || ly > RY - 4) continue;
    const int gx = fx0 - 4 + lx, gy = fy0 - 4 + ly;
    c32 sv = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) {
      const c32 nb = cadd(cadd(sB[ly][lx - 1], sB[ly][lx + 1]), cadd(sB[ly - 1][lx], sB[ly + 1][lx]));
      sv = cadd(cscale(wa[it], 1.0f - omega), nb);
    }
    sA[ly][lx] = sv;
  }
  __syncthreads();
  // ---- rc = 4 R s at the tile's coarse points
  const int tx = threadIdx.x % TCX, ty = threadIdx.x / TCX;
  const int I = cx0 + tx, J = cy0 + ty;
  if (I < nc && J < nc) {
    const int sx = 4 + 2 * tx, sy = 4 + 2 * ty;
    c32 acc = cscale(sA[sy][sx], 4.0f);
    acc = cadd(acc, cscale(cadd(cadd(sA[sy][sx - 1], sA[sy][sx + 1]), cadd(sA[sy - 1][sx], sA[sy + 1][sx])), 2.0f));
    acc = cadd(acc, cadd(cadd(sA[sy - 1][sx - 1], sA[sy - 1][sx + 1]), cadd(sA[sy + 1][sx - 1], sA[sy + 1][sx + 1])));
    rc.p[(long long)b * rc.stride + (long long)J * nc + I] = cscale(acc, 0.25f);
  }
}

// ------------------------------------------------------------ generic (2D/3D)
__global__ void k_jacobi_zero(int dim, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet v,
                              const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= lv.N) return;
  const Coord c = coord_of32((unsigned)p, (unsigned)lv.n, dim);
  const c32 rv = cscale(r.p[(long long)b * r.stride + p], scale_of(rs, b));
  v.p[(long long)b * v.stride + p] = cscale(cmul(rv, crcp(diag_at(lv, p, ghosts_of(c, lv.n, dim), dim))), omega);
}

__global__ void k_jacobi(int dim, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet v, VecSet vout,
                         const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= lv.N) return;
  const Coord c = coord_of32((unsigned)p, (unsigned)lv.n, dim);
  const c32* vb = v.p + (long long)b * v.stride;
  const c32 rv = cscale(r.p[(long long)b * r.stride + p], scale_of(rs, b));
  const c32 D = diag_at(lv, p, ghosts_of(c, lv.n, dim), dim);
  // v + w D^-1 (r - K v), K v = D v - sum of neighbours
  const c32 res = csub(cadd(rv, neighbour_sum(vb, p, c, lv.n, dim)), cmul(D, vb[p]));
  vout.p[(long long)b * vout.stride + p] = cadd(vb[p], cscale(cmul(res, crcp(D)), omega));
}

__global__ void k_restrict_residual(int dim, VecSet r, ScaleSet rs, VecSet v, LevelArgs lv, VecSet rc, int nc,
                                    const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long ncN = dim == 2 ? (long long)nc * nc : (long long)nc * nc * nc;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncN) return;
  const Coord C = coord_of32((unsigned)q, (unsigned)nc, dim);
  const int n = lv.n;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const c32* vb = v.p ? v.p + (long long)b * v.stride : nullptr;
  const float w1[3] = {0.25f, 0.5f, 0.25f};
  c32 acc = make_float2(0.f, 0.f);
  const int zlo = dim == 3 ? -1 : 0, zhi = dim == 3 ? 1 : 0;
  for (int dz = zlo; dz <= zhi; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        Coord f{2 * C.x + dx, 2 * C.y + dy, dim == 3 ? 2 * C.z + dz : 0};
        if (f.x < 0 || f.x >= n || f.y < 0 || f.y >= n || f.z < 0 || f.z >= n) continue;
        const long long p = ((long long)f.z * n + f.y) * n + f.x;
        c32 s = cscale(rb[p], sc);
        if (vb) {
          const c32 D = diag_at(lv, p, ghosts_of(f, n, dim), dim);
          s = cadd(csub(s, cmul(D, vb[p])), neighbour_sum(vb, p, f, n, dim));
        }
        const float wgt = w1[dx + 1] * w1[dy + 1] * (dim == 3 ? w1[dz + 1] : 1.0f);
        acc = cadd(acc, cscale(s, wgt));
      }
  rc.p[(long long)b * rc.stride + q] = cscale(acc, 4.0f);
}

// vout = v + P ec (vout may be v)
__global__ void k_prolong_add(int dim, VecSet ec, int nc, VecSet v, VecSet vout, int n, long long N,
                              const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const Coord f = coord_of32((unsigned)p, (unsigned)n, dim);
  const c32* eb = ec.p + (long long)b * ec.stride;
  c32 acc = make_float2(0.f, 0.f);
  const int oz = dim == 3 ? (f.z & 1) : 0;
  for (int kz = 0; kz <= oz; ++kz)
    for (int ky = 0; ky <= (f.y & 1); ++ky)
      for (int kx = 0; kx <= (f.x & 1); ++kx) {
        const int I = (f.x >> 1) + kx, J = (f.y >> 1) + ky, K = dim == 3 ? (f.z >> 1) + kz : 0;
        float wgt = ((f.x & 1) ? 0.5f : 1.0f) * ((f.y & 1) ? 0.5f : 1.0f) * (oz ? 0.5f : 1.0f);
        acc = cadd(acc, cscale(eb[((long long)K * nc + J) * nc + I], wgt));
      }
  const c32* vb = v.p + (long long)b * v.stride;
  vout.p[(long long)b * vout.stride + p] = cadd(vb[p], acc);
}

// out = s_b b - K v on a level (the right-hand side of a repeated coarse visit:
// MG(b, v) = v + MG(b - K v, 0) for the affine multigrid cycle; the residual
// ahead of a restriction in the generic legs)
__global__ void k_level_residual(int dim, VecSet bvec, ScaleSet bs, VecSet v, LevelArgs lv, VecSet out,
                                 const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= lv.N) return;
  const Coord c = coord_of32((unsigned)p, (unsigned)lv.n, dim);
  const c32* vb = v.p + (long long)b * v.stride;
  const c32 D = diag_at(lv, p, ghosts_of(c, lv.n, dim), dim);
  const c32 kv = csub(cmul(D, vb[p]), neighbour_sum(vb, p, c, lv.n, dim));
  out.p[(long long)b * out.stride + p] = csub(cscale(bvec.p[(long long)b * bvec.stride + p], scale_of(bs, b)), kv);
}

// y += x for every active right-hand side
__global__ void k_add(VecSet x, VecSet y, long long N, const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  c32* yb = y.p + (long long)b * y.stride;
  yb[p] = cadd(yb[p], x.p[(long long)b * x.stride + p]);
}

// y = out_scale * (D x - sum of neighbours), D = 2d - coef - g #ghosts
__global__ void k_apply(int dim, VecSet x, ScaleSet xs, LevelArgs lv, float out_scale, VecSet y,
                        const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= lv.N) return;
  const Coord c = coord_of32((unsigned)p, (unsigned)lv.n, dim);
  const c32* xb = x.p + (long long)b * x.stride;
  const c32 D = diag_at(lv, p, ghosts_of(c, lv.n, dim), dim);
  const c32 out = csub(cmul(D, xb[p]), neighbour_sum(xb, p, c, lv.n, dim));
  y.p[(long long)b * y.stride + p] = cscale(out, out_scale * scale_of(xs, b));
}

// z_b = M r_b with M given transposed (minvT[k * Nc + row] = M[row][k]):
// one thread per (row, right-hand side); r_b is staged in LDS and broadcast,
// rows are read coalesced from the transposed inverse.
constexpr int CS_MAX = 4096;
__global__ __launch_bounds__(256) void k_coarse_solve(const c32* minvT, int Nc, VecSet r, VecSet z,
                                                      const int* active) {
  __shared__ c32 sr[CS_MAX];
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const c32* rb = r.p + (long long)b * r.stride;
  for (int k = threadIdx.x; k < Nc; k += blockDim.x) sr[k] = rb[k];
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= Nc) return;
  c32 acc0 = make_float2(0.f, 0.f), acc1 = acc0;
  int k = 0;
  for (; k + 1 < Nc; k += 2) {
    acc0 = cfma(minvT[(long long)k * Nc + row], sr[k], acc0);
    acc1 = cfma(minvT[(long long)(k + 1) * Nc + row], sr[k + 1], acc1);
  }
  if (k < Nc) acc0 = cfma(minvT[(long long)k * Nc + row], sr[k], acc0);
  z.p[(long long)b * z.stride + row] = cadd(acc0, acc1);
}

// The same product for all right-hand sides as one complex matrix product
// Z = M R: a block computes 64 rows x 16 right-hand sides over one of
// CS_KSPLIT slices of the inner index (tiles of 32 staged in LDS, 2 x 2
// outputs per thread), writing its slice's partial sums; k_coarse_reduce adds
// the slices in a fixed order.  The inverse is read once per 16 right-hand
// sides instead of once per right-hand side.
constexpr int CS_KSPLIT = 8, CS_RT = 64, CS_BT = 16, CS_KC = 32;
__global__ __launch_bounds__(256) void k_coarse_gemm(const c32* minvT, int Nc, int B, VecSet r, c32* part) {
  __shared__ c32 sA[CS_KC][CS_RT];
  __shared__ c32 sR[CS_KC][CS_BT];
  const int r0 = blockIdx.x * CS_RT, b0 = blockIdx.y * CS_BT;
  const int klen = ((Nc + CS_KSPLIT - 1) / CS_KSPLIT + CS_KC - 1) / CS_KC * CS_KC;
  const int kb = blockIdx.z * klen, ke = min(Nc, kb + klen);
  const int ry = threadIdx.x % 32, bx = threadIdx.x / 32;
  c32 a00 = make_float2(0.f, 0.f), a01 = a00, a10 = a00, a11 = a00;
  for (int k0 = kb; k0 < ke; k0 += CS_KC) {
    for (int i = threadIdx.x; i < CS_KC * CS_RT; i += 256) {
      const int kk = i / CS_RT, rr = i % CS_RT;
      const bool ok = k0 + kk < ke && r0 + rr < Nc;
      sA[kk][rr] = ok ? minvT[(long long)(k0 + kk) * Nc + r0 + rr] : make_float2(0.f, 0.f);
    }
    for (int i = threadIdx.x; i < CS_KC * CS_BT; i += 256) {
      const int q = i / CS_KC, kk = i % CS_KC;
      const bool ok = k0 + kk < ke && b0 + q < B;
      sR[kk][q] = ok ? r.p[(long long)(b0 + q) * r.stride + k0 + kk] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < CS_KC; ++kk) {
      const c32 m0 = sA[kk][ry], m1 = sA[kk][ry + 32], v0 = sR[kk][bx], v1 = sR[kk][bx + 8];
      a00 = cfma(m0, v0, a00);
      a01 = cfma(m0, v1, a01);
      a10 = cfma(m1, v0, a10);
      a11 = cfma(m1, v1, a11);
    }
    __syncthreads();
  }
  c32* pp = part + (long long)blockIdx.z * B * Nc;
  const int ra = r0 + ry, rb = r0 + ry + 32, ba = b0 + bx, bb = b0 + bx + 8;
  if (ra < Nc && ba < B) pp[(long long)ba * Nc + ra] = a00;
  if (ra < Nc && bb < B) pp[(long long)bb * Nc + ra] = a01;
  if (rb < Nc && ba < B) pp[(long long)ba * Nc + rb] = a10;
  if (rb < Nc && bb < B) pp[(long long)bb * Nc + rb] = a11;
}

__global__ __launch_bounds__(256) void k_coarse_reduce(const c32* part, int Nc, int B, VecSet z, const int* active) {
  const int b = blockIdx.y;
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= Nc || (active && !active[b])) return;
  c32 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < CS_KSPLIT; ++q) acc = cadd(acc, part[((long long)q * B + b) * Nc + row]);
  z.p[(long long)b * z.stride + row] = acc;
}

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// Tile shapes of the fused legs the autotuner chooses from (index 0 = default):
// down-leg coarse TCX x TCY per block, up-leg fine TX x TY with PY points per thread.
namespace {
struct DownTile {
  int tcx, tcy;
};
struct UpTile {
  int tx, ty, py;
};
// the last entry of each is the column-layout kernel (k_down_col / k_up_col)
constexpr DownTile kDown[] = {{32, 8}, {16, 16}, {64, 4}, {32, 4}, {16, 8}, {30, 8}};
constexpr UpTile kUp[] = {{64, 16, 4}, {32, 16, 2}, {64, 8, 2}, {32, 32, 4}, {64, 32, 8}, {62, 14, 0}};
constexpr int kDownCol = 5, kUpCol = 5;

template <int TCX, int TCY>
void down_tile(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet rc, int nc,
               const int* active, VecSet e) {
  const int tiles = ((nc + TCX - 1) / TCX) * ((nc + TCY - 1) / TCY);
  if (e.p)
    hipLaunchKernelGGL((k_down_fused2<TCX, TCY, true>), dim3(B * tiles), dim3(TCX * TCY), 0, s, B, r, rs, lv, omega,
                       rc, nc, active, e);
  else
    hipLaunchKernelGGL((k_down_fused2<TCX, TCY, false>), dim3(B * tiles), dim3(TCX * TCY), 0, s, B, r, rs, lv,
                       omega, rc, nc, active, e);
}
template <int TX, int TY, int PY>
void up_tile(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet ec, int nc, VecSet z,
             const int* active, VecSet e) {
  const int tiles = ((lv.n + TX - 1) / TX) * ((lv.n + TY - 1) / TY);
  if (e.p)
    hipLaunchKernelGGL((k_up_fused2<TX, TY, PY, true>), dim3(B * tiles), dim3(TX * (TY / PY)), 0, s, B, r, rs, lv,
                       omega, ec, nc, z, active, e);
  else
    hipLaunchKernelGGL((k_up_fused2<TX, TY, PY, false>), dim3(B * tiles), dim3(TX * (TY / PY)), 0, s, B, r, rs, lv,
                       omega, ec, nc, z, active, e);
}
}  // namespace

void launch_down_fused3(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet rc, int nc,
                        const int* active) {
#ifndef HELM_DOWN3_MARCH
#define HELM_DOWN3_MARCH 1
#endif
  if (HELM_DOWN3_MARCH) {
    constexpr int TCX = 16, TCY = 8, KZ = 8;
    const int tiles = ((nc + TCX - 1) / TCX) * ((nc + TCY - 1) / TCY) * ((nc + KZ - 1) / KZ);
    hipLaunchKernelGGL((k_down_march3<TCX, TCY, KZ>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, rc, nc,
                       active);
    return;
  }
  constexpr int TCX = 8, TCY = 4, TCZ = 4;
  const int tiles = ((nc + TCX - 1) / TCX) * ((nc + TCY - 1) / TCY) * ((nc + TCZ - 1) / TCZ);
  hipLaunchKernelGGL((k_down_fused3<TCX, TCY, TCZ>), dim3(B * tiles), dim3(TCX * TCY * TCZ), 0, s, B, r, rs, lv,
                     omega, rc, nc, active);
}

void launch_up_fused3(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet ec, int nc,
                      VecSet z, const int* active) {
#ifndef HELM_UP3_MARCH
#define HELM_UP3_MARCH 1
#endif
  if (HELM_UP3_MARCH) {
    constexpr int TX = 32, TY = 16, FZ = 16;
    const int n = lv.n;
    const int tiles = ((n + TX - 1) / TX) * ((n + TY - 1) / TY) * ((n + FZ - 1) / FZ);
    hipLaunchKernelGGL((k_up_march3<TX, TY, FZ>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z,
                       active);
    return;
  }
  constexpr int TX = 16, TY = 8, TZ = 8;
  const int n = lv.n;
  const int tiles = ((n + TX - 1) / TX) * ((n + TY - 1) / TY) * ((n + TZ - 1) / TZ);
  hipLaunchKernelGGL((k_up_fused3<TX, TY, TZ>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z,
                     active);
}

void launch_up_mv2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la, float omega, VecSet ec,
                   int nc, VecSet z, VecSet w, const int* active) {
#ifndef HELM_UPMV_WIDE
#define HELM_UPMV_WIDE 12
#endif
  if (HELM_UPMV_WIDE > 0) {
    constexpr int TX = 60, TY = HELM_UPMV_WIDE > 0 ? HELM_UPMV_WIDE : 16;
    const int n = lv.n;
    const int tiles = ((n + TX - 1) / TX) * ((n + TY - 1) / TY);
    hipLaunchKernelGGL((k_up_mv2w<TY>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, la, omega, ec, nc, z, w,
                       active);
    return;
  }
  constexpr int TX = 64, TY = 16;
  const int n = lv.n;
  const int tiles = ((n + TX - 1) / TX) * ((n + TY - 1) / TY);
  hipLaunchKernelGGL((k_up_mv2<TX, TY>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, la, omega, ec, nc, z, w,
                     active);
}

void launch_step_fused2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la, float omega,
                        VecSet ec, int nc, VecSet z, VecSet w, VecSet rc, const int* active) {
  constexpr int TCX = 16, TCY = 16;
  const int tiles = ((nc + TCX - 1) / TCX) * ((nc + TCY - 1) / TCY);
  hipLaunchKernelGGL((k_step_fused2<TCX, TCY>), dim3(B * tiles), dim3(TCX * TCY), 0, s, B, r, rs, lv, la, omega, ec,
                     nc, z, w, rc, active);
}

int mg_down_variants() { return (int)(sizeof(kDown) / sizeof(kDown[0])); }
int mg_up_variants() { return (int)(sizeof(kUp) / sizeof(kUp[0])); }
void mg_down_shape(int cfg, int* tcx, int* tcy) {
  *tcx = kDown[cfg].tcx;
  *tcy = kDown[cfg].tcy;
}
void mg_up_shape(int cfg, int* tx, int* ty, int* py) {
  *tx = kUp[cfg].tx;
  *ty = kUp[cfg].ty;
  *py = kUp[cfg].py;
}

void launch_down_fused2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet rc, int nc,
                        const int* active, int cfg, VecSet e) {
  if (cfg == kDownCol) {
    constexpr int TCX = 30, TCY = 8;
    const int tiles = ((nc + TCX - 1) / TCX) * ((nc + TCY - 1) / TCY);
    if (e.p)
      hipLaunchKernelGGL((k_down_col<TCY, true>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, rc, nc,
                         active, e);
    else
      hipLaunchKernelGGL((k_down_col<TCY, false>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, rc, nc,
                         active, e);
    return;
  }
  switch (cfg) {
    case 1: down_tile<16, 16>(s, B, r, rs, lv, omega, rc, nc, active, e); break;
    case 2: down_tile<64, 4>(s, B, r, rs, lv, omega, rc, nc, active, e); break;
    case 3: down_tile<32, 4>(s, B, r, rs, lv, omega, rc, nc, active, e); break;
    case 4: down_tile<16, 8>(s, B, r, rs, lv, omega, rc, nc, active, e); break;
    default: down_tile<32, 8>(s, B, r, rs, lv, omega, rc, nc, active, e); break;
  }
}

void launch_up_fused2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet ec, int nc,
                      VecSet z, const int* active, int cfg, VecSet e) {
  if (cfg == kUpCol) {
    constexpr int TX = 62, TY = 14;
    const int tiles = ((lv.n + TX - 1) / TX) * ((lv.n + TY - 1) / TY);
    if (e.p)
      hipLaunchKernelGGL((k_up_col<TY, true>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z,
                         active, e);
    else
      hipLaunchKernelGGL((k_up_col<TY, false>), dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z,
                         active, e);
    return;
  }
  switch (cfg) {
    case 1: up_tile<32, 16, 2>(s, B, r, rs, lv, omega, ec, nc, z, active, e); break;
    case 2: up_tile<64, 8, 2>(s, B, r, rs, lv, omega, ec, nc, z, active, e); break;
    case 3: up_tile<32, 32, 4>(s, B, r, rs, lv, omega, ec, nc, z, active, e); break;
    case 4: up_tile<64, 32, 8>(s, B, r, rs, lv, omega, ec, nc, z, active, e); break;
    default: up_tile<64, 16, 4>(s, B, r, rs, lv, omega, ec, nc, z, active, e); break;
  }
}

void launch_jacobi_zero(hipStream_t s, int dim, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet v,
                        const int* active) {
  hipLaunchKernelGGL(k_jacobi_zero, dim3(nblocks(lv.N, 256), B), dim3(256), 0, s, dim, r, rs, lv, omega, v, active);
}

void launch_jacobi(hipStream_t s, int dim, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet v,
                   VecSet vout, const int* active) {
  hipLaunchKernelGGL(k_jacobi, dim3(nblocks(lv.N, 256), B), dim3(256), 0, s, dim, r, rs, lv, omega, v, vout,
                     active);
}

void launch_restrict_residual(hipStream_t s, int dim, int B, VecSet r, ScaleSet rs, VecSet v, LevelArgs lv,
                              VecSet rc, int nc, const int* active) {
  const long long ncN = dim == 2 ? (long long)nc * nc : (long long)nc * nc * nc;
  hipLaunchKernelGGL(k_restrict_residual, dim3(nblocks(ncN, 256), B), dim3(256), 0, s, dim, r, rs, v, lv, rc, nc,
                     active);
}

void launch_prolong_add(hipStream_t s, int dim, int B, VecSet ec, int nc, VecSet v, int n, const int* active,
                        VecSet vout) {
  const long long N = dim == 2 ? (long long)n * n : (long long)n * n * n;
  hipLaunchKernelGGL(k_prolong_add, dim3(nblocks(N, 256), B), dim3(256), 0, s, dim, ec, nc, v, vout.p ? vout : v, n,
                     N, active);
}

void launch_coarse_solve(hipStream_t s, int B, const c32* minvT, int Nc, VecSet r, VecSet z, const int* active,
                         c32* part) {
  if (part && B >= 4) {  // as one matrix product (part: coarse_solve_part_size(B, Nc) entries)
    hipLaunchKernelGGL(k_coarse_gemm, dim3(nblocks(Nc, CS_RT), nblocks(B, CS_BT), CS_KSPLIT), dim3(256), 0, s, minvT,
                       Nc, B, r, part);
    hipLaunchKernelGGL(k_coarse_reduce, dim3(nblocks(Nc, 256), B), dim3(256), 0, s, part, Nc, B, z, active);
    return;
  }
  hipLaunchKernelGGL(k_coarse_solve, dim3(nblocks(Nc, 256), B), dim3(256), 0, s, minvT, Nc, r, z, active);
}

size_t coarse_solve_part_size(int B, int Nc) { return (size_t)CS_KSPLIT * B * Nc; }

void launch_apply(hipStream_t s, int dim, int B, VecSet x, ScaleSet xs, LevelArgs lv, float out_scale, VecSet y,
                  const int* active) {
  hipLaunchKernelGGL(k_apply, dim3(nblocks(lv.N, 256), B), dim3(256), 0, s, dim, x, xs, lv, out_scale, y, active);
}

void launch_level_residual(hipStream_t s, int dim, int B, VecSet bvec, VecSet v, LevelArgs lv, VecSet out,
                           const int* active, ScaleSet bs) {
  hipLaunchKernelGGL(k_level_residual, dim3(nblocks(lv.N, 256), B), dim3(256), 0, s, dim, bvec, bs, v, lv, out,
                     active);
}

void launch_add(hipStream_t s, int B, VecSet x, VecSet y, long long N, const int* active) {
  hipLaunchKernelGGL(k_add, dim3(nblocks(N, 256), B), dim3(256), 0, s, x, y, N, active);
}
