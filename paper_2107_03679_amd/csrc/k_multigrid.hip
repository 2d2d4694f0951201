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
  // issue every global load first, back to back: clamped in-grid addresses without
  // predicates, so that none waits for another; zeros outside the grid are put in at the
  // LDS stores, and values of points outside the grid are never used (every use below is
  // guarded by the same condition); the scale of r is applied after the loads
  constexpr int NE = CX * CY, ITE = (NE + NT - 1) / NT, ITF = RES ? (FX * FY + NT - 1) / NT : 0;
  c32 ev_c[ITE], fv[ITF > 0 ? ITF : 1], rv[PY + 1], wv[PY + 1];
#pragma unroll
  for (int it = 0; it < ITE; ++it) {
    const int idx = min((int)threadIdx.x + it * NT, NE - 1);
    const int I = min(max(cxs + idx % CX, 0), nc - 1), J = min(max(cys + idx / CX, 0), nc - 1);
    ev_c[it] = eb[(long long)J * nc + I];
  }
  c32 kv[RES ? PY + 1 : 1];
  if constexpr (RES) {
    const c32* fb = ev.p + (long long)b * ev.stride;
#pragma unroll
    for (int it = 0; it < ITF; ++it) {
      const int idx = min((int)threadIdx.x + it * NT, FX * FY - 1);
      const int gx = min(max(fx0 - 2 + idx % FX, 0), n - 1), gy = min(max(fy0 - 2 + idx / FX, 0), n - 1);
      fv[it] = fb[(long long)gy * n + gx];
    }
  }
#pragma unroll
  for (int k = 0; k <= PY; ++k) {
    const int gx = min(max(k < PY ? fx0 + tx : fx0 - 1 + rlx, 0), n - 1);
    const int gy = min(max(k < PY ? fy0 + ty0 + k : fy0 - 1 + rly, 0), n - 1);
    const long long p = (long long)gy * n + gx;
    rv[k] = rb[p];
    wv[k] = lv.wd[p];
    if constexpr (RES) kv[k] = lv.coef[p];
  }
#pragma unroll
  for (int it = 0; it < ITE; ++it) {
    const int idx = threadIdx.x + it * NT;
    const int I = cxs + idx % CX, J = cys + idx / CX;
    const bool ok = I >= 0 && I < nc && J >= 0 && J < nc;
    if (idx < NE) sE[idx / CX][idx % CX] = ok ? ev_c[it] : make_float2(0.f, 0.f);
  }
  if constexpr (RES) {
#pragma unroll
    for (int it = 0; it < ITF; ++it) {
      const int idx = threadIdx.x + it * NT;
      const int gx = fx0 - 2 + idx % FX, gy = fy0 - 2 + idx / FX;
      const bool ok = gx >= 0 && gx < n && gy >= 0 && gy < n;
      if (idx < FX * FY) sF[idx / FX][idx % FX] = ok ? fv[it] : make_float2(0.f, 0.f);
    }
  }
#pragma unroll
  for (int k = 0; k <= PY; ++k) rv[k] = cscale(rv[k], sc);
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

// The same fused up-leg and matvec with a wavefront-wide column layout: the
// region is 64 columns wide (a 60-column tile and a two-point ring), each
// thread owns one column (lane) and every fourth row, so that the v2, z and
// output stages are done by the thread that loaded the point's r, W and A
// coefficient (kept in registers, no reloads), and no index needs a division.
// A block walks K right-hand sides of one tile: the coefficient rows (shared by
// the batch) are loaded once, and the next right-hand side's r and coarse tile
// are loaded while the current one is computed, so that the memory system has
// work in every stage.  A wavefront's rows are uniform (its index is read into
// a scalar register), so every row's base address is scalar and all loads and
// stores of a lane share one 32-bit column offset.  Loads go to the nearest
// in-grid point without predicates; values of points outside the grid are
// never used (every use is guarded by the same condition).
template <int TY, int K>
__global__ __launch_bounds__(256) void k_up_mv2w(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la,
                                                 float omega, VecSet ec, int nc, VecSet z, VecSet w,
                                                 const int* active) {
  constexpr int TX = 60, VX = 64, VY = TY + 4, ZY = TY + 2, RPI = 4, IV = VY / RPI;
  static_assert(VY % RPI == 0, "whole row groups");
  constexpr int CX = TX / 2 + 3, CY = TY / 2 + 3, IE = (CX * CY + 255) / 256;
  __shared__ c32 sE[CY][CX];
  __shared__ c32 sV[VY][VX];
  __shared__ c32 sZ[ZY][VX];  // z of region point (lx, ly) at sZ[ly - 1][lx]
  const int n = lv.n;
  // workgroup order (xcd_stretch): "groups of K right-hand sides fastest, then tiles in
  // raster order", one contiguous stretch per XCD
  const unsigned groups = (unsigned)(nrhs + K - 1) / K, tiles_x = (unsigned)(n + TX - 1) / TX;
  const unsigned l = xcd_stretch(blockIdx.x, gridDim.x);
  const unsigned t = l / groups, grp = l - t * groups;
  const int b_end = min(nrhs, (int)(grp + 1) * K);
  int b = (int)grp * K;
  if (active)
    while (b < b_end && !active[b]) ++b;
  if (b >= b_end) return;
  const int fx0 = (int)(t % tiles_x) * TX, fy0 = (int)(t / tiles_x) * TY;
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1;
  const int lx0 = threadIdx.x & 63;
  const int r0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wavefront's first region row
  const unsigned ob0 = (unsigned)min(max(fx0 - 2 + lx0, 0), n - 1) * (unsigned)sizeof(c32);  // nearest in-grid column
  unsigned eo[IE];  // coarse-tile items of this thread: nearest in-grid coarse point
#pragma unroll
  for (int it = 0; it < IE; ++it) {
    const int idx = min((int)threadIdx.x + it * 256, CX * CY - 1);
    const int I = min(max(cxs + idx % CX, 0), nc - 1), J = min(max(cys + idx / CX, 0), nc - 1);
    eo[it] = (unsigned)(J * nc + I);
  }
  auto load_e = [&](int bb, c32* ev_) {  // the coarse tile of right-hand side bb
    const c32* eb = ec.p + (long long)bb * ec.stride;
#pragma unroll
    for (int it = 0; it < IE; ++it) ev_[it] = eb[eo[it]];
  };
  auto load_r = [&](int bb, c32* rv_) {  // r of right-hand side bb on the region
    const c32* rb = r.p + (long long)bb * r.stride;
#pragma unroll
    for (int it = 0; it < IV; ++it) {
      const int gy = fy0 - 2 + r0 + RPI * it;
      if (gy >= 0 && gy < n) rv_[it] = at_byte(rb + (long long)gy * n, ob0);
    }
  };
  c32 rv[IV], evc[IE], wv[IV], kv[IV];
  load_e(b, evc);
  load_r(b, rv);
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // the coefficient rows, once for all right-hand sides
    const int ly = r0 + RPI * it, gy = fy0 - 2 + ly;
    if (gy >= 0 && gy < n) {
      const long long row = (long long)gy * n;
      wv[it] = at_byte(lv.wd + row, ob0);
      if (ly >= 2 && ly < TY + 2) kv[it] = at_byte(la.coef + row, ob0);
    }
  }
  while (true) {
    // the lane's geometry, recomputed every pass from an opaque copy of its column (cheaper
    // than the registers the hoisted addresses and predicates would hold across the loop)
    int lx = lx0;
    asm volatile("" : "+v"(lx));
    const int gx = fx0 - 2 + lx;
    const bool inx = gx >= 0 && gx < n;
    const unsigned ob = (unsigned)min(max(gx, 0), n - 1) * (unsigned)sizeof(c32);
    const bool tcol = lx >= 2 && lx < TX + 2 && gx < n;
    int bn = b + 1;  // the next iterating right-hand side of the block
    if (active)
      while (bn < b_end && !active[bn]) ++bn;
#pragma unroll
    for (int it = 0; it < IE; ++it) {
      const int idx = threadIdx.x + it * 256;
      const int I = cxs + idx % CX, J = cys + idx / CX;
      const bool ok = I >= 0 && I < nc && J >= 0 && J < nc;
      if (idx < CX * CY) sE[idx / CX][idx % CX] = ok ? evc[it] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    c32 rn[IV], en[IE];  // the next right-hand side's r and coarse tile, loaded during the stages below
    if constexpr (K > 1)
      if (bn < b_end) {
        load_e(bn, en);
        load_r(bn, rn);
      }
    const float sc = scale_of(rs, b);
#pragma unroll
    for (int it = 0; it < IV; ++it) {  // v2 = W r + P e (zero outside the grid)
      const int ly = r0 + RPI * it, gy = fy0 - 2 + ly;
      c32 v2 = make_float2(0.f, 0.f);
      if (inx && gy >= 0 && gy < n) {
        rv[it] = cscale(rv[it], sc);
        const int I = (gx >> 1) - cxs, J = (gy >> 1) - cys, ox1 = gx & 1, oy = gy & 1;
        const c32 a = sE[J][I], bb = sE[J][I + ox1], c = sE[J + oy][I], d = sE[J + oy][I + ox1];
        v2 = cadd(cmul(rv[it], wv[it]), cscale(cadd(cadd(a, bb), cadd(c, d)), 0.25f));
      }
      sV[ly][lx] = v2;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IV; ++it) {  // z on the tile and a one-point ring (zero outside the grid)
      const int ly = r0 + RPI * it, gy = fy0 - 2 + ly;
      if (ly < 1 || ly > VY - 2) continue;
      if (lx < 1 || lx > VX - 2) continue;
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
      if (ly < 2 || ly >= TY + 2 || gy >= n) continue;
      if (!tcol) continue;
      const long long row = (long long)gy * n;
      const c32 zc = sZ[ly - 1][lx];
      const int ng = ghosts2(gx, gy, n);
      const c32 D = make_float2(4.0f - kv[it].x - ng * la.ghost.x, -kv[it].y - ng * la.ghost.y);
      const c32 nb = cadd(cadd(sZ[ly - 1][lx - 1], sZ[ly - 1][lx + 1]), cadd(sZ[ly - 2][lx], sZ[ly][lx]));
      at_byte(zb + row, ob) = zc;
      at_byte(wb + row, ob) = csub(cmul(D, zc), nb);
    }
    if (K == 1 || bn >= b_end) break;
    b = bn;
#pragma unroll
    for (int it = 0; it < IV; ++it) rv[it] = rn[it];
#pragma unroll
    for (int it = 0; it < IE; ++it) evc[it] = en[it];
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
__global__ __launch_bounds__(256) void k_down_col(VecSet r, ScaleSet rs, LevelArgs lv, float omega,
                                                  VecSet rc, int nc, const int* active, VecSet ev) {
  constexpr int TCX = 30, RXU = 2 * TCX + 3, RYU = 2 * TCY + 3, RPI = 4, VY = (RYU + RPI - 1) / RPI * RPI,
                IV = VY / RPI;
  constexpr int FX = RES ? RXU + 2 : 1, FY = RES ? RYU + 2 : 1;
  __shared__ c32 sV[VY][64];
  __shared__ c32 sS[VY][64];
  __shared__ c32 sF[FY][FX];
  const int n = lv.n;
  const int b = blockIdx.x;  // grid (right-hand side, tile column, tile row)
  if (active && !active[b]) return;
  const int cx0 = blockIdx.y * TCX, cy0 = blockIdx.z * TCY;
  const int fx0 = 2 * cx0 - 2, fy0 = 2 * cy0 - 2;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const int lx = threadIdx.x & 63;
  const int r0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wavefront's first region row
  const int gx = fx0 + lx;
  const bool inx = lx < RXU && gx >= 0 && gx < n;
  const unsigned ob = (unsigned)min(max(gx, 0), n - 1) * (unsigned)sizeof(c32);  // nearest in-grid column, bytes
  // with RES the fine correction, loaded from clamped in-grid addresses back to back with
  // the row loads; zeros outside the grid are put in at the LDS stores
  constexpr int IF = RES ? (FX * FY + 255) / 256 : 0;
  c32 fv[IF > 0 ? IF : 1];
  if constexpr (RES) {
    const c32* fb = ev.p + (long long)b * ev.stride;
#pragma unroll
    for (int it = 0; it < IF; ++it) {
      const int idx = min((int)threadIdx.x + it * 256, FX * FY - 1);
      const int fx = min(max(fx0 - 1 + idx % FX, 0), n - 1), fy = min(max(fy0 - 1 + idx / FX, 0), n - 1);
      fv[it] = fb[(long long)fy * n + fx];
    }
  }
  // rows are loaded from clamped in-grid columns without lane predicates; values of lanes
  // outside the grid are never used (every use below is guarded by the same condition)
  c32 rv[IV], wv[IV], kv[RES ? IV : 1];
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 + ly;
    if (ly < RYU && gy >= 0 && gy < n) {
      const long long row = (long long)gy * n;
      rv[it] = at_byte(rb + row, ob);
      wv[it] = at_byte(lv.wd + row, ob);
      if constexpr (RES) kv[it] = at_byte(lv.coef + row, ob);
    }
  }
  if constexpr (RES) {
#pragma unroll
    for (int it = 0; it < IF; ++it) {
      const int idx = threadIdx.x + it * 256;
      const int fx = fx0 - 1 + idx % FX, fy = fy0 - 1 + idx / FX;
      const bool ok = fx >= 0 && fx < n && fy >= 0 && fy < n;
      if (idx < FX * FY) sF[idx / FX][idx % FX] = ok ? fv[it] : make_float2(0.f, 0.f);
    }
    __syncthreads();
  }
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 + ly;
    c32 v1 = make_float2(0.f, 0.f);  // W r, zero outside the grid
    if (inx && ly < RYU && gy >= 0 && gy < n) {
      rv[it] = cscale(rv[it], sc);
      if constexpr (RES) {
        // r - K e with K e = D e - (sum of in-grid neighbours); sF is zero outside the grid
        const int ng = ghosts2(gx, gy, n);
        const c32 D = make_float2(4.0f - kv[it].x - ng * lv.ghost.x, -kv[it].y - ng * lv.ghost.y);
        const int fx = lx + 1, fy = ly + 1;
        const c32 nb = cadd(cadd(sF[fy][fx - 1], sF[fy][fx + 1]), cadd(sF[fy - 1][fx], sF[fy + 1][fx]));
        rv[it] = cadd(csub(rv[it], cmul(D, sF[fy][fx])), nb);
      }
      v1 = cmul(rv[it], wv[it]);
    }
    sV[ly][lx] = v1;
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
  for (int q = threadIdx.x; q < TCX * TCY; q += 256) {  // 30 x TCY coarse points may exceed the block
    const int tx = q % TCX, ty = q / TCX;
    const int I = cx0 + tx, J = cy0 + ty;
    if (I < nc && J < nc) {
      const int sx = 2 * tx + 2, sy = 2 * ty + 2;
      c32 acc = cscale(sS[sy][sx], 4.0f);
      acc = cadd(acc, cscale(cadd(cadd(sS[sy][sx - 1], sS[sy][sx + 1]), cadd(sS[sy - 1][sx], sS[sy + 1][sx])), 2.0f));
      acc = cadd(acc, cadd(cadd(sS[sy - 1][sx - 1], sS[sy - 1][sx + 1]), cadd(sS[sy + 1][sx - 1], sS[sy + 1][sx + 1])));
      at_byte(rc.p + (long long)b * rc.stride + (long long)J * nc, (unsigned)I * (unsigned)sizeof(c32)) =
          cscale(acc, 0.25f);
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
  // workgroup order (xcd_stretch): "right-hand sides fastest, then tiles in raster order",
  // one contiguous stretch per XCD
  const unsigned tiles_x = (unsigned)(n + TX - 1) / TX;
  const unsigned l = xcd_stretch(blockIdx.x, gridDim.x);
  const unsigned t = l / (unsigned)nrhs;
  const int b = (int)(l - t * (unsigned)nrhs);
  if (active && !active[b]) return;
  const int fx0 = (int)(t % tiles_x) * TX, fy0 = (int)(t / tiles_x) * TY;
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const c32* rb = r.p + (long long)b * r.stride;
  const float sc = scale_of(rs, b);
  const int lx = threadIdx.x & 63;
  const int r0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wavefront's first region row
  const int gx = fx0 - 1 + lx;
  const bool inx = gx >= 0 && gx < n;
  const unsigned ob = (unsigned)min(max(gx, 0), n - 1) * (unsigned)sizeof(c32);  // nearest in-grid column, bytes
  // the coarse tile (and with RES the fine correction) loaded from clamped in-grid
  // addresses, back to back with the row loads; zeros outside the grid are put in at
  // the LDS stores
  constexpr int IE = (CX * CY + 255) / 256, IF = RES ? (FX * FY + 255) / 256 : 0;
  c32 evc[IE], fv[IF > 0 ? IF : 1];
#pragma unroll
  for (int it = 0; it < IE; ++it) {
    const int idx = min((int)threadIdx.x + it * 256, CX * CY - 1);
    const int I = min(max(cxs + idx % CX, 0), nc - 1), J = min(max(cys + idx / CX, 0), nc - 1);
    evc[it] = eb[(long long)J * nc + I];
  }
  if constexpr (RES) {
    const c32* fb = ev.p + (long long)b * ev.stride;
#pragma unroll
    for (int it = 0; it < IF; ++it) {
      const int idx = min((int)threadIdx.x + it * 256, FX * FY - 1);
      const int fx = min(max(fx0 - 2 + idx % FX, 0), n - 1), fy = min(max(fy0 - 2 + idx / FX, 0), n - 1);
      fv[it] = fb[(long long)fy * n + fx];
    }
  }
  // rows from clamped in-grid columns without lane predicates; values of lanes outside
  // the grid are never used (every use below is guarded by the same condition)
  c32 rv[IV], wv[IV], kv[RES ? IV : 1];
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int gy = fy0 - 1 + r0 + RPI * it;
    if (gy >= 0 && gy < n) {
      const long long row = (long long)gy * n;
      rv[it] = at_byte(rb + row, ob);
      wv[it] = at_byte(lv.wd + row, ob);
      if constexpr (RES) kv[it] = at_byte(lv.coef + row, ob);
    }
  }
#pragma unroll
  for (int it = 0; it < IE; ++it) {
    const int idx = threadIdx.x + it * 256;
    const int I = cxs + idx % CX, J = cys + idx / CX;
    const bool ok = I >= 0 && I < nc && J >= 0 && J < nc;
    if (idx < CX * CY) sE[idx / CX][idx % CX] = ok ? evc[it] : make_float2(0.f, 0.f);
  }
  if constexpr (RES) {
#pragma unroll
    for (int it = 0; it < IF; ++it) {
      const int idx = threadIdx.x + it * 256;
      const int fx = fx0 - 2 + idx % FX, fy = fy0 - 2 + idx / FX;
      const bool ok = fx >= 0 && fx < n && fy >= 0 && fy < n;
      if (idx < FX * FY) sF[idx / FX][idx % FX] = ok ? fv[it] : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // v2 = W r + P e on the region (zero outside the grid)
    const int ly = r0 + RPI * it, gy = fy0 - 1 + ly;
    c32 v2 = make_float2(0.f, 0.f);
    if (inx && gy >= 0 && gy < n) {
      rv[it] = cscale(rv[it], sc);
      if constexpr (RES) {
        const int ng = ghosts2(gx, gy, n);
        const c32 D = make_float2(4.0f - kv[it].x - ng * lv.ghost.x, -kv[it].y - ng * lv.ghost.y);
        const int fx = lx + 1, fy = ly + 1;
        const c32 nb = cadd(cadd(sF[fy][fx - 1], sF[fy][fx + 1]), cadd(sF[fy - 1][fx], sF[fy + 1][fx]));
        rv[it] = cadd(csub(rv[it], cmul(D, sF[fy][fx])), nb);
      }
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
    at_byte(zb + (long long)gy * n, ob) = zv;
  }
}

// The finest-level step of the s-step basis in the column layout: up-leg of
// Z_j, W_{j+1} = A Z_j and the down-leg of W_{j+1} in one launch.  A 56 x 12
// tile; the region is 64 x 20 (a four-point ring): v2 on all of it, z on a
// three-point ring, W_{j+1} on a two-point ring (its v1 = W W_{j+1}), s on a
// one-point ring, and the coarse right-hand side of the 28 x 6 coarse points
// whose fine points lie in the tile.  The basis vector W_{j+1} carries scale 1.
// Same arithmetic per point as the separate kernels.
__global__ __launch_bounds__(256) void k_step_col(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la,
                                                  float omega, VecSet ec, int nc, VecSet z, VecSet w, VecSet rc,
                                                  const int* active) {
  constexpr int TX = 56, TY = 12, VY = TY + 8, RPI = 4, IV = VY / RPI;
  constexpr int CX = 33, CY = TY / 2 + 5, KX = TX / 2, KY = TY / 2;
  __shared__ c32 sE[CY][CX];
  __shared__ c32 sA[VY][64];  // v2, then v1 = W W_{j+1}
  __shared__ c32 sB[VY][64];  // z, then s
  const int n = lv.n;
  const int tiles_x = (n + TX - 1) / TX;
  const unsigned tiles = (unsigned)(tiles_x * ((n + TY - 1) / TY));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int fx0 = (id.t % tiles_x) * TX, fy0 = (id.t / tiles_x) * TY;
  const int cxs = fx0 / 2 - 2, cys = fy0 / 2 - 2;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const c32* rb = r.p + (long long)b * r.stride;
  const float sc = scale_of(rs, b);
  const int lx = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int gx = fx0 - 4 + lx;
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
  c32 rv[IV], wv[IV], kv[IV];
  bool ing[IV];
#pragma unroll
  for (int it = 0; it < IV; ++it) {
    const int ly = r0 + RPI * it, gy = fy0 - 4 + ly;
    ing[it] = inx && gy >= 0 && gy < n;
    const long long p = ing[it] ? (long long)gy * n + gx : 0;
    rv[it] = ing[it] ? cscale(rb[p], sc) : make_float2(0.f, 0.f);
    wv[it] = ing[it] ? lv.wd[p] : make_float2(0.f, 0.f);
    kv[it] = ing[it] && lx >= 2 && lx <= 61 && ly >= 2 && ly <= VY - 3 ? la.coef[p] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int it = 0; it < IE; ++it) {
    const int idx = threadIdx.x + it * 256;
    if (idx < CX * CY) sE[idx / CX][idx % CX] = evc[it];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // v2 = W r + P e
    const int ly = r0 + RPI * it, gy = fy0 - 4 + ly;
    c32 v2 = make_float2(0.f, 0.f);
    if (ing[it]) {
      const int I = (gx >> 1) - cxs, J = (gy >> 1) - cys, ox = gx & 1, oy = gy & 1;
      const c32 a = sE[J][I], bb = sE[J][I + ox], c = sE[J + oy][I], d = sE[J + oy][I + ox];
      v2 = cadd(cmul(rv[it], wv[it]), cscale(cadd(cadd(a, bb), cadd(c, d)), 0.25f));
    }
    sA[ly][lx] = v2;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // z on the three-point ring
    const int ly = r0 + RPI * it;
    if (lx < 1 || lx > 62 || ly < 1 || ly > VY - 2) continue;
    c32 zv = make_float2(0.f, 0.f);
    if (ing[it]) {
      const c32 nb = cadd(cadd(sA[ly][lx - 1], sA[ly][lx + 1]), cadd(sA[ly - 1][lx], sA[ly + 1][lx]));
      zv = cadd(cscale(sA[ly][lx], 1.0f - omega), cmul(wv[it], cadd(rv[it], nb)));
    }
    sB[ly][lx] = zv;
  }
  __syncthreads();
  c32* zb = z.p + (long long)b * z.stride;
  c32* wb = w.p + (long long)b * w.stride;
  c32 wn[IV];
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // W_{j+1} = A z on the two-point ring; v1 = W W_{j+1}
    const int ly = r0 + RPI * it, gy = fy0 - 4 + ly;
    wn[it] = make_float2(0.f, 0.f);
    if (lx < 2 || lx > 61 || ly < 2 || ly > VY - 3) continue;
    c32 v1 = make_float2(0.f, 0.f);
    if (ing[it]) {
      const c32 zc = sB[ly][lx];
      const int ng = ghosts2(gx, gy, n);
      const c32 D = make_float2(4.0f - kv[it].x - ng * la.ghost.x, -kv[it].y - ng * la.ghost.y);
      const c32 nb = cadd(cadd(sB[ly][lx - 1], sB[ly][lx + 1]), cadd(sB[ly - 1][lx], sB[ly + 1][lx]));
      wn[it] = csub(cmul(D, zc), nb);
      v1 = cmul(wn[it], wv[it]);
      if (lx >= 4 && lx < TX + 4 && ly >= 4 && ly < TY + 4) {
        const long long p = (long long)gy * n + gx;
        zb[p] = zc;
        wb[p] = wn[it];
      }
    }
    sA[ly][lx] = v1;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IV; ++it) {  // s = W_{j+1} - K v1 on the one-point ring
    const int ly = r0 + RPI * it;
    if (lx < 3 || lx > 60 || ly < 3 || ly > VY - 4) continue;
    c32 sv = make_float2(0.f, 0.f);
    if (ing[it]) {
      const c32 nb = cadd(cadd(sA[ly][lx - 1], sA[ly][lx + 1]), cadd(sA[ly - 1][lx], sA[ly + 1][lx]));
      sv = cadd(cscale(wn[it], 1.0f - omega), nb);
    }
    sB[ly][lx] = sv;
  }
  __syncthreads();
  if (threadIdx.x < KX * KY) {  // the coarse right-hand side 4 R s
    const int tx = threadIdx.x % KX, ty = threadIdx.x / KX;
    const int I = fx0 / 2 + tx, J = fy0 / 2 + ty;
    if (I < nc && J < nc) {
      const int sx = 2 * tx + 4, sy = 2 * ty + 4;
      c32 acc = cscale(sB[sy][sx], 4.0f);
      acc = cadd(acc, cscale(cadd(cadd(sB[sy][sx - 1], sB[sy][sx + 1]), cadd(sB[sy - 1][sx], sB[sy + 1][sx])), 2.0f));
      acc = cadd(acc, cadd(cadd(sB[sy - 1][sx - 1], sB[sy - 1][sx + 1]), cadd(sB[sy + 1][sx - 1], sB[sy + 1][sx + 1])));
      rc.p[(long long)b * rc.stride + (long long)J * nc + I] = cscale(acc, 0.25f);
    }
  }
}

// ------------------------------------------------------------ fused 3D legs
// The down-leg marching in z with a fixed thread map: 30 x 8 coarse points,
// fine region 63 x 19 (2 c0 - 2 origin); each lane owns one region column and
// every fourth row, keeping v1 of the planes f - 2 .. f and r of the plane it
// forms s on in registers (the next plane's loads in flight); only in-plane
// neighbours go through LDS.  Per fine plane f (bottom to top): v1(f) = W r;
// then s(f - 1) = r - K v1 on the region's interior; then the plane's in-plane
// full weighting is added to the coarse plane(s) it belongs to (weight 1/2 for
// f - 1 = 2K, 1/4 to K - 1 and K for f - 1 = 2K - 1), accumulated in
// registers; a coarse plane is written once complete.
constexpr int DCX = 30, DCY = 8, DKZ = 8, DRX = 2 * DCX + 3, DRY = 2 * DCY + 3, DIV = (DRY + 3) / 4;
__global__ __launch_bounds__(256) void k_down_march3c(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, float omega,
                                                      VecSet rc, int nc, const int* active) {
  __shared__ c32 sV[2][4 * DIV][64];
  __shared__ c32 sS[4 * DIV][64];
  const int n = lv.n;
  const int tx_n = (nc + DCX - 1) / DCX, ty_n = (nc + DCY - 1) / DCY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((nc + DKZ - 1) / DKZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int cx0 = (id.t % tx_n) * DCX, cy0 = ((id.t / tx_n) % ty_n) * DCY, kz0 = (id.t / (tx_n * ty_n)) * DKZ;
  const int kz1 = min(nc, kz0 + DKZ);
  const int fx0 = 2 * cx0 - 2, fy0 = 2 * cy0 - 2;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const long long n2 = (long long)n * n;
  const int lx = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int gx = fx0 + lx;
  const bool inx = lx < DRX && gx >= 0 && gx < n;
  bool in[DIV];
  long long off[DIV];
#pragma unroll
  for (int it = 0; it < DIV; ++it) {
    const int ly = r0 + 4 * it, gy = fy0 + ly;
    in[it] = inx && ly < DRY && gy >= 0 && gy < n;
    off[it] = in[it] ? (long long)gy * n + gx : 0;
  }
  c32 rn[DIV], wn[DIV];
  auto fetch = [&](int f) {
    const bool inz = f >= 0 && f < n;
#pragma unroll
    for (int it = 0; it < DIV; ++it) {
      const bool ok = inz && in[it];
      const long long p = ok ? f * n2 + off[it] : 0;
      rn[it] = ok ? rb[p] : make_float2(0.f, 0.f);
      wn[it] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
    }
  };
  const int f0 = 2 * kz0 - 2, f1 = 2 * kz1;  // fine planes whose v1 is needed
  fetch(f0);
  const int tx = threadIdx.x % DCX, ty = threadIdx.x / DCX;
  const bool coarse = threadIdx.x < DCX * DCY && cx0 + tx < nc && cy0 + ty < nc;
  c32 acc = make_float2(0.f, 0.f);
  c32 vm[DIV], vc[DIV], rp[DIV];
#pragma unroll
  for (int it = 0; it < DIV; ++it) vm[it] = vc[it] = rp[it] = make_float2(0.f, 0.f);
  for (int f = f0; f <= f1; ++f) {
    c32 rf[DIV], vf[DIV];
#pragma unroll
    for (int it = 0; it < DIV; ++it) {
      rf[it] = cscale(rn[it], sc);
      vf[it] = cmul(rf[it], wn[it]);
      sV[f & 1][r0 + 4 * it][lx] = vf[it];
    }
    if (f < f1) fetch(f + 1);
    __syncthreads();
    const int g = f - 1;  // the plane whose s is formed now
    if (g >= f0 + 1) {
      const bool ing = g >= 0 && g < n;
      const c32(*P)[64] = sV[g & 1];
#pragma unroll
      for (int it = 0; it < DIV; ++it) {
        const int ly = r0 + 4 * it;
        if (lx < 1 || lx > DRX - 2 || ly < 1 || ly > DRY - 2) continue;
        c32 sv = make_float2(0.f, 0.f);
        if (ing && in[it]) {
          const c32 nb = cadd(cadd(cadd(P[ly][lx - 1], P[ly][lx + 1]), cadd(P[ly - 1][lx], P[ly + 1][lx])),
                              cadd(vm[it], vf[it]));
          sv = cadd(cscale(rp[it], 1.0f - omega), nb);
        }
        sS[ly][lx] = sv;
      }
    }
    __syncthreads();
    if (g >= f0 + 1 && coarse) {
      const int sx = 2 * tx + 2, sy = 2 * ty + 2;
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
    for (int it = 0; it < DIV; ++it) {
      vm[it] = vc[it];
      vc[it] = vf[it];
      rp[it] = rf[it];
    }
  }
}

// The up-leg marching in z with a fixed thread map: a 64 x 8 column, two own
// points per thread (x and x + 32) and a one-point in-plane ring (148 threads
// take one ring point each).  Each thread keeps its own points' v2 of the
// planes f - 2 .. f and r, W of the plane it smooths in registers, with the
// next plane's loads in flight; only the in-plane neighbours go through LDS
// (two planes).  Per fine plane f: v2(f) = W r + P e (the coarse planes that P
// reads are kept two at a time in LDS), then z(f - 1) from v2(f - 2 .. f).  With acc
// the leg adds z to the output instead of overwriting it (a repeated coarse visit:
// e + MG(r - K e, 0) without a separate pass).
constexpr int UX = 64, UY = 8, UZ = 16, URING = 2 * (UX + 2) + 2 * UY;
__global__ __launch_bounds__(256) void k_up_march3c(int nrhs, VecSet r, ScaleSet rs, LevelArgs lv, float omega,
                                                    VecSet ec, int nc, VecSet z, const int* active, int acc) {
  constexpr int CX = UX / 2 + 2, CY = UY / 2 + 2, NCP = CX * CY, ITC = (NCP + 255) / 256;
  __shared__ c32 sE[2][CY][CX];
  __shared__ c32 sV[2][UY + 2][UX + 2];
  const int n = lv.n;
  const int tx_n = (n + UX - 1) / UX, ty_n = (n + UY - 1) / UY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((n + UZ - 1) / UZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int fx0 = (id.t % tx_n) * UX, fy0 = ((id.t / tx_n) % ty_n) * UY, fz0 = (id.t / (tx_n * ty_n)) * UZ;
  const int fz1 = min(n, fz0 + UZ);
  const int cxs = fx0 / 2 - 1, cys = fy0 / 2 - 1;
  const float sc = scale_of(rs, b);
  const c32* rb = r.p + (long long)b * r.stride;
  const c32* eb = ec.p + (long long)b * ec.stride;
  const long long n2 = (long long)n * n, nc2 = (long long)nc * nc;
  // points of this thread: q = 0, 1 own, q = 2 the ring point (if any); LDS coordinates (lx, ly)
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  int lxq[3], lyq[3];
  lxq[0] = tx + 1, lyq[0] = ty + 1, lxq[1] = tx + 33, lyq[1] = ty + 1;
  {
    const int t = threadIdx.x;
    int rx = -1, ry = -1;
    if (t < UX + 2) rx = t, ry = 0;
    else if (t < 2 * (UX + 2)) rx = t - (UX + 2), ry = UY + 1;
    else if (t < 2 * (UX + 2) + UY) rx = 0, ry = t - 2 * (UX + 2) + 1;
    else if (t < URING) rx = UX + 1, ry = t - 2 * (UX + 2) - UY + 1;
    lxq[2] = rx, lyq[2] = ry;
  }
  bool in[3];
  long long off[3];
  int gxq[3], gyq[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    gxq[q] = fx0 - 1 + lxq[q], gyq[q] = fy0 - 1 + lyq[q];
    in[q] = lxq[q] >= 0 && gxq[q] >= 0 && gxq[q] < n && gyq[q] >= 0 && gyq[q] < n;
    off[q] = in[q] ? (long long)gyq[q] * n + gxq[q] : 0;
  }
  long long coff[ITC];
  bool cin[ITC];
#pragma unroll
  for (int it = 0; it < ITC; ++it) {
    const int idx = threadIdx.x + it * 256;
    const int I = cxs + idx % CX, J = cys + idx / CX;
    cin[it] = idx < NCP && I >= 0 && I < nc && J >= 0 && J < nc;
    coff[it] = cin[it] ? (long long)J * nc + I : 0;
  }
  c32 rn[3], wn[3], cn[ITC];
  auto fetch = [&](int f) {
    const bool inz = f >= 0 && f < n;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const bool ok = inz && in[q];
      const long long p = ok ? f * n2 + off[q] : 0;
      rn[q] = ok ? rb[p] : make_float2(0.f, 0.f);
      wn[q] = ok ? lv.wd[p] : make_float2(0.f, 0.f);
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
      const int idx = threadIdx.x + it * 256;
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
  __syncthreads();
  c32 vm[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)}, vc[2] = {vm[0], vm[1]};
  c32 rc[2] = {vm[0], vm[1]}, wc[2] = {vm[0], vm[1]};  // r (scaled) and W of plane f - 1
  c32* zb = z.p + (long long)b * z.stride;
  for (int f = fa; f <= fb; ++f) {
    c32 rf[3], wf[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      rf[q] = cscale(rn[q], sc);
      wf[q] = wn[q];
    }
    const int knext = (f + 2) >> 1;  // the higher coarse plane that v2(f + 1) reads
    if (f < fb) {
      fetch(f + 1);
      if (knext > khi) fetch_coarse(knext);
    }
    // v2(f) = W r + P e at the own points and the ring point
    c32 vf[3];
    const bool inz = f >= 0 && f < n;
    const int klo = f >> 1;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      vf[q] = make_float2(0.f, 0.f);
      if (inz && in[q]) {
        c32 pe = prolong_lds<CX>(sE[klo & 1], gxq[q], gyq[q], cxs, cys);
        if (f & 1) pe = cscale(cadd(pe, prolong_lds<CX>(sE[(klo + 1) & 1], gxq[q], gyq[q], cxs, cys)), 0.5f);
        vf[q] = cadd(cmul(rf[q], wf[q]), pe);
      }
      if (lxq[q] >= 0) sV[f & 1][lyq[q]][lxq[q]] = vf[q];
    }
    __syncthreads();
    if (f < fb && knext > khi) {  // the coarse plane that replaces one no longer read
      store_coarse(knext);
      khi = knext;
    }
    const int g = f - 1;  // output plane
    if (g >= fz0) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (!in[q]) continue;
        const int lx = lxq[q], ly = lyq[q];
        const c32(*P)[UX + 2] = sV[g & 1];
        const c32 nb = cadd(cadd(cadd(P[ly][lx - 1], P[ly][lx + 1]), cadd(P[ly - 1][lx], P[ly + 1][lx])),
                            cadd(vm[q], vf[q]));
        const c32 zv = cadd(cscale(vc[q], 1.0f - omega), cmul(wc[q], cadd(rc[q], nb)));
        const long long p = g * n2 + off[q];
        zb[p] = acc ? cadd(zb[p], zv) : zv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      vm[q] = vc[q];
      vc[q] = vf[q];
      rc[q] = rf[q];
      wc[q] = wf[q];
    }
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

// The same residual in 3D, marching in z: a 64 x 8 column over 16 planes, two
// points per thread, the in-plane neighbours from an LDS copy of the plane and a
// one-point ring, the planes below and above in registers with the next plane's
// loads in flight (the flat kernel's z-neighbours, a plane apart, mostly miss the
// L2).  Neighbours summed in the order of neighbour_sum (zero outside the grid).
constexpr int RMX = 64, RMY = 8, RMZ = 16;
__global__ __launch_bounds__(256) void k_level_residual_march3(int nrhs, VecSet bvec, ScaleSet bs, VecSet v,
                                                               LevelArgs lv, VecSet out, const int* active) {
  __shared__ c32 sP[RMY + 2][RMX + 2];
  const int n = lv.n;
  const int tx_n = (n + RMX - 1) / RMX, ty_n = (n + RMY - 1) / RMY;
  const unsigned tiles = (unsigned)(tx_n * ty_n * ((n + RMZ - 1) / RMZ));
  const TileId id = xcd_tile(blockIdx.x, nrhs, tiles, HELM_RHS_GROUP);
  const int b = id.b;
  if (active && !active[b]) return;
  const int x0 = (id.t % tx_n) * RMX, y0 = ((id.t / tx_n) % ty_n) * RMY, z0 = (id.t / (tx_n * ty_n)) * RMZ;
  const int z1 = min(n, z0 + RMZ);
  const c32* vb = v.p + (long long)b * v.stride;
  const c32* bb = bvec.p + (long long)b * bvec.stride;
  c32* ob = out.p + (long long)b * out.stride;
  const float sc = scale_of(bs, b);
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
    if (t < RMX + 2) rx = t, ry = 0;
    else if (t < 2 * (RMX + 2)) rx = t - (RMX + 2), ry = RMY + 1;
    else if (t < 2 * (RMX + 2) + RMY) rx = 0, ry = t - 2 * (RMX + 2) + 1;
    else if (t < 2 * (RMX + 2) + 2 * RMY) rx = RMX + 1, ry = t - 2 * (RMX + 2) - RMY + 1;
  }
  const int rgx = x0 - 1 + rx, rgy = y0 - 1 + ry;
  const bool ring = rx >= 0 && rgx >= 0 && rgx < n && rgy >= 0 && rgy < n;
  const long long ro = ring ? (long long)rgy * n + rgx : 0;
  auto at = [&](bool ok, int zz, long long off) {
    return ok && zz >= 0 && zz < n ? vb[zz * n2 + off] : make_float2(0.f, 0.f);
  };
  c32 vm[2], vc[2], vp[2], kc[2], bc[2];
  c32 vr = at(ring, z0, ro);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    vm[h] = at(own[h], z0 - 1, o[h]);
    vc[h] = at(own[h], z0, o[h]);
    vp[h] = at(own[h], z0 + 1, o[h]);
    kc[h] = own[h] ? lv.coef[z0 * n2 + o[h]] : make_float2(0.f, 0.f);
    bc[h] = own[h] ? bb[z0 * n2 + o[h]] : make_float2(0.f, 0.f);
  }
  for (int zz = z0; zz < z1; ++zz) {
#pragma unroll
    for (int h = 0; h < 2; ++h) sP[ty + 1][tx + 1 + 32 * h] = vc[h];
    if (rx >= 0) sP[ry][rx] = vr;
    c32 vn[2], kn[2], bn[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      vn[h] = at(own[h], zz + 2, o[h]);
      const bool nx = own[h] && zz + 1 < n;
      kn[h] = nx ? lv.coef[(zz + 1) * n2 + o[h]] : make_float2(0.f, 0.f);
      bn[h] = nx ? bb[(zz + 1) * n2 + o[h]] : make_float2(0.f, 0.f);
    }
    const c32 vrn = at(ring, zz + 1, ro);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!own[h]) continue;
      const int lx = tx + 1 + 32 * h, ly = ty + 1;
      const int ng = ghosts3(x0 + tx + 32 * h, y0 + ty, zz, n);
      const c32 D = make_float2(6.0f - kc[h].x - ng * lv.ghost.x, -kc[h].y - ng * lv.ghost.y);
      c32 nb = make_float2(0.f, 0.f);
      nb = cadd(nb, sP[ly][lx - 1]);
      nb = cadd(nb, sP[ly][lx + 1]);
      nb = cadd(nb, sP[ly - 1][lx]);
      nb = cadd(nb, sP[ly + 1][lx]);
      nb = cadd(nb, vm[h]);
      nb = cadd(nb, vp[h]);
      ob[zz * n2 + o[h]] = csub(cscale(bc[h], sc), csub(cmul(D, vc[h]), nb));
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      vm[h] = vc[h];
      vc[h] = vp[h];
      vp[h] = vn[h];
      kc[h] = kn[h];
      bc[h] = bn[h];
    }
    vr = vrn;
  }
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
constexpr DownTile kDown[] = {{32, 8}, {16, 16}, {64, 4}, {32, 4}, {16, 8}, {30, 8}, {30, 16}};
constexpr UpTile kUp[] = {{64, 16, 4}, {32, 16, 2}, {64, 8, 2}, {32, 32, 4}, {64, 32, 8}, {62, 14, 0}, {62, 30, 0}};
constexpr int kDownCol = 5, kDownCol16 = 6, kUpCol = 5, kUpCol30 = 6;

// launch shapes of the fused finest up-leg + basis matvec (k_up_mv2w), one autotuner
// choice: tile height and right-hand sides per block
struct UpMvShape {
  int rows, k;
};
constexpr UpMvShape kUpMv[] = {{16, 4}, {12, 1}, {20, 1}, {28, 1}, {12, 2}, {12, 4}, {12, 6}, {20, 2}, {20, 4}};

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
  const int tiles = ((nc + DCX - 1) / DCX) * ((nc + DCY - 1) / DCY) * ((nc + DKZ - 1) / DKZ);
  hipLaunchKernelGGL(k_down_march3c, dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, rc, nc, active);
}

void launch_up_fused3(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet ec, int nc,
                      VecSet z, const int* active, int acc) {
  const int n = lv.n;
  const int tiles = ((n + UX - 1) / UX) * ((n + UY - 1) / UY) * ((n + UZ - 1) / UZ);
  hipLaunchKernelGGL(k_up_march3c, dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z, active, acc);
}

template <int TY, int K>
void up_mv2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la, float omega, VecSet ec, int nc,
            VecSet z, VecSet w, const int* active) {
  constexpr int TX = 60;
  const int n = lv.n;
  const int blocks = (B + K - 1) / K * ((n + TX - 1) / TX) * ((n + TY - 1) / TY);
  hipLaunchKernelGGL((k_up_mv2w<TY, K>), dim3(blocks), dim3(256), 0, s, B, r, rs, lv, la, omega, ec, nc, z, w, active);
}

int mg_up_mv_variants() { return (int)(sizeof(kUpMv) / sizeof(kUpMv[0])); }
int mg_up_mv_rows(int cfg) { return kUpMv[cfg].rows; }
int mg_up_mv_rhs_per_block(int cfg) { return kUpMv[cfg].k; }

void launch_up_mv2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la, float omega, VecSet ec,
                   int nc, VecSet z, VecSet w, const int* active, int cfg) {
#define HELM_UP_MV(TY_, K_)                                                     \
  if (kUpMv[cfg].rows == TY_ && kUpMv[cfg].k == K_) {                           \
    up_mv2<TY_, K_>(s, B, r, rs, lv, la, omega, ec, nc, z, w, active);          \
    return;                                                                     \
  }
  HELM_UP_MV(12, 1) HELM_UP_MV(20, 1) HELM_UP_MV(28, 1) HELM_UP_MV(12, 2) HELM_UP_MV(12, 4)
  HELM_UP_MV(12, 6) HELM_UP_MV(20, 2) HELM_UP_MV(20, 4)
#undef HELM_UP_MV
  up_mv2<16, 4>(s, B, r, rs, lv, la, omega, ec, nc, z, w, active);
}

void launch_step_fused2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la, float omega,
                        VecSet ec, int nc, VecSet z, VecSet w, VecSet rc, const int* active) {
  constexpr int TX = 56, TY = 12;
  const int tiles = ((lv.n + TX - 1) / TX) * ((lv.n + TY - 1) / TY);
  hipLaunchKernelGGL(k_step_col, dim3(B * tiles), dim3(256), 0, s, B, r, rs, lv, la, omega, ec, nc, z, w, rc,
                     active);
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
    const dim3 grid(B, (nc + TCX - 1) / TCX, (nc + TCY - 1) / TCY);
    if (e.p)
      hipLaunchKernelGGL((k_down_col<TCY, true>), grid, dim3(256), 0, s, r, rs, lv, omega, rc, nc, active, e);
    else
      hipLaunchKernelGGL((k_down_col<TCY, false>), grid, dim3(256), 0, s, r, rs, lv, omega, rc, nc, active, e);
    return;
  }
  if (cfg == kDownCol16) {  // taller column tile: fewer halo rows per coarse row
    constexpr int TCX = 30, TCY = 16;
    const dim3 grid(B, (nc + TCX - 1) / TCX, (nc + TCY - 1) / TCY);
    if (e.p)
      hipLaunchKernelGGL((k_down_col<TCY, true>), grid, dim3(256), 0, s, r, rs, lv, omega, rc, nc, active, e);
    else
      hipLaunchKernelGGL((k_down_col<TCY, false>), grid, dim3(256), 0, s, r, rs, lv, omega, rc, nc, active, e);
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
    const int blocks = B * ((lv.n + TX - 1) / TX) * ((lv.n + TY - 1) / TY);
    if (e.p)
      hipLaunchKernelGGL((k_up_col<TY, true>), dim3(blocks), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z, active,
                         e);
    else
      hipLaunchKernelGGL((k_up_col<TY, false>), dim3(blocks), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z, active,
                         e);
    return;
  }
  if (cfg == kUpCol30) {  // taller column tile
    constexpr int TX = 62, TY = 30;
    const int blocks = B * ((lv.n + TX - 1) / TX) * ((lv.n + TY - 1) / TY);
    if (e.p)
      hipLaunchKernelGGL((k_up_col<TY, true>), dim3(blocks), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z, active,
                         e);
    else
      hipLaunchKernelGGL((k_up_col<TY, false>), dim3(blocks), dim3(256), 0, s, B, r, rs, lv, omega, ec, nc, z, active,
                         e);
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
  if (dim == 3) {
    const int n = lv.n;
    const int tiles = ((n + RMX - 1) / RMX) * ((n + RMY - 1) / RMY) * ((n + RMZ - 1) / RMZ);
    hipLaunchKernelGGL(k_level_residual_march3, dim3(B * tiles), dim3(256), 0, s, B, bvec, bs, v, lv, out, active);
    return;
  }
  hipLaunchKernelGGL(k_level_residual, dim3(nblocks(lv.N, 256), B), dim3(256), 0, s, dim, bvec, bs, v, lv, out,
                     active);
}

void launch_add(hipStream_t s, int B, VecSet x, VecSet y, long long N, const int* active) {
  hipLaunchKernelGGL(k_add, dim3(nblocks(N, 256), B), dim3(256), 0, s, x, y, N, active);
}
