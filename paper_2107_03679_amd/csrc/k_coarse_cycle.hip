// The coarse part of a V-cycle (Alg. 2, nu1 = nu2 = 1, zero initial guess)
// for levels lp .. L-1 in ONE launch: one workgroup per right-hand side.
// The right-hand sides are independent, so every sweep of a level only
// needs a workgroup barrier; the level buffers of one right-hand side stay
// in L2.  Per level l (h_l^2-scaled operators, W = omega / diag(K_l)):
//   down: e = W r;  t = r - K e = (1 - w) r + sum of neighbours of e;  r_{l+1} = 4 R t
//   coarsest: e = K^-1 r (explicit inverse)
//   up:   t = e + P e_{l+1};  e = (1 - w) t + W (r + sum of neighbours of t)
#include "dev_common.h"
#include "kernels.h"

namespace {

constexpr int CC_NT = 1024;

// 4 * full weighting of s at coarse point C (neighbours outside the fine grid count as 0)
__device__ __forceinline__ c32 fw4(const c32* s, const Coord& C, int nf, int dim) {
  const float w1[3] = {0.25f, 0.5f, 0.25f};
  c32 acc = make_float2(0.f, 0.f);
  const int zr = dim == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int fx = 2 * C.x + dx, fy = 2 * C.y + dy, fz = dim == 3 ? 2 * C.z + dz : 0;
        if (fx < 0 || fx >= nf || fy < 0 || fy >= nf || fz < 0 || fz >= nf) continue;
        const float wgt = w1[dx + 1] * w1[dy + 1] * (dim == 3 ? w1[dz + 1] : 1.0f);
        acc = cadd(acc, cscale(s[((long long)fz * nf + fy) * nf + fx], wgt));
      }
  return cscale(acc, 4.0f);
}

// (P e)(f): bilinear / trilinear prolongation from the coarse grid (nc points per side)
__device__ __forceinline__ c32 prolong_at(const c32* e, const Coord& f, int nc, int dim) {
  c32 acc = make_float2(0.f, 0.f);
  const int oz = dim == 3 ? (f.z & 1) : 0;
  for (int kz = 0; kz <= oz; ++kz)
    for (int ky = 0; ky <= (f.y & 1); ++ky)
      for (int kx = 0; kx <= (f.x & 1); ++kx) {
        const int I = (f.x >> 1) + kx, J = (f.y >> 1) + ky, K = dim == 3 ? (f.z >> 1) + kz : 0;
        const float wgt = ((f.x & 1) ? 0.5f : 1.0f) * ((f.y & 1) ? 0.5f : 1.0f) * (oz ? 0.5f : 1.0f);
        acc = cadd(acc, cscale(e[((long long)K * nc + J) * nc + I], wgt));
      }
  return acc;
}

__global__ __launch_bounds__(CC_NT) void k_coarse_cycle(CoarseCycleArgs a) {
  __shared__ c32 red[CC_NT];
  const int b = blockIdx.x;
  if (a.active && !a.active[b]) return;
  const int dim = a.dim;
  const float om = a.omega;
  // ---- down ----
  for (int l = a.lp; l < a.L - 1; ++l) {
    const CoarseLevel& F = a.lv[l];
    const CoarseLevel& C = a.lv[l + 1];
    const c32* r = F.rc + (long long)b * F.N;
    c32* e = F.e + (long long)b * F.N;
    c32* t = F.t + (long long)b * F.N;
    for (int p = threadIdx.x; p < F.N; p += CC_NT) e[p] = cmul(F.wd[p], r[p]);
    __syncthreads();
    for (int p = threadIdx.x; p < F.N; p += CC_NT) {
      const Coord c = coord_of32((unsigned)p, (unsigned)F.n, dim);
      t[p] = cadd(cscale(r[p], 1.0f - om), neighbour_sum(e, p, c, F.n, dim));
    }
    __syncthreads();
    c32* rcn = C.rc + (long long)b * C.N;
    for (int q = threadIdx.x; q < C.N; q += CC_NT) {
      const Coord cq = coord_of32((unsigned)q, (unsigned)C.n, dim);
      rcn[q] = fw4(t, cq, F.n, dim);
    }
    __syncthreads();
  }
  // ---- coarsest: e = M r, rows split over thread groups, partial sums reduced in LDS ----
  {
    const CoarseLevel& Q = a.lv[a.L - 1];
    const int Nc = (int)Q.N;
    const c32* r = Q.rc + (long long)b * Nc;
    c32* e = Q.e + (long long)b * Nc;
    const int groups = max(1, CC_NT / max(Nc, 1));  // k-split factor when Nc < CC_NT
    for (int row0 = 0; row0 < Nc; row0 += CC_NT / groups) {
      const int rows = min(CC_NT / groups, Nc - row0);
      const int g = threadIdx.x / (CC_NT / groups), rr = threadIdx.x % (CC_NT / groups);
      c32 acc = make_float2(0.f, 0.f);
      if (g < groups && rr < rows) {
        for (int k = g; k < Nc; k += groups) acc = cfma(a.minvT[(long long)k * Nc + row0 + rr], r[k], acc);
      }
      red[threadIdx.x] = acc;
      __syncthreads();
      if (threadIdx.x < rows) {
        c32 s2 = make_float2(0.f, 0.f);
        for (int q = 0; q < groups; ++q) s2 = cadd(s2, red[q * (CC_NT / groups) + threadIdx.x]);
        e[row0 + threadIdx.x] = s2;
      }
      __syncthreads();
    }
  }
  // ---- up ----
  for (int l = a.L - 2; l >= a.lp; --l) {
    const CoarseLevel& F = a.lv[l];
    const CoarseLevel& C = a.lv[l + 1];
    const c32* r = F.rc + (long long)b * F.N;
    c32* e = F.e + (long long)b * F.N;
    c32* t = F.t + (long long)b * F.N;
    const c32* ec = C.e + (long long)b * C.N;
    for (int p = threadIdx.x; p < F.N; p += CC_NT) {
      const Coord c = coord_of32((unsigned)p, (unsigned)F.n, dim);
      t[p] = cadd(e[p], prolong_at(ec, c, C.n, dim));
    }
    __syncthreads();
    for (int p = threadIdx.x; p < F.N; p += CC_NT) {
      const Coord c = coord_of32((unsigned)p, (unsigned)F.n, dim);
      e[p] = cadd(cscale(t[p], 1.0f - om), cmul(F.wd[p], cadd(r[p], neighbour_sum(t, p, c, F.n, dim))));
    }
    __syncthreads();
  }
}

// The same cycle with every level's right-hand side, solution and scratch in
// LDS (dynamic shared memory, laid out level after level, then CC_NT
// reduction slots): the input right-hand side is read once and the solution
// written once; every other access of the cycle stays on the CU.  Used when
// the levels fit (see coarse_cycle_lds_bytes).
// Offset in the LDS layout of level l's block (r, e, t; r, e on the coarsest;
// the reduction slots after the coarsest).  Uniform scalar arithmetic: the
// per-level pointers are formed where used instead of living in a
// dynamically indexed (scratch) array.
__device__ __forceinline__ int lds_base(const CoarseCycleArgs& a, int l) {
  int o = 0;
  for (int q = a.lp; q < l; ++q) o += (q < a.L - 1 ? 3 : 2) * (int)a.lv[q].N;
  return o;
}

__global__ __launch_bounds__(CC_NT) void k_coarse_cycle_lds(CoarseCycleArgs a) {
  extern __shared__ c32 lds[];
  const int b = blockIdx.x;
  if (a.active && !a.active[b]) return;
  const int dim = a.dim;
  const float om = a.omega;
  auto R = [&](int l) { return lds + lds_base(a, l); };
  auto E = [&](int l) { return lds + lds_base(a, l) + (int)a.lv[l].N; };
  auto T = [&](int l) { return l < a.L - 1 ? lds + lds_base(a, l) + 2 * (int)a.lv[l].N : lds + lds_base(a, a.L); };
  // The coarsest solve's entries of this thread, loaded now when they fit in
  // registers (one pass of rows, at most MK per thread), so that the solve
  // waits on no global load.
  constexpr int MK = 10;
  const int Ncst = (int)a.lv[a.L - 1].N;
  const int groups = max(1, CC_NT / max(Ncst, 1));
  const bool pre = Ncst <= CC_NT && (Ncst + groups - 1) / groups <= MK;
  c32 mk[MK];
  if (pre) {
    const int g = threadIdx.x / (CC_NT / groups), rr = threadIdx.x % (CC_NT / groups);
    const bool mine = g < groups && rr < Ncst;
#pragma unroll
    for (int u = 0; u < MK; ++u) {
      const int k = g + u * groups;
      mk[u] = mine && k < Ncst ? a.minvT[(long long)k * Ncst + rr] : make_float2(0.f, 0.f);
    }
  }
  {
    const CoarseLevel& F = a.lv[a.lp];
    const c32* rg = F.rc + (long long)b * F.N;
    for (int p = threadIdx.x; p < F.N; p += CC_NT) R(a.lp)[p] = rg[p];
  }
  __syncthreads();
  // ---- down ----
  for (int l = a.lp; l < a.L - 1; ++l) {
    const CoarseLevel& F = a.lv[l];
    const CoarseLevel& C = a.lv[l + 1];
    const int Nf = (int)F.N, Ncl = (int)C.N;
    c32 *r = R(l), *e = E(l), *t = T(l);
    for (int p = threadIdx.x; p < Nf; p += CC_NT) e[p] = cmul(F.wd[p], r[p]);
    __syncthreads();
    for (int p = threadIdx.x; p < Nf; p += CC_NT) {
      const Coord c = coord_of32((unsigned)p, (unsigned)F.n, dim);
      t[p] = cadd(cscale(r[p], 1.0f - om), neighbour_sum(e, p, c, F.n, dim));
    }
    __syncthreads();
    for (int q = threadIdx.x; q < Ncl; q += CC_NT) {
      const Coord cq = coord_of32((unsigned)q, (unsigned)C.n, dim);
      R(l + 1)[q] = fw4(t, cq, F.n, dim);
    }
    __syncthreads();
  }
  // ---- coarsest: e = M r, rows split over thread groups, partial sums reduced in LDS ----
  {
    const int Nc = Ncst;
    const c32* r = R(a.L - 1);
    c32* e = E(a.L - 1);
    c32* red = T(a.L - 1);
    for (int row0 = 0; row0 < Nc; row0 += CC_NT / groups) {
      const int rows = min(CC_NT / groups, Nc - row0);
      const int g = threadIdx.x / (CC_NT / groups), rr = threadIdx.x % (CC_NT / groups);
      c32 acc = make_float2(0.f, 0.f);
      if (g < groups && rr < rows) {
        if (pre) {
#pragma unroll
          for (int u = 0; u < MK; ++u) {
            const int k = g + u * groups;
            if (k < Nc) acc = cfma(mk[u], r[k], acc);
          }
        } else {
          for (int k = g; k < Nc; k += groups) acc = cfma(a.minvT[(long long)k * Nc + row0 + rr], r[k], acc);
        }
      }
      red[threadIdx.x] = acc;
      __syncthreads();
      if (threadIdx.x < rows) {
        c32 s2 = make_float2(0.f, 0.f);
        for (int q = 0; q < groups; ++q) s2 = cadd(s2, red[q * (CC_NT / groups) + threadIdx.x]);
        e[row0 + threadIdx.x] = s2;
      }
      __syncthreads();
    }
    if (a.lp == a.L - 1) {  // the coarsest level alone
      c32* eg = a.lv[a.lp].e + (long long)b * Nc;
      for (int p = threadIdx.x; p < Nc; p += CC_NT) eg[p] = e[p];
    }
  }
  // ---- up ----
  for (int l = a.L - 2; l >= a.lp; --l) {
    const CoarseLevel& F = a.lv[l];
    const CoarseLevel& C = a.lv[l + 1];
    const int Nf = (int)F.N;
    c32 *r = R(l), *e = E(l), *t = T(l);
    const c32* ec = E(l + 1);
    for (int p = threadIdx.x; p < Nf; p += CC_NT) {
      const Coord c = coord_of32((unsigned)p, (unsigned)F.n, dim);
      t[p] = cadd(e[p], prolong_at(ec, c, C.n, dim));
    }
    __syncthreads();
    if (l == a.lp) {
      c32* eg = F.e + (long long)b * F.N;
      for (int p = threadIdx.x; p < Nf; p += CC_NT) {
        const Coord c = coord_of32((unsigned)p, (unsigned)F.n, dim);
        eg[p] = cadd(cscale(t[p], 1.0f - om), cmul(F.wd[p], cadd(r[p], neighbour_sum(t, p, c, F.n, dim))));
      }
    } else {
      for (int p = threadIdx.x; p < Nf; p += CC_NT) {
        const Coord c = coord_of32((unsigned)p, (unsigned)F.n, dim);
        e[p] = cadd(cscale(t[p], 1.0f - om), cmul(F.wd[p], cadd(r[p], neighbour_sum(t, p, c, F.n, dim))));
      }
      __syncthreads();
    }
  }
}

}  // namespace

// LDS bytes k_coarse_cycle_lds needs for levels lp .. L-1 (r, e, t per level,
// r, e on the coarsest, CC_NT reduction slots)
size_t coarse_cycle_lds_bytes(const CoarseCycleArgs& a) {
  size_t n = CC_NT;
  for (int l = a.lp; l < a.L; ++l) n += (size_t)(l < a.L - 1 ? 3 : 2) * (size_t)a.lv[l].N;
  return n * sizeof(c32);
}

void launch_coarse_cycle(hipStream_t s, int B, const CoarseCycleArgs& a) {
  const size_t lds = coarse_cycle_lds_bytes(a);
  if (lds <= kCoarseCycleMaxLds)
    hipLaunchKernelGGL(k_coarse_cycle_lds, dim3(B), dim3(CC_NT), lds, s, a);
  else
    hipLaunchKernelGGL(k_coarse_cycle, dim3(B), dim3(CC_NT), 0, s, a);
}
