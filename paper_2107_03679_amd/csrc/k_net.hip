// Kernels of the learned preconditioner network (BF16 storage, FP32
// accumulation, v_mfma_f32_16x16x32_bf16 on gfx950).
//
// Activations are NHWC (NDHWC in 3D): element (pixel p, channel c) of a buffer
// with channel stride ct at channel offset off is buf[p * ct + off + c]; pixels
// are flattened over (image, z, y, x), with depth 1 for the 2D network.  A 3x3
// (3x3x3) convolution is an implicit GEMM
//     out[p][co] = bias[co] + sum_k in[p + shift(tap(k))][ci(k)] * Wt[co][k],
//     k = tap * cin + ci,  tap = 3 (dy + 1) + (dx + 1)  (+ 9 (dz + 1) in 3D),
// with the weights packed as Wt[co][k] (k padded to a multiple of 32).
// MFMA 16x16x32 operand layout (lane l, g = l / 16):
//     A[i][k]: i = l % 16, k = 8 g + v (v = 0..7)      (16 pixels x 32 k)
//     B[k][j]: j = l % 16, k = 8 g + v                 (32 k x 16 channels)
//     D[i][j]: j = l % 16, i = 4 g + r (r = 0..3)
// The forward / backward-data convolution passes the weights as A and the
// activations as B, so that D is [output channel][pixel].
#include <algorithm>
#include <type_traits>

#include "dev_common.h"
#include "net.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ bf16x8 load8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int v = 0; v < 8; ++v) z[v] = (__bf16)0.0f;
  return z;
}

// ---------------------------------------------------------------- layer inputs
// Address of 8 input channels [ci0, ci0 + 8) of pixel (z, y, x) of one image for the
// convolution's halo staging (MODE 0: plain, 2: upsample + skip), with (z, y, x) clamped
// into the layer (depth D, 1 in 2D); for MODE 1 (pool) the first of the 2^NDIM source
// pixels, clamped likewise.  in_img: the input's image (in_off applied), up_img: the
// upsampled tensor's image; offsets inside an image fit 32 bits.
template <int MODE, int NDIM>
__device__ __forceinline__ const bf16* src_ptr(const bf16* in_img, const bf16* up_img, const NetSrc& s, int D, int H,
                                               int W, int z, int y, int x, int ci0) {
  const int zc = NDIM == 3 ? min(max(z, 0), D - 1) : 0;
  const int yc = min(max(y, 0), H - 1), xc = min(max(x, 0), W - 1);
  if (MODE == 1) return in_img + (((NDIM == 3 ? 2 * zc : 0) * s.Hs + 2 * yc) * s.Ws + 2 * xc) * s.in_ct + ci0;
  if (MODE == 2 && ci0 < s.cup) {
    const int Hu = (H + 1) / 2, Wu = (W + 1) / 2;
    return up_img + (((zc >> 1) * Hu + (yc >> 1)) * Wu + (xc >> 1)) * s.up_ct + ci0;
  }
  return in_img + ((zc * H + yc) * W + xc) * s.in_ct + (ci0 - s.cup);
}

// one input channel ci of pixel (img, z, y, x) inside the layer, the value the staging gives
template <int NDIM>
__device__ __forceinline__ float fetch1(const NetSrc& s, long long img, int D, int H, int W, int z, int y, int x,
                                        int ci) {
  if (ci < s.cup) {
    const int Du = NDIM == 3 ? (D + 1) / 2 : 1, Hu = (H + 1) / 2, Wu = (W + 1) / 2;
    return (float)s.up[(((img * Du + (z >> 1)) * Hu + (y >> 1)) * Wu + (x >> 1)) * s.up_ct + ci];
  }
  const int c = ci - s.cup;
  if (!s.pool) return (float)s.in[(((img * D + z) * H + y) * W + x) * s.in_ct + s.in_off + c];
  const int Ds = NDIM == 3 ? s.Ds : 1;
  float acc = 0.f;
  for (int e = 0; e < (NDIM == 3 ? 2 : 1); ++e)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const int zz = NDIM == 3 ? 2 * z + e : 0, yy = 2 * y + a, xx = 2 * x + b;
        if (zz < Ds && yy < s.Hs && xx < s.Ws)
          acc += (float)s.in[(((img * Ds + zz) * s.Hs + yy) * s.Ws + xx) * s.in_ct + s.in_off + c];
      }
  return (float)(bf16)((NDIM == 3 ? 0.125f : 0.25f) * acc);
}

// ---------------------------------------------------------------- conv, LDS-tiled (MFMA)
// Block = TH x TW output pixels of one image plane, all output channels (NCO tiles
// of 16).  The (TH + 2) x (TW + 2) input halo tile (in 3D: three planes of it,
// z - 1 .. z + 1), all cin channels, is staged once in LDS (pixel stride PS channels,
// padded so that the 16-byte reads of 8 consecutive lanes hit distinct bank groups);
// the four wavefronts then take MT = TH TW / 64 row segments of 16 pixels each and
// run the implicit GEMM over k = tap * cin + ci with A from LDS and B (weights) from
// global memory (small, cache resident).  Pixels outside the layer read zeros.
// With WL (weights larger than the L1), the weights pass through LDS instead, in
// chunks of WKC k-values, double-buffered: the chunk after the current one is read
// from global memory into registers while the current one is used, so no k-step
// waits on an L2 round trip.  Same products in the same order either way.
__device__ __forceinline__ int conv_pixel_stride(int cin) { return cin == 8 ? 8 : cin + 8; }
constexpr int WKC = 64, WROW = WKC + 8;  // k per weight chunk; LDS row stride (bf16, padded against bank conflicts)

// With ZM > 0 (3D, plain or upsample-and-skip inputs of at most 64 channels) a block
// marches through ZM output planes: four plane slots in LDS, the three a plane's
// taps read and the next one, loaded into registers while the plane is computed
// (a plane's halo is staged once instead of three times).
template <int NCO, int TH, int TW, int MODE, int NDIM, bool WL, int ZM>
__global__ __launch_bounds__(256) void k_conv_lds(ConvArgs a) {
  static_assert(ZM == 0 || (NDIM == 3 && MODE != 1 && !WL), "marching: 3D, no pooled input, weights in L1");
  extern __shared__ __align__(16) bf16 tile[];
  constexpr int TW2 = TW + 2, SEG = TW / 16, MT = TH * TW / 64;
  constexpr int NZ = NDIM == 3 ? 3 : 1, NT = NDIM == 3 ? 27 : 9, PLANE = (TH + 2) * TW2;
  constexpr int NZS = ZM ? 4 : NZ;  // plane slots in LDS
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64, g = l / 16, i16 = l % 16;
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
  const int D = NDIM == 3 ? a.D : 1;
  const int nzb = ZM ? (D + ZM - 1) / ZM : D;  // blocks along z per image
  const long long img = NDIM == 3 ? (long long)blockIdx.z / nzb : (long long)blockIdx.z;
  const int z0 = NDIM == 3 ? (int)(blockIdx.z % nzb) * (ZM ? ZM : 1) : 0;
  const int zend = ZM ? min(D, z0 + ZM) : z0 + 1;
  const int cin = a.cin, ps = conv_pixel_stride(cin), cg8 = cin / 8;
  // stage the halo tile: NZ (TH + 2)(TW + 2) pixels x cin / 8 chunks of 16 bytes; a batch
  // of loads is in flight per thread before any is used (points outside the layer store 0)
  constexpr int NSRC = MODE == 1 ? (NDIM == 3 ? 8 : 4) : 1;
  constexpr int BATCH = MODE == 1 ? (NDIM == 3 ? 1 : 2) : 8;
  const int nchunk = NZ * PLANE * cg8;
  // per-image base pointers (offsets inside an image fit 32 bits) and 1 / cg8 for the
  // chunk index: (t + 1/2) / cg8 is at least 1 / 32 away from an integer, far above
  // the rounding of the product for t < 2^20
  const bf16* in_img;
  if (MODE == 1)
    in_img = a.src.in + img * ((long long)(NDIM == 3 ? a.src.Ds : 1) * a.src.Hs * a.src.Ws * a.src.in_ct) + a.src.in_off;
  else
    in_img = a.src.in + img * ((long long)D * a.H * a.W * a.src.in_ct) + a.src.in_off;
  const bf16* up_img = MODE == 2 ? a.src.up + img * ((long long)(NDIM == 3 ? (D + 1) / 2 : 1) * ((a.H + 1) / 2) *
                                                     ((a.W + 1) / 2) * a.src.up_ct)
                                 : nullptr;
  const float rcg = 1.0f / (float)cg8;
  // weight chunks (WL): 16 NCO rows x WKC k, 16-byte pieces, zero past kpad
  constexpr int WPC = 16 * NCO * (WKC / 8), WPT = (WPC + 255) / 256, WBUF = 16 * NCO * WROW;
  bf16* wl = tile + NZS * PLANE * ps;
  bf16x8 wreg[WPT];
  auto wfetch = [&](int c) {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int q = threadIdx.x + 256 * u, row = q / (WKC / 8), k = c * WKC + (q % (WKC / 8)) * 8;
      wreg[u] = (q < WPC && k < a.kpad) ? load8(a.wt + (long long)row * a.kpad + k) : zero8();
    }
  };
  auto wstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int q = threadIdx.x + 256 * u;
      if (q < WPC) *reinterpret_cast<bf16x8*>(wl + buf * WBUF + (q / (WKC / 8)) * WROW + (q % (WKC / 8)) * 8) = wreg[u];
    }
  };
  if constexpr (WL) {
    wfetch(0);
    wstore(0);
  }
  for (int tb = 0; tb < nchunk; tb += 256 * BATCH) {
    const int t0 = tb + threadIdx.x;
    const int nslot = min(BATCH, (nchunk - tb + 255) / 256);  // uniform over the block
    bf16x8 v[BATCH][NSRC];
    int dst[BATCH];  // LDS element offset of the chunk (-1: none); bit 30 set: outside the layer
    int pm[BATCH];   // pooled input: which children lie inside the source (x, y, z bits)
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      dst[u] = -1;
      pm[u] = 0;
      if (u < nslot) {
        const int t = t0 + 256 * u, tt = min(t, nchunk - 1);
        const int q = __float2int_rd(((float)tt + 0.5f) * rcg), cg = tt - q * cg8;
        const int pz = q / PLANE, rq = q - pz * PLANE, r = rq / TW2, c = rq - r * TW2;
        const int zz = z0 - (NZ - 1) / 2 + pz, yy = y0 - 1 + r, xx = x0 - 1 + c;
        const bf16* p = src_ptr<MODE, NDIM>(in_img, up_img, a.src, D, a.H, a.W, zz, yy, xx, cg * 8);
        if (MODE == 1) {
          // the 2 x 2 (x 2) children, clamped into the source (weights applied below)
          const int yc = min(max(yy, 0), a.H - 1), xc = min(max(xx, 0), a.W - 1);
          const int dx = (2 * xc + 1 < a.src.Ws) ? a.src.in_ct : 0;
          const int dy = (2 * yc + 1 < a.src.Hs) ? a.src.Ws * a.src.in_ct : 0;
          v[u][0] = load8(p);
          v[u][NSRC > 1 ? 1 : 0] = load8(p + dx);
          v[u][NSRC > 2 ? 2 : 0] = load8(p + dy);
          v[u][NSRC > 3 ? 3 : 0] = load8(p + dy + dx);
          int zb = 0;
          if (NDIM == 3) {
            const int zc = min(max(zz, 0), D - 1);
            const int dz = (2 * zc + 1 < a.src.Ds) ? a.src.Hs * a.src.Ws * a.src.in_ct : 0;
            v[u][NSRC > 4 ? 4 : 0] = load8(p + dz);
            v[u][NSRC > 5 ? 5 : 0] = load8(p + dz + dx);
            v[u][NSRC > 6 ? 6 : 0] = load8(p + dz + dy);
            v[u][NSRC > 7 ? 7 : 0] = load8(p + dz + dy + dx);
            zb = 2 * zz + 1 < a.src.Ds ? 4 : 0;
          }
          pm[u] = (2 * xx + 1 < a.src.Ws ? 1 : 0) | (2 * yy + 1 < a.src.Hs ? 2 : 0) | zb;
        } else {
          v[u][0] = load8(p);
        }
        const bool valid = zz >= 0 && zz < D && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
        if (t < nchunk) dst[u] = (q * ps + cg * 8) | (valid ? 0 : 1 << 30);
      }
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      if (dst[u] < 0) continue;
      const bool valid = !(dst[u] & (1 << 30));
      bf16x8 o = zero8();
      if (MODE == 1) {
        // average with zero padding: children past the source edge count 0
        const bool hx = pm[u] & 1, hy = pm[u] & 2;
        const float w1 = hx ? 1.f : 0.f, w2 = hy ? 1.f : 0.f, w3 = (hx && hy) ? 1.f : 0.f;
        if (NDIM == 3) {
          const bool hz = pm[u] & 4;
          const float w4 = hz ? 1.f : 0.f, w5 = hz && hx ? 1.f : 0.f, w6 = hz && hy ? 1.f : 0.f,
                      w7 = hz && hx && hy ? 1.f : 0.f;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float acc = (float)v[u][0][e];
            acc += w1 * (float)v[u][NSRC > 1 ? 1 : 0][e];
            acc += w2 * (float)v[u][NSRC > 2 ? 2 : 0][e];
            acc += w3 * (float)v[u][NSRC > 3 ? 3 : 0][e];
            acc += w4 * (float)v[u][NSRC > 4 ? 4 : 0][e];
            acc += w5 * (float)v[u][NSRC > 5 ? 5 : 0][e];
            acc += w6 * (float)v[u][NSRC > 6 ? 6 : 0][e];
            acc += w7 * (float)v[u][NSRC > 7 ? 7 : 0][e];
            o[e] = (bf16)(0.125f * acc);
          }
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float acc = (float)v[u][0][e];
            acc += w1 * (float)v[u][NSRC > 1 ? 1 : 0][e];
            acc += w2 * (float)v[u][NSRC > 2 ? 2 : 0][e];
            acc += w3 * (float)v[u][NSRC > 3 ? 3 : 0][e];
            o[e] = (bf16)(0.25f * acc);
          }
        }
      } else {
        o = v[u][0];
      }
      *reinterpret_cast<bf16x8*>(tile + (dst[u] & ((1 << 30) - 1))) = valid ? o : zero8();
    }
  }
  __syncthreads();
  // LDS offset of this lane's pixel in segment m (tap (0, 0, 0) = the first plane's top-left)
  int base[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int seg = wave * MT + m, r = seg / SEG, c = (seg - r * SEG) * 16 + i16;
    base[m] = (r * TW2 + c) * ps;
  }
  // marching (ZM): the next plane's halo, 16-byte pieces in registers (cin <= 64)
  constexpr int SPT = ZM ? (PLANE * 8 + 255) / 256 : 1;
  bf16x8 spre[SPT];
  auto sfetch = [&](int zz) {
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int t = threadIdx.x + 256 * u;
      spre[u] = zero8();
      if (t < PLANE * cg8) {
        const int q = t / cg8, cg = t - q * cg8, r = q / TW2, c = q - r * TW2;
        const int yy = y0 - 1 + r, xx = x0 - 1 + c;
        if (zz >= 0 && zz < D && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
          spre[u] = load8(src_ptr<MODE, NDIM>(in_img, up_img, a.src, D, a.H, a.W, zz, yy, xx, cg * 8));
      }
    }
  };
  auto sstore = [&](int slot) {
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int t = threadIdx.x + 256 * u;
      if (t < PLANE * cg8) {
        const int q = t / cg8, cg = t - q * cg8;
        *reinterpret_cast<bf16x8*>(tile + (slot * PLANE + q) * ps + cg * 8) = spre[u];
      }
    }
  };
  // the epilogue's bias values and output image base
  const int cout = a.cout;
  float bsv[NCO][4];
#pragma unroll
  for (int t = 0; t < NCO; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = t * 16 + 4 * g + q;
      bsv[t][q] = (a.bias && ch < cout) ? a.bias[ch] : 0.f;
    }
  const long long oimg = img * ((long long)D * a.H * a.W * a.out_ct) + a.out_off;
  for (int zc = z0; zc < zend; ++zc) {
    if constexpr (ZM > 0) {
      if (zc + 1 < zend) sfetch(zc + 2);  // the plane the next output plane adds
    }
    f32x4 acc[MT][NCO];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < NCO; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // Two register sets, two k-steps per iteration: the operands of one step are read
    // (A from LDS, B = weights from global memory) while the MFMAs of the other run.
    // Past the last tap (NT cin <= k < kpad) the packed weights are zero (the padding
    // of every weight matrix stays zero) and past kpad B is set to zero, so those
    // steps add exact zeros whatever A they read (a real pixel of the last tap).
    int tap = (8 * g) / cin, ci0 = 8 * g - tap * cin;  // k = 8 g at the first step
    const int dtap = cin < 32 ? 32 / cin : 0, dci = cin < 32 ? 0 : 32;
    const bf16* wrow = a.wt + (long long)i16 * a.kpad + 8 * g;
    const long long wstride = 16LL * a.kpad;
    const int iz = zc - z0;  // slot of tap plane dz: (iz + dz) mod 4 when marching
    auto read_step = [&](int kc, bf16x8* A, bf16x8* Bw) {
      const int tc = min(tap, NT - 1), dz = NDIM == 3 ? tc / 9 : 0, tp = tc - 9 * dz, dy = tp / 3, dx = tp - 3 * dy;
      const int pl = ZM ? ((iz + dz) & 3) : dz;
      const int off = ((pl * (TH + 2) + dy) * TW2 + dx) * ps + ci0;
#pragma unroll
      for (int m = 0; m < MT; ++m) A[m] = *reinterpret_cast<const bf16x8*>(tile + base[m] + off);
      const bool kin = kc < a.kpad;  // uniform over the block
#pragma unroll
      for (int t = 0; t < NCO; ++t) Bw[t] = kin ? load8(wrow + t * wstride + kc) : zero8();
      // advance k by 32: cin < 32 divides 32 (whole taps), else at most one wrap
      ci0 += dci;
      const int wrap = ci0 >= cin;
      ci0 -= wrap * cin;
      tap += dtap + wrap;
    };
    auto mfma_step = [&](const bf16x8* A, const bf16x8* Bw) {
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NCO; ++t)
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Bw[t], A[m], acc[m][t], 0, 0, 0);
    };
    bf16x8 a0[MT], b0[NCO], a1[MT], b1[NCO];
    if constexpr (WL) {
      // the same k-steps, two per chunk, with B from the chunk's LDS buffer
      auto read_lds = [&](const bf16* wb, bf16x8* A, bf16x8* Bw) {
        const int tc = min(tap, NT - 1), dz = NDIM == 3 ? tc / 9 : 0, tp = tc - 9 * dz, dy = tp / 3, dx = tp - 3 * dy;
        const int off = ((dz * (TH + 2) + dy) * TW2 + dx) * ps + ci0;
#pragma unroll
        for (int m = 0; m < MT; ++m) A[m] = *reinterpret_cast<const bf16x8*>(tile + base[m] + off);
#pragma unroll
        for (int t = 0; t < NCO; ++t) Bw[t] = *reinterpret_cast<const bf16x8*>(wb + t * 16 * WROW);
        ci0 += dci;
        const int wrap = ci0 >= cin;
        ci0 -= wrap * cin;
        tap += dtap + wrap;
      };
      const int nwc = (a.kpad + WKC - 1) / WKC;
      for (int c = 0; c < nwc; ++c) {
        if (c + 1 < nwc) wfetch(c + 1);
        const bf16* wb = wl + (c & 1) * WBUF + i16 * WROW + 8 * g;
        read_lds(wb, a0, b0);
        read_lds(wb + 32, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        mfma_step(a0, b0);
        mfma_step(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        if (c + 1 < nwc) wstore((c + 1) & 1);
        __syncthreads();
      }
    } else {
      read_step(0, a0, b0);
      for (int kc = 0; kc < a.kpad; kc += 64) {
        read_step(kc + 32, a1, b1);
        __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the MFMAs that do not need them
        mfma_step(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        read_step(kc + 64, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        mfma_step(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // epilogue: with the weights as the MFMA's first operand, acc[m][t][r] is output
    // channel t * 16 + 4 g + r of pixel i16 of segment m, so each lane writes four
    // consecutive channels of one pixel (8 bytes in BF16, 16 in FP32)
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int seg = wave * MT + m, r = seg / SEG;
      const int y = y0 + r, xo = x0 + (seg - r * SEG) * 16 + i16;
      if (y >= a.H || xo >= a.W) continue;
      const int po = ((zc * a.H + y) * a.W + xo) * a.out_ct;  // inside the image
#pragma unroll
      for (int t = 0; t < NCO; ++t) {
        const int c0 = t * 16 + 4 * g;
        if (c0 >= cout) continue;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          v[q] = acc[m][t][q] + bsv[t][q];
          if (a.relu) v[q] = fmaxf(v[q], 0.f);
        }
        if (a.out32) {
          float* dst = a.out32 + oimg + po + c0;
          if (c0 + 4 <= cout) *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
          else
            for (int q = 0; q < cout - c0; ++q) dst[q] = v[q];
        } else {
          // BF16 outputs have a multiple of 8 channels
          typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
          bf16x4 o;
#pragma unroll
          for (int q = 0; q < 4; ++q) o[q] = (bf16)v[q];
          *reinterpret_cast<bf16x4*>(a.out + oimg + po + c0) = o;
        }
      }
    }
    if constexpr (ZM > 0) {
      // the prefetched plane zc + 2 replaces plane zc - 2 (read by no output plane from here on)
      if (zc + 1 < zend) sstore((iz + 3) & 3);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- conv, channel-specialised (2D)
// The 2D layers with the input channel count CIN fixed at compile time.  Same implicit
// GEMM as k_conv_lds, term for term: the same k order, products and sums, so the same
// outputs bit for bit.  What changes is where the index arithmetic runs:
//  * a k-step's 32 k-values fall on at most four taps, so the LDS offset of a lane's
//    8 channels is one of four constants picked by its lane group (one constant plus
//    8 g when the step stays on one tap), and the offsets of a wavefront's pixel
//    segments from its first one are constants; the k-loop is unrolled;
//  * the halo tile (pixel stride PS channels, as in k_conv_lds) is staged by halo row:
//    each thread keeps one column chunk (its x clamp, source and channel offsets
//    computed once) and walks the rows;
//  * without WL every k-step's weight fragments sit in registers, loaded before the
//    halo; with WL the 64-k chunks pass through LDS as in k_conv_lds, at constant
//    offsets.
// (Storing the halo tile by 8-channel group, [group][pixel][8], removes the LDS bank
// conflicts of the padded pixel stride but made the level-0 decoder layer slower.)
// A k-step past the last one with real k-values (k_conv_lds runs one when the step
// count is odd) multiplies zero weights, so it is left out.
template <int S, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (S < N) {
    f(std::integral_constant<int, S>{});
    static_for<S + 1, N>(f);
  }
}

// LDS element offset, from the lane's pixel, of the 8 channels lane group g reads at
// k-step s: k = 32 s + 8 g = tap * CIN + ci (k past the last tap reads the last tap)
template <int CIN, int TW2, int PS>
__host__ __device__ constexpr int conv_tap_off(int s, int g) {
  const int k = 32 * s + 8 * g, tap = k / CIN < 8 ? k / CIN : 8;
  return ((tap / 3) * TW2 + tap % 3) * PS + k % CIN;
}

template <int CIN, int NCO, int TH, int TW, int MODE, bool WL>
__global__ __launch_bounds__(256) void k_conv2c(ConvArgs a) {
  constexpr int PS = CIN == 8 ? 8 : CIN + 8, CG8 = CIN / 8;
  constexpr int TW2 = TW + 2, SEG = TW / 16, MT = TH * TW / 64, PLANE = (TH + 2) * TW2;
  constexpr int KS = (9 * CIN + 31) / 32, KPAD = 32 * KS;
  static_assert(CIN % 8 == 0 && MT % SEG == 0, "whole 8-channel groups; a wavefront's segments fill tile rows");
  extern __shared__ __align__(16) bf16 tile[];
  const int tid = threadIdx.x, l = tid % 64, g = l / 16, i16 = l % 16;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, H = a.H, W = a.W;
  const long long img = blockIdx.z;
  const NetSrc& sr = a.src;

  // weights: all k-steps in registers, or (WL) 64-k chunks through two LDS buffers
  // (issuing them after the first batch of halo loads, so that the halo's wait does not
  // also wait for them, made the level-0 decoder layer 9% slower)
  bf16x8 Bw[WL ? 1 : KS][NCO];
  if constexpr (!WL) {
    const bf16* wrow = a.wt + i16 * KPAD + 8 * g;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int t = 0; t < NCO; ++t) Bw[s][t] = load8(wrow + t * 16 * KPAD + 32 * s);
  }
  constexpr int WPC = 16 * NCO * (WKC / 8), WPT = (WPC + 255) / 256, WBUF = 16 * NCO * WROW;
  constexpr int NWC = (KPAD + WKC - 1) / WKC;
  bf16* wl = tile + PLANE * PS;
  bf16x8 wreg[WPT];
  auto wfetch = [&](auto cc) {
    constexpr int c = decltype(cc)::value;
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int q = tid + 256 * u, kq = (q % (WKC / 8)) * 8;
      wreg[u] = (q < WPC && c * WKC + kq < KPAD) ? load8(a.wt + (q / (WKC / 8)) * KPAD + c * WKC + kq) : zero8();
    }
  };
  auto wstore = [&](auto bc) {
    constexpr int buf = decltype(bc)::value;
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
      const int q = tid + 256 * u;
      if (q < WPC) *reinterpret_cast<bf16x8*>(wl + buf * WBUF + (q / (WKC / 8)) * WROW + (q % (WKC / 8)) * 8) = wreg[u];
    }
  };
  if constexpr (WL) {
    wfetch(std::integral_constant<int, 0>{});
    wstore(std::integral_constant<int, 0>{});
  }

  // ---- halo staging, by halo row: RW 16-byte chunks per row; a thread keeps the
  // column chunk j (of each of NP passes over a row) and walks rows r0, r0 + RPP, ...
  constexpr int RW = TW2 * CG8, NP = (RW + 255) / 256, RPP = RW <= 256 ? 256 / RW : 1;
  constexpr int NRI = (TH + 2 + RPP - 1) / RPP;
  constexpr int NSRC = MODE == 1 ? 4 : 1;
  constexpr int RB0 = (WL ? 16 : 8) / (NP * NSRC), RB = RB0 < 1 ? 1 : (RB0 > NRI ? NRI : RB0);  // rows per load batch
  const int r0 = RW <= 256 ? tid / RW : 0;
  const bf16* in_img;
  if (MODE == 1)
    in_img = sr.in + img * ((long long)sr.Hs * sr.Ws * sr.in_ct) + sr.in_off;
  else
    in_img = sr.in + img * ((long long)H * W * sr.in_ct) + sr.in_off;
  const int Hu = (H + 1) / 2, Wu = (W + 1) / 2;
  const bf16* up_img = MODE == 2 ? sr.up + img * ((long long)Hu * Wu * sr.up_ct) : nullptr;
  const bf16* colp[NP];  // source of the column chunk at row 0 (MODE 2: of the source it reads)
  int dst0[NP], dxp[NP];
  bool act[NP], xin[NP], hx[NP], isup[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int j = RW <= 256 ? tid - r0 * RW : tid + 256 * p;
    act[p] = RW <= 256 ? r0 < RPP : j < RW;
    const int c = min(j / CG8, TW2 - 1), cg = j - (j / CG8) * CG8;
    const int xx = x0 - 1 + c, xc = min(max(xx, 0), W - 1);
    xin[p] = xx >= 0 && xx < W;
    dst0[p] = (r0 * TW2 + c) * PS + cg * 8;
    isup[p] = false;
    dxp[p] = 0;
    hx[p] = false;
    if (MODE == 1) {
      colp[p] = in_img + 2 * xc * sr.in_ct + cg * 8;
      dxp[p] = (2 * xc + 1 < sr.Ws) ? sr.in_ct : 0;
      hx[p] = 2 * xx + 1 < sr.Ws;
    } else if (MODE == 2 && cg * 8 < sr.cup) {
      isup[p] = true;
      colp[p] = up_img + (xc >> 1) * sr.up_ct + cg * 8;
    } else {
      colp[p] = in_img + xc * sr.in_ct + (cg * 8 - sr.cup);
    }
  }
  static_for<0, (NRI + RB - 1) / RB>([&](auto bc) {
    constexpr int i0 = decltype(bc)::value * RB, i1 = i0 + RB < NRI ? i0 + RB : NRI;
    bf16x8 v[RB][NP][NSRC];
    bool yin[RB], hy[RB];
#pragma unroll
    for (int i = i0; i < i1; ++i) {
      const int r = min(r0 + i * RPP, TH + 1), yy = y0 - 1 + r, yc = min(max(yy, 0), H - 1);
      yin[i - i0] = yy >= 0 && yy < H;
      hy[i - i0] = 2 * yy + 1 < sr.Hs;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (MODE == 1) {
          const bf16* q = colp[p] + (long long)2 * yc * sr.Ws * sr.in_ct;
          const int dy = (2 * yc + 1 < sr.Hs) ? sr.Ws * sr.in_ct : 0;
          v[i - i0][p][0] = load8(q);
          v[i - i0][p][NSRC > 1 ? 1 : 0] = load8(q + dxp[p]);
          v[i - i0][p][NSRC > 2 ? 2 : 0] = load8(q + dy);
          v[i - i0][p][NSRC > 3 ? 3 : 0] = load8(q + dy + dxp[p]);
        } else {
          const int ro = MODE == 2 && isup[p] ? (yc >> 1) * Wu * sr.up_ct : yc * W * sr.in_ct;
          v[i - i0][p][0] = load8(colp[p] + ro);
        }
      }
    }
#pragma unroll
    for (int i = i0; i < i1; ++i) {
      if (r0 + i * RPP >= TH + 2) continue;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (!act[p]) continue;
        bf16x8 o;
        if (MODE == 1) {
          // average with zero padding: children past the source edge count 0
          const float w1 = hx[p] ? 1.f : 0.f, w2 = hy[i - i0] ? 1.f : 0.f, w3 = (hx[p] && hy[i - i0]) ? 1.f : 0.f;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float acc = (float)v[i - i0][p][0][e];
            acc += w1 * (float)v[i - i0][p][NSRC > 1 ? 1 : 0][e];
            acc += w2 * (float)v[i - i0][p][NSRC > 2 ? 2 : 0][e];
            acc += w3 * (float)v[i - i0][p][NSRC > 3 ? 3 : 0][e];
            o[e] = (bf16)(0.25f * acc);
          }
        } else {
          o = v[i - i0][p][0];
        }
        *reinterpret_cast<bf16x8*>(tile + dst0[p] + i * RPP * TW2 * PS) = (xin[p] && yin[i - i0]) ? o : zero8();
      }
    }
  });
  __syncthreads();

  // ---- implicit GEMM: segment m of this wavefront is tile row wave * MT / SEG + m / SEG,
  // columns (m % SEG) * 16 + 0..15; its LDS offset from segment 0 is a constant
  const int base0 = ((wave * (MT / SEG)) * TW2 + i16) * PS, base8 = base0 + 8 * g;
  const bool g1 = g & 1, g2 = g & 2;
  auto readA = [&](auto sc, bf16x8* A) {
    constexpr int s = decltype(sc)::value;
    constexpr int o0 = conv_tap_off<CIN, TW2, PS>(s, 0), o1 = conv_tap_off<CIN, TW2, PS>(s, 1);
    constexpr int o2 = conv_tap_off<CIN, TW2, PS>(s, 2), o3 = conv_tap_off<CIN, TW2, PS>(s, 3);
    int off;
    if constexpr (o1 == o0 + 8 && o2 == o0 + 16 && o3 == o0 + 24)
      off = base8 + o0;  // one tap, 32 consecutive channels
    else
      off = base0 + (g2 ? (g1 ? o3 : o2) : (g1 ? o1 : o0));
#pragma unroll
    for (int m = 0; m < MT; ++m)
      A[m] = *reinterpret_cast<const bf16x8*>(tile + off + ((m / SEG) * TW2 + (m % SEG) * 16) * PS);
  };
  f32x4 acc[MT][NCO];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NCO; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto mfma_step = [&](const bf16x8* A, const bf16x8* Bv) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < NCO; ++t) acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Bv[t], A[m], acc[m][t], 0, 0, 0);
  };
  bf16x8 Ab[2][MT];
  if constexpr (!WL) {
    readA(std::integral_constant<int, 0>{}, Ab[0]);
    static_for<0, KS>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      if constexpr (s + 1 < KS) readA(std::integral_constant<int, s + 1>{}, Ab[(s + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
      mfma_step(Ab[s & 1], Bw[s]);
      __builtin_amdgcn_sched_barrier(0);
    });
  } else {
    const bf16* wlane = wl + i16 * WROW + 8 * g;
    static_for<0, NWC>([&](auto cc) {
      constexpr int c = decltype(cc)::value, s0 = 2 * c;
      constexpr bool two = s0 + 1 < KS;
      if constexpr (c + 1 < NWC) wfetch(std::integral_constant<int, c + 1>{});
      const bf16* wb = wlane + (c & 1) * WBUF;
      bf16x8 b0[NCO], b1[NCO];
      readA(std::integral_constant<int, s0>{}, Ab[0]);
#pragma unroll
      for (int t = 0; t < NCO; ++t) b0[t] = *reinterpret_cast<const bf16x8*>(wb + t * 16 * WROW);
      if constexpr (two) {
        readA(std::integral_constant<int, s0 + 1>{}, Ab[1]);
#pragma unroll
        for (int t = 0; t < NCO; ++t) b1[t] = *reinterpret_cast<const bf16x8*>(wb + 32 + t * 16 * WROW);
      }
      __builtin_amdgcn_sched_barrier(0);
      mfma_step(Ab[0], b0);
      if constexpr (two) mfma_step(Ab[1], b1);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (c + 1 < NWC) wstore(std::integral_constant<int, (c + 1) & 1>{});
      __syncthreads();
    });
  }

  // ---- epilogue, as in k_conv_lds: lane (i16, g) holds channels t * 16 + 4 g + 0..3 of
  // pixel i16 of each segment
  const int cout = a.cout;
  float bsv[NCO][4];
#pragma unroll
  for (int t = 0; t < NCO; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = t * 16 + 4 * g + q;
      bsv[t][q] = (a.bias && ch < cout) ? a.bias[ch] : 0.f;
    }
  const long long oimg = img * ((long long)H * W * a.out_ct) + a.out_off;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int y = y0 + wave * (MT / SEG) + m / SEG, xo = x0 + (m % SEG) * 16 + i16;
    if (y >= H || xo >= W) continue;
    const int po = (y * W + xo) * a.out_ct;  // inside the image
#pragma unroll
    for (int t = 0; t < NCO; ++t) {
      const int c0 = t * 16 + 4 * g;
      if (c0 >= cout) continue;
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] = acc[m][t][q] + bsv[t][q];
        if (a.relu) v[q] = fmaxf(v[q], 0.f);
      }
      if (a.out32) {
        float* dst = a.out32 + oimg + po + c0;
        if (c0 + 4 <= cout) *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
        else
          for (int q = 0; q < cout - c0; ++q) dst[q] = v[q];
      } else {
        typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
        bf16x4 o;
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = (bf16)v[q];
        *reinterpret_cast<bf16x4*>(a.out + oimg + po + c0) = o;
      }
    }
  }
}

// ---------------------------------------------------------------- conv, 2D marching form
// k_conv2c's sums (outputs equal bit for bit) for 2D layers with plain or
// upsample-and-skip inputs: every k-step's weights sit in registers (loaded once per
// block), a block walks NIT tiles down one column, the next tile's halo is loaded into
// registers while the current tile is computed, and the A operands are read PD k-steps
// ahead.  Used for the level-0 decoder layer (48 -> 16), whose halo loads k_conv2c
// waits for: 783 -> 701 us at 60 x 577^2 with 16 tiles per block.  The first layer and
// the output layer ran slower marching (238 -> 328 and 317 -> 323 us), and so did the
// 96 -> 32 layer with its 27 k-steps of weights in registers at one wavefront per SIMD
// (534 -> 710 us, against k_conv2c's weights through LDS at three blocks per CU).
template <int CIN, int NCO, int TH, int TW, int MODE, int NIT, int PD>
__global__ __launch_bounds__(256) void k_conv2m(ConvArgs a) {
  constexpr int PS = CIN == 8 ? 8 : CIN + 8, CG8 = CIN / 8;
  constexpr int TW2 = TW + 2, SEG = TW / 16, MT = TH * TW / 64;
  constexpr int KS = (9 * CIN + 31) / 32, KPAD = 32 * KS;
  static_assert(CIN % 8 == 0 && MT % SEG == 0 && MODE != 1, "whole channel groups and tile rows; no pooled input");
  extern __shared__ __align__(16) bf16 tile[];
  const int tid = threadIdx.x, l = tid % 64, g = l / 16, i16 = l % 16;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int H = a.H, W = a.W, x0 = blockIdx.x * TW, ty0 = blockIdx.y * NIT;
  const int ntile = min(NIT, (H + TH - 1) / TH - ty0);  // uniform
  const long long img = blockIdx.z;
  const NetSrc& sr = a.src;
  const bf16* in_img = sr.in + img * ((long long)H * W * sr.in_ct) + sr.in_off;
  const int Hu = (H + 1) / 2, Wu = (W + 1) / 2;
  const bf16* up_img = MODE == 2 ? sr.up + img * ((long long)Hu * Wu * sr.up_ct) : nullptr;
  bf16x8 Bw[KS][NCO];
  {
    const bf16* wrow = a.wt + i16 * KPAD + 8 * g;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int t = 0; t < NCO; ++t) Bw[s][t] = load8(wrow + t * 16 * KPAD + 32 * s);
  }

  // ---- halo staging by halo row, as in k_conv2c (all rows in one batch)
  constexpr int RW = TW2 * CG8, NP = (RW + 255) / 256, RPP = RW <= 256 ? 256 / RW : 1;
  constexpr int NRI = (TH + 2 + RPP - 1) / RPP;
  const int r0 = RW <= 256 ? tid / RW : 0;
  const bf16* colp[NP];
  int dst0[NP];
  bool act[NP], xin[NP], isup[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int j = RW <= 256 ? tid - r0 * RW : tid + 256 * p;
    act[p] = RW <= 256 ? r0 < RPP : j < RW;
    const int c = min(j / CG8, TW2 - 1), cg = j - (j / CG8) * CG8;
    const int xx = x0 - 1 + c, xc = min(max(xx, 0), W - 1);
    xin[p] = xx >= 0 && xx < W;
    dst0[p] = (r0 * TW2 + c) * PS + cg * 8;
    isup[p] = MODE == 2 && cg * 8 < sr.cup;
    colp[p] = isup[p] ? up_img + (xc >> 1) * sr.up_ct + cg * 8 : in_img + xc * sr.in_ct + (cg * 8 - sr.cup);
  }
  typedef bf16x8 HaloRegs[NRI][NP];
  auto load_tile = [&](int y0, HaloRegs& v, bool (&ok)[NRI]) {
#pragma unroll
    for (int i = 0; i < NRI; ++i) {
      const int r = min(r0 + i * RPP, TH + 1), yy = y0 - 1 + r, yc = min(max(yy, 0), H - 1);
      ok[i] = yy >= 0 && yy < H;
      const int oin = yc * W * sr.in_ct, oup = MODE == 2 ? (yc >> 1) * Wu * sr.up_ct : 0;
#pragma unroll
      for (int p = 0; p < NP; ++p) v[i][p] = load8(colp[p] + (isup[p] ? oup : oin));
    }
  };
  auto store_tile = [&](const HaloRegs& v, const bool (&ok)[NRI]) {
#pragma unroll
    for (int i = 0; i < NRI; ++i) {
      if (r0 + i * RPP >= TH + 2) continue;
#pragma unroll
      for (int p = 0; p < NP; ++p)
        if (act[p])
          *reinterpret_cast<bf16x8*>(tile + dst0[p] + i * RPP * TW2 * PS) = (xin[p] && ok[i]) ? v[i][p] : zero8();
    }
  };
  {
    HaloRegs v;
    bool ok[NRI];
    load_tile(ty0 * TH, v, ok);
    store_tile(v, ok);
  }
  __syncthreads();

  const int base0 = ((wave * (MT / SEG)) * TW2 + i16) * PS, base8 = base0 + 8 * g;
  const bool g1 = g & 1, g2 = g & 2;
  auto readA = [&](auto sc, bf16x8* A) {
    constexpr int s = decltype(sc)::value;
    constexpr int o0 = conv_tap_off<CIN, TW2, PS>(s, 0), o1 = conv_tap_off<CIN, TW2, PS>(s, 1);
    constexpr int o2 = conv_tap_off<CIN, TW2, PS>(s, 2), o3 = conv_tap_off<CIN, TW2, PS>(s, 3);
    int off;
    if constexpr (o1 == o0 + 8 && o2 == o0 + 16 && o3 == o0 + 24)
      off = base8 + o0;
    else
      off = base0 + (g2 ? (g1 ? o3 : o2) : (g1 ? o1 : o0));
#pragma unroll
    for (int m = 0; m < MT; ++m)
      A[m] = *reinterpret_cast<const bf16x8*>(tile + off + ((m / SEG) * TW2 + (m % SEG) * 16) * PS);
  };
  const int cout = a.cout;
  const long long oimg = img * ((long long)H * W * a.out_ct) + a.out_off;
  HaloRegs vn;
  bool kn[NRI];
  for (int it = 0; it < ntile; ++it) {
    const int y0 = (ty0 + it) * TH;
    const bool more = it + 1 < ntile;  // uniform
    if (more) load_tile(y0 + TH, vn, kn);  // in flight during the tile's GEMM
    f32x4 acc[MT][NCO];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < NCO; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    constexpr int NB = PD + 1;
    bf16x8 Ab[NB][MT];
    static_for<0, (PD < KS ? PD : KS)>([&](auto sc) { readA(sc, Ab[decltype(sc)::value]); });
    static_for<0, KS>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      if constexpr (s + PD < KS) readA(std::integral_constant<int, s + PD>{}, Ab[(s + PD) % NB]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NCO; ++t)
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Bw[s][t], Ab[s % NB][m], acc[m][t], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    });
    // epilogue, as in k_conv_lds
    float bsv[NCO][4];
#pragma unroll
    for (int t = 0; t < NCO; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ch = t * 16 + 4 * g + q;
        bsv[t][q] = (a.bias && ch < cout) ? a.bias[ch] : 0.f;
      }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int y = y0 + wave * (MT / SEG) + m / SEG, xo = x0 + (m % SEG) * 16 + i16;
      if (y >= H || xo >= W) continue;
      const int po = (y * W + xo) * a.out_ct;  // inside the image
#pragma unroll
      for (int t = 0; t < NCO; ++t) {
        const int c0 = t * 16 + 4 * g;
        if (c0 >= cout) continue;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          v[q] = acc[m][t][q] + bsv[t][q];
          if (a.relu) v[q] = fmaxf(v[q], 0.f);
        }
        if (a.out32) {
          float* dst = a.out32 + oimg + po + c0;
          if (c0 + 4 <= cout) *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
          else
            for (int q = 0; q < cout - c0; ++q) dst[q] = v[q];
        } else {
          typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
          bf16x4 o;
#pragma unroll
          for (int q = 0; q < 4; ++q) o[q] = (bf16)v[q];
          *reinterpret_cast<bf16x4*>(a.out + oimg + po + c0) = o;
        }
      }
    }
    __syncthreads();  // every wavefront done with the tile's halo
    if (more) {
      store_tile(vn, kn);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- conv, channel-specialised (3D)
// 3D layers (plain, pooled or upsample-and-skip inputs), CIN fixed at compile time: the
// products and sums of k_conv_lds (whose marching form these follow) in the same order,
// so the outputs are equal bit for bit, with the index arithmetic at compile time as in
// k_conv2c.  A block computes ZM output planes of a TH x TW tile; four plane slots hold
// the halo planes z - 1, z, z + 1 and the prefetched z + 2.  A k-step's lane group reads
// tap (dz, dy, dx), channel ci: its LDS offset is the (uniform, per output plane) base of
// slot (z - z0 + dz) mod 4 plus a compile-time constant.  The weights of every k-step
// sit in registers; the A operands are read PD k-steps ahead.
template <int CIN>
__host__ __device__ constexpr int conv3_tap(int s, int g) {  // tap of lane group g at k-step s
  return (32 * s + 8 * g) / CIN < 26 ? (32 * s + 8 * g) / CIN : 26;
}
template <int CIN, int TW2, int PS>
__host__ __device__ constexpr int conv3_off(int s, int g) {  // in-plane offset of that read
  const int k = 32 * s + 8 * g, tp = conv3_tap<CIN>(s, g) % 9;
  return ((tp / 3) * TW2 + tp % 3) * PS + k % CIN;
}

template <int CIN, int NCO, int TH, int TW, int MODE, int ZM, int PD>
__global__ __launch_bounds__(256) void k_conv3c(ConvArgs a) {
  constexpr int PS = CIN == 8 ? 8 : CIN + 8, CG8 = CIN / 8;
  constexpr int TW2 = TW + 2, SEG = TW / 16, MT = TH * TW / 64, PLANE = (TH + 2) * TW2, SLOT = PLANE * PS;
  constexpr int KS = (27 * CIN + 31) / 32, KPAD = 32 * KS;
  static_assert(CIN % 8 == 0 && MT % SEG == 0, "whole channel groups and tile rows");
  extern __shared__ __align__(16) bf16 tile[];
  const int tid = threadIdx.x, l = tid % 64, g = l / 16, i16 = l % 16;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int D = a.D, H = a.H, W = a.W, x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
  const int nzb = (D + ZM - 1) / ZM;
  const long long img = blockIdx.z / nzb;
  const int z0 = (int)(blockIdx.z % nzb) * ZM, zend = min(D, z0 + ZM);
  const NetSrc& sr = a.src;
  // MODE 1: the 2 x 2 x 2 average (zero padding) of the source at Ds x Hs x Ws
  const bf16* in_img = sr.in + img * ((long long)(MODE == 1 ? (long long)sr.Ds * sr.Hs * sr.Ws : (long long)D * H * W) * sr.in_ct) + sr.in_off;
  const int Du = (D + 1) / 2, Hu = (H + 1) / 2, Wu = (W + 1) / 2;
  const bf16* up_img = MODE == 2 ? sr.up + img * ((long long)Du * Hu * Wu * sr.up_ct) : nullptr;
  // every k-step's weight fragments in registers, loaded once per block (the LDS of the
  // four plane slots allows two blocks per CU, so there is room for them)
  bf16x8 Bw[KS][NCO];
  {
    const bf16* wrow = a.wt + i16 * KPAD + 8 * g;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int t = 0; t < NCO; ++t) Bw[s][t] = load8(wrow + t * 16 * KPAD + 32 * s);
  }

  // ---- plane staging, by halo row (as in k_conv2c), every row of a plane in one batch
  constexpr int RW = TW2 * CG8, NP = (RW + 255) / 256, RPP = RW <= 256 ? 256 / RW : 1;
  constexpr int NRI = (TH + 2 + RPP - 1) / RPP;
  const int r0 = RW <= 256 ? tid / RW : 0;
  constexpr int NSRC = MODE == 1 ? 8 : 1;
  const bf16* colp[NP];
  int dst0[NP], dxp[NP];
  bool act[NP], xin[NP], isup[NP], hx[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int j = RW <= 256 ? tid - r0 * RW : tid + 256 * p;
    act[p] = RW <= 256 ? r0 < RPP : j < RW;
    const int c = min(j / CG8, TW2 - 1), cg = j - (j / CG8) * CG8;
    const int xx = x0 - 1 + c, xc = min(max(xx, 0), W - 1);
    xin[p] = xx >= 0 && xx < W;
    dst0[p] = (r0 * TW2 + c) * PS + cg * 8;
    isup[p] = MODE == 2 && cg * 8 < sr.cup;
    dxp[p] = MODE == 1 && 2 * xc + 1 < sr.Ws ? sr.in_ct : 0;
    hx[p] = 2 * xx + 1 < sr.Ws;
    if (MODE == 1)
      colp[p] = in_img + 2 * xc * sr.in_ct + cg * 8;
    else
      colp[p] = isup[p] ? up_img + (xc >> 1) * sr.up_ct + cg * 8 : in_img + xc * sr.in_ct + (cg * 8 - sr.cup);
  }
  // a plane's loads; fl[i]: bit 0 the row is inside the layer, bits 1 and 2 (pooled input)
  // the second child along y and along z lies inside the source
  typedef bf16x8 PlaneRegs[NRI][NP][NSRC];
  auto load_plane = [&](int zz, PlaneRegs& v, int (&fl)[NRI]) {
    const int zc = min(max(zz, 0), D - 1);
    const bool zin = zz >= 0 && zz < D;
    const long long dz = MODE == 1 && 2 * zc + 1 < sr.Ds ? (long long)sr.Hs * sr.Ws * sr.in_ct : 0;
    const int hz = MODE == 1 && 2 * zz + 1 < sr.Ds ? 4 : 0;
#pragma unroll
    for (int i = 0; i < NRI; ++i) {
      const int r = min(r0 + i * RPP, TH + 1), yy = y0 - 1 + r, yc = min(max(yy, 0), H - 1);
      fl[i] = (zin && yy >= 0 && yy < H ? 1 : 0) | (MODE == 1 && 2 * yy + 1 < sr.Hs ? 2 : 0) | hz;
      if (MODE == 1) {
        const long long dy = 2 * yc + 1 < sr.Hs ? (long long)sr.Ws * sr.in_ct : 0;
        const long long o = ((long long)2 * zc * sr.Hs + 2 * yc) * sr.Ws * sr.in_ct;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const bf16* q = colp[p] + o;
          v[i][p][0] = load8(q);
          v[i][p][NSRC > 1 ? 1 : 0] = load8(q + dxp[p]);
          v[i][p][NSRC > 2 ? 2 : 0] = load8(q + dy);
          v[i][p][NSRC > 3 ? 3 : 0] = load8(q + dy + dxp[p]);
          v[i][p][NSRC > 4 ? 4 : 0] = load8(q + dz);
          v[i][p][NSRC > 5 ? 5 : 0] = load8(q + dz + dxp[p]);
          v[i][p][NSRC > 6 ? 6 : 0] = load8(q + dz + dy);
          v[i][p][NSRC > 7 ? 7 : 0] = load8(q + dz + dy + dxp[p]);
        }
      } else {
        const long long oin = ((long long)zc * H + yc) * W * sr.in_ct;
        const long long oup = MODE == 2 ? ((long long)(zc >> 1) * Hu + (yc >> 1)) * Wu * sr.up_ct : 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) v[i][p][0] = load8(colp[p] + (isup[p] ? oup : oin));
      }
    }
  };
  auto store_plane = [&](int slot, const PlaneRegs& v, const int (&fl)[NRI]) {
#pragma unroll
    for (int i = 0; i < NRI; ++i) {
      if (r0 + i * RPP >= TH + 2) continue;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (!act[p]) continue;
        bf16x8 o;
        if (MODE == 1) {
          // average with zero padding, as in k_conv_lds: children past the source edge count 0
          const bool bx = hx[p], by = fl[i] & 2, bz = fl[i] & 4;
          const float w1 = bx ? 1.f : 0.f, w2 = by ? 1.f : 0.f, w3 = (bx && by) ? 1.f : 0.f;
          const float w4 = bz ? 1.f : 0.f, w5 = bz && bx ? 1.f : 0.f, w6 = bz && by ? 1.f : 0.f,
                      w7 = bz && bx && by ? 1.f : 0.f;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            float acc = (float)v[i][p][0][e];
            acc += w1 * (float)v[i][p][NSRC > 1 ? 1 : 0][e];
            acc += w2 * (float)v[i][p][NSRC > 2 ? 2 : 0][e];
            acc += w3 * (float)v[i][p][NSRC > 3 ? 3 : 0][e];
            acc += w4 * (float)v[i][p][NSRC > 4 ? 4 : 0][e];
            acc += w5 * (float)v[i][p][NSRC > 5 ? 5 : 0][e];
            acc += w6 * (float)v[i][p][NSRC > 6 ? 6 : 0][e];
            acc += w7 * (float)v[i][p][NSRC > 7 ? 7 : 0][e];
            o[e] = (bf16)(0.125f * acc);
          }
        } else {
          o = v[i][p][0];
        }
        *reinterpret_cast<bf16x8*>(tile + slot * SLOT + dst0[p] + i * RPP * TW2 * PS) =
            (xin[p] && (fl[i] & 1)) ? o : zero8();
      }
    }
  };
  if constexpr (MODE == 1) {
    // eight sources per chunk: one plane at a time
    for (int k = 0; k < 3; ++k) {
      PlaneRegs v;
      int f[NRI];
      load_plane(z0 - 1 + k, v, f);
      store_plane(k, v, f);
    }
  } else {
    PlaneRegs v0, v1, v2;
    int k0[NRI], k1[NRI], k2[NRI];
    load_plane(z0 - 1, v0, k0);
    load_plane(z0, v1, k1);
    load_plane(z0 + 1, v2, k2);
    store_plane(0, v0, k0);
    store_plane(1, v1, k1);
    store_plane(2, v2, k2);
  }
  __syncthreads();

  const int base0 = ((wave * (MT / SEG)) * TW2 + i16) * PS;
  const bool g1 = g & 1, g2 = g & 2;
  const int cout = a.cout;
  const long long oimg = img * ((long long)D * H * W * a.out_ct) + a.out_off;
  PlaneRegs vn;
  int kn[NRI];
  for (int zc = z0; zc < zend; ++zc) {
    const int iz = zc - z0;
    const bool more = zc + 1 < zend;  // uniform
    if (more) load_plane(zc + 2, vn, kn);  // the plane the next output plane adds
    // per tap plane dz: the LDS base of its slot for this lane, plus 8 g / 8 (g & 1)
    int sb[3], sb8[3], sbh[3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
      sb[dz] = base0 + ((iz + dz) & 3) * SLOT;
      sb8[dz] = sb[dz] + 8 * g;
      sbh[dz] = sb[dz] + 8 * (g & 1);
    }
    auto readA = [&](auto sc, bf16x8* A) {
      constexpr int s = decltype(sc)::value;
      constexpr int t0 = conv3_tap<CIN>(s, 0), t1 = conv3_tap<CIN>(s, 1);
      constexpr int t2 = conv3_tap<CIN>(s, 2), t3 = conv3_tap<CIN>(s, 3);
      constexpr int o0 = conv3_off<CIN, TW2, PS>(s, 0), o1 = conv3_off<CIN, TW2, PS>(s, 1);
      constexpr int o2 = conv3_off<CIN, TW2, PS>(s, 2), o3 = conv3_off<CIN, TW2, PS>(s, 3);
      int off;
      if constexpr (t0 == t3 && o1 == o0 + 8 && o2 == o0 + 16 && o3 == o0 + 24)
        off = sb8[t0 / 9] + o0;  // one tap, 32 consecutive channels
      else if constexpr (t0 == t1 && t2 == t3 && o1 == o0 + 8 && o3 == o2 + 8)
        off = g2 ? sbh[t2 / 9] + o2 : sbh[t0 / 9] + o0;  // two taps, 16 channels each
      else
        off = g2 ? (g1 ? sb[t3 / 9] + o3 : sb[t2 / 9] + o2) : (g1 ? sb[t1 / 9] + o1 : sb[t0 / 9] + o0);
#pragma unroll
      for (int m = 0; m < MT; ++m)
        A[m] = *reinterpret_cast<const bf16x8*>(tile + off + ((m / SEG) * TW2 + (m % SEG) * 16) * PS);
    };
    f32x4 acc[MT][NCO];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < NCO; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // A read PD k-steps ahead of the MFMAs that use it
    constexpr int NB = PD + 1;
    bf16x8 Ab[NB][MT];
    static_for<0, (PD < KS ? PD : KS)>([&](auto sc) { readA(sc, Ab[decltype(sc)::value]); });
    static_for<0, KS>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      if constexpr (s + PD < KS) readA(std::integral_constant<int, s + PD>{}, Ab[(s + PD) % NB]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NCO; ++t)
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Bw[s][t], Ab[s % NB][m], acc[m][t], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    });
    // epilogue, as in k_conv_lds
    float bsv[NCO][4];
#pragma unroll
    for (int t = 0; t < NCO; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ch = t * 16 + 4 * g + q;
        bsv[t][q] = (a.bias && ch < cout) ? a.bias[ch] : 0.f;
      }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int y = y0 + wave * (MT / SEG) + m / SEG, xo = x0 + (m % SEG) * 16 + i16;
      if (y >= H || xo >= W) continue;
      const int po = ((zc * H + y) * W + xo) * a.out_ct;  // inside the image
#pragma unroll
      for (int t = 0; t < NCO; ++t) {
        const int c0 = t * 16 + 4 * g;
        if (c0 >= cout) continue;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          v[q] = acc[m][t][q] + bsv[t][q];
          if (a.relu) v[q] = fmaxf(v[q], 0.f);
        }
        if (a.out32) {
          float* dst = a.out32 + oimg + po + c0;
          if (c0 + 4 <= cout) *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
          else
            for (int q = 0; q < cout - c0; ++q) dst[q] = v[q];
        } else {
          typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
          bf16x4 o;
#pragma unroll
          for (int q = 0; q < 4; ++q) o[q] = (bf16)v[q];
          *reinterpret_cast<bf16x4*>(a.out + oimg + po + c0) = o;
        }
      }
    }
    if (more) store_plane((iz + 3) & 3, vn, kn);  // plane zc + 2 replaces plane zc - 2
    __syncthreads();
  }
}

// ---------------------------------------------------------------- weight gradient (MFMA)
// dW[co][k] = sum_p in[p + shift(tap(k))][ci(k)] * g[p][co]: a GEMM over pixels.
// Block (k tile of 16, channel tile of 16, pixel chunk); each wavefront takes a
// quarter of the chunk, the four partial tiles are summed in LDS and written
// to part[chunk][co][k] (reduced in a fixed order by k_wgrad_reduce).
template <int NDIM>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  constexpr int NT = NDIM == 3 ? 27 : 9;
  __shared__ float red[4][16][17];
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64, gq = l / 16, i16 = l % 16;
  const int kt = blockIdx.x, ct = blockIdx.y, chunk = blockIdx.z;
  const int D = NDIM == 3 ? a.D : 1;
  const long long P = (long long)a.nimg * D * a.H * a.W;
  const long long p_begin = (long long)chunk * a.chunk + (long long)wave * (a.chunk / 4);
  const long long p_end = min(p_begin + a.chunk / 4, P);
  const int krow = kt * 16 + i16;                  // A row of this lane
  const int tap = krow / a.cin, ci = krow - tap * a.cin;
  const int dz = NDIM == 3 ? tap / 9 - 1 : 0, tp = NDIM == 3 ? tap % 9 : tap;
  const int dy = tp / 3 - 1, dx = tp % 3 - 1;
  const int co = ct * 16 + i16;                    // B column of this lane
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  // pixel (img, pz, py, px) of this lane's first element, advanced by one pixel per
  // element and by 32 per step instead of divided out of p each time
  long long img0;
  int px0, py0, pz0;
  {
    const long long p = p_begin + 8 * gq;
    px0 = (int)(p % a.W);
    const long long r = p / a.W;
    py0 = (int)(r % a.H);
    const long long r2 = r / a.H;
    pz0 = NDIM == 3 ? (int)(r2 % D) : 0;
    img0 = NDIM == 3 ? r2 / D : r2;
  }
  auto next_row = [&](int& py, int& pz, long long& img) {
    if (++py == a.H) {
      py = 0;
      if (NDIM == 3 && ++pz < D) return;
      pz = 0;
      ++img;
    }
  };
  for (long long pc = p_begin; pc < p_end; pc += 32) {
    bf16x8 av, bv;
    int px = px0, py = py0, pz = pz0;
    long long img = img0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const long long p = pc + 8 * gq + v;
      float xa = 0.f, gb = 0.f;
      if (p < p_end) {
        const int zz = pz + dz, yy = py + dy, xx = px + dx;
        if (tap < NT && zz >= 0 && zz < D && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
          xa = fetch1<NDIM>(a.src, img, D, a.H, a.W, zz, yy, xx, ci);
        gb = (float)a.g[p * a.g_ct + co];
      }
      av[v] = (__bf16)xa;
      bv[v] = (__bf16)gb;
      if (++px == a.W) {
        px = 0;
        next_row(py, pz, img);
      }
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    px0 += 32;
    while (px0 >= a.W) {
      px0 -= a.W;
      next_row(py0, pz0, img0);
    }
  }
  // D[i][j]: i = k row (4 gq + r), j = co column (i16)
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave][4 * gq + r][i16] = acc[r];
  __syncthreads();
  const int i = threadIdx.x / 16, j = threadIdx.x % 16;  // 256 threads = 16 x 16 outputs
  const float s = red[0][i][j] + red[1][i][j] + red[2][i][j] + red[3][i][j];
  a.part[((long long)chunk * a.cout_pad + ct * 16 + j) * a.kpad + kt * 16 + i] = s;
}

__global__ void k_wgrad_reduce(int nchunk, int n, const float* part, float* dw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(long long)c * n + t];
  dw[t] = s;
}

// db[co] = sum_p g[p][co], first stage: block `chunk` sums its pixels [chunk * n, ...)
// into part[chunk][co]; thread t takes channel t % g_ct of every (256 / g_ct)-th pixel, so
// a block reads consecutive 512-byte rows of g.  The chunk partials are then summed in
// chunk order (k_wgrad_reduce): the same order on every call.  g_ct divides 256.
__global__ __launch_bounds__(256) void k_bias_part(long long P, int n, const bf16* g, int g_ct, int cout,
                                                   float* part) {
  __shared__ float red[256];
  const int c = threadIdx.x % g_ct, lane = threadIdx.x / g_ct, lanes = 256 / g_ct;
  const long long p0 = (long long)blockIdx.x * n, p1 = min(p0 + n, P);
  float s = 0.f;
  long long p = p0 + lane;
  // 16 loads in flight, added in the order of p
  for (; p + 15 * lanes < p1; p += 16 * lanes) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = (float)g[(p + u * lanes) * g_ct + c];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u];
  }
  for (; p < p1; p += lanes) s += (float)g[p * g_ct + c];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < cout) {
    float t = 0.f;
    for (int k = 0; k < lanes; ++k) t += red[k * g_ct + threadIdx.x];
    part[(long long)blockIdx.x * cout + threadIdx.x] = t;
  }
}

// db[co] = sum_p g[p][co] in one block per channel (channel strides that do not divide 256)
__global__ void k_bias_grad(long long P, const bf16* g, int g_ct, float* db) {
  __shared__ float red[256];
  const int co = blockIdx.x;
  float s = 0.f;
  for (long long p = threadIdx.x; p < P; p += 256) s += (float)g[p * g_ct + co];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[co] = red[0];
}

// ---------------------------------------------------------------- elementwise
// gm[p][c] = (c < creal) ? g[p][c] * (mask ? act[p][c] > 0 : 1) : 0, bf16 out (cpad channels)
__global__ void k_grad_prep(long long P, const float* g, int g_ct, int g_off, const bf16* act, int act_ct,
                            int act_off, int creal, int cpad, bf16* gm) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * cpad) return;
  const long long p = t / cpad;
  const int c = (int)(t % cpad);
  float v = 0.f;
  if (c < creal) {
    v = g[p * g_ct + g_off + c];
    if (act && !((float)act[p * act_ct + act_off + c] > 0.f)) v = 0.f;
  }
  gm[t] = (bf16)v;
}

// gin[p][off + c] += 2^-NDIM g[parent(p)][c]   (fp32; depth D = 1 in 2D)
template <int NDIM>
__global__ void k_pool_back(int nimg, int D, int H, int W, int C, const float* g, int g_ct, float* gin, int gin_ct,
                            int gin_off) {
  const int Dc = NDIM == 3 ? (D + 1) / 2 : 1, Hc = (H + 1) / 2, Wc = (W + 1) / 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nimg * D * H * W * C) return;
  const int c = (int)(t % C);
  const long long p = t / C;
  const int x = (int)(p % W);
  const long long r = p / W;
  const int y = (int)(r % H);
  const long long r2 = r / H;
  const int z = NDIM == 3 ? (int)(r2 % D) : 0;
  const long long img = NDIM == 3 ? r2 / D : r2;
  const long long q = ((img * Dc + z / 2) * Hc + y / 2) * Wc + x / 2;
  gin[p * gin_ct + gin_off + c] += (NDIM == 3 ? 0.125f : 0.25f) * g[q * g_ct + c];
}

// gc[q][c] = sum over the children p of q of g[p][off + c]   (fp32)
template <int NDIM>
__global__ void k_upsample_back(int nimg, int D, int H, int W, int C, const float* g, int g_ct, int g_off, float* gc) {
  const int Dc = NDIM == 3 ? (D + 1) / 2 : 1, Hc = (H + 1) / 2, Wc = (W + 1) / 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nimg * Dc * Hc * Wc * C) return;
  const int c = (int)(t % C);
  const long long q = t / C;
  const int X = (int)(q % Wc);
  const long long r = q / Wc;
  const int Y = (int)(r % Hc);
  const long long r2 = r / Hc;
  const int Z = NDIM == 3 ? (int)(r2 % Dc) : 0;
  const long long img = NDIM == 3 ? r2 / Dc : r2;
  float s = 0.f;
  for (int e = 0; e < (NDIM == 3 ? 2 : 1); ++e)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const int zz = NDIM == 3 ? 2 * Z + e : 0, yy = 2 * Y + a, xx = 2 * X + b;
        if (zz < D && yy < H && xx < W) s += g[(((img * D + zz) * H + yy) * W + xx) * g_ct + g_off + c];
      }
  gc[q * C + c] = s;
}

// gy = (y - target) / nimg, and per-block partial sums of 1/2 (y - target)^2 / nimg
__global__ void k_loss(long long n, const float* y, const float* tgt, float inv_nimg, float* gy, float* part) {
  __shared__ float red[256];
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.f;
  if (t < n) {
    const float d = y[t] - tgt[t];
    gy[t] = d * inv_nimg;
    s = 0.5f * d * d * inv_nimg;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Residual term of the training loss.  With r = (x0 + j x1), c = cb (1 + x2 + j x3)
// taken from the FP32 network input x [P][4] and the output y [P][2] read as
// complex, q = r - gamma A' y on the interior of every image (one-pixel border
// excluded: the crop's neighbours outside it are unknown), where A' y =
// (2 NDIM - c) y - (sum of the 2 NDIM neighbours).  part[block] = w/2 sum |q|^2.
// Pixels are (image, z, y, x) with depth D (1 in 2D).
template <int NDIM>
__device__ __forceinline__ bool res_interior(long long p, int D, int H, int W) {
  const int px = (int)(p % W), py = (int)((p / W) % H);
  bool in = px > 0 && px < W - 1 && py > 0 && py < H - 1;
  if (NDIM == 3) {
    const int pz = (int)((p / ((long long)W * H)) % D);
    in = in && pz > 0 && pz < D - 1;
  }
  return in;
}

// A' applied at an interior pixel p of the complex field f (interleaved pairs) with coefficient c
template <int NDIM>
__device__ __forceinline__ c32 res_apply(const float* f, long long p, int H, int W, c32 c) {
  const long long sy = W, sz = (long long)W * H;
  const c32 fc = make_float2(f[p * 2], f[p * 2 + 1]);
  c32 nbs = make_float2(f[(p - 1) * 2] + f[(p + 1) * 2] + f[(p - sy) * 2] + f[(p + sy) * 2],
                        f[(p - 1) * 2 + 1] + f[(p + 1) * 2 + 1] + f[(p - sy) * 2 + 1] + f[(p + sy) * 2 + 1]);
  if (NDIM == 3)
    nbs = cadd(nbs, make_float2(f[(p - sz) * 2] + f[(p + sz) * 2], f[(p - sz) * 2 + 1] + f[(p + sz) * 2 + 1]));
  return csub(cmul(make_float2((float)(2 * NDIM) - c.x, -c.y), fc), nbs);
}

template <int NDIM>
__global__ void k_res_q(int nimg, int D, int H, int W, const float* x, const float* y, float gamma, c32 cb, float w,
                        float2* q, float* part) {
  __shared__ float red[256];
  const long long P = (long long)nimg * D * H * W;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.f;
  if (p < P) {
    float2 qq = make_float2(0.f, 0.f);
    if (res_interior<NDIM>(p, D, H, W)) {
      const float* xp = x + p * 4;
      const c32 c = cmul(cb, make_float2(1.f + xp[2], xp[3]));
      const c32 ay = res_apply<NDIM>(y, p, H, W, c);
      qq = make_float2(xp[0] - gamma * ay.x, xp[1] - gamma * ay.y);
      s = 0.5f * w * (qq.x * qq.x + qq.y * qq.y);
    }
    q[p] = qq;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int t = 128; t > 0; t >>= 1) {
    if (threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// gy += -w gamma A'^H q, A'^H q = (2 NDIM - conj c) q - (sum of the neighbours of q); q is zero
// on the border, and neighbours outside the image count as zero.
template <int NDIM>
__global__ void k_res_grad(int nimg, int D, int H, int W, const float* x, const float2* q, float gamma, c32 cb,
                           float w, float* gy) {
  const long long P = (long long)nimg * D * H * W;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int px = (int)(p % W), py = (int)((p / W) % H);
  const float* xp = x + p * 4;
  const c32 c = cmul(cb, make_float2(1.f + xp[2], xp[3]));
  float2 nbs = make_float2(0.f, 0.f);
  if (px > 0) nbs = cadd(nbs, q[p - 1]);
  if (px < W - 1) nbs = cadd(nbs, q[p + 1]);
  if (py > 0) nbs = cadd(nbs, q[p - W]);
  if (py < H - 1) nbs = cadd(nbs, q[p + W]);
  if (NDIM == 3) {
    const long long sz = (long long)W * H;
    const int pz = (int)((p / sz) % D);
    if (pz > 0) nbs = cadd(nbs, q[p - sz]);
    if (pz < D - 1) nbs = cadd(nbs, q[p + sz]);
  }
  const c32 g = csub(cmul(make_float2((float)(2 * NDIM) - c.x, c.y), q[p]), nbs);
  gy[p * 2] -= w * gamma * g.x;
  gy[p * 2 + 1] -= w * gamma * g.y;
}

// Per image: sums over the interior of |r - gamma A' y|^2 and |r|^2 (r, c, y as in k_res_q),
// one block per image, fixed-order reduction; sums[2 img], sums[2 img + 1].
template <int NDIM>
__global__ __launch_bounds__(256) void k_res_ratio(int D, int H, int W, const float* x, const float* y, float gamma,
                                                   c32 cb, double* sums) {
  __shared__ double red[2][256 / HELM_WAVE];
  const long long img = blockIdx.x, npx = (long long)D * H * W, base = img * npx;
  double sq = 0.0, sr = 0.0;
  for (long long t = threadIdx.x; t < npx; t += 256) {
    const long long p = base + t;
    if (!res_interior<NDIM>(p, D, H, W)) continue;
    const float* xp = x + p * 4;
    const c32 c = cmul(cb, make_float2(1.f + xp[2], xp[3]));
    const c32 ay = res_apply<NDIM>(y, p, H, W, c);
    const float qx = xp[0] - gamma * ay.x, qy = xp[1] - gamma * ay.y;
    sq += (double)qx * qx + (double)qy * qy;
    sr += (double)xp[0] * xp[0] + (double)xp[1] * xp[1];
  }
  sq = wave_sum_d(sq);
  sr = wave_sum_d(sr);
  if (threadIdx.x % HELM_WAVE == 0) {
    red[0][threadIdx.x / HELM_WAVE] = sq;
    red[1][threadIdx.x / HELM_WAVE] = sr;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double v = 0.0;
    for (int w = 0; w < 256 / HELM_WAVE; ++w) v += red[threadIdx.x][w];
    sums[2 * img + threadIdx.x] = v;
  }
}

// Adam on the FP32 master weights (entries with mask 0 -- the padding -- stay 0)
__global__ void k_adam(int n, float* w, const float* dw, float* m, float* v, const unsigned char* mask, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (mask && !mask[t]) {
    w[t] = 0.f;
    return;
  }
  const float gr = dw[t];
  const float mt = b1 * m[t] + (1.f - b1) * gr;
  const float vt = b2 * v[t] + (1.f - b2) * gr * gr;
  m[t] = mt;
  v[t] = vt;
  w[t] -= lr * (mt * c1) / (sqrtf(vt * c2) + eps);
}

// Pack FP32 master weights W[co][k] (k = tap * cin + ci) into the BF16 forward layout and the
// BF16 backward-data layout Wb[ci][tap' * cob + co] = W[co][(ntaps - 1 - tap') * cin + ci]
// (wb_rows >= cin rows; rows past cin, read by the last output tile, are zero).
__global__ void k_pack(int ntaps, int cout_pad, int cin, int kpad, int cob, int kbpad, int wb_rows, const float* w,
                       bf16* wt, bf16* wb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cout_pad * kpad) wt[t] = (bf16)w[t];
  if (wb && t < wb_rows * kbpad) {
    const int ci = t / kbpad, kb = t % kbpad;
    const int tapb = kb / cob, co = kb - tapb * cob;
    float v = 0.f;
    if (ci < cin && tapb < ntaps && co < cout_pad) v = w[(long long)co * kpad + (ntaps - 1 - tapb) * cin + ci];
    wb[t] = (bf16)v;
  }
}

// Network input / output on the solver grid: x[p] = (Re, Im of s v[p], Re, Im of the
// coefficient contrast (c - c_b) / c_b, 0 ...) for one image per right-hand side.
__global__ void k_net_input(int B, long long N, const c32* v, long long v_stride, const float* vscale, int vs_stride,
                            float gain, const c32* coef, c32 cb, bf16* x, int x_ct) {
  const int b = blockIdx.y;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const float s = gain * (vscale ? vscale[(long long)b * vs_stride] : 1.f);
  const c32 r = cscale(v[(long long)b * v_stride + p], s);
  const c32 c = coef[p];
  const float inv = 1.f / (cb.x * cb.x + cb.y * cb.y);
  const c32 d = make_float2(c.x - cb.x, c.y - cb.y);
  const c32 q = make_float2((d.x * cb.x + d.y * cb.y) * inv, (d.y * cb.x - d.x * cb.y) * inv);
  bf16* xp = x + ((long long)b * N + p) * x_ct;
  if (x_ct == 8) {  // one 16-byte store per pixel
    bf16x8 o = zero8();
    o[0] = (bf16)r.x;
    o[1] = (bf16)r.y;
    o[2] = (bf16)q.x;
    o[3] = (bf16)q.y;
    *reinterpret_cast<bf16x8*>(xp) = o;
    return;
  }
  xp[0] = (bf16)r.x;
  xp[1] = (bf16)r.y;
  xp[2] = (bf16)q.x;
  xp[3] = (bf16)q.y;
  for (int c2 = 4; c2 < x_ct; ++c2) xp[c2] = (bf16)0.f;
}

// z[b][p] = gain * (y[p][0] + j y[p][1])
__global__ void k_net_output(int B, long long N, const float* y, float gain, c32* z, long long z_stride,
                             const int* mask) {
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const float* yp = y + ((long long)b * N + p) * 2;
  z[(long long)b * z_stride + p] = make_float2(gain * yp[0], gain * yp[1]);
}

// out[p][c] = bf16(x[p][c]) for c < cin, 0 up to cpad channels
__global__ void k_to_bf16_pad(long long P, int cin, const float* x, int cpad, bf16* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P * cpad) return;
  const long long p = t / cpad;
  const int c = (int)(t % cpad);
  out[t] = (bf16)(c < cin ? x[p * cin + c] : 0.f);
}
// the same for 4 input channels padded to 8: one pixel per thread, 16-byte load and store
__global__ void k_to_bf16_pad48(long long P, const float4* x, bf16x8* out) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float4 v = x[p];
  bf16x8 o = zero8();
  o[0] = (bf16)v.x;
  o[1] = (bf16)v.y;
  o[2] = (bf16)v.z;
  o[3] = (bf16)v.w;
  out[p] = o;
}

// Training examples from solver snapshots: crop c = (rhs b, y0, x0) of size S x S;
// r' = r_scale * r (the scaled residual), e = x_final - x_k; features are r' / rms_crop(r')
// and the coefficient contrast, targets e / rms_crop(r') / gamma.
// ss[b] = sum over the grid of |r_scale r[b]|^2 (one block per right-hand side, fixed order)
__global__ __launch_bounds__(256) void k_field_sumsq(long long N, const c32* r, float r_scale, float* ss) {
  __shared__ float red[256];
  const int b = blockIdx.x;
  const c32* rb = r + (long long)b * N;
  float s = 0.f;
  for (long long p = threadIdx.x; p < N; p += 256) {
    const c32 v = cscale(rb[p], r_scale);
    s = fmaf(v.x, v.x, fmaf(v.y, v.y, s));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) ss[b] = red[0];
}

// One block per crop: features (r_scale r / rms, contrast) and target (x* - x_k) / rms / gamma,
// with rms the root mean square of r_scale r[b] over the whole grid of its right-hand side.
// Crop c = (rhs, (z0,) y0, x0) of S^NDIM points.
template <int NDIM>
__global__ __launch_bounds__(256) void k_examples(int S, int n_e, const int* crops, const float* ss, const c32* r,
                                                  const c32* xfin, const c32* xk, long long N, const c32* coef, c32 cb,
                                                  float r_scale, float inv_gamma, float* feat, float* tgt) {
  const int c = blockIdx.x;
  const int* cr = crops + (1 + NDIM) * c;
  const int b = cr[0], z0 = NDIM == 3 ? cr[1] : 0, y0 = cr[NDIM - 1], x0 = cr[NDIM];
  const long long base = (long long)b * N;
  const float rms = sqrtf(ss[b] / (float)N);
  const float inv = rms > 0.f ? 1.f / rms : 0.f;
  const float invc = 1.f / (cb.x * cb.x + cb.y * cb.y);
  const long long npx = NDIM == 3 ? (long long)S * S * S : (long long)S * S;
  for (long long t = threadIdx.x; t < npx; t += 256) {
    const int tx = (int)(t % S), ty = (int)((t / S) % S), tz = NDIM == 3 ? (int)(t / ((long long)S * S)) : 0;
    const long long p = ((long long)(z0 + tz) * n_e + (y0 + ty)) * n_e + (x0 + tx);
    const c32 v = cscale(r[base + p], r_scale * inv);
    const c32 e = cscale(csub(xfin[base + p], xk[base + p]), inv * inv_gamma);
    const c32 cc = coef[p];
    const c32 d = make_float2(cc.x - cb.x, cc.y - cb.y);
    float* f = feat + ((long long)c * npx + t) * 4;
    f[0] = v.x;
    f[1] = v.y;
    f[2] = (d.x * cb.x + d.y * cb.y) * invc;
    f[3] = (d.y * cb.x - d.x * cb.y) * invc;
    float* o = tgt + ((long long)c * npx + t) * 2;
    o[0] = e.x;
    o[1] = e.y;
  }
}

inline unsigned nb(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_to_bf16_pad(hipStream_t s, long long P, int cin, const float* x, int cpad, bf16* out) {
  if (cin == 4 && cpad == 8 && ((uintptr_t)x % 16) == 0 && ((uintptr_t)out % 16) == 0)
    hipLaunchKernelGGL(k_to_bf16_pad48, dim3(nb(P, 256)), dim3(256), 0, s, P, reinterpret_cast<const float4*>(x),
                       reinterpret_cast<bf16x8*>(out));
  else
    hipLaunchKernelGGL(k_to_bf16_pad, dim3(nb(P * cpad, 256)), dim3(256), 0, s, P, cin, x, cpad, out);
}
void launch_examples(hipStream_t s, int dim, int B, int ncrop, int S, int n_e, const int* crops, float* ss,
                     const c32* r, const c32* xfin, const c32* xk, long long N, const c32* coef, c32 cb,
                     float r_scale, float inv_gamma, float* feat, float* tgt) {
  hipLaunchKernelGGL(k_field_sumsq, dim3(B), dim3(256), 0, s, N, r, r_scale, ss);
  if (dim == 3)
    hipLaunchKernelGGL(k_examples<3>, dim3(ncrop), dim3(256), 0, s, S, n_e, crops, ss, r, xfin, xk, N, coef, cb,
                       r_scale, inv_gamma, feat, tgt);
  else
    hipLaunchKernelGGL(k_examples<2>, dim3(ncrop), dim3(256), 0, s, S, n_e, crops, ss, r, xfin, xk, N, coef, cb,
                       r_scale, inv_gamma, feat, tgt);
}

template <int NCO, int TH, int TW, int NDIM>
void conv_lds(hipStream_t s, const ConvArgs& a) {
  constexpr int ZM = 8;  // output planes per block of the marching 3D form
  if constexpr (NDIM == 3) {
    const bool wl3 = 16LL * NCO * a.kpad * (long long)sizeof(bf16) > 32768;
    if (!a.src.pool && !wl3 && a.cin <= 64) {
      const size_t lz = (size_t)4 * (TH + 2) * (TW + 2) * (a.cin == 8 ? 8 : a.cin + 8) * sizeof(bf16);
      const dim3 gz((a.W + TW - 1) / TW, (a.H + TH - 1) / TH, a.nimg * ((a.D + ZM - 1) / ZM));
      if (a.src.cup > 0) hipLaunchKernelGGL((k_conv_lds<NCO, TH, TW, 2, 3, false, ZM>), gz, dim3(256), lz, s, a);
      else hipLaunchKernelGGL((k_conv_lds<NCO, TH, TW, 0, 3, false, ZM>), gz, dim3(256), lz, s, a);
      return;
    }
  }
  const size_t lds = (size_t)(NDIM == 3 ? 3 : 1) * (TH + 2) * (TW + 2) * (a.cin == 8 ? 8 : a.cin + 8) * sizeof(bf16);
  const dim3 grid((a.W + TW - 1) / TW, (a.H + TH - 1) / TH, a.nimg * (NDIM == 3 ? a.D : 1));
  // weights above the 32 KB L1 pass through LDS (two chunk buffers)
  const bool wl = 16LL * NCO * a.kpad * (long long)sizeof(bf16) > 32768;
  const size_t lw = lds + (wl ? 2 * 16 * NCO * WROW * sizeof(bf16) : 0);
  if (wl) {
    if (a.src.pool) hipLaunchKernelGGL((k_conv_lds<NCO, TH, TW, 1, NDIM, true, 0>), grid, dim3(256), lw, s, a);
    else if (a.src.cup > 0) hipLaunchKernelGGL((k_conv_lds<NCO, TH, TW, 2, NDIM, true, 0>), grid, dim3(256), lw, s, a);
    else hipLaunchKernelGGL((k_conv_lds<NCO, TH, TW, 0, NDIM, true, 0>), grid, dim3(256), lw, s, a);
    return;
  }
  if (a.src.pool) hipLaunchKernelGGL((k_conv_lds<NCO, TH, TW, 1, NDIM, false, 0>), grid, dim3(256), lds, s, a);
  else if (a.src.cup > 0) hipLaunchKernelGGL((k_conv_lds<NCO, TH, TW, 2, NDIM, false, 0>), grid, dim3(256), lds, s, a);
  else hipLaunchKernelGGL((k_conv_lds<NCO, TH, TW, 0, NDIM, false, 0>), grid, dim3(256), lds, s, a);
}

template <int CIN, int NCO, int TH, int MODE>
void conv2c(hipStream_t s, const ConvArgs& a) {
  constexpr int TW = 32, KPAD = (9 * CIN + 31) / 32 * 32;
  constexpr bool WL = 16 * NCO * KPAD * (int)sizeof(bf16) > 32768;  // weights above the 32 KB L1
  const size_t lds = (size_t)(TH + 2) * (TW + 2) * (CIN == 8 ? 8 : CIN + 8) * sizeof(bf16) + (WL ? 2 * 16 * NCO * WROW * sizeof(bf16) : 0);
  const dim3 grid((a.W + TW - 1) / TW, (a.H + TH - 1) / TH, a.nimg);
  hipLaunchKernelGGL((k_conv2c<CIN, NCO, TH, TW, MODE, WL>), grid, dim3(256), lds, s, a);
}

template <int CIN, int NCO, int TH, int MODE, int NIT, int PD>
void conv2m(hipStream_t s, const ConvArgs& a) {
  constexpr int TW = 32;
  const size_t lds = (size_t)(TH + 2) * (TW + 2) * (CIN == 8 ? 8 : CIN + 8) * sizeof(bf16);
  const int ty = (a.H + TH - 1) / TH;
  const dim3 grid((a.W + TW - 1) / TW, (ty + NIT - 1) / NIT, a.nimg);
  hipLaunchKernelGGL((k_conv2m<CIN, NCO, TH, TW, MODE, NIT, PD>), grid, dim3(256), lds, s, a);
}

// The channel-specialised kernels of the 2D network's forward layers (their tile shapes
// those of the generic kernel); false when the layer has none.  The pooled 16-channel
// layer (A1) stays on the generic kernel: its specialised form, holding 40 weight
// registers beside four pooled sources per chunk, runs at 3 wavefronts per SIMD and was
// slower (272-288 against 247 us at 60 x 577^2).
bool conv2c_dispatch(hipStream_t s, const ConvArgs& a, int nco) {
  if (a.kpad != (9 * a.cin + 31) / 32 * 32) return false;
  const int mode = a.src.pool ? 1 : (a.src.cup > 0 ? 2 : 0);
  switch ((a.cin << 8) | (nco << 4) | mode) {
    case (8 << 8) | (1 << 4) | 0: conv2c<8, 1, 8, 0>(s, a); return true;       // A0
    case (32 << 8) | (4 << 4) | 1: conv2c<32, 4, 8, 1>(s, a); return true;     // A2
    case (64 << 8) | (4 << 4) | 1: conv2c<64, 4, 8, 1>(s, a); return true;     // A3
    case (128 << 8) | (4 << 4) | 2: conv2c<128, 4, 4, 2>(s, a); return true;   // B2
    case (96 << 8) | (2 << 4) | 2: conv2c<96, 2, 4, 2>(s, a); return true;     // B1
    case (48 << 8) | (1 << 4) | 2: conv2m<48, 1, 8, 2, 16, 1>(s, a); return true;     // B0 (marching)
    case (16 << 8) | (1 << 4) | 0: conv2c<16, 1, 8, 0>(s, a); return true;     // O
    default: return false;
  }
}

template <int CIN, int MODE, int PD = 1, int NCO = 1>
void conv3c(hipStream_t s, const ConvArgs& a) {
  constexpr int TH = 4, TW = 32, ZM = 8;
  const size_t lds = (size_t)4 * (TH + 2) * (TW + 2) * (CIN == 8 ? 8 : CIN + 8) * sizeof(bf16);
  const dim3 grid((a.W + TW - 1) / TW, (a.H + TH - 1) / TH, a.nimg * ((a.D + ZM - 1) / ZM));
  hipLaunchKernelGGL((k_conv3c<CIN, NCO, TH, TW, MODE, ZM, PD>), grid, dim3(256), lds, s, a);
}

// The channel-specialised kernels of the 3D network's layers (the generic marching
// kernel's 4 x 32 tile and 8 planes per block).  B1, whose weights exceed the L1, and
// the pooled A1 and A2 march here too, where the generic kernel stages three planes per
// output plane; B1 runs one wavefront per SIMD and reads its operands three k-steps
// ahead.  False when the layer has none (A3 and B2: weights of 55 and 110 KB).
bool conv3c_dispatch(hipStream_t s, const ConvArgs& a, int nco) {
  if (a.kpad != (27 * a.cin + 31) / 32 * 32) return false;
  const int mode = a.src.pool ? 1 : (a.src.cup > 0 ? 2 : 0);
  if (nco == 2) {
    if (a.cin == 16 && mode == 1) {
      conv3c<16, 1, 1, 2>(s, a);  // A2 (pooled input, two output tiles)
      return true;
    }
    return false;
  }
  if (nco != 1) return false;
  switch ((a.cin << 4) | mode) {
    case (16 << 4) | 1: conv3c<16, 1>(s, a); return true;  // A1 (pooled input)
    case (8 << 4) | 0: conv3c<8, 0>(s, a); return true;    // A0
    case (32 << 4) | 2: conv3c<32, 2>(s, a); return true;  // B0
    case (48 << 4) | 2: conv3c<48, 2, 3>(s, a); return true;  // B1
    case (16 << 4) | 0: conv3c<16, 0>(s, a); return true;  // O
    default: return false;
  }
}

// 2D tile: 8 x 32 pixels (four 16-pixel segments per wavefront) while the halo tile stays
// within 50 KB of LDS and the accumulators within 64 registers, else 4 x 32.  3D: three
// staged planes, so 4 x 32 up to 32 input channels and 2 x 32 above (under 60 KB).
// Unless `generic`, a layer with a channel-specialised kernel runs that one (same result).
void launch_conv3x3(hipStream_t s, const ConvArgs& a, int nco, int dim, bool generic) {
  if (dim == 2 && !generic && conv2c_dispatch(s, a, nco)) return;
  if (dim == 3 && !generic && conv3c_dispatch(s, a, nco)) return;
  if (dim == 3) {
    const bool wide = a.cin > 32;
    switch (nco) {
      case 1: wide ? conv_lds<1, 2, 32, 3>(s, a) : conv_lds<1, 4, 32, 3>(s, a); break;
      case 2: wide ? conv_lds<2, 2, 32, 3>(s, a) : conv_lds<2, 4, 32, 3>(s, a); break;
      case 3: wide ? conv_lds<3, 2, 32, 3>(s, a) : conv_lds<3, 4, 32, 3>(s, a); break;
      case 4: wide ? conv_lds<4, 2, 32, 3>(s, a) : conv_lds<4, 4, 32, 3>(s, a); break;
      default: break;
    }
    return;
  }
  const bool big = a.cin > 64 || nco > 4;
  switch (nco) {
    case 1: big ? conv_lds<1, 4, 32, 2>(s, a) : conv_lds<1, 8, 32, 2>(s, a); break;
    case 2: big ? conv_lds<2, 4, 32, 2>(s, a) : conv_lds<2, 8, 32, 2>(s, a); break;
    case 3: big ? conv_lds<3, 4, 32, 2>(s, a) : conv_lds<3, 8, 32, 2>(s, a); break;
    case 4: big ? conv_lds<4, 4, 32, 2>(s, a) : conv_lds<4, 8, 32, 2>(s, a); break;
    case 6: conv_lds<6, 4, 32, 2>(s, a); break;
    case 8: conv_lds<8, 4, 32, 2>(s, a); break;
    default: break;
  }
}

void launch_wgrad(hipStream_t s, const WgradArgs& a, int nchunk, float* dw, const bf16* g_for_bias, float* db,
                  int cout_real) {
  const dim3 grid(a.kpad / 16, a.cout_pad / 16, nchunk);
  if (a.dim == 3) hipLaunchKernelGGL(k_wgrad<3>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_wgrad<2>, grid, dim3(256), 0, s, a);
  const int n = a.cout_pad * a.kpad;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb(n, 256)), dim3(256), 0, s, nchunk, n, a.part, dw);
  const long long P = (long long)a.nimg * (a.dim == 3 ? a.D : 1) * a.H * a.W;
  if (256 % a.g_ct == 0 && cout_real <= a.g_ct) {
    // the weight partials are consumed by now (stream order): reuse the buffer
    hipLaunchKernelGGL(k_bias_part, dim3(nchunk), dim3(256), 0, s, P, a.chunk, g_for_bias, a.g_ct, cout_real, a.part);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb(cout_real, 256)), dim3(256), 0, s, nchunk, cout_real, a.part, db);
  } else {
    hipLaunchKernelGGL(k_bias_grad, dim3(cout_real), dim3(256), 0, s, P, g_for_bias, a.g_ct, db);
  }
}

void launch_grad_prep(hipStream_t s, long long P, const float* g, int g_ct, int g_off, const bf16* act, int act_ct,
                      int act_off, int creal, int cpad, bf16* gm) {
  hipLaunchKernelGGL(k_grad_prep, dim3(nb(P * cpad, 256)), dim3(256), 0, s, P, g, g_ct, g_off, act, act_ct, act_off,
                     creal, cpad, gm);
}
void launch_pool_back(hipStream_t s, int dim, int nimg, int D, int H, int W, int C, const float* g, int g_ct,
                      float* gin, int gin_ct, int gin_off) {
  const long long n = (long long)nimg * D * H * W * C;
  if (dim == 3)
    hipLaunchKernelGGL(k_pool_back<3>, dim3(nb(n, 256)), dim3(256), 0, s, nimg, D, H, W, C, g, g_ct, gin, gin_ct,
                       gin_off);
  else
    hipLaunchKernelGGL(k_pool_back<2>, dim3(nb(n, 256)), dim3(256), 0, s, nimg, 1, H, W, C, g, g_ct, gin, gin_ct,
                       gin_off);
}
void launch_upsample_back(hipStream_t s, int dim, int nimg, int D, int H, int W, int C, const float* g, int g_ct,
                          int g_off, float* gc) {
  const long long n = (long long)nimg * (dim == 3 ? (D + 1) / 2 : 1) * ((H + 1) / 2) * ((W + 1) / 2) * C;
  if (dim == 3)
    hipLaunchKernelGGL(k_upsample_back<3>, dim3(nb(n, 256)), dim3(256), 0, s, nimg, D, H, W, C, g, g_ct, g_off, gc);
  else
    hipLaunchKernelGGL(k_upsample_back<2>, dim3(nb(n, 256)), dim3(256), 0, s, nimg, 1, H, W, C, g, g_ct, g_off, gc);
}
int loss_partials(long long n) { return (int)nb(n, 256); }
void launch_loss(hipStream_t s, long long n, const float* y, const float* tgt, float inv_nimg, float* gy,
                 float* part) {
  hipLaunchKernelGGL(k_loss, dim3(nb(n, 256)), dim3(256), 0, s, n, y, tgt, inv_nimg, gy, part);
}
void launch_res_loss(hipStream_t s, int dim, int nimg, int D, int H, int W, const float* x, const float* y,
                     float gamma, c32 cb, float w, float2* q, float* part, float* gy) {
  const long long P = (long long)nimg * D * H * W;
  if (dim == 3) {
    hipLaunchKernelGGL(k_res_q<3>, dim3(nb(P, 256)), dim3(256), 0, s, nimg, D, H, W, x, y, gamma, cb, w, q, part);
    hipLaunchKernelGGL(k_res_grad<3>, dim3(nb(P, 256)), dim3(256), 0, s, nimg, D, H, W, x, q, gamma, cb, w, gy);
  } else {
    hipLaunchKernelGGL(k_res_q<2>, dim3(nb(P, 256)), dim3(256), 0, s, nimg, 1, H, W, x, y, gamma, cb, w, q, part);
    hipLaunchKernelGGL(k_res_grad<2>, dim3(nb(P, 256)), dim3(256), 0, s, nimg, 1, H, W, x, q, gamma, cb, w, gy);
  }
}
void launch_res_ratio(hipStream_t s, int dim, int nimg, int D, int H, int W, const float* x, const float* y,
                      float gamma, c32 cb, double* sums) {
  if (dim == 3) hipLaunchKernelGGL(k_res_ratio<3>, dim3(nimg), dim3(256), 0, s, D, H, W, x, y, gamma, cb, sums);
  else hipLaunchKernelGGL(k_res_ratio<2>, dim3(nimg), dim3(256), 0, s, 1, H, W, x, y, gamma, cb, sums);
}
void launch_adam(hipStream_t s, int n, float* w, const float* dw, float* m, float* v, const unsigned char* mask,
                 float lr, float b1, float b2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_adam, dim3(nb(n, 256)), dim3(256), 0, s, n, w, dw, m, v, mask, lr, b1, b2, eps, c1, c2);
}
void launch_pack(hipStream_t s, int ntaps, int cout_pad, int cin, int kpad, int cob, int kbpad, int wb_rows,
                 const float* w, bf16* wt, bf16* wb) {
  const int n = std::max(cout_pad * kpad, wb ? wb_rows * kbpad : 0);
  hipLaunchKernelGGL(k_pack, dim3(nb(n, 256)), dim3(256), 0, s, ntaps, cout_pad, cin, kpad, cob, kbpad, wb_rows, w,
                     wt, wb);
}
void launch_net_input(hipStream_t s, int B, long long N, const c32* v, long long v_stride, const float* vscale,
                      int vs_stride, float gain, const c32* coef, c32 cb, bf16* x, int x_ct) {
  hipLaunchKernelGGL(k_net_input, dim3(nb(N, 256), B), dim3(256), 0, s, B, N, v, v_stride, vscale, vs_stride, gain,
                     coef, cb, x, x_ct);
}
void launch_net_output(hipStream_t s, int B, long long N, const float* y, float gain, c32* z, long long z_stride,
                       const int* mask) {
  hipLaunchKernelGGL(k_net_output, dim3(nb(N, 256), B), dim3(256), 0, s, B, N, y, gain, z, z_stride, mask);
}
