// Kernels of the learned preconditioner network (BF16 storage, FP32
// accumulation, v_mfma_f32_16x16x32_bf16 on gfx950).
//
// Activations are NHWC: element (pixel p, channel c) of a buffer with
// channel stride ct at channel offset off is buf[p * ct + off + c]; pixels
// are flattened over (image, y, x).  A 3x3 convolution is an implicit GEMM
//     out[p][co] = bias[co] + sum_k in[p + shift(tap(k))][ci(k)] * Wt[co][k],
//     k = tap * cin + ci,  tap = 3 (dy + 1) + (dx + 1),
// with the weights packed as Wt[co][k] (k padded to a multiple of 32).
// MFMA 16x16x32 operand layout (lane l, g = l / 16):
//     A[i][k]: i = l % 16, k = 8 g + v (v = 0..7)      (16 pixels x 32 k)
//     B[k][j]: j = l % 16, k = 8 g + v                 (32 k x 16 channels)
//     D[i][j]: j = l % 16, i = 4 g + r (r = 0..3)
#include <algorithm>

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

// ---------------------------------------------------------------- conv (MFMA)
// One wavefront computes 16 consecutive pixels of one image row for all
// output channels (NCO tiles of 16); four wavefronts per block.
template <int NCO>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a) {
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64, g = l / 16, i16 = l % 16;
  const int xt = (a.W + 15) / 16;
  const long long tile = (long long)blockIdx.x * 4 + wave;
  const long long ntiles = (long long)a.nimg * a.H * xt;
  if (tile >= ntiles) return;
  const int x0 = (int)(tile % xt) * 16;
  const long long rowid = tile / xt;  // image * H + y
  const int y = (int)(rowid % a.H);
  const long long img = rowid / a.H;
  const int x = x0 + i16;
  f32x4 acc[NCO];
#pragma unroll
  for (int t = 0; t < NCO; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < a.kpad; kc += 32) {
    const int k0 = kc + 8 * g;
    const int tap = k0 / a.cin, ci0 = k0 - tap * a.cin;
    bf16x8 av = zero8();
    if (tap < 9) {
      const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
      if (x < a.W && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
        av = load8(a.in + ((img * a.H + yy) * a.W + xx) * a.in_ct + a.in_off + ci0);
    }
#pragma unroll
    for (int t = 0; t < NCO; ++t) {
      const bf16x8 bv = load8(a.wt + (long long)(t * 16 + i16) * a.kpad + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NCO; ++t) {
    const int co = t * 16 + i16;
    if (co >= a.cout) continue;
    const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int xo = x0 + 4 * g + r;
      if (xo >= a.W) continue;
      float v = acc[t][r] + bias;
      if (a.relu) v = fmaxf(v, 0.f);
      const long long p = (img * a.H + y) * a.W + xo;
      if (a.out32) a.out32[p * a.out_ct + a.out_off + co] = v;
      else a.out[p * a.out_ct + a.out_off + co] = (bf16)v;
    }
  }
}

// ---------------------------------------------------------------- weight gradient (MFMA)
// dW[co][k] = sum_p in[p + shift(tap(k))][ci(k)] * g[p][co]: a GEMM over pixels.
// Block (k tile of 16, channel tile of 16, pixel chunk); each wavefront takes a
// quarter of the chunk, the four partial tiles are summed in LDS and written
// to part[chunk][co][k] (reduced in a fixed order by k_wgrad_reduce).
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
  __shared__ float red[4][16][17];
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64, gq = l / 16, i16 = l % 16;
  const int kt = blockIdx.x, ct = blockIdx.y, chunk = blockIdx.z;
  const long long P = (long long)a.nimg * a.H * a.W;
  const long long p_begin = (long long)chunk * a.chunk + (long long)wave * (a.chunk / 4);
  const long long p_end = min(p_begin + a.chunk / 4, P);
  const int krow = kt * 16 + i16;                  // A row of this lane
  const int tap = krow / a.cin, ci = krow - tap * a.cin;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int co = ct * 16 + i16;                    // B column of this lane
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (long long pc = p_begin; pc < p_end; pc += 32) {
    bf16x8 av, bv;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const long long p = pc + 8 * gq + v;
      float xa = 0.f, gb = 0.f;
      if (p < p_end) {
        const int px = (int)(p % a.W);
        const long long r = p / a.W;
        const int py = (int)(r % a.H);
        const int yy = py + dy, xx = px + dx;
        if (tap < 9 && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
          xa = (float)a.in[(p + (long long)dy * a.W + dx) * a.in_ct + a.in_off + ci];
        gb = (float)a.g[p * a.g_ct + co];
      }
      av[v] = (__bf16)xa;
      bv[v] = (__bf16)gb;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
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

// db[co] = sum_p g[p][co] (one block per channel, fixed-order reduction)
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

// out[P'][off + c] = 1/4 sum of the 2x2 window of in (zero padding), C channels
__global__ void k_pool(int nimg, int H, int W, int C, const bf16* in, int in_ct, int in_off, bf16* out, int out_ct,
                       int out_off) {
  const int Hc = (H + 1) / 2, Wc = (W + 1) / 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nimg * Hc * Wc * C) return;
  const int c = (int)(t % C);
  const long long q = t / C;
  const int X = (int)(q % Wc);
  const long long r = q / Wc;
  const int Y = (int)(r % Hc);
  const long long img = r / Hc;
  float s = 0.f;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int yy = 2 * Y + a, xx = 2 * X + b;
      if (yy < H && xx < W) s += (float)in[((img * H + yy) * W + xx) * in_ct + in_off + c];
    }
  out[q * out_ct + out_off + c] = (bf16)(0.25f * s);
}

// gin[p][off + c] += 1/4 g[parent(p)][c]   (fp32)
__global__ void k_pool_back(int nimg, int H, int W, int C, const float* g, int g_ct, float* gin, int gin_ct,
                            int gin_off) {
  const int Hc = (H + 1) / 2, Wc = (W + 1) / 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nimg * H * W * C) return;
  const int c = (int)(t % C);
  const long long p = t / C;
  const int x = (int)(p % W);
  const long long r = p / W;
  const int y = (int)(r % H);
  const long long img = r / H;
  const long long q = (img * Hc + y / 2) * Wc + x / 2;
  gin[p * gin_ct + gin_off + c] += 0.25f * g[q * g_ct + c];
}

// out[p][off + c] = in[parent(p)][c]   (nearest neighbour up to H x W)
__global__ void k_upsample(int nimg, int H, int W, int C, const bf16* in, int in_ct, bf16* out, int out_ct,
                           int out_off) {
  const int Hc = (H + 1) / 2, Wc = (W + 1) / 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nimg * H * W * C) return;
  const int c = (int)(t % C);
  const long long p = t / C;
  const int x = (int)(p % W);
  const long long r = p / W;
  const int y = (int)(r % H);
  const long long img = r / H;
  out[p * out_ct + out_off + c] = in[((img * Hc + y / 2) * Wc + x / 2) * in_ct + c];
}

// gc[q][c] = sum over the children p of q of g[p][off + c]   (fp32)
__global__ void k_upsample_back(int nimg, int H, int W, int C, const float* g, int g_ct, int g_off, float* gc) {
  const int Hc = (H + 1) / 2, Wc = (W + 1) / 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nimg * Hc * Wc * C) return;
  const int c = (int)(t % C);
  const long long q = t / C;
  const int X = (int)(q % Wc);
  const long long r = q / Wc;
  const int Y = (int)(r % Hc);
  const long long img = r / Hc;
  float s = 0.f;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int yy = 2 * Y + a, xx = 2 * X + b;
      if (yy < H && xx < W) s += g[((img * H + yy) * W + xx) * g_ct + g_off + c];
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
// complex, q = r - gamma A' y on the interior of every image (one-pixel
// border excluded: the crop's neighbours outside it are unknown), where
// A' y = (4 - c) y - (sum of the 4 neighbours).  part[block] = w/2 sum |q|^2.
__global__ void k_res_q(int nimg, int H, int W, const float* x, const float* y, float gamma, c32 cb, float w,
                        float2* q, float* part) {
  __shared__ float red[256];
  const long long P = (long long)nimg * H * W;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.f;
  if (p < P) {
    const int px = (int)(p % W), py = (int)((p / W) % H);
    float2 qq = make_float2(0.f, 0.f);
    if (px > 0 && px < W - 1 && py > 0 && py < H - 1) {
      const float* xp = x + p * 4;
      const c32 f = make_float2(xp[2], xp[3]);
      const c32 c = cmul(cb, make_float2(1.f + f.x, f.y));
      const c32 yc = make_float2(y[p * 2], y[p * 2 + 1]);
      const c32 nbs = make_float2(y[(p - 1) * 2] + y[(p + 1) * 2] + y[(p - W) * 2] + y[(p + W) * 2],
                                  y[(p - 1) * 2 + 1] + y[(p + 1) * 2 + 1] + y[(p - W) * 2 + 1] + y[(p + W) * 2 + 1]);
      const c32 ay = csub(cmul(make_float2(4.f - c.x, -c.y), yc), nbs);
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

// gy += -w gamma A'^H q, A'^H q = (4 - conj c) q - (sum of the neighbours of q); q is zero
// on the border, and neighbours outside the image count as zero.
__global__ void k_res_grad(int nimg, int H, int W, const float* x, const float2* q, float gamma, c32 cb, float w,
                           float* gy) {
  const long long P = (long long)nimg * H * W;
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
  const c32 g = csub(cmul(make_float2(4.f - c.x, c.y), q[p]), nbs);
  gy[p * 2] -= w * gamma * g.x;
  gy[p * 2 + 1] -= w * gamma * g.y;
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

// Pack FP32 master weights W[co][k] (k = tap * cin + ci) into the BF16 forward
// layout and the BF16 backward-data layout Wb[ci][tap' * cob + co] = W[co][(8 - tap') * cin + ci].
__global__ void k_pack(int cout_pad, int cin, int kpad, int cob, int kbpad, const float* w, bf16* wt, bf16* wb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cout_pad * kpad) wt[t] = (bf16)w[t];
  if (wb && t < cin * kbpad) {
    const int ci = t / kbpad, kb = t % kbpad;
    const int tapb = kb / cob, co = kb - tapb * cob;
    float v = 0.f;
    if (tapb < 9 && co < cout_pad) v = w[(long long)co * kpad + (8 - tapb) * cin + ci];
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
__global__ __launch_bounds__(256) void k_examples(int S, int n_e, const int* crops, const float* ss, const c32* r,
                                                  const c32* xfin, const c32* xk, long long N, const c32* coef, c32 cb,
                                                  float r_scale, float inv_gamma, float* feat, float* tgt) {
  const int c = blockIdx.x;
  const int b = crops[3 * c], y0 = crops[3 * c + 1], x0 = crops[3 * c + 2];
  const long long base = (long long)b * N;
  const float rms = sqrtf(ss[b] / (float)N);
  const float inv = rms > 0.f ? 1.f / rms : 0.f;
  const float invc = 1.f / (cb.x * cb.x + cb.y * cb.y);
  for (int t = threadIdx.x; t < S * S; t += 256) {
    const long long p = (long long)(y0 + t / S) * n_e + (x0 + t % S);
    const c32 v = cscale(r[base + p], r_scale * inv);
    const c32 e = cscale(csub(xfin[base + p], xk[base + p]), inv * inv_gamma);
    const c32 cc = coef[p];
    const c32 d = make_float2(cc.x - cb.x, cc.y - cb.y);
    float* f = feat + ((long long)c * S * S + t) * 4;
    f[0] = v.x;
    f[1] = v.y;
    f[2] = (d.x * cb.x + d.y * cb.y) * invc;
    f[3] = (d.y * cb.x - d.x * cb.y) * invc;
    float* o = tgt + ((long long)c * S * S + t) * 2;
    o[0] = e.x;
    o[1] = e.y;
  }
}

inline unsigned nb(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_to_bf16_pad(hipStream_t s, long long P, int cin, const float* x, int cpad, bf16* out) {
  hipLaunchKernelGGL(k_to_bf16_pad, dim3(nb(P * cpad, 256)), dim3(256), 0, s, P, cin, x, cpad, out);
}
void launch_examples(hipStream_t s, int B, int ncrop, int S, int n_e, const int* crops, float* ss, const c32* r,
                     const c32* xfin, const c32* xk, long long N, const c32* coef, c32 cb, float r_scale,
                     float inv_gamma, float* feat, float* tgt) {
  hipLaunchKernelGGL(k_field_sumsq, dim3(B), dim3(256), 0, s, N, r, r_scale, ss);
  hipLaunchKernelGGL(k_examples, dim3(ncrop), dim3(256), 0, s, S, n_e, crops, ss, r, xfin, xk, N, coef, cb, r_scale,
                     inv_gamma, feat, tgt);
}

void launch_conv3x3(hipStream_t s, const ConvArgs& a, int nco) {
  const long long tiles = (long long)a.nimg * a.H * ((a.W + 15) / 16);
  const unsigned blocks = nb(tiles, 4);
  switch (nco) {
    case 1: hipLaunchKernelGGL(k_conv3x3<1>, dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_conv3x3<2>, dim3(blocks), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_conv3x3<3>, dim3(blocks), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_conv3x3<4>, dim3(blocks), dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_conv3x3<6>, dim3(blocks), dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_conv3x3<8>, dim3(blocks), dim3(256), 0, s, a); break;
    default: break;
  }
}

void launch_wgrad(hipStream_t s, const WgradArgs& a, int nchunk, float* dw, const bf16* g_for_bias, float* db,
                  int cout_real) {
  hipLaunchKernelGGL(k_wgrad, dim3(a.kpad / 16, a.cout_pad / 16, nchunk), dim3(256), 0, s, a);
  const int n = a.cout_pad * a.kpad;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb(n, 256)), dim3(256), 0, s, nchunk, n, a.part, dw);
  const long long P = (long long)a.nimg * a.H * a.W;
  hipLaunchKernelGGL(k_bias_grad, dim3(cout_real), dim3(256), 0, s, P, g_for_bias, a.g_ct, db);
}

void launch_grad_prep(hipStream_t s, long long P, const float* g, int g_ct, int g_off, const bf16* act, int act_ct,
                      int act_off, int creal, int cpad, bf16* gm) {
  hipLaunchKernelGGL(k_grad_prep, dim3(nb(P * cpad, 256)), dim3(256), 0, s, P, g, g_ct, g_off, act, act_ct, act_off,
                     creal, cpad, gm);
}
void launch_pool(hipStream_t s, int nimg, int H, int W, int C, const bf16* in, int in_ct, int in_off, bf16* out,
                 int out_ct, int out_off) {
  const long long n = (long long)nimg * ((H + 1) / 2) * ((W + 1) / 2) * C;
  hipLaunchKernelGGL(k_pool, dim3(nb(n, 256)), dim3(256), 0, s, nimg, H, W, C, in, in_ct, in_off, out, out_ct,
                     out_off);
}
void launch_pool_back(hipStream_t s, int nimg, int H, int W, int C, const float* g, int g_ct, float* gin, int gin_ct,
                      int gin_off) {
  const long long n = (long long)nimg * H * W * C;
  hipLaunchKernelGGL(k_pool_back, dim3(nb(n, 256)), dim3(256), 0, s, nimg, H, W, C, g, g_ct, gin, gin_ct, gin_off);
}
void launch_upsample(hipStream_t s, int nimg, int H, int W, int C, const bf16* in, int in_ct, bf16* out, int out_ct,
                     int out_off) {
  const long long n = (long long)nimg * H * W * C;
  hipLaunchKernelGGL(k_upsample, dim3(nb(n, 256)), dim3(256), 0, s, nimg, H, W, C, in, in_ct, out, out_ct, out_off);
}
void launch_upsample_back(hipStream_t s, int nimg, int H, int W, int C, const float* g, int g_ct, int g_off,
                          float* gc) {
  const long long n = (long long)nimg * ((H + 1) / 2) * ((W + 1) / 2) * C;
  hipLaunchKernelGGL(k_upsample_back, dim3(nb(n, 256)), dim3(256), 0, s, nimg, H, W, C, g, g_ct, g_off, gc);
}
int loss_partials(long long n) { return (int)nb(n, 256); }
void launch_loss(hipStream_t s, long long n, const float* y, const float* tgt, float inv_nimg, float* gy,
                 float* part) {
  hipLaunchKernelGGL(k_loss, dim3(nb(n, 256)), dim3(256), 0, s, n, y, tgt, inv_nimg, gy, part);
}
void launch_res_loss(hipStream_t s, int nimg, int H, int W, const float* x, const float* y, float gamma, c32 cb,
                     float w, float2* q, float* part, float* gy) {
  const long long P = (long long)nimg * H * W;
  hipLaunchKernelGGL(k_res_q, dim3(nb(P, 256)), dim3(256), 0, s, nimg, H, W, x, y, gamma, cb, w, q, part);
  hipLaunchKernelGGL(k_res_grad, dim3(nb(P, 256)), dim3(256), 0, s, nimg, H, W, x, q, gamma, cb, w, gy);
}
void launch_adam(hipStream_t s, int n, float* w, const float* dw, float* m, float* v, const unsigned char* mask,
                 float lr, float b1, float b2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_adam, dim3(nb(n, 256)), dim3(256), 0, s, n, w, dw, m, v, mask, lr, b1, b2, eps, c1, c2);
}
void launch_pack(hipStream_t s, int cout_pad, int cin, int kpad, int cob, int kbpad, const float* w, bf16* wt,
                 bf16* wb) {
  const int n = std::max(cout_pad * kpad, wb ? cin * kbpad : 0);
  hipLaunchKernelGGL(k_pack, dim3(nb(n, 256)), dim3(256), 0, s, cout_pad, cin, kpad, cob, kbpad, w, wt, wb);
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
