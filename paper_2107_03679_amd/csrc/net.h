// Learned-preconditioner network: kernel argument types and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

typedef __bf16 bf16;

// Input of a convolution: channels [0, cup) are the nearest-neighbour upsampling
// of `up` (half resolution, up_ct channels per pixel), channels [cup, cin) come
// from `in` at channel offset in_off (in_ct per pixel): at the convolution's
// resolution, or, with pool = 1, as the 2 x 2 (2D) or 2 x 2 x 2 (3D) average
// (zero padding) of `in` at resolution (Ds x) Hs x Ws.  Channel strides and
// offsets are multiples of 8.  Pixels are flattened over (image, z, y, x); 2D
// layers have depth 1.
struct NetSrc {
  const bf16* in;
  int in_ct, in_off;
  const bf16* up;
  int up_ct, cup;
  int pool, Hs, Ws;
  int Ds;
};

struct ConvArgs {
  NetSrc src;
  int cin;  // channels (multiple of 8)
  int nimg, H, W;
  int D;    // depth (1 in 2D)
  const bf16* wt;  // [cout_pad][kpad] packed weights
  int kpad;
  const float* bias;  // [cout] or NULL
  int cout;           // channels written (<= 16 * NCO)
  int relu;
  bf16* out;     // NHWC output (bf16) ...
  float* out32;  // ... or FP32 output when non-NULL
  int out_ct, out_off;
};

struct WgradArgs {
  NetSrc src;  // layer input
  int cin;
  int nimg, H, W;
  int D;       // depth (1 in 2D)
  int dim;     // 2: 3x3 taps, 3: 3x3x3 taps
  const bf16* g;  // masked output gradient [P][g_ct]
  int g_ct;
  int kpad, cout_pad;
  int chunk;    // pixels per block (multiple of 128)
  float* part;  // [nchunk][cout_pad][kpad]
};

// 3x3 (dim 2) or 3x3x3 (dim 3) convolution, nco output tiles of 16 channels
// generic: the channel-generic kernel even where a channel-specialised one exists
void launch_conv3x3(hipStream_t s, const ConvArgs& a, int nco, int dim, bool generic);
void launch_wgrad(hipStream_t s, const WgradArgs& a, int nchunk, float* dw, const bf16* g_for_bias, float* db,
                  int cout_real);
void launch_grad_prep(hipStream_t s, long long P, const float* g, int g_ct, int g_off, const bf16* act, int act_ct,
                      int act_off, int creal, int cpad, bf16* gm);
// pooling and upsampling adjoints at the fine resolution D x H x W (D = 1 in 2D)
void launch_pool_back(hipStream_t s, int dim, int nimg, int D, int H, int W, int C, const float* g, int g_ct,
                      float* gin, int gin_ct, int gin_off);
void launch_upsample_back(hipStream_t s, int dim, int nimg, int D, int H, int W, int C, const float* g, int g_ct,
                          int g_off, float* gc);
int loss_partials(long long n);
void launch_loss(hipStream_t s, long long n, const float* y, const float* tgt, float inv_nimg, float* gy, float* part);
// residual loss term w/2 sum |r - gamma A' y|^2 over image interiors; adds its gradient to gy
// (part: loss_partials(P) block sums)
void launch_res_loss(hipStream_t s, int dim, int nimg, int D, int H, int W, const float* x, const float* y,
                     float gamma, c32 cb, float w, float2* q, float* part, float* gy);
// per image: interior sums of |r - gamma A' y|^2 and |r|^2 into sums[2 img], sums[2 img + 1] (FP64)
void launch_res_ratio(hipStream_t s, int dim, int nimg, int D, int H, int W, const float* x, const float* y,
                      float gamma, c32 cb, double* sums);
void launch_adam(hipStream_t s, int n, float* w, const float* dw, float* m, float* v, const unsigned char* mask,
                 float lr, float b1, float b2, float eps, float c1, float c2);
// forward weights (bf16) and flipped backward-data weights over ntaps = 9 or 27 taps; wb has
// wb_rows >= cin rows (the rows past cin are zero)
void launch_pack(hipStream_t s, int ntaps, int cout_pad, int cin, int kpad, int cob, int kbpad, int wb_rows,
                 const float* w, bf16* wt, bf16* wb);
void launch_net_input(hipStream_t s, int B, long long N, const c32* v, long long v_stride, const float* vscale,
                      int vs_stride, float gain, const c32* coef, c32 cb, bf16* x, int x_ct);
void launch_net_output(hipStream_t s, int B, long long N, const float* y, float gain, c32* z, long long z_stride,
                       const int* mask);
void launch_to_bf16_pad(hipStream_t s, long long P, int cin, const float* x, int cpad, bf16* out);
// training crops S^dim of the solver grid; crops [ncrop][1 + dim] = (rhs, (z0,) y0, x0)
void launch_examples(hipStream_t s, int dim, int B, int ncrop, int S, int n_e, const int* crops, float* ss,
                     const c32* r, const c32* xfin, const c32* xk, long long N, const c32* coef, c32 cb,
                     float r_scale, float inv_gamma, float* feat, float* tgt);
