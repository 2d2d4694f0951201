// Learned preconditioner network: layers, NHWC (NDHWC) buffers, forward, backward,
// Adam, and the C ABI entry points helm_net_* (include/helm.h).
//
// U-Net, 4 levels, BF16 weights and activations, FP32 accumulation on MFMA, FP32
// master weights; 2D: 16/32/64/64 channels and 3x3 convolutions, 3D: 16/16/32/32
// channels and 3x3x3 convolutions:
//   e0 = relu(A0 x)  e1 = relu(A1 pool e0)  e2 = relu(A2 pool e1)  e3 = relu(A3 pool e2)
//   d2 = relu(B2 [up e3, e2])  d1 = relu(B1 [up d2, e1])  d0 = relu(B0 [up d1, e0])  y = O d0
// Concatenations are channel ranges of one buffer (the upsampled part first).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/helm.h"
#include "net.h"
#include "net_internal.h"

namespace {

struct LayerDef {
  const char* name;
  int cin, cout, relu;
};
const LayerDef kLayers[HELM_NET_LAYERS] = {
    {"A0", 4, 16, 1},  {"A1", 16, 32, 1}, {"A2", 32, 64, 1}, {"A3", 64, 64, 1},
    {"B2", 128, 64, 1}, {"B1", 96, 32, 1}, {"B0", 48, 16, 1}, {"O", 16, 2, 0},
};
const LayerDef kLayers3[HELM_NET_LAYERS] = {
    {"A0", 4, 16, 1},  {"A1", 16, 16, 1}, {"A2", 16, 32, 1}, {"A3", 32, 32, 1},
    {"B2", 64, 32, 1}, {"B1", 48, 16, 1}, {"B0", 32, 16, 1}, {"O", 16, 2, 0},
};
enum { A0, A1, A2, A3, B2, B1, B0, OUT };

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct NetErr {
  hipError_t code;
  const char* what;
};
void ck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw NetErr{e, what};
}

// splitmix64 + Box-Muller for the He-normal initialisation
struct Rng {
  unsigned long long s;
  unsigned long long next() {
    unsigned long long z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() { return std::sqrt(-2.0 * std::log(uniform())) * std::cos(6.283185307179586 * uniform()); }
};

// One set of activation / gradient buffers for up to cap_nimg images of (cap_D x) cap_H x cap_W.
struct NetBufs {
  long long capP0 = 0;
  int cap_nimg = 0, cap_D = 0, cap_H = 0, cap_W = 0;
  int cur_nimg = 0;  // images of the current call (<= cap_nimg)
  bool cap_train = false;
  std::vector<void*> bufs;
  bf16 *x0 = nullptr, *e0 = nullptr, *e1 = nullptr, *e2 = nullptr, *e3 = nullptr, *d2 = nullptr, *d1 = nullptr,
       *d0 = nullptr, *gm = nullptr;
  float2* q = nullptr;  // residual of the residual loss term
  float* rpart = nullptr;
  float *y = nullptr, *gy = nullptr, *g_d0 = nullptr, *g_cat0 = nullptr, *g_d1 = nullptr, *g_cat1 = nullptr,
        *g_d2 = nullptr, *g_cat2 = nullptr, *g_e3 = nullptr, *g_p = nullptr, *part = nullptr, *lpart = nullptr;
  long long part_n = 0;
  int D[4] = {1, 1, 1, 1}, H[4] = {0}, W[4] = {0};
  long long P[4] = {0};
};

}  // namespace

struct helm_net {
  int dim = 2;          // 2: 3x3 convolutions on images, 3: 3x3x3 on volumes
  int ntaps = 9;
  int ch[4] = {0};      // channels of the four levels
  NetLayer L[HELM_NET_LAYERS];
  hipStream_t s = nullptr;
  std::vector<void*> allocs;
  std::string err;
  int step = 0;
  bool generic_conv = false;  // channel-generic convolution kernels only (helm_net_set_conv_kernels)
  // training loss: err_w / 2 sum (y - t)^2 + res_w / 2 sum |r - gamma A' y|^2, per image
  double err_w = 1.0, res_w = 0.0, gamma = 1.0, cb = 0.0;
  NetBufs tb;              // buffers of the user calls (forward / backward)
  NetBufs* cur = &tb;      // the set the kernels of the current call use (a solver
                           // context's own set during its preconditioner applications)

  template <class T>
  T* alloc(size_t n, std::vector<void*>& list) {
    void* p = nullptr;
    ck(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)), "hipMalloc");
    list.push_back(p);
    return (T*)p;
  }
};

namespace {

constexpr int WCHUNK = 4096;

void free_bufs(helm_net* n) {
  for (void* p : n->cur->bufs) hipFree(p);
  n->cur->bufs.clear();
  n->cur->capP0 = 0;
}

void shape(helm_net* n, int nimg, int D0, int H0, int W0) {
  n->cur->D[0] = D0;
  n->cur->H[0] = H0;
  n->cur->W[0] = W0;
  for (int l = 1; l < 4; ++l) {
    n->cur->D[l] = n->dim == 3 ? (n->cur->D[l - 1] + 1) / 2 : 1;
    n->cur->H[l] = (n->cur->H[l - 1] + 1) / 2;
    n->cur->W[l] = (n->cur->W[l - 1] + 1) / 2;
  }
  for (int l = 0; l < 4; ++l) n->cur->P[l] = (long long)nimg * n->cur->D[l] * n->cur->H[l] * n->cur->W[l];
}

// Buffers for up to nimg images of D0 x H0 x W0 (reallocated only when they do not fit).
void ensure(helm_net* n, int nimg, int D0, int H0, int W0, bool train) {
  bool ok = n->cur->capP0 > 0 && nimg <= n->cur->cap_nimg && D0 == n->cur->cap_D && H0 == n->cur->cap_H &&
            W0 == n->cur->cap_W && (!train || n->cur->cap_train);
  if (ok) return;
  shape(n, nimg, D0, H0, W0);
  const long long P0 = n->cur->P[0];
  free_bufs(n);
  auto& B = n->cur->bufs;  // (allocations of this set)
  const long long *P = n->cur->P;
  const int* c = n->ch;
  n->cur->x0 = n->alloc<bf16>(P[0] * 8, B);
  n->cur->e0 = n->alloc<bf16>(P[0] * c[0], B);
  n->cur->e1 = n->alloc<bf16>(P[1] * c[1], B);
  n->cur->e2 = n->alloc<bf16>(P[2] * c[2], B);
  n->cur->e3 = n->alloc<bf16>(P[3] * c[3], B);
  n->cur->d2 = n->alloc<bf16>(P[2] * c[2], B);
  n->cur->d1 = n->alloc<bf16>(P[1] * c[1], B);
  n->cur->d0 = n->alloc<bf16>(P[0] * c[0], B);
  n->cur->y = n->alloc<float>(P[0] * 2, B);
  if (train) {
    n->cur->gy = n->alloc<float>(P[0] * 2, B);
    n->cur->g_d0 = n->alloc<float>(P[0] * c[0], B);
    n->cur->g_cat0 = n->alloc<float>(P[0] * (c[1] + c[0]), B);
    n->cur->g_d1 = n->alloc<float>(P[1] * c[1], B);
    n->cur->g_cat1 = n->alloc<float>(P[1] * (c[2] + c[1]), B);
    n->cur->g_d2 = n->alloc<float>(P[2] * c[2], B);
    n->cur->g_cat2 = n->alloc<float>(P[2] * (c[3] + c[2]), B);
    n->cur->g_e3 = n->alloc<float>(P[3] * c[3], B);
    n->cur->g_p = n->alloc<float>(std::max({P[1] * c[0], P[2] * c[1], P[3] * c[2]}), B);
    n->cur->gm = n->alloc<bf16>(std::max({P[0] * c[0], P[1] * c[1], P[2] * c[2], P[3] * c[3]}), B);
    long long pn = 0;
    const int lvl[HELM_NET_LAYERS] = {0, 1, 2, 3, 2, 1, 0, 0};
    for (int i = 0; i < HELM_NET_LAYERS; ++i) {
      const long long nch = (P[lvl[i]] + WCHUNK - 1) / WCHUNK;
      pn = std::max(pn, nch * n->L[i].cout_pad * n->L[i].kpad);
    }
    n->cur->part = n->alloc<float>(pn, B);
    n->cur->part_n = pn;
    n->cur->lpart = n->alloc<float>(loss_partials(P[0] * 2), B);
    n->cur->q = n->alloc<float2>(P[0], B);
    n->cur->rpart = n->alloc<float>(loss_partials(P[0]), B);
  }
  n->cur->capP0 = P0;
  n->cur->cap_nimg = nimg;
  n->cur->cap_D = D0;
  n->cur->cap_H = H0;
  n->cur->cap_W = W0;
  n->cur->cap_train = train;
}

void set_current(helm_net* n, int nimg, int D0, int H0, int W0) {
  shape(n, nimg, D0, H0, W0);
  n->cur->cur_nimg = nimg;
}

// rows of the backward-data weights: the input channels rounded up to whole 16-channel tiles
int wb_rows(const NetLayer& L) { return round_up(L.cin_pad, 16); }

void pack(helm_net* n, int i) {
  NetLayer& L = n->L[i];
  launch_pack(n->s, n->ntaps, L.cout_pad, L.cin_pad, L.kpad, L.cob, L.kbpad, wb_rows(L), L.w, L.wt, L.wb);
}

// plain input: in[p][0, ct)
NetSrc src_of(const bf16* in, int ct) { return NetSrc{in, ct, 0, nullptr, 0, 0, 0, 0, 0, 1}; }
// 2 x 2 (x 2) average of a layer at level lvl - 1
NetSrc src_pool(helm_net* n, const bf16* in, int ct, int lvl) {
  return NetSrc{in, ct, 0, nullptr, 0, 0, 1, n->cur->H[lvl - 1], n->cur->W[lvl - 1], n->cur->D[lvl - 1]};
}
// [upsampled `up` (cup channels), skip (ct channels)]
NetSrc src_cat(const bf16* up, int cup, const bf16* skip, int ct) {
  return NetSrc{skip, ct, 0, up, cup, cup, 0, 0, 0, 1};
}

void conv(helm_net* n, int i, const NetSrc& src, int lvl, bf16* out, float* out32, int out_ct, int out_off) {
  const NetLayer& L = n->L[i];
  ConvArgs a{};
  a.src = src;
  a.cin = L.cin_pad;
  a.nimg = n->cur->cur_nimg;
  a.D = n->cur->D[lvl];
  a.H = n->cur->H[lvl];
  a.W = n->cur->W[lvl];
  a.wt = L.wt;
  a.kpad = L.kpad;
  a.bias = L.b;
  a.cout = L.cout;
  a.relu = L.relu;
  a.out = out;
  a.out32 = out32;
  a.out_ct = out_ct;
  a.out_off = out_off;
  launch_conv3x3(n->s, a, L.cout_pad / 16, n->dim, n->generic_conv);
}

// backward-data: g_in (fp32, cin channels at g_ct/g_off) = conv of the masked gradient n->cur->gm with flipped weights
void conv_back(helm_net* n, int i, int lvl, float* gin, int g_ct) {
  const NetLayer& L = n->L[i];
  ConvArgs a{};
  a.src = src_of(n->cur->gm, L.cob);
  a.cin = L.cob;
  a.nimg = n->cur->cur_nimg;
  a.D = n->cur->D[lvl];
  a.H = n->cur->H[lvl];
  a.W = n->cur->W[lvl];
  a.wt = L.wb;
  a.kpad = L.kbpad;
  a.bias = nullptr;
  a.cout = L.cin_pad;
  a.relu = 0;
  a.out = nullptr;
  a.out32 = gin;
  a.out_ct = g_ct;
  a.out_off = 0;
  launch_conv3x3(n->s, a, wb_rows(L) / 16, n->dim, n->generic_conv);
}

void wgrad(helm_net* n, int i, const NetSrc& src, int lvl) {
  NetLayer& L = n->L[i];
  WgradArgs a{};
  a.src = src;
  a.cin = L.cin_pad;
  a.nimg = n->cur->cur_nimg;
  a.D = n->cur->D[lvl];
  a.H = n->cur->H[lvl];
  a.W = n->cur->W[lvl];
  a.dim = n->dim;
  a.g = n->cur->gm;
  a.g_ct = L.cout_pad;
  a.kpad = L.kpad;
  a.cout_pad = L.cout_pad;
  a.chunk = WCHUNK;
  a.part = n->cur->part;
  const int nchunk = (int)((n->cur->P[lvl] + WCHUNK - 1) / WCHUNK);
  launch_wgrad(n->s, a, nchunk, L.dw, n->cur->gm, L.db, L.cout);
}

void forward(helm_net* n) {
  NetBufs& b = *n->cur;
  const int* c = n->ch;
  conv(n, A0, src_of(b.x0, 8), 0, b.e0, nullptr, c[0], 0);
  conv(n, A1, src_pool(n, b.e0, c[0], 1), 1, b.e1, nullptr, c[1], 0);
  conv(n, A2, src_pool(n, b.e1, c[1], 2), 2, b.e2, nullptr, c[2], 0);
  conv(n, A3, src_pool(n, b.e2, c[2], 3), 3, b.e3, nullptr, c[3], 0);
  conv(n, B2, src_cat(b.e3, c[3], b.e2, c[2]), 2, b.d2, nullptr, c[2], 0);
  conv(n, B1, src_cat(b.d2, c[2], b.e1, c[1]), 1, b.d1, nullptr, c[1], 0);
  conv(n, B0, src_cat(b.d1, c[1], b.e0, c[0]), 0, b.d0, nullptr, c[0], 0);
  conv(n, OUT, src_of(b.d0, c[0]), 0, nullptr, b.y, 2, 0);
}

// Concatenation gradients g_cat{l} hold [upsampled part, skip part]; the skip part
// also collects the pooled-path gradient of the encoder.
void backward(helm_net* n) {
  NetBufs& b = *n->cur;
  const int N = b.cur_nimg, dim = n->dim;
  const long long* P = b.P;
  const int* c = n->ch;
  hipStream_t s = n->s;
  // output layer (no ReLU): gy is the loss gradient of y
  launch_grad_prep(s, P[0], b.gy, 2, 0, nullptr, 0, 0, 2, n->L[OUT].cout_pad, b.gm);
  wgrad(n, OUT, src_of(b.d0, c[0]), 0);
  conv_back(n, OUT, 0, b.g_d0, c[0]);
  // decoder
  launch_grad_prep(s, P[0], b.g_d0, c[0], 0, b.d0, c[0], 0, c[0], c[0], b.gm);
  wgrad(n, B0, src_cat(b.d1, c[1], b.e0, c[0]), 0);
  conv_back(n, B0, 0, b.g_cat0, c[1] + c[0]);
  launch_upsample_back(s, dim, N, b.D[0], b.H[0], b.W[0], c[1], b.g_cat0, c[1] + c[0], 0, b.g_d1);
  launch_grad_prep(s, P[1], b.g_d1, c[1], 0, b.d1, c[1], 0, c[1], c[1], b.gm);
  wgrad(n, B1, src_cat(b.d2, c[2], b.e1, c[1]), 1);
  conv_back(n, B1, 1, b.g_cat1, c[2] + c[1]);
  launch_upsample_back(s, dim, N, b.D[1], b.H[1], b.W[1], c[2], b.g_cat1, c[2] + c[1], 0, b.g_d2);
  launch_grad_prep(s, P[2], b.g_d2, c[2], 0, b.d2, c[2], 0, c[2], c[2], b.gm);
  wgrad(n, B2, src_cat(b.e3, c[3], b.e2, c[2]), 2);
  conv_back(n, B2, 2, b.g_cat2, c[3] + c[2]);
  launch_upsample_back(s, dim, N, b.D[2], b.H[2], b.W[2], c[3], b.g_cat2, c[3] + c[2], 0, b.g_e3);
  // encoder
  launch_grad_prep(s, P[3], b.g_e3, c[3], 0, b.e3, c[3], 0, c[3], c[3], b.gm);
  wgrad(n, A3, src_pool(n, b.e2, c[2], 3), 3);
  conv_back(n, A3, 3, b.g_p, c[2]);
  launch_pool_back(s, dim, N, b.D[2], b.H[2], b.W[2], c[2], b.g_p, c[2], b.g_cat2, c[3] + c[2], c[3]);
  launch_grad_prep(s, P[2], b.g_cat2, c[3] + c[2], c[3], b.e2, c[2], 0, c[2], c[2], b.gm);
  wgrad(n, A2, src_pool(n, b.e1, c[1], 2), 2);
  conv_back(n, A2, 2, b.g_p, c[1]);
  launch_pool_back(s, dim, N, b.D[1], b.H[1], b.W[1], c[1], b.g_p, c[1], b.g_cat1, c[2] + c[1], c[2]);
  launch_grad_prep(s, P[1], b.g_cat1, c[2] + c[1], c[2], b.e1, c[1], 0, c[1], c[1], b.gm);
  wgrad(n, A1, src_pool(n, b.e0, c[0], 1), 1);
  conv_back(n, A1, 1, b.g_p, c[0]);
  launch_pool_back(s, dim, N, b.D[0], b.H[0], b.W[0], c[0], b.g_p, c[0], b.g_cat0, c[1] + c[0], c[1]);
  launch_grad_prep(s, P[0], b.g_cat0, c[1] + c[0], c[1], b.e0, c[0], 0, c[0], c[0], b.gm);
  wgrad(n, A0, src_of(b.x0, 8), 0);
}

int fail(helm_net* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  return code;
}

#define NET_TRY try {
#define NET_CATCH                                                                   \
  }                                                                                 \
  catch (const NetErr& e) {                                                         \
    return fail(n, e.code == hipErrorOutOfMemory ? HELM_ENOMEM : HELM_EHIP,         \
                std::string(e.what) + ": " + hipGetErrorString(e.code));            \
  }

}  // namespace

struct NetSolveBufs {
  NetBufs b;
};

NetSolveBufs* net_bufs_create(helm_net* n, int B, int ngrid) {
  NetSolveBufs* sb = new NetSolveBufs();
  n->cur = &sb->b;
  try {
    ensure(n, B, n->dim == 3 ? ngrid : 1, ngrid, ngrid, false);
  } catch (...) {
    free_bufs(n);
    n->cur = &n->tb;
    delete sb;
    throw;
  }
  n->cur = &n->tb;
  return sb;
}

void net_bufs_destroy(NetSolveBufs* sb) {
  if (!sb) return;
  for (void* p : sb->b.bufs) hipFree(p);
  delete sb;
}

hipError_t net_apply(helm_net* n, NetSolveBufs* sb, hipStream_t s, int B, int ngrid, const c32* v,
                     long long v_stride, const float* vscale, int vs_stride, float in_gain, const c32* coef, c32 cb,
                     float out_gain, c32* z, long long z_stride, const int* mask) {
  const int depth = n->dim == 3 ? ngrid : 1;
  if (!sb || B > sb->b.cap_nimg || depth != sb->b.cap_D || ngrid != sb->b.cap_H || ngrid != sb->b.cap_W)
    return hipErrorInvalidValue;
  hipStream_t keep = n->s;
  n->s = s;
  n->cur = &sb->b;
  set_current(n, B, depth, ngrid, ngrid);
  const long long N = (long long)depth * ngrid * ngrid;
  launch_net_input(s, B, N, v, v_stride, vscale, vs_stride, in_gain, coef, cb, n->cur->x0, 8);
  forward(n);
  launch_net_output(s, B, N, n->cur->y, out_gain, z, z_stride, mask);
  n->s = keep;
  n->cur = &n->tb;
  return hipSuccess;
}

namespace {

// shared body of the network entry points (2D: D = 1)
int create(unsigned long long seed, void* hip_stream, int dim, helm_net** out) {
  if (!out) return HELM_EINVAL;
  *out = nullptr;
  helm_net* n = new (std::nothrow) helm_net();
  if (!n) return HELM_ENOMEM;
  try {
    n->s = (hipStream_t)hip_stream;
    n->dim = dim;
    n->ntaps = dim == 3 ? 27 : 9;
    const LayerDef* defs = dim == 3 ? kLayers3 : kLayers;
    for (int l = 0; l < 4; ++l) n->ch[l] = defs[l].cout;  // A0..A3 outputs
    Rng rng{seed};
    for (int i = 0; i < HELM_NET_LAYERS; ++i) {
      NetLayer& L = n->L[i];
      L.cin = defs[i].cin;
      L.cout = defs[i].cout;
      L.relu = defs[i].relu;
      L.cin_pad = round_up(L.cin, 8);
      L.cout_pad = round_up(L.cout, 16);
      L.kpad = round_up(n->ntaps * L.cin_pad, 32);
      L.cob = L.cout_pad;
      L.kbpad = round_up(n->ntaps * L.cob, 32);
      const size_t nw = (size_t)L.cout_pad * L.kpad;
      L.w = n->alloc<float>(nw, n->allocs);
      L.dw = n->alloc<float>(nw, n->allocs);
      L.mw = n->alloc<float>(nw, n->allocs);
      L.vw = n->alloc<float>(nw, n->allocs);
      L.b = n->alloc<float>(L.cout, n->allocs);
      L.db = n->alloc<float>(L.cout, n->allocs);
      L.mb = n->alloc<float>(L.cout, n->allocs);
      L.vb = n->alloc<float>(L.cout, n->allocs);
      L.mask = n->alloc<unsigned char>(nw, n->allocs);
      L.wt = n->alloc<bf16>(nw, n->allocs);
      L.wb = n->alloc<bf16>((size_t)wb_rows(L) * L.kbpad, n->allocs);
      // He-normal initialisation, zero bias, zero Adam moments
      std::vector<float> w(nw, 0.f), zero(nw, 0.f);
      std::vector<unsigned char> m(nw, 0);
      const double std = std::sqrt(2.0 / ((double)n->ntaps * L.cin));
      for (int tap = 0; tap < n->ntaps; ++tap)
        for (int ci = 0; ci < L.cin; ++ci)
          for (int co = 0; co < L.cout; ++co) {
            const size_t idx = (size_t)co * L.kpad + tap * L.cin_pad + ci;
            w[idx] = (float)(std * rng.normal());
            m[idx] = 1;
          }
      ck(hipMemcpy(L.w, w.data(), nw * 4, hipMemcpyHostToDevice), "upload");
      ck(hipMemcpy(L.mw, zero.data(), nw * 4, hipMemcpyHostToDevice), "upload");
      ck(hipMemcpy(L.vw, zero.data(), nw * 4, hipMemcpyHostToDevice), "upload");
      ck(hipMemcpy(L.mask, m.data(), nw, hipMemcpyHostToDevice), "upload");
      ck(hipMemcpy(L.b, zero.data(), L.cout * 4, hipMemcpyHostToDevice), "upload");
      ck(hipMemcpy(L.mb, zero.data(), L.cout * 4, hipMemcpyHostToDevice), "upload");
      ck(hipMemcpy(L.vb, zero.data(), L.cout * 4, hipMemcpyHostToDevice), "upload");
      pack(n, i);
    }
    ck(hipStreamSynchronize(n->s), "sync");
  } catch (const NetErr& e) {
    for (void* p : n->allocs) hipFree(p);
    delete n;
    return e.code == hipErrorOutOfMemory ? HELM_ENOMEM : HELM_EHIP;
  }
  *out = n;
  return HELM_OK;
}

int forward_call(helm_net* n, int nimg, int D, int H, int W, const float* x, float* y) {
  NET_TRY
  ensure(n, nimg, D, H, W,
         n->cur->cap_train && n->cur->cap_nimg == nimg && n->cur->cap_D == D && n->cur->cap_H == H &&
             n->cur->cap_W == W);
  set_current(n, nimg, D, H, W);
  launch_to_bf16_pad(n->s, n->cur->P[0], 4, x, 8, n->cur->x0);
  forward(n);
  ck(hipMemcpyAsync(y, n->cur->y, n->cur->P[0] * 2 * sizeof(float), hipMemcpyDeviceToDevice, n->s), "copy");
  ck(hipGetLastError(), "launch");
  ck(hipStreamSynchronize(n->s), "sync");
  NET_CATCH
  return HELM_OK;
}

int backward_call(helm_net* n, int nimg, int D, int H, int W, const float* x, const float* target, double* loss) {
  NET_TRY
  ensure(n, nimg, D, H, W, true);
  set_current(n, nimg, D, H, W);
  launch_to_bf16_pad(n->s, n->cur->P[0], 4, x, 8, n->cur->x0);
  forward(n);
  const long long ny = n->cur->P[0] * 2;
  launch_loss(n->s, ny, n->cur->y, target, (float)(n->err_w / nimg), n->cur->gy, n->cur->lpart);
  const bool res = n->res_w > 0.0;
  if (res)
    launch_res_loss(n->s, n->dim, nimg, D, H, W, x, n->cur->y, (float)n->gamma, make_float2((float)n->cb, 0.f),
                    (float)(n->res_w / nimg), n->cur->q, n->cur->rpart, n->cur->gy);
  backward(n);
  ck(hipGetLastError(), "launch");
  if (loss) {
    std::vector<float> part(loss_partials(ny)), rpart(res ? loss_partials(n->cur->P[0]) : 0);
    ck(hipMemcpyAsync(part.data(), n->cur->lpart, part.size() * 4, hipMemcpyDeviceToHost, n->s), "loss");
    if (res)
      ck(hipMemcpyAsync(rpart.data(), n->cur->rpart, rpart.size() * 4, hipMemcpyDeviceToHost, n->s), "loss");
    ck(hipStreamSynchronize(n->s), "sync");
    double sum = 0.0;
    for (float v : part) sum += v;
    for (float v : rpart) sum += v;
    *loss = sum;
  }
  ck(hipStreamSynchronize(n->s), "sync");
  NET_CATCH
  return HELM_OK;
}

int ratio_call(helm_net* n, int nimg, int D, int H, int W, const float* x, double gamma, double cb,
               double* ratio_host) {
  NET_TRY
  ensure(n, nimg, D, H, W,
         n->cur->cap_train && n->cur->cap_nimg >= nimg && n->cur->cap_D == D && n->cur->cap_H == H &&
             n->cur->cap_W == W);
  set_current(n, nimg, D, H, W);
  launch_to_bf16_pad(n->s, n->cur->P[0], 4, x, 8, n->cur->x0);
  forward(n);
  std::vector<double> sums(2 * (size_t)nimg);
  double* d_sums = nullptr;
  ck(hipMalloc((void**)&d_sums, sums.size() * sizeof(double)), "hipMalloc");
  launch_res_ratio(n->s, n->dim, nimg, D, H, W, x, n->cur->y, (float)gamma, make_float2((float)cb, 0.f), d_sums);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(sums.data(), d_sums, sums.size() * sizeof(double), hipMemcpyDeviceToHost, n->s);
  if (e == hipSuccess) e = hipStreamSynchronize(n->s);
  hipFree(d_sums);
  ck(e, "residual ratio");
  for (int i = 0; i < nimg; ++i) ratio_host[i] = sums[2 * i + 1] > 0.0 ? std::sqrt(sums[2 * i] / sums[2 * i + 1]) : 0.0;
  NET_CATCH
  return HELM_OK;
}

}  // namespace

int net_dim(const helm_net* n) { return n ? n->dim : 0; }

extern "C" {

int helm_net_layers(void) { return HELM_NET_LAYERS; }

int helm_net_layer_shape(int i, int* cin, int* cout) {
  if (i < 0 || i >= HELM_NET_LAYERS) return HELM_EINVAL;
  if (cin) *cin = kLayers[i].cin;
  if (cout) *cout = kLayers[i].cout;
  return HELM_OK;
}

int helm_net_dim(const helm_net* n) { return n ? n->dim : HELM_EINVAL; }

int helm_net_set_conv_kernels(helm_net* n, int generic) {
  if (!n || (generic != 0 && generic != 1)) return HELM_EINVAL;
  n->generic_conv = generic == 1;
  return HELM_OK;
}

int helm_net_shape(const helm_net* n, int i, int* cin, int* cout) {
  if (!n || i < 0 || i >= HELM_NET_LAYERS) return HELM_EINVAL;
  if (cin) *cin = n->L[i].cin;
  if (cout) *cout = n->L[i].cout;
  return HELM_OK;
}

int helm_net_create(unsigned long long seed, void* hip_stream, helm_net** out) {
  return create(seed, hip_stream, 2, out);
}

int helm_net_create3(unsigned long long seed, void* hip_stream, helm_net** out) {
  return create(seed, hip_stream, 3, out);
}

void helm_net_destroy(helm_net* n) {
  if (!n) return;
  hipStreamSynchronize(n->s);
  n->cur = &n->tb;
  free_bufs(n);
  for (void* p : n->allocs) hipFree(p);
  delete n;
}

const char* helm_net_last_error(const helm_net* n) { return n ? n->err.c_str() : ""; }

int helm_net_set_layer(helm_net* n, int i, const float* w_host, const float* b_host) {
  if (!n || i < 0 || i >= HELM_NET_LAYERS || !w_host || !b_host) return fail(n, HELM_EINVAL, "bad argument");
  NET_TRY
  NetLayer& L = n->L[i];
  std::vector<float> w((size_t)L.cout_pad * L.kpad, 0.f);
  for (int tap = 0; tap < n->ntaps; ++tap)
    for (int ci = 0; ci < L.cin; ++ci)
      for (int co = 0; co < L.cout; ++co)
        w[(size_t)co * L.kpad + tap * L.cin_pad + ci] = w_host[((size_t)tap * L.cin + ci) * L.cout + co];
  ck(hipMemcpy(L.w, w.data(), w.size() * 4, hipMemcpyHostToDevice), "upload");
  ck(hipMemcpy(L.b, b_host, L.cout * 4, hipMemcpyHostToDevice), "upload");
  pack(n, i);
  ck(hipStreamSynchronize(n->s), "sync");
  NET_CATCH
  return HELM_OK;
}

static int get_tensor(helm_net* n, int i, const float* wdev, const float* bdev, float* w_host, float* b_host) {
  NetLayer& L = n->L[i];
  std::vector<float> w((size_t)L.cout_pad * L.kpad);
  ck(hipStreamSynchronize(n->s), "sync");
  ck(hipMemcpy(w.data(), wdev, w.size() * 4, hipMemcpyDeviceToHost), "download");
  if (w_host)
    for (int tap = 0; tap < n->ntaps; ++tap)
      for (int ci = 0; ci < L.cin; ++ci)
        for (int co = 0; co < L.cout; ++co)
          w_host[((size_t)tap * L.cin + ci) * L.cout + co] = w[(size_t)co * L.kpad + tap * L.cin_pad + ci];
  if (b_host) ck(hipMemcpy(b_host, bdev, L.cout * 4, hipMemcpyDeviceToHost), "download");
  return HELM_OK;
}

int helm_net_get_layer(helm_net* n, int i, float* w_host, float* b_host) {
  if (!n || i < 0 || i >= HELM_NET_LAYERS) return fail(n, HELM_EINVAL, "bad argument");
  NET_TRY
  return get_tensor(n, i, n->L[i].w, n->L[i].b, w_host, b_host);
  NET_CATCH
}

int helm_net_get_grad(helm_net* n, int i, float* dw_host, float* db_host) {
  if (!n || i < 0 || i >= HELM_NET_LAYERS) return fail(n, HELM_EINVAL, "bad argument");
  NET_TRY
  return get_tensor(n, i, n->L[i].dw, n->L[i].db, dw_host, db_host);
  NET_CATCH
}

int helm_net_forward(helm_net* n, int nimg, int H, int W, const float* x, float* y) {
  if (!n || !x || !y || nimg < 1 || H < 1 || W < 1) return fail(n, HELM_EINVAL, "bad argument");
  if (n->dim != 2) return fail(n, HELM_EINVAL, "a 3D network takes helm_net_forward3");
  return forward_call(n, nimg, 1, H, W, x, y);
}

int helm_net_forward3(helm_net* n, int nimg, int D, int H, int W, const float* x, float* y) {
  if (!n || !x || !y || nimg < 1 || D < 1 || H < 1 || W < 1) return fail(n, HELM_EINVAL, "bad argument");
  if (n->dim != 3) return fail(n, HELM_EINVAL, "a 2D network takes helm_net_forward");
  return forward_call(n, nimg, D, H, W, x, y);
}

int helm_net_backward(helm_net* n, int nimg, int H, int W, const float* x, const float* target, double* loss) {
  if (!n || !x || !target || nimg < 1 || H < 1 || W < 1) return fail(n, HELM_EINVAL, "bad argument");
  if (n->dim != 2) return fail(n, HELM_EINVAL, "a 3D network takes helm_net_backward3");
  return backward_call(n, nimg, 1, H, W, x, target, loss);
}

int helm_net_backward3(helm_net* n, int nimg, int D, int H, int W, const float* x, const float* target,
                       double* loss) {
  if (!n || !x || !target || nimg < 1 || D < 1 || H < 1 || W < 1) return fail(n, HELM_EINVAL, "bad argument");
  if (n->dim != 3) return fail(n, HELM_EINVAL, "a 2D network takes helm_net_backward");
  return backward_call(n, nimg, D, H, W, x, target, loss);
}

int helm_net_residual_ratio(helm_net* n, int nimg, int H, int W, const float* x, double gamma, double cb,
                            double* ratio_host) {
  if (!n || !x || !ratio_host || nimg < 1 || H < 3 || W < 3 || !(gamma > 0.0) || !(cb > 0.0))
    return fail(n, HELM_EINVAL, "bad argument");
  if (n->dim != 2) return fail(n, HELM_EINVAL, "a 3D network takes helm_net_residual_ratio3");
  return ratio_call(n, nimg, 1, H, W, x, gamma, cb, ratio_host);
}

int helm_net_residual_ratio3(helm_net* n, int nimg, int D, int H, int W, const float* x, double gamma, double cb,
                             double* ratio_host) {
  if (!n || !x || !ratio_host || nimg < 1 || D < 3 || H < 3 || W < 3 || !(gamma > 0.0) || !(cb > 0.0))
    return fail(n, HELM_EINVAL, "bad argument");
  if (n->dim != 3) return fail(n, HELM_EINVAL, "a 2D network takes helm_net_residual_ratio");
  return ratio_call(n, nimg, D, H, W, x, gamma, cb, ratio_host);
}

int helm_net_set_loss(helm_net* n, double err_weight, double res_weight, double gamma, double cb) {
  if (!n || !(err_weight >= 0.0) || !(res_weight >= 0.0) || !(gamma > 0.0) || !(cb > 0.0))
    return fail(n, HELM_EINVAL, "bad argument");
  n->err_w = err_weight;
  n->res_w = res_weight;
  n->gamma = gamma;
  n->cb = cb;
  return HELM_OK;
}

int helm_net_adam_step(helm_net* n, double lr) {
  if (!n || !(lr > 0)) return fail(n, HELM_EINVAL, "bad argument");
  NET_TRY
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, n->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, n->step)));
  for (int i = 0; i < HELM_NET_LAYERS; ++i) {
    NetLayer& L = n->L[i];
    launch_adam(n->s, L.cout_pad * L.kpad, L.w, L.dw, L.mw, L.vw, L.mask, (float)lr, b1, b2, eps, c1, c2);
    launch_adam(n->s, L.cout, L.b, L.db, L.mb, L.vb, nullptr, (float)lr, b1, b2, eps, c1, c2);
    pack(n, i);
  }
  ck(hipGetLastError(), "launch");
  ck(hipStreamSynchronize(n->s), "sync");
  NET_CATCH
  return HELM_OK;
}

}  // extern "C"
