// Model kernels: plane-wave right-hand sides (Sec. II-A), the refractive-index
// gradient of Prop. 1 (Sec. V), and small elementwise helpers.
#include "dev_common.h"
#include "kernels.h"

namespace {

// rhs_q(p) = f(p) * prod_axis T_q,axis(coord_axis(p)): the plane wave
// exp(j k_b <d_q, x - x_c>) factorises over axes; the per-axis factors are
// tabulated on the host in FP64 and rounded once to complex64.
__global__ void k_plane_wave(int dim, int n, long long N, const float* fplane, const c32* tables, c32* rhs,
                             c32* uin) {
  const int b = blockIdx.y;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const Coord c = coord_of32((unsigned)p, (unsigned)n, dim);
  const c32* t = tables + (long long)b * dim * n;
  c32 u = cmul(t[c.x], t[n + c.y]);
  if (dim == 3) u = cmul(u, t[2 * n + c.z]);
  rhs[(long long)b * N + p] = cscale(u, fplane[p]);
  if (uin) uin[(long long)b * N + p] = u;
}

// grad[i] = scale * n_i * sum_q Re(conj(u_q) lam_q) at interior point i
__global__ void k_grad_n(int dim, int B, int ne, int w, int n, const c32* u, const c32* lam, const float* nmap,
                         float scale, float* grad) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Ni) return;
  const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
  const long long Ne = dim == 2 ? (long long)ne * ne : (long long)ne * ne * ne;
  const long long p = dim == 2 ? (long long)(c.y + w) * ne + (c.x + w)
                               : ((long long)(c.z + w) * ne + (c.y + w)) * ne + (c.x + w);
  float s = 0.f;
  for (int b = 0; b < B; ++b) {
    const c32 a = u[(long long)b * Ne + p], l = lam[(long long)b * Ne + p];
    s = fmaf(a.x, l.x, fmaf(a.y, l.y, s));
  }
  grad[i] = scale * nmap[i] * s;
}

__global__ void k_conj_copy(long long count, const c32* in, c32* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    const c32 v = in[i];
    out[i] = make_float2(v.x, -v.y);
  }
}

__global__ void k_zero(long long count, c32* p) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = make_float2(0.f, 0.f);
}

inline unsigned nb(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_plane_wave(hipStream_t s, int dim, int B, int n, const float* fplane, const c32* tables, c32* rhs,
                       c32* uin) {
  const long long N = dim == 2 ? (long long)n * n : (long long)n * n * n;
  hipLaunchKernelGGL(k_plane_wave, dim3(nb(N, 256), B), dim3(256), 0, s, dim, n, N, fplane, tables, rhs, uin);
}
void launch_grad_n(hipStream_t s, int dim, int B, int n_e, int w, int n, const c32* u, const c32* lam,
                   const float* nmap, float scale, float* grad) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  hipLaunchKernelGGL(k_grad_n, dim3(nb(Ni, 256)), dim3(256), 0, s, dim, B, n_e, w, n, u, lam, nmap, scale, grad);
}
void launch_conj_copy(hipStream_t s, long long count, const c32* in, c32* out) {
  hipLaunchKernelGGL(k_conj_copy, dim3(nb(count, 256)), dim3(256), 0, s, count, in, out);
}
void launch_zero(hipStream_t s, long long count, c32* p) {
  hipLaunchKernelGGL(k_zero, dim3(nb(count, 256)), dim3(256), 0, s, count, p);
}
