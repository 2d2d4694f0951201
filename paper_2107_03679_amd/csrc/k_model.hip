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

// grad[i] = scale * n_i * sum_q Re(conj(u_in,q + u_sc,q) (lam_q + lam2_q)) at interior point i
// (n_i = 1 without nmap, lam2 = 0 when NULL)
__global__ void k_grad_n(int dim, int B, int ne, int w, int n, const c32* uin, const c32* u, const c32* lam,
                         const c32* lam2, const float* nmap, float scale, int accumulate, float* grad) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Ni) return;
  const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
  const long long Ne = dim == 2 ? (long long)ne * ne : (long long)ne * ne * ne;
  const long long p = dim == 2 ? (long long)(c.y + w) * ne + (c.x + w)
                               : ((long long)(c.z + w) * ne + (c.y + w)) * ne + (c.x + w);
  float s = 0.f;
  for (int b = 0; b < B; ++b) {
    c32 a = u[(long long)b * Ne + p];
    if (uin) a = cadd(a, uin[(long long)b * Ne + p]);
    c32 l = lam[(long long)b * Ne + p];
    if (lam2) l = cadd(l, lam2[(long long)b * Ne + p]);
    s = fmaf(a.x, l.x, fmaf(a.y, l.y, s));
  }
  const float g = scale * (nmap ? nmap[i] : 1.0f) * s;
  grad[i] = accumulate ? grad[i] + g : g;
}

__global__ void k_conj_copy(long long count, const c32* in, c32* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    const c32 v = in[i];
    out[i] = make_float2(v.x, -v.y);
  }
}

// the iterate of each right-hand side from the buffer of the pair its last update wrote
__global__ void k_x_select(long long N, const int* xpar, const c32* in0, const c32* in1, c32* out, int conj) {
  const int b = blockIdx.y;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const c32* in = xpar && xpar[b] ? in1 : in0;
  c32 v = in[(long long)b * N + i];
  if (conj) v.y = -v.y;
  out[(long long)b * N + i] = v;
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
void launch_grad_n(hipStream_t s, int dim, int B, int n_e, int w, int n, const c32* uin, const c32* u,
                   const c32* lam, const float* nmap, float scale, float* grad, const c32* lam2, int accumulate) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  hipLaunchKernelGGL(k_grad_n, dim3(nb(Ni, 256)), dim3(256), 0, s, dim, B, n_e, w, n, uin, u, lam, lam2, nmap, scale,
                     accumulate, grad);
}
void launch_conj_copy(hipStream_t s, long long count, const c32* in, c32* out) {
  hipLaunchKernelGGL(k_conj_copy, dim3(nb(count, 256)), dim3(256), 0, s, count, in, out);
}
void launch_x_select(hipStream_t s, int B, long long N, const int* xpar, const c32* in0, const c32* in1, c32* out,
                     int conj) {
  hipLaunchKernelGGL(k_x_select, dim3(nb(N, 256), B), dim3(256), 0, s, N, xpar, in0, in1, out, conj);
}
void launch_zero(hipStream_t s, long long count, c32* p) {
  hipLaunchKernelGGL(k_zero, dim3(nb(count, 256)), dim3(256), 0, s, count, p);
}

// ---- receivers (the sampling operator S of the data term) and smoothed TV ----
namespace {

// y[q][i] = u[q][idx[i]]
__global__ void k_gather(int B, int M, long long N, const int* idx, const c32* u, c32* y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B * M) return;
  const int q = (int)(t / M), i = (int)(t % M);
  y[t] = u[(long long)q * N + idx[i]];
}

// u[q][idx[i]] = y[q][i] (u zero-filled beforehand; receiver indices are distinct)
__global__ void k_scatter(int B, int M, long long N, const int* idx, const c32* y, c32* u) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)B * M) return;
  const int q = (int)(t / M), i = (int)(t % M);
  u[(long long)q * N + idx[i]] = y[t];
}

// Smoothed isotropic TV on the interior map: per point the magnitude
// m = sqrt(sum_axis (forward difference)^2 + eps^2) (zero difference across the
// last row/column) and its gradient, assembled by a second kernel.
__global__ void k_tv_terms(int dim, int n, const float* nm, float eps, float* mag, float* part) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float v = 0.f;
  if (i < Ni) {
    const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
    const float x0 = nm[i];
    const float dx = c.x < n - 1 ? nm[i + 1] - x0 : 0.f;
    const float dy = c.y < n - 1 ? nm[i + n] - x0 : 0.f;
    const float dz = (dim == 3 && c.z < n - 1) ? nm[i + (long long)n * n] - x0 : 0.f;
    v = sqrtf(dx * dx + dy * dy + dz * dz + eps * eps);
    mag[i] = v;
  }
  v = wave_sum(v);
  __shared__ float red[4];
  if (threadIdx.x % HELM_WAVE == 0) red[threadIdx.x / HELM_WAVE] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_tv_grad(int dim, int n, const float* nm, const float* mag, float scale, float* grad) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Ni) return;
  const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
  const float x0 = nm[i];
  float g = 0.f;
  // own forward differences: d/dx0 of (x_next - x0) = -1
  if (c.x < n - 1) g -= (nm[i + 1] - x0) / mag[i];
  if (c.y < n - 1) g -= (nm[i + n] - x0) / mag[i];
  if (dim == 3 && c.z < n - 1) g -= (nm[i + (long long)n * n] - x0) / mag[i];
  // as the "next" point of the left / lower / previous-plane neighbour
  if (c.x > 0) g += (x0 - nm[i - 1]) / mag[i - 1];
  if (c.y > 0) g += (x0 - nm[i - n]) / mag[i - n];
  if (dim == 3 && c.z > 0) g += (x0 - nm[i - (long long)n * n]) / mag[i - (long long)n * n];
  grad[i] = scale * g;
}

}  // namespace

void launch_gather(hipStream_t s, int B, int M, long long N, const int* idx, const c32* u, c32* y) {
  const long long T = (long long)B * M;
  hipLaunchKernelGGL(k_gather, dim3(nb(T, 256)), dim3(256), 0, s, B, M, N, idx, u, y);
}
void launch_scatter(hipStream_t s, int B, int M, long long N, const int* idx, const c32* y, c32* u) {
  const long long T = (long long)B * M;
  hipLaunchKernelGGL(k_scatter, dim3(nb(T, 256)), dim3(256), 0, s, B, M, N, idx, y, u);
}
int tv_partials(int dim, int n) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  return (int)nb(Ni, 256);
}
void launch_tv(hipStream_t s, int dim, int n, const float* nm, float eps, float scale, float* mag, float* part,
               float* grad) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  hipLaunchKernelGGL(k_tv_terms, dim3(nb(Ni, 256)), dim3(256), 0, s, dim, n, nm, eps, mag, part);
  hipLaunchKernelGGL(k_tv_grad, dim3(nb(Ni, 256)), dim3(256), 0, s, dim, n, nm, mag, scale, grad);
}
