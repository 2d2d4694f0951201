// Inverse-problem steps of Sec. V on the interior grid Omega (n^dim points,
// x fastest): the TV proximal operator with a lower bound (eq. proximalOpt),
// computed by fast gradient projection on its dual, the update of the
// accelerated forward-backward splitting (Alg. 4), the data residual of the
// quadratic fidelity term, and the medium from the scattering potential.
//
// TV(w) = sum_i ||(D w)_i||, (D w)_{a,i} = w_{i+e_a} - w_i (0 across the last
// index of axis a).  Dual field p: dim components per point, ||p_i|| <= 1.
// One FGP step (t the Nesterov sequence, beta = (t - 1) / t'):
//   w = max(v - lam D^T r, lo)                              k_fgp_primal
//   q = P_B(r + D w / (4 dim lam));  r = q + beta (q - p);  p = q   k_fgp_dual
// and the answer is max(v - lam D^T p, lo).
#include <cmath>

#include "dev_common.h"
#include "kernels.h"

namespace {

__device__ __forceinline__ long long axis_stride(int a, int n) {
  return a == 0 ? 1LL : (a == 1 ? (long long)n : (long long)n * n);
}
__device__ __forceinline__ int coord_a(const Coord& c, int a) { return a == 0 ? c.x : (a == 1 ? c.y : c.z); }

// w = max(v - lam D^T r, lo); (D^T r)_i = sum_a (r_{a, i - e_a} [i_a > 0] - r_{a,i} [i_a < n - 1])
__global__ void k_fgp_primal(int dim, int n, long long Ni, const float* v, const float* r, float lam, float lo,
                             float* w) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < Ni; i += (long long)gridDim.x * blockDim.x) {
    const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
    float dt = 0.f;
    for (int a = 0; a < dim; ++a) {
      const float* ra = r + (long long)a * Ni;
      const int ca = coord_a(c, a);
      if (ca > 0) dt += ra[i - axis_stride(a, n)];
      if (ca < n - 1) dt -= ra[i];
    }
    w[i] = fmaxf(v[i] - lam * dt, lo);
  }
}

__global__ void k_fgp_dual(int dim, int n, long long Ni, const float* w, float step, float beta, float* p, float* r) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < Ni; i += (long long)gridDim.x * blockDim.x) {
    const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
    float q[3] = {0.f, 0.f, 0.f};
    float nn = 0.f;
    for (int a = 0; a < dim; ++a) {
      const float g = coord_a(c, a) < n - 1 ? w[i + axis_stride(a, n)] - w[i] : 0.f;
      q[a] = fmaf(step, g, r[(long long)a * Ni + i]);
      nn = fmaf(q[a], q[a], nn);
    }
    const float sc = 1.0f / fmaxf(1.0f, sqrtf(nn));
    for (int a = 0; a < dim; ++a) {
      const float qa = q[a] * sc;
      const long long k = (long long)a * Ni + i;
      r[k] = fmaf(beta, qa - p[k], qa);
      p[k] = qa;
    }
  }
}

__global__ void k_fill(long long count, float val, float* x) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    x[i] = val;
}

// out = a - s * b
__global__ void k_axmy(long long count, const float* a, float s, const float* b, float* out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    out[i] = fmaf(-s, b[i], a[i]);
}

// fbar = f_new + beta (f_new - f);  f = f_new
__global__ void k_fbs_momentum(long long count, const float* f_new, float beta, float* f, float* fbar) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x) {
    const float fn = f_new[i];
    fbar[i] = fmaf(beta, fn - f[i], fn);
    f[i] = fn;
  }
}

// res[q][i] = u[q][idx[i]] - y[q][i];  per-block partial sums of |res|^2 (FP64)
__global__ void k_data_residual(int B, int M, long long N, const int* idx, const c32* u, const c32* y, c32* res,
                                double* part) {
  __shared__ double red[256 / HELM_WAVE];
  double s = 0.0;
  const long long T = (long long)B * M;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(t / M), i = (int)(t - (long long)q * M);
    const c32 d = csub(u[(long long)q * N + idx[i]], y[t]);
    res[t] = d;
    s += (double)d.x * d.x + (double)d.y * d.y;
  }
  s = wave_sum_d(s);
  if (threadIdx.x % HELM_WAVE == 0) red[threadIdx.x / HELM_WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < 256 / HELM_WAVE; ++q) t += red[q];
    part[blockIdx.x] = t;
  }
}

// n = sqrt(n_b^2 + f / k0^2) (f >= -k0^2 n_b^2 is clamped to n = 0)
__global__ void k_index_from_f(long long count, const float* f, double inv_k02, double nb2, float* nmap) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    nmap[i] = (float)sqrt(fmax(0.0, nb2 + (double)f[i] * inv_k02));
}

inline unsigned grid_of(long long n) {
  const long long g = (n + 255) / 256;
  return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

void launch_tv_prox(hipStream_t s, int dim, int n, const float* v, float lam, float lo, int iters, float* p, float* r,
                    float* w) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  const unsigned g = grid_of(Ni);
  if (!(lam > 0.0f) || iters <= 0) {
    hipLaunchKernelGGL(k_fill, dim3(g), dim3(256), 0, s, (long long)dim * Ni, 0.0f, p);
    hipLaunchKernelGGL(k_fgp_primal, dim3(g), dim3(256), 0, s, dim, n, Ni, v, p, 0.0f, lo, w);
    return;
  }
  hipLaunchKernelGGL(k_fill, dim3(grid_of(dim * Ni)), dim3(256), 0, s, (long long)dim * Ni, 0.0f, p);
  hipLaunchKernelGGL(k_fill, dim3(grid_of(dim * Ni)), dim3(256), 0, s, (long long)dim * Ni, 0.0f, r);
  const float step = 1.0f / (4.0f * dim * lam);
  double t = 1.0;
  for (int k = 0; k < iters; ++k) {
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    const float beta = (float)((t - 1.0) / tn);
    hipLaunchKernelGGL(k_fgp_primal, dim3(g), dim3(256), 0, s, dim, n, Ni, v, r, lam, lo, w);
    hipLaunchKernelGGL(k_fgp_dual, dim3(g), dim3(256), 0, s, dim, n, Ni, w, step, beta, p, r);
    t = tn;
  }
  hipLaunchKernelGGL(k_fgp_primal, dim3(g), dim3(256), 0, s, dim, n, Ni, v, p, lam, lo, w);
}

void launch_axmy(hipStream_t s, long long count, const float* a, float sc, const float* b, float* out) {
  hipLaunchKernelGGL(k_axmy, dim3(grid_of(count)), dim3(256), 0, s, count, a, sc, b, out);
}

void launch_fbs_momentum(hipStream_t s, long long count, const float* f_new, float beta, float* f, float* fbar) {
  hipLaunchKernelGGL(k_fbs_momentum, dim3(grid_of(count)), dim3(256), 0, s, count, f_new, beta, f, fbar);
}

namespace {
// per-block partial sums of x[i]^2 (FP64), grid-stride
__global__ void k_sumsq(long long n, const float* x, double* part) {
  __shared__ double red[256 / HELM_WAVE];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    s += (double)x[i] * x[i];
  s = wave_sum_d(s);
  if (threadIdx.x % HELM_WAVE == 0) red[threadIdx.x / HELM_WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < 256 / HELM_WAVE; ++q) t += red[q];
    part[blockIdx.x] = t;
  }
}

__global__ void k_scale(long long n, float* x, float a) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] *= a;
}
}  // namespace

int sumsq_blocks(long long n) { return (int)grid_of(n); }
void launch_sumsq(hipStream_t s, long long n, const float* x, double* part) {
  hipLaunchKernelGGL(k_sumsq, dim3(sumsq_blocks(n)), dim3(256), 0, s, n, x, part);
}
void launch_scale(hipStream_t s, long long n, float* x, float a) {
  hipLaunchKernelGGL(k_scale, dim3(grid_of(n)), dim3(256), 0, s, n, x, a);
}

int data_residual_blocks(int B, int M) { return (int)grid_of((long long)B * M); }

void launch_data_residual(hipStream_t s, int B, int M, long long N, const int* idx, const c32* u, const c32* y,
                          c32* res, double* part) {
  hipLaunchKernelGGL(k_data_residual, dim3(data_residual_blocks(B, M)), dim3(256), 0, s, B, M, N, idx, u, y, res,
                     part);
}

void launch_index_from_f(hipStream_t s, long long count, const float* f, double inv_k02, double nb2, float* nmap) {
  hipLaunchKernelGGL(k_index_from_f, dim3(grid_of(count)), dim3(256), 0, s, count, f, inv_k02, nb2, nmap);
}
