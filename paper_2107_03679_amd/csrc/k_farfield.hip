// Sensor operator G~ of eq. DiscreteForward / DiscreteForwardHelm: the field
// scattered by the induced source s = f u (u the total field) on Omega,
// observed at M sensors outside Omega, by the Lippmann-Schwinger integral
// (eq. LSIntegral) with the free-space Green's function (eq. green) and the
// rectangle rule on the grid:
//     y_m = sum_{z in Omega} g(x_m - z) s(z) h^d,
//     g(x) = (j/4) H0^(1)(k_b |x|)  (2D),   e^{j k_b |x|} / (4 pi |x|)  (3D).
// G~ [M][n^dim] is formed once per sensor set (2D: H0^(1) by cubic Hermite
// interpolation in a host FP64 table of H0^(1) and its derivative; 3D: in
// closed form in FP64), then applied as a split-K product and its adjoint.
#include "dev_common.h"
#include "kernels.h"

namespace {

constexpr int TT = 32;  // tile edge of the products (32 x 32 outputs, 256 threads, 4 outputs each)

__global__ void k_ff_matrix(int dim, int n, int M, const double* sens, double kbh, double h, const double2* tab,
                            double x0, double dx, int ntab, c32* G) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (i >= Ni || m >= M) return;
  const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
  const double ctr = 0.5 * (n - 1);
  const double ddx = sens[m * dim + 0] - (c.x - ctr), ddy = sens[m * dim + 1] - (c.y - ctr);
  const double ddz = dim == 3 ? sens[m * dim + 2] - (c.z - ctr) : 0.0;
  const double r = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);  // in cells
  double gr, gi;
  if (dim == 2) {
    // H0(x) on the table: value/derivative pairs (tab[2k], tab[2k+1]) at x0 + k dx
    const double x = kbh * r;
    double t = (x - x0) / dx;
    int k = (int)floor(t);
    k = k < 0 ? 0 : (k > ntab - 2 ? ntab - 2 : k);
    t -= k;
    const double h00 = (1 + 2 * t) * (1 - t) * (1 - t), h10 = t * (1 - t) * (1 - t);
    const double h01 = t * t * (3 - 2 * t), h11 = t * t * (t - 1);
    const double2 v0 = tab[2 * k], d0 = tab[2 * k + 1], v1 = tab[2 * k + 2], d1 = tab[2 * k + 3];
    const double hr = h00 * v0.x + h10 * dx * d0.x + h01 * v1.x + h11 * dx * d1.x;
    const double hi = h00 * v0.y + h10 * dx * d0.y + h01 * v1.y + h11 * dx * d1.y;
    // (j/4) H0 = (-Im H0 + j Re H0) / 4, times the cell area h^2
    gr = -0.25 * hi * h * h;
    gi = 0.25 * hr * h * h;
  } else {
    const double rr = r * h, kb = kbh / h;
    double sn, cs;
    sincos(kb * rr, &sn, &cs);
    const double a = h * h * h / (4.0 * 3.14159265358979323846 * rr);
    gr = a * cs;
    gi = a * sn;
  }
  G[(long long)m * Ni + i] = make_float2((float)gr, (float)gi);
}

// s[b][i] = f_i (u_in + u_sc)[b][p(i)] on Omega (compact [B][n^dim])
__global__ void k_ff_source(int dim, int B, int ne, int w, int n, const float* fpl, const c32* uin, const c32* usc,
                            c32* s) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  const long long Ne = dim == 2 ? (long long)ne * ne : (long long)ne * ne * ne;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= Ni) return;
  const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
  const long long p = dim == 2 ? (long long)(c.y + w) * ne + (c.x + w)
                               : ((long long)(c.z + w) * ne + (c.y + w)) * ne + (c.x + w);
  c32 u = usc[(long long)b * Ne + p];
  if (uin) u = cadd(u, uin[(long long)b * Ne + p]);
  s[(long long)b * Ni + i] = cscale(u, fpl[p]);
}

// part[k][b][m] = sum over pixel chunk k of G[m][i] s[b][i]; block: 32 sensors x 32 RHS, chunk k
__global__ __launch_bounds__(256) void k_ff_apply(int B, int M, long long Ni, long long chunk, const c32* G,
                                                   const c32* s, c32* part) {
  __shared__ c32 sg[TT][TT + 1];
  __shared__ c32 ss[TT][TT + 1];
  const int m0 = blockIdx.x * TT, b0 = blockIdx.y * TT, k = blockIdx.z;
  const long long i0 = (long long)k * chunk, i1 = i0 + chunk < Ni ? i0 + chunk : Ni;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;  // ty in 0..7: rows ty, ty+8, ty+16, ty+24
  c32 acc[4];
  for (int q = 0; q < 4; ++q) acc[q] = make_float2(0.f, 0.f);
  for (long long ib = i0; ib < i1; ib += TT) {
    for (int q = 0; q < 4; ++q) {
      const int row = ty + 8 * q;
      const long long i = ib + tx;
      const bool ok = i < i1;
      sg[row][tx] = (ok && m0 + row < M) ? G[(long long)(m0 + row) * Ni + i] : make_float2(0.f, 0.f);
      ss[row][tx] = (ok && b0 + row < B) ? s[(long long)(b0 + row) * Ni + i] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    // thread (tx, ty): sensor m0 + tx, RHS b0 + ty + 8 q
    for (int t = 0; t < TT; ++t) {
      const c32 gv = sg[tx][t];
      for (int q = 0; q < 4; ++q) acc[q] = cfma(gv, ss[ty + 8 * q][t], acc[q]);
    }
    __syncthreads();
  }
  for (int q = 0; q < 4; ++q) {
    const int b = b0 + ty + 8 * q, m = m0 + tx;
    if (b < B && m < M) part[((long long)k * B + b) * M + m] = acc[q];
  }
}

// y[b][m] = sum over chunks (fixed order)
__global__ void k_ff_reduce(int B, int M, int nsplit, const c32* part, c32* y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * M) return;
  c32 a = make_float2(0.f, 0.f);
  for (int k = 0; k < nsplit; ++k) a = cadd(a, part[(long long)k * B * M + t]);
  y[t] = a;
}

// s_ext[b][p(i)] = sum_m conj(G[m][i]) r[b][m] on Omega (0 in the layer), rhs_ext = f s_ext;
// block: 32 pixels x 32 RHS, sensors in tiles of 32
__global__ __launch_bounds__(256) void k_ff_adjoint(int dim, int B, int M, int ne, int w, int n, const c32* G,
                                                     const c32* r, const float* fpl, c32* s_ext, c32* rhs_ext) {
  __shared__ c32 sg[TT][TT + 1];  // [sensor][pixel]
  __shared__ c32 sr[TT][TT + 1];  // [rhs][sensor]
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  const long long Ne = dim == 2 ? (long long)ne * ne : (long long)ne * ne * ne;
  const long long i0 = (long long)blockIdx.x * TT;
  const int b0 = blockIdx.y * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  c32 acc[4];
  for (int q = 0; q < 4; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int mb = 0; mb < M; mb += TT) {
    for (int q = 0; q < 4; ++q) {
      const int row = ty + 8 * q;
      const long long i = i0 + tx;
      sg[row][tx] = (mb + row < M && i < Ni) ? G[(long long)(mb + row) * Ni + i] : make_float2(0.f, 0.f);
      sr[row][tx] = (b0 + row < B && mb + tx < M) ? r[(long long)(b0 + row) * M + mb + tx] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    // thread (tx, ty): pixel i0 + tx, RHS b0 + ty + 8 q
    for (int t = 0; t < TT; ++t) {
      const c32 gv = sg[t][tx];
      for (int q = 0; q < 4; ++q) acc[q] = cadd(acc[q], cconjmul(gv, sr[ty + 8 * q][t]));
    }
    __syncthreads();
  }
  const long long i = i0 + tx;
  if (i >= Ni) return;
  const Coord c = coord_of32((unsigned)i, (unsigned)n, dim);
  const long long p = dim == 2 ? (long long)(c.y + w) * ne + (c.x + w)
                               : ((long long)(c.z + w) * ne + (c.y + w)) * ne + (c.x + w);
  for (int q = 0; q < 4; ++q) {
    const int b = b0 + ty + 8 * q;
    if (b < B) {
      s_ext[(long long)b * Ne + p] = acc[q];
      if (rhs_ext) rhs_ext[(long long)b * Ne + p] = cscale(acc[q], fpl[p]);
    }
  }
}

inline unsigned nb(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_ff_matrix(hipStream_t s, int dim, int n, int M, const double* sens, double kbh, double h,
                      const double2* tab, double x0, double dx, int ntab, c32* G) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  hipLaunchKernelGGL(k_ff_matrix, dim3(nb(Ni, 256), M), dim3(256), 0, s, dim, n, M, sens, kbh, h, tab, x0, dx, ntab,
                     G);
}

int ff_splits(long long Ni) {
  // pixel chunks of at least 1024 points, at most 64 chunks
  long long k = Ni / 1024;
  return (int)(k < 1 ? 1 : (k > 64 ? 64 : k));
}

void launch_ff_forward(hipStream_t s, int dim, int B, int M, int ne, int w, int n, const float* fpl, const c32* uin,
                       const c32* usc, const c32* G, c32* src, c32* part, c32* y) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  hipLaunchKernelGGL(k_ff_source, dim3(nb(Ni, 256), B), dim3(256), 0, s, dim, B, ne, w, n, fpl, uin, usc, src);
  const int ns = ff_splits(Ni);
  const long long chunk = (Ni + ns - 1) / ns;
  hipLaunchKernelGGL(k_ff_apply, dim3(nb(M, TT), nb(B, TT), ns), dim3(256), 0, s, B, M, Ni, chunk, G, src, part);
  hipLaunchKernelGGL(k_ff_reduce, dim3(nb((long long)B * M, 256)), dim3(256), 0, s, B, M, ns, part, y);
}

void launch_ff_adjoint(hipStream_t s, int dim, int B, int M, int ne, int w, int n, const c32* G, const c32* r,
                       const float* fpl, c32* s_ext, c32* rhs_ext) {
  const long long Ni = dim == 2 ? (long long)n * n : (long long)n * n * n;
  hipLaunchKernelGGL(k_ff_adjoint, dim3(nb(Ni, TT), nb(B, TT)), dim3(256), 0, s, dim, B, M, ne, w, n, G, r, fpl, s_ext,
                     rhs_ext);
}
