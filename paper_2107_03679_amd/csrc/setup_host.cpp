// Host FP64 set-up of the level hierarchy (runs once per medium):
//  * coefficient c = (k0 h)^2 eta^2 alpha on Omega_e (Sec. IV-A), with the
//    absorbing-layer factor alpha = 1 + j sign gamma(x);
//  * coarse coefficients (Sec. IV-C): 4 x full weighting of the finer
//    coefficient at interior coarse points (the factor 4 = (2h)^2 / h^2 of the
//    h_l^2-scaled operators), background value k_b^2 h_l^2 alpha(x) on the
//    outermost ring;
//  * the explicit inverse of the coarsest shifted operator (Gauss-Jordan with
//    partial pivoting), which the GPU applies as a dense product.
#include "setup_host.h"

#include <algorithm>
#include <cmath>

namespace helm_host {

int extended_size(int n, int w, int levels) {
  if (n < 1 || w < 0 || levels < 1 || levels > 20) return -1;
  const long long step = 1LL << std::max(levels - 1, 1);
  long long ne = (long long)n + 2LL * w;
  while ((ne - 1) % step != 0) ++ne;
  return (int)ne;
}

// gamma(x) of the absorbing layer at fine index (ix, iy, iz).  Distances to
// Omega are measured in cells; profile 0 is the printed form in the unit
// normalisation of Omega_e (x in [0, 1], L = w / (n_e - 1)):
//   gamma = beta d^2 / L  = beta d_cells^2 / (w (n_e - 1));
// profile 1 is beta (d / L)^2 = beta d_cells^2 / w^2.
static double layer_gamma(const Geometry& g, const int* idx) {
  if (g.w <= 0 || g.beta == 0.0) return 0.0;
  const double lo = g.w, hi = g.w + g.n - 1;
  double d2 = 0.0;
  for (int a = 0; a < g.dim; ++a) {
    const double x = idx[a];
    const double d = std::max(0.0, std::max(lo - x, x - hi));
    d2 += d * d;
  }
  if (g.profile == 1) return g.beta * d2 / ((double)g.w * g.w);
  return g.beta * d2 / ((double)g.w * (g.ne - 1));
}

static cd layer_alpha(const Geometry& g, const int* idx) { return cd(1.0, g.sign * layer_gamma(g, idx)); }

static long long npts(int n, int dim) { return dim == 2 ? (long long)n * n : (long long)n * n * n; }

std::vector<cd> fine_coefficient(const Geometry& g, const std::vector<double>& nmap) {
  const long long N = npts(g.ne, g.dim);
  std::vector<cd> c(N);
  const double k2 = g.k0h * g.k0h;
  int idx[3] = {0, 0, 0};
  for (long long p = 0; p < N; ++p) {
    idx[0] = (int)(p % g.ne);
    idx[1] = (int)((p / g.ne) % g.ne);
    idx[2] = g.dim == 3 ? (int)(p / ((long long)g.ne * g.ne)) : 0;
    bool inside = true;
    for (int a = 0; a < g.dim; ++a) inside = inside && idx[a] >= g.w && idx[a] < g.w + g.n;
    double eta = g.n_b;
    if (inside) {
      const long long q = g.dim == 2 ? (long long)(idx[1] - g.w) * g.n + (idx[0] - g.w)
                                     : ((long long)(idx[2] - g.w) * g.n + (idx[1] - g.w)) * g.n + (idx[0] - g.w);
      eta = nmap[q];
    }
    c[p] = k2 * eta * eta * layer_alpha(g, idx);
  }
  return c;
}

std::vector<cd> coarse_coefficient(const Geometry& g, const std::vector<cd>& cf, int nf, int level) {
  const int nc = (nf - 1) / 2 + 1;
  const long long Nc = npts(nc, g.dim);
  std::vector<cd> cc(Nc);
  const double w1[3] = {0.25, 0.5, 0.25};
  const double kb = g.k0h * g.n_b * std::ldexp(1.0, level);
  for (long long q = 0; q < Nc; ++q) {
    int C[3] = {(int)(q % nc), (int)((q / nc) % nc), g.dim == 3 ? (int)(q / ((long long)nc * nc)) : 0};
    bool ring = false;
    for (int a = 0; a < g.dim; ++a) ring = ring || C[a] == 0 || C[a] == nc - 1;
    if (ring) {
      int fidx[3] = {0, 0, 0};
      for (int a = 0; a < g.dim; ++a) fidx[a] = C[a] << level;
      cc[q] = kb * kb * layer_alpha(g, fidx);
      continue;
    }
    cd acc = 0.0;
    const int zr = g.dim == 3 ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const long long fx = 2 * C[0] + dx, fy = 2 * C[1] + dy, fz = g.dim == 3 ? 2 * C[2] + dz : 0;
          const double wgt = w1[dx + 1] * w1[dy + 1] * (g.dim == 3 ? w1[dz + 1] : 1.0);
          acc += wgt * cf[(fz * nf + fy) * nf + fx];
        }
    cc[q] = 4.0 * acc;
  }
  return cc;
}

bool dense_inverse_transposed(const Geometry& g, const std::vector<cd>& cl, int nl, int level, cd kappa,
                              std::vector<cd>& inv_t) {
  const long long N = npts(nl, g.dim);
  const cd ghost(1.0, g.k0h * g.n_b * std::ldexp(1.0, level));
  // assemble K'_l = -Lap'_l - kappa c_l as a dense row-major matrix
  std::vector<cd> a(N * N, cd(0.0));
  for (long long p = 0; p < N; ++p) {
    const int x = (int)(p % nl), y = (int)((p / nl) % nl), z = g.dim == 3 ? (int)(p / ((long long)nl * nl)) : 0;
    int ng = (x == 0) + (x == nl - 1) + (y == 0) + (y == nl - 1);
    if (g.dim == 3) ng += (z == 0) + (z == nl - 1);
    a[p * N + p] = 2.0 * g.dim - kappa * cl[p] - (double)ng * ghost;
    const long long s2 = (long long)nl * nl;
    if (x > 0) a[p * N + p - 1] = -1.0;
    if (x < nl - 1) a[p * N + p + 1] = -1.0;
    if (y > 0) a[p * N + p - nl] = -1.0;
    if (y < nl - 1) a[p * N + p + nl] = -1.0;
    if (g.dim == 3) {
      if (z > 0) a[p * N + p - s2] = -1.0;
      if (z < nl - 1) a[p * N + p + s2] = -1.0;
    }
  }
  // Gauss-Jordan with partial pivoting on [A | I]
  std::vector<cd> inv(N * N, cd(0.0));
  for (long long i = 0; i < N; ++i) inv[i * N + i] = 1.0;
  for (long long col = 0; col < N; ++col) {
    long long piv = col;
    double best = std::abs(a[col * N + col]);
    for (long long r = col + 1; r < N; ++r) {
      const double v = std::abs(a[r * N + col]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (best == 0.0 || !std::isfinite(best)) return false;
    if (piv != col) {
      std::swap_ranges(a.begin() + piv * N, a.begin() + piv * N + N, a.begin() + col * N);
      std::swap_ranges(inv.begin() + piv * N, inv.begin() + piv * N + N, inv.begin() + col * N);
    }
    const cd d = 1.0 / a[col * N + col];
    for (long long k = 0; k < N; ++k) {
      a[col * N + k] *= d;
      inv[col * N + k] *= d;
    }
    for (long long r = 0; r < N; ++r) {
      if (r == col) continue;
      const cd f = a[r * N + col];
      if (f == cd(0.0)) continue;
      cd* ar = &a[r * N];
      cd* ir = &inv[r * N];
      const cd* ac = &a[col * N];
      const cd* ic = &inv[col * N];
      for (long long k = col; k < N; ++k) ar[k] -= f * ac[k];
      for (long long k = 0; k < N; ++k) ir[k] -= f * ic[k];
    }
  }
  inv_t.assign(N * N, cd(0.0));
  for (long long r = 0; r < N; ++r)
    for (long long k = 0; k < N; ++k) inv_t[k * N + r] = inv[r * N + k];
  return true;
}

}  // namespace helm_host
