// Host FP64 set-up of the level hierarchy (runs once per medium):
//  * coefficient c = (k0 h)^2 eta^2 alpha on Omega_e (Sec. IV-A), with the
//    absorbing-layer factor alpha = 1 + j sign gamma(x);
//  * coarse coefficients (Sec. IV-C): 4 x full weighting of the finer
//    coefficient at interior coarse points (the factor 4 = (2h)^2 / h^2 of the
//    h_l^2-scaled operators), background value k_b^2 h_l^2 alpha(x) on the
//    outermost ring;
//  * the explicit inverse of the coarsest shifted operator, which the GPU applies
//    as a dense product: banded LU without pivoting where the operator is
//    diagonally dominant (the usual case: the shifted coefficient of the
//    coarsest grid is large), else Gauss-Jordan with partial pivoting.
#include "setup_host.h"

#include <algorithm>
#include <cmath>
#include <thread>

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

// Inverse of a matrix that is diagonally dominant by rows (so LU without pivoting is stable)
// and banded with half-bandwidth bw (the h^2-scaled Laplacian plus a diagonal on an nl^d grid:
// bw = nl^(d-1)).  LU in band storage costs N bw^2; column j of the inverse needs the forward
// substitution from row j on and, since K is complex symmetric (so is its inverse), only the
// back substitution down to row j: entry (i, j) for i >= j, mirrored to (j, i).  Columns are
// split over host threads.  Returns the transposed inverse (row-major inv_t[k][r] = inv[r][k]).
static void banded_inverse(const std::vector<cd>& a, long long N, long long bw, std::vector<cd>& inv_t) {
  const long long W = 2 * bw + 1;  // band row: columns p - bw .. p + bw
  std::vector<cd> band(N * W, cd(0.0));
  auto B = [&](long long r, long long col) -> cd& { return band[r * W + (col - r + bw)]; };
  for (long long r = 0; r < N; ++r)
    for (long long col = std::max(0LL, r - bw); col <= std::min(N - 1, r + bw); ++col) B(r, col) = a[r * N + col];
  // LU without pivoting: L (unit lower) below the diagonal, U on and above it, fill stays in the band
  for (long long k = 0; k < N; ++k) {
    const cd piv = B(k, k);
    const long long end = std::min(N - 1, k + bw);
    for (long long i = k + 1; i <= end; ++i) {
      cd& lik = B(i, k);
      if (lik == cd(0.0)) continue;
      lik /= piv;
      for (long long j = k + 1; j <= end; ++j) B(i, j) -= lik * B(k, j);
    }
  }
  inv_t.assign(N * N, cd(0.0));
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t)
    pool.emplace_back([&, t] {
      std::vector<cd> v(N);
      for (long long j = t; j < N; j += nth) {
        // forward: L y = e_j (y_i = 0 for i < j)
        std::fill(v.begin(), v.end(), cd(0.0));
        v[j] = 1.0;
        for (long long i = j + 1; i < N; ++i) {
          cd s = 0.0;
          for (long long k = std::max(j, i - bw); k < i; ++k) s += B(i, k) * v[k];
          v[i] = -s;
        }
        // back: U x = y, rows N-1 down to j
        for (long long i = N - 1; i >= j; --i) {
          cd s = v[i];
          const long long end = std::min(N - 1, i + bw);
          for (long long k = i + 1; k <= end; ++k) s -= B(i, k) * v[k];
          v[i] = s / B(i, i);
        }
        // inv[i][j] = inv[j][i] = v[i] for i >= j; inv_t[k][r] = inv[r][k]
        for (long long i = j; i < N; ++i) {
          inv_t[j * N + i] = v[i];
          inv_t[i * N + j] = v[i];
        }
      }
    });
  for (auto& th : pool) th.join();
}

bool dense_inverse_transposed(const Geometry& g, const std::vector<cd>& kcl, int nl, int level,
                              std::vector<cd>& inv_t) {
  const long long N = npts(nl, g.dim);
  const cd ghost(1.0, g.k0h * g.n_b * std::ldexp(1.0, level));
  // assemble K'_l = -Lap'_l - kappa c_l (kcl = kappa c_l) as a dense row-major matrix
  std::vector<cd> a(N * N, cd(0.0));
  bool dominant = true;
  for (long long p = 0; p < N; ++p) {
    const int x = (int)(p % nl), y = (int)((p / nl) % nl), z = g.dim == 3 ? (int)(p / ((long long)nl * nl)) : 0;
    int ng = (x == 0) + (x == nl - 1) + (y == 0) + (y == nl - 1);
    if (g.dim == 3) ng += (z == 0) + (z == nl - 1);
    a[p * N + p] = 2.0 * g.dim - kcl[p] - (double)ng * ghost;
    dominant = dominant && std::abs(a[p * N + p]) > 2.0 * g.dim - ng;  // off-diagonal row sum
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
  for (long long p = 0; p < N; ++p)
    if (!std::isfinite(std::abs(a[p * N + p]))) return false;
  if (dominant) {
    banded_inverse(a, N, g.dim == 2 ? nl : (long long)nl * nl, inv_t);
    return true;
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
