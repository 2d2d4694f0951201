// Host FP64 set-up numerics (coefficients per level, coarsest inverse).
#pragma once

#include <complex>
#include <vector>

namespace helm_host {

typedef std::complex<double> cd;

struct Geometry {
  int dim;      // 2 or 3
  int n;        // interior points per axis
  int w;        // low-side layer width (cells)
  int ne;       // extended points per axis
  double k0h;   // k0 * h
  double n_b;   // background index
  double beta;  // layer strength
  int sign;     // +1 dissipative, -1 printed sign
  int profile;  // 0 printed (unit normalisation), 1 beta (d/L)^2
};

int extended_size(int n, int w, int levels);
std::vector<cd> fine_coefficient(const Geometry& g, const std::vector<double>& nmap);
std::vector<cd> coarse_coefficient(const Geometry& g, const std::vector<cd>& cf, int nf, int level);
// transposed inverse of K'_l = -Lap'_l (with the level's ghost rows) - kcl, kcl = kappa c_l
bool dense_inverse_transposed(const Geometry& g, const std::vector<cd>& kcl, int nl, int level,
                              std::vector<cd>& inv_t);

}  // namespace helm_host
