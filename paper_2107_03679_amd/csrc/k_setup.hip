// Medium-dependent set-up on the GPU (helm_setup / helm_update_n), once per
// medium, i.e. once per evaluation of the inverse problem's gradient:
//  * on Omega: c = (k0 h)^2 eta^2 (alpha = 1 inside Omega, Sec. IV-A), the
//    float-float diagonal of A' = h^2 A_Hel for the true residual,
//    f = k0^2 (eta^2 - eta_b^2) for the right-hand sides, and the finest level's
//    shifted coefficient kappa c and Jacobi factor omega / diag(K);
//  * per coarser level, at interior coarse points: kappa c_{l+1} = 4 x full
//    weighting of kappa c_l (Sec. IV-C; the 4 is (2h)^2 / h^2 of the scaled
//    operators, and the shift commutes with the linear restriction) and
//    omega / diag(K_l).
// The absorbing layer and the outermost coarse rings carry the background
// index whatever the medium, so they are written once by the host (FP64) and
// left alone here.
#include "dev_common.h"
#include "kernels.h"

namespace {

__global__ void k_setup_fine(SetupFineArgs a) {
  const long long Ni = a.dim == 2 ? (long long)a.n * a.n : (long long)a.n * a.n * a.n;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Ni) return;
  const int ix = (int)(q % a.n), iy = (int)((q / a.n) % a.n), iz = a.dim == 3 ? (int)(q / ((long long)a.n * a.n)) : 0;
  const int x = ix + a.w, y = iy + a.w, z = a.dim == 3 ? iz + a.w : 0;
  const long long p = a.dim == 2 ? (long long)y * a.ne + x : ((long long)z * a.ne + y) * a.ne + x;
  int ng = (x == 0) + (x == a.ne - 1) + (y == 0) + (y == a.ne - 1);
  if (a.dim == 3) ng += (z == 0) + (z == a.ne - 1);
  const float eta = a.nmap[q];
  // c = (k0 h)^2 eta^2 in float-float (eta^2 exact by TwoProd)
  const ff eta2 = two_prod(eta, eta);
  const ff c = ff_mul({a.k2_hi, a.k2_lo}, eta2);
  // diagonal of A': 2d - c - ng (1 + j k_b h)
  const ff dre = ff_sub(ff_from((float)(2 * a.dim - ng)), c);
  const ff dim_ = ff_neg(ff_mul(ff_from((float)ng), ff{a.kbh_hi, a.kbh_lo}));
  a.dhi[p] = make_float2(dre.hi, dim_.hi);
  a.dlo[p] = make_float2(dre.lo, dim_.lo);
  const float cf = c.hi;
  a.chi[p] = make_float2(cf, 0.f);
  // f = k0^2 (eta^2 - eta_b^2), unscaled
  const ff df = ff_sub(eta2, ff{a.nb2_hi, a.nb2_lo});
  const ff fv = ff_mul({a.k02_hi, a.k02_lo}, df);
  a.f[p] = fv.hi;
  // finest level of the preconditioner: kappa c (float-float, the start of the coarse chain)
  // and omega / (2d - kappa c - ng g0)
  const ff kre = ff_mul(c, ff_from(a.kappa.x)), kim = ff_mul(c, ff_from(a.kappa.y));
  const c32 kc = make_float2(kre.hi, kim.hi);
  a.kc0[p] = kc;
  a.kc0lo[p] = make_float2(kre.lo, kim.lo);
  const c32 D = make_float2((float)(2 * a.dim) - kc.x - (float)ng * a.g0.x, -kc.y - (float)ng * a.g0.y);
  a.wd0[p] = cscale(crcp(D), a.omega);
}

// interior points of level l (ring excluded): kc = 4 FW(kc of level l - 1), wd = omega / (2d - kc).
// kc is carried in float-float (hi, lo planes): the weights are powers of two, so every
// weighted term is exact and only the float-float sums round (about 2^-44), which keeps
// the chain over the levels as accurate as an FP64 one.
__global__ void k_setup_coarse(int dim, int nf, int nc, const c32* kcf, const c32* kcflo, float omega, c32* kcc,
                               c32* kcclo, c32* wdc) {
  const int m = nc - 2;  // interior points per axis
  const long long Nint = dim == 2 ? (long long)m * m : (long long)m * m * m;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Nint) return;
  const int X = 1 + (int)(t % m), Y = 1 + (int)((t / m) % m), Z = dim == 3 ? 1 + (int)(t / ((long long)m * m)) : 0;
  const float w1[3] = {0.25f, 0.5f, 0.25f};
  ff are = ff_from(0.f), aim = ff_from(0.f);
  const int zr = dim == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const long long fx = 2 * X + dx, fy = 2 * Y + dy, fz = dim == 3 ? 2 * Z + dz : 0;
        // 4 x the full-weighting weight: a power of two, so the products below are exact
        const float wgt = 4.f * w1[dx + 1] * w1[dy + 1] * (dim == 3 ? w1[dz + 1] : 1.f);
        const long long i = (fz * nf + fy) * nf + fx;
        const c32 vh = kcf[i], vl = kcflo[i];
        are = ff_add(are, ff_add(ff_from(wgt * vh.x), ff_from(wgt * vl.x)));
        aim = ff_add(aim, ff_add(ff_from(wgt * vh.y), ff_from(wgt * vl.y)));
      }
  const long long q = dim == 2 ? (long long)Y * nc + X : ((long long)Z * nc + Y) * nc + X;
  const c32 kc = make_float2(are.hi, aim.hi);
  kcc[q] = kc;
  kcclo[q] = make_float2(are.lo, aim.lo);
  wdc[q] = cscale(crcp(make_float2((float)(2 * dim) - kc.x, -kc.y)), omega);
}

}  // namespace

void launch_setup_fine(hipStream_t s, const SetupFineArgs& a) {
  const long long Ni = a.dim == 2 ? (long long)a.n * a.n : (long long)a.n * a.n * a.n;
  hipLaunchKernelGGL(k_setup_fine, dim3((unsigned)((Ni + 255) / 256)), dim3(256), 0, s, a);
}

void launch_setup_coarse(hipStream_t s, int dim, int nf, int nc, const c32* kcf, const c32* kcflo, float omega,
                         c32* kcc, c32* kcclo, c32* wdc) {
  const long long m = nc - 2;
  if (m <= 0) return;
  const long long Nint = dim == 2 ? m * m : m * m * m;
  hipLaunchKernelGGL(k_setup_coarse, dim3((unsigned)((Nint + 255) / 256)), dim3(256), 0, s, dim, nf, nc, kcf, kcflo,
                     omega, kcc, kcclo, wdc);
}
