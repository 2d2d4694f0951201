// Kernel argument types and launcher declarations shared by the HIP sources
// and the host engine.  All fields are complex64 (float2) arrays.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

typedef float2 c32;

// A set of per-right-hand-side vectors: vector q starts at p + q * stride.
struct VecSet {
  c32* p;
  long long stride;
};
// Optional per-right-hand-side scale factors: factor of q is p[q * stride] (p = NULL -> 1).
struct ScaleSet {
  const float* p;
  int stride;
};
// One multigrid level of the vertex-centred hierarchy.
struct LevelArgs {
  int n;            // points per side
  long long N;      // n^dim
  const c32* coef;  // operator coefficient: kappa * c_l (K_kappa) or c (A)
  c32 ghost;        // Sommerfeld ghost factor 1 + j k_b h_l
  const c32* wd;    // omega_S / diag(K_kappa) per point (multigrid levels only)
};

// per-RHS solver status on the device (the final values match helm.h's HELM_STATUS_*)
enum {
  HELM_RUNNING = -1,
  HELM_STATUS_CONVERGED_DEV = 0,
  HELM_STATUS_NOT_CONVERGED_DEV = 1,
  HELM_STATUS_BREAKDOWN_DEV = 2
};

// ---- multigrid legs (2D) ----
// fused 2D legs; cfg selects one of the tile shapes (0 = default, see mg_*_shape).
// e.p != NULL: repeated visit from the current solution e (right-hand side r - K e;
// the up-leg writes e + correction to z, which must not alias e).
void launch_down_fused2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet rc, int nc,
                        const int* active, int cfg, VecSet e = VecSet{nullptr, 0});
void launch_up_fused2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet ec, int nc,
                      VecSet z, const int* active, int cfg, VecSet e = VecSet{nullptr, 0});
// fused 3D legs (same roles as the 2D legs; fixed tiles)
void launch_down_fused3(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet rc, int nc,
                        const int* active);
void launch_up_fused3(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet ec, int nc,
                      VecSet z, const int* active, int acc = 0);  // acc: z += the leg's result
// up-leg of Z_j and W_{j+1} = A Z_j in one launch (2D; la = the A operator)
void launch_up_mv2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la, float omega, VecSet ec,
                   int nc, VecSet z, VecSet w, const int* active, int cfg = 0);
// finest-level step of the s-step basis (2D): up-leg of Z_j, W_{j+1} = A Z_j (la = the A
// operator), down-leg of W_{j+1} into rc; one launch
void launch_step_fused2(hipStream_t s, int B, VecSet r, ScaleSet rs, LevelArgs lv, LevelArgs la, float omega,
                        VecSet ec, int nc, VecSet z, VecSet w, VecSet rc, const int* active);
int mg_down_variants();
int mg_up_variants();
// launch shapes of the fused finest up-leg + basis matvec (autotuner choices): tile
// height and right-hand sides per block
int mg_up_mv_variants();
int mg_up_mv_rows(int cfg);
int mg_up_mv_rhs_per_block(int cfg);
void mg_down_shape(int cfg, int* tcx, int* tcy);
void mg_up_shape(int cfg, int* tx, int* ty, int* py);
void launch_jacobi_zero(hipStream_t s, int dim, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet v,
                        const int* active);
void launch_jacobi(hipStream_t s, int dim, int B, VecSet r, ScaleSet rs, LevelArgs lv, float omega, VecSet v,
                   VecSet vout, const int* active);
void launch_restrict_residual(hipStream_t s, int dim, int B, VecSet r, ScaleSet rs, VecSet v, LevelArgs lv,
                              VecSet rc, int nc, const int* active);
// v (or vout when given) = v + P ec
void launch_prolong_add(hipStream_t s, int dim, int B, VecSet ec, int nc, VecSet v, int n, const int* active,
                        VecSet vout = VecSet{nullptr, 0});
// z = M r with the explicit inverse (M^T stored); with `part` (coarse_solve_part_size
// entries) and B >= 4 as one matrix product over all right-hand sides
void launch_coarse_solve(hipStream_t s, int B, const c32* minvT, int Nc, VecSet r, VecSet z, const int* active,
                         c32* part = nullptr);
size_t coarse_solve_part_size(int B, int Nc);
void launch_apply(hipStream_t s, int dim, int B, VecSet x, ScaleSet xs, LevelArgs lv, float out_scale, VecSet y,
                  const int* active);
// out = s_b bvec - K v (bs = per-RHS scale of bvec, NULL = 1)
void launch_level_residual(hipStream_t s, int dim, int B, VecSet bvec, VecSet v, LevelArgs lv, VecSet out,
                           const int* active, ScaleSet bs = ScaleSet{nullptr, 0});
void launch_add(hipStream_t s, int B, VecSet x, VecSet y, long long N, const int* active);

// ---- coarse levels of a V-cycle in one launch (one workgroup per right-hand side) ----
struct CoarseLevel {
  int n;
  long long N;
  const c32* wd;  // omega / diag(K_l)
  c32* rc;        // [B][N] right-hand side
  c32* e;         // [B][N] solution
  c32* t;         // [B][N] scratch
};
constexpr int HELM_MAX_LEVELS = 12;
struct CoarseCycleArgs {
  int dim, lp, L;  // levels lp .. L-1 are handled; lp's rc is the input, its e the output
  float omega;
  const c32* minvT;
  const int* active;
  CoarseLevel lv[HELM_MAX_LEVELS];
};
// LDS-resident variant when the levels' vectors fit in this many bytes, else through L2
constexpr size_t kCoarseCycleMaxLds = 64 * 1024;
size_t coarse_cycle_lds_bytes(const CoarseCycleArgs& a);
void launch_coarse_cycle(hipStream_t s, int B, const CoarseCycleArgs& a);

// ---- Krylov (FGMRES / float-float outer loop), flat over the fine grid ----
// a float-float field pair, [B][N] each
struct XPair {
  c32* hi;
  c32* lo;
};

struct KrylovArgs {
  int dim;
  int n;
  long long N;
  int m;          // restart length
  int nblk;       // partial-reduction blocks per right-hand side
  c32* V;         // [B][m+1][N] basis (unnormalised; v_i = vs[i] * V_i)
  c32* Z;         // [B][m][N] preconditioned vectors
  float* vs;      // [B][m+1] scale of each basis vector
  c32* P1;        // [B][nblk][m+1] partial dots
  float* P2;      // [B][nblk] partial squared norms ([B][nres] after a true residual)
  int nres;       // partial squared norms per right-hand side of the last true residual
  int* xpar;      // [B] which buffer of the pair holds x (the fused update of 2D grids alternates)
  int flip_x;     // 1: k_finalize flips xpar (after the fused update and residual)
  double2* H;     // [B][m+1][m] Hessenberg (rotated in place)
  double* cs;     // [B][m]
  double2* sn;    // [B][m]
  double2* g;     // [B][m+1]
  c32* coef;      // [B][m+1] h_i * vs_i for the update pass
  c32* y;         // [B][m] least-squares solution of the cycle
  int* active;    // [B] 1 while the current cycle iterates
  int* status;    // [B] HELM_RUNNING or a final status
  int* jcount;    // [B] steps taken in the current cycle
  int* iters;     // [B] total preconditioner applications
  double* bnorm;  // [B] ||h^2 b||
  double* tol;    // [B] absolute stop level of the Givens estimate
  double* relres; // [B] true relative residual of the last evaluation
  int max_iters;
  double rtol;
  double inner_factor;
  int bicg;       // 1: Bi-CGSTAB (the true residual skips right-hand sides still iterating)
};

void launch_arnoldi_dots(hipStream_t s, int B, const KrylovArgs& k, int j, const LevelArgs* fine, int with_matvec);
void launch_arnoldi_reduce(hipStream_t s, int B, const KrylovArgs& k, int j, int accumulate);
void launch_arnoldi_update(hipStream_t s, int B, const KrylovArgs& k, int j);
void launch_givens(hipStream_t s, int B, const KrylovArgs& k, int j);
void launch_x_update(hipStream_t s, int B, const KrylovArgs& k, c32* x_hi, c32* x_lo);
// partial squared norms per right-hand side that launch_residual_ff writes (block or column tiles)
int krylov_residual_partials(const KrylovArgs& k, int x_zero);
void launch_residual_ff(hipStream_t s, int B, const KrylovArgs& k, const c32* rhs, long long rhs_stride,
                        int conj_rhs, const c32* x_hi, const c32* x_lo, int x_zero, const c32* d_hi,
                        const c32* d_lo, float h2_hi, float h2_lo, c32* r_out, long long r_stride, float out_scale);
// 2D grids: x += sum_i y_i Z_i and the true residual of the new x in one pass
// (the partial norms of krylov_xres_tiles(n) tiles per right-hand side)
int krylov_xres_tiles(int n);
void launch_x_update_residual(hipStream_t s, int B, const KrylovArgs& k, XPair x0, XPair x1, const c32* rhs,
                              long long rhs_stride, int conj_rhs, const c32* d_hi, const c32* d_lo, float h2_hi,
                              float h2_lo, c32* r_out, long long r_stride);
void launch_finalize(hipStream_t s, int B, const KrylovArgs& k, int first);
void launch_accept(hipStream_t s, int B, const KrylovArgs& k, int j, const LevelArgs& fine, double tol, int* mg_mask,
                   int* fallbacks, VecSet resid);
void launch_reject_reset(hipStream_t s, int B, const KrylovArgs& k, int j, const int* mg_mask, VecSet resid);

// ---- model kernels ----
void launch_plane_wave(hipStream_t s, int dim, int B, int n, const float* fplane, const c32* tables, c32* rhs,
                       c32* uin);
void launch_grad_n(hipStream_t s, int dim, int B, int n_e, int w, int n, const c32* uin, const c32* u,
                   const c32* lam, const float* nmap, float scale, float* grad,
                   const c32* lam2 = nullptr, int accumulate = 0);
void launch_conj_copy(hipStream_t s, long long count, const c32* in, c32* out);
// out[b] = (xpar && xpar[b] ? in1 : in0)[b] for b < B, N points each, conjugated when conj
void launch_x_select(hipStream_t s, int B, long long N, const int* xpar, const c32* in0, const c32* in1, c32* out,
                     int conj);
void launch_gather(hipStream_t s, int B, int M, long long N, const int* idx, const c32* u, c32* y);
void launch_scatter(hipStream_t s, int B, int M, long long N, const int* idx, const c32* y, c32* u);
int tv_partials(int dim, int n);
void launch_tv(hipStream_t s, int dim, int n, const float* nm, float eps, float scale, float* mag, float* part,
               float* grad);
void launch_zero(hipStream_t s, long long count, c32* p);
void launch_status_init(hipStream_t s, int B, const KrylovArgs& k);
int krylov_blocks_per_rhs(long long N);
int krylov_max_restart();
// Bi-CGSTAB (Alg. 3), slots and scalars documented in k_bicgstab.hip
void launch_bicg_dir(hipStream_t s, int B, const KrylovArgs& k);
void launch_bicg_apply(hipStream_t s, int B, const KrylovArgs& k, int zs, int vs, const LevelArgs& fine, int second);
void launch_bicg_alpha(hipStream_t s, int B, const KrylovArgs& k);
void launch_bicg_s(hipStream_t s, int B, const KrylovArgs& k);
void launch_bicg_sigma(hipStream_t s, int B, const KrylovArgs& k);
void launch_bicg_update(hipStream_t s, int B, const KrylovArgs& k, c32* x_hi, c32* x_lo);
void launch_bicg_rho(hipStream_t s, int B, const KrylovArgs& k);
void launch_bicg_finalize(hipStream_t s, int B, const KrylovArgs& k, int first);
// s-step GMRES(m): basis matvec W_{j+1} = A Z_j; Gram pass (fused with the last
// matvec) + per-RHS Cholesky-QR least squares.  part: [B][nblk][sstep_gram_entries(m)].
int sstep_max_restart();
long long sstep_gram_entries(int m);
void launch_sstep_matvec(hipStream_t s, int B, const KrylovArgs& k, int j, const LevelArgs& fine);
void launch_sstep_gram_solve(hipStream_t s, int B, const KrylovArgs& k, const LevelArgs& fine, double2* part);

// ---- inverse problem (Sec. V, Alg. 4), interior grid n^dim ----
void launch_tv_prox(hipStream_t s, int dim, int n, const float* v, float lam, float lo, int iters, float* p, float* r,
                    float* w);
void launch_axmy(hipStream_t s, long long count, const float* a, float sc, const float* b, float* out);
void launch_fbs_momentum(hipStream_t s, long long count, const float* f_new, float beta, float* f, float* fbar);
// ---- medium-dependent set-up (k_setup.hip) ----
struct SetupFineArgs {
  int dim, n, w, ne;
  const float* nmap;            // interior index [n^dim]
  float k2_hi, k2_lo;           // (k0 h)^2, float-float
  float kbh_hi, kbh_lo;         // k_b h (imaginary part of the fine ghost factor), float-float
  float k02_hi, k02_lo;         // k0^2 (the unscaled f), float-float
  float nb2_hi, nb2_lo;         // eta_b^2, float-float
  c32 kappa, g0;                // shift; fine ghost factor 1 + j k_b h
  float omega;                  // damped-Jacobi factor
  c32 *chi, *dhi, *dlo, *kc0, *kc0lo, *wd0;
  float* f;
};
// Omega points of the fine level: c, float-float diagonal of A', f, kappa c, omega / diag(K_0)
void launch_setup_fine(hipStream_t s, const SetupFineArgs& a);
// interior points of a coarse level (nc per axis) from the finer level's kappa c (nf per axis),
// kappa c carried as float-float (hi, lo planes)
void launch_setup_coarse(hipStream_t s, int dim, int nf, int nc, const c32* kcf, const c32* kcflo, float omega,
                         c32* kcc, c32* kcclo, c32* wdc);

// Fixed device scratch of the allocation-free data residual (k_static.hip): per-device
// address from hipGetSymbolAddress (static_scratch_init once per device, with it current),
// partial capacity, and the check / total kernels working inside it.
int static_scratch_partials();
hipError_t static_scratch_init();
double* static_scratch();  // current device's copy, nullptr before static_scratch_init
void launch_static_check(hipStream_t s, int M, long long N, const int* idx, double* scr);
void launch_static_total(hipStream_t s, int nbk, double* scr);
const double* static_flag(const double* scr);
const double* static_total(const double* scr);
// FP32 vector helpers: block partial sums of squares (FP64) and an in-place scaling
int sumsq_blocks(long long n);
void launch_sumsq(hipStream_t s, long long n, const float* x, double* part);
void launch_scale(hipStream_t s, long long n, float* x, float a);
int data_residual_blocks(int B, int M);
void launch_data_residual(hipStream_t s, int B, int M, long long N, const int* idx, const c32* u, const c32* y,
                          c32* res, double* part);
void launch_index_from_f(hipStream_t s, long long count, const float* f, double inv_k02, double nb2, float* nmap);

// ---- sensor operator (far field through the Lippmann-Schwinger integral) ----
void launch_ff_matrix(hipStream_t s, int dim, int n, int M, const double* sens, double kbh, double h,
                      const double2* tab, double x0, double dx, int ntab, c32* G);
int ff_splits(long long Ni);
void launch_ff_forward(hipStream_t s, int dim, int B, int M, int ne, int w, int n, const float* fpl, const c32* uin,
                       const c32* usc, const c32* G, c32* src, c32* part, c32* y);
void launch_ff_adjoint(hipStream_t s, int dim, int B, int M, int ne, int w, int n, const c32* G, const c32* r,
                       const float* fpl, c32* s_ext, c32* rhs_ext);
