/*
 * helm.h -- C ABI of the MI355X Helmholtz solver library (libhelm.so).
 *
 * The library computes the scattered field of the discretised Helmholtz
 * equation of Hong, Pham, Treister and Unser, "Diffraction Tomography with
 * Helmholtz Equation: Efficient and Robust Multigrid-Based Solver"
 * (arXiv 2107.03679):
 *
 *     A_Hel u_sc = b,  b = f u_in,  f = k0^2 (eta^2 - eta_b^2)
 *
 * (Sec. II-A eq. HelmScatterRightIncident; Sec. IV-A eq. discretizedHelm and
 * the first-order Sommerfeld ghost rows), one solve per incident plane wave,
 * batched over all waves of a scan, by a Krylov method (restarted GMRES in
 * s-step form by default, flexible GMRES, or the paper's Bi-CGSTAB of Alg. 3)
 * preconditioned with one multigrid cycle (V, W, or two coarse-grid corrections
 * on the finest level; Alg. 2) on the shifted operator
 * K_kappa = -Lap - kappa k0^2 eta^2 (Sec. IV-B/IV-C), and the adjoint solves
 * and refractive-index gradient of Sec. V (Prop. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Fields are complex64, interleaved {re, im} (helm_c32), on the EXTENDED
 *    grid Omega_e (interior Omega plus the absorbing layer), laid out
 *    [B][n_e][n_e] (2D) or [B][n_e][n_e][n_e] (3D), x fastest: point (m, n)
 *    of right-hand side q is element q*n_e^2 + n*n_e + m (row order of
 *    eq. discretizedHelm).  Omega is indices [w, w+n) per axis, w = the layer
 *    width; n_e comes from helm_extended_size().
 *  - Field pointers are DEVICE pointers (hipMalloc'd or torch tensors) unless
 *    the name ends in _host.  The caller owns every buffer it passes and keeps
 *    it alive until the call returns; calls are stream-ordered on the stream
 *    given to helm_setup and return after that stream has finished the work.
 *  - All operator semantics refer to the UNSCALED matrix A_Hel of
 *    eq. discretizedHelm (1/h^2 Laplacian).  Internally the library solves the
 *    h^2-scaled system, which has the same solution.
 *  - Return codes: 0 = OK; HELM_NOT_CONVERGED (> 0) is soft: outputs hold the
 *    best iterate and the per-RHS stats are valid; negative codes are hard
 *    errors (outputs undefined), described by helm_last_error().  No C++
 *    exception crosses this boundary.
 *  - One context per stream; calls on one context are not thread-safe.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HELM_OK 0
#define HELM_NOT_CONVERGED 1
#define HELM_EINVAL (-1)
#define HELM_EHIP (-2)
#define HELM_ENOMEM (-3)
#define HELM_ESTATE (-4)

/* per-RHS status in helm_stats.status */
#define HELM_STATUS_CONVERGED 0
#define HELM_STATUS_NOT_CONVERGED 1
#define HELM_STATUS_BREAKDOWN 2 /* non-finite data or a Krylov breakdown */

typedef struct {
  float re, im;
} helm_c32;

/* Grid (Sec. IV-A).  dim = 2 or 3; n = interior points per axis; abl_width =
 * low-side absorbing-layer width in cells (the high side gets at least as
 * many; see helm_extended_size); h = mesh size in the unit of 1/k0, or <= 0
 * for the paper's normalisation of Omega_e to the unit square/cube,
 * h = 1/(n_e - 1). */
typedef struct {
  int dim;
  int n;
  int abl_width;
  double h;
} helm_grid;

/* Absorbing layer (Sec. IV-A): k0^2 eta^2 is multiplied on Omega_e \ Omega by
 * alpha = 1 + j*sign*beta*|x - P_Omega(x)|^2 / L, L = abl_width*h.  sign = +1
 * (default) is the dissipative reading under the e^{-j w t} convention;
 * sign = -1 reproduces the printed sign.  profile 0 = the printed form
 * (distances in the mesh's unit); profile 1 = beta*(|x - P x| / L)^2. */
typedef struct {
  double beta;
  int sign;
  int profile;
} helm_abl;

/* Solver options.  helm_default_opts() fills the defaults quoted here. */
typedef struct {
  double n_b;       /* background refractive index eta_b (1.333) */
  double kappa_re;  /* shift of the preconditioning operator K_kappa (1.0) */
  double kappa_im;  /*   ... imaginary part (0.5) */
  double omega_jac; /* damped-Jacobi factor omega_S, eq. dampedJ (0.8) */
  double rtol;      /* stop when ||b - A x|| <= rtol ||b||, true residual (1e-6) */
  int levels;       /* multigrid levels incl. the exactly solved coarsest (4) */
  int nu1, nu2;     /* pre/post relaxations (1, 1) */
  int cycle;        /* 1 = V-cycle, 2 = W-cycle (Alg. 2 CycleType); 3 = two coarse-grid
                       corrections on the finest level and V-cycles below (1) */
  int restart;      /* restart length m of GMRES (s-step form or FGMRES); for Bi-CGSTAB the
                       iterations between status checks (10) */
  int max_iters;    /* max preconditioner applications per RHS (4000) */
  int max_batch;    /* largest B accepted by the solve calls (64) */
  int reorth;       /* 1 = one re-orthogonalisation pass (CGS2) (0) */
  int fused;        /* 1 = fused multigrid leg kernels (2D and 3D) when nu1 = nu2 = 1 (1) */
  int use_graph;    /* 1 = replay each restart cycle as a captured hipGraph (1) */
  int coarse_single_launch; /* 1 = V-cycle levels with <= 48^2 (2D) / 16^3 (3D) points run
                               in one launch, one workgroup per right-hand side (1) */
  int krylov;       /* HELM_KRYLOV_SSTEP (default), HELM_KRYLOV_FGMRES or HELM_KRYLOV_BICGSTAB */
  int fused_step;   /* finest level of the s-step form (2D, fused legs): 0 = separate kernels;
                       1 = the work between two coarse visits (up-leg, basis matvec, next
                       down-leg) is one kernel: 36% fewer bytes, but the wider region and six
                       barrier stages leave it slower than option 2 on MI355X (200 against
                       138 + 56 us per step at 512^2 x 60);
                       2 = the up-leg and the basis matvec W_{j+1} = A Z_j in one kernel, which
                       saves the matvec's pass over Z_j (2) */
} helm_opts;

/* Krylov forms (helm_opts.krylov).  Both minimise the residual over the same
 * space (GMRES(m) right-preconditioned by the multigrid cycle: the Krylov
 * part of the Krylov + multigrid scheme of Sec. IV-C) and restart from a
 * float-float true residual.
 *   HELM_KRYLOV_FGMRES  flexible GMRES, Arnoldi with classical Gram-Schmidt
 *                       (reorth = 1: twice); admits a nonlinear preconditioner.
 *   HELM_KRYLOV_SSTEP   s-step form: the basis W_{j+1} = A M(W_j) is built by
 *                       plain matvecs, one Gram pass per cycle and an FP64
 *                       Cholesky QR give the least squares; restart <= 12;
 *                       needs a linear preconditioner, so a context with a
 *                       learned network (helm_set_preconditioner) runs FGMRES. */
#define HELM_KRYLOV_FGMRES 0
#define HELM_KRYLOV_SSTEP 1
/*   HELM_KRYLOV_BICGSTAB  the paper's Alg. 3 (Bi-CGSTAB, two multigrid cycles per
 *                       iteration; sigma is van der Vorst's omega), batched, with
 *                       the float-float solution; `restart` (>= 4) is the number of
 *                       iterations between status checks, not a restart: the
 *                       recurrence restarts from the true residual only when its
 *                       own residual met the tolerance and the true one did not.
 *                       helm_stats.iters counts multigrid cycles (2 per iteration).
 *                       A context with a learned network runs FGMRES instead. */
#define HELM_KRYLOV_BICGSTAB 2

typedef struct {
  int iters;            /* preconditioner applications */
  int status;           /* HELM_STATUS_* */
  double rel_res_true;  /* ||b - A x|| / ||b|| of the returned x (float-float evaluation) */
  int fallbacks;        /* learned-preconditioner outputs rejected for the V-cycle (0 without a network) */
  double ms;            /* wall time of the whole batched call on the GPU (HIP events on the context
                           stream, from the copy of the right-hand sides to the last status read);
                           the same value for every right-hand side of the batch */
} helm_stats;

typedef struct {
  int dim, n, abl_width, n_e, levels, coarsest_n;
  double h, k0, n_b;
  size_t workspace_bytes;
} helm_info;

typedef struct helm_ctx helm_ctx;
typedef struct helm_net helm_net;

/* Defaults of helm_opts (see the field comments). */
void helm_default_opts(helm_opts* opts);

/* Extended grid size n_e for n interior points, a low-side layer of
 * abl_width cells and `levels` multigrid levels: the smallest odd
 * n_e >= n + 2*abl_width with (n_e - 1) divisible by 2^(levels-1), which the
 * vertex-centred coarsening of Sec. IV-C needs.  Returns -1 on bad input. */
int helm_extended_size(int n, int abl_width, int levels);

/* Create a context: coefficient c = (k0 h)^2 eta^2 alpha on Omega_e and its
 * restrictions per level (Sec. IV-C: full weighting, background ring), the
 * exact inverse of the coarsest K_kappa (factorised on the host in FP64),
 * the Krylov workspace for opts->max_batch right-hand sides.
 *   n_map_dev : device float[n^dim], the refractive index on Omega (copied)
 *   k0        : free-space wavenumber omega/c in the unit of 1/h
 *   abl, opts : NULL = defaults (beta 0.15, sign +1, profile 0)
 *   hip_stream: hipStream_t the context issues all work on (NULL = default)
 * Errors: HELM_EINVAL for bad sizes, HELM_ENOMEM, HELM_EHIP. */
int helm_setup(const helm_grid* grid, const float* n_map_dev, double k0, const helm_abl* abl,
               const helm_opts* opts, void* hip_stream, helm_ctx** out);

/* Replace the refractive index (FBS iterations): recompute coefficients and
 * the coarsest inverse; no reallocation. */
int helm_update_n(helm_ctx* ctx, const float* n_map_dev);

int helm_get_info(const helm_ctx* ctx, helm_info* info);

/* Plane-wave right-hand sides (Sec. II-A): for q < B and unit directions
 * dirs_host[q*dim .. q*dim+dim) (x, y[, z]),
 *   u_in = exp(j k0 eta_b <d, x - x_c>) with x_c the centre of Omega,
 *   rhs  = f * u_in, f = k0^2 (eta^2 - eta_b^2) on Omega, 0 in the layer.
 * rhs: device [B][grid] (written).  u_in: device [B][grid] or NULL. */
int helm_plane_wave_rhs(helm_ctx* ctx, int B, const double* dirs_host, helm_c32* rhs, helm_c32* u_in);

/* Solve A_Hel x_q = rhs_q for q < B (B <= max_batch), x0 = 0, to
 * ||rhs - A x|| <= rtol ||rhs|| (true residual, evaluated in float-float).
 * rhs and x must not alias.  stats_host: B entries or NULL.
 * Returns HELM_NOT_CONVERGED if any RHS did not converge. */
int helm_solve_batch(helm_ctx* ctx, int B, const helm_c32* rhs, helm_c32* x, helm_stats* stats_host);

/* Low-order part of the float-float iterate of the last solve on ctx:
 * the returned complex64 field x is x_hi, and x_hi + x_lo is the iterate whose
 * residual helm_stats.rel_res_true reports (the complex64 rounding of the
 * exact solution alone leaves a relative residual of order 1e-6..1e-5, so
 * x_lo is what certifies tolerances near 1e-6).  For an adjoint solve the
 * conjugation is applied.  x_lo: device [B][grid], B <= the last call's B. */
int helm_solution_lo(helm_ctx* ctx, int B, helm_c32* x_lo);

/* Adjoint solves A_Hel^H lam_q = rhs_q.  A_Hel is complex symmetric (the
 * Sommerfeld terms only touch the diagonal), so lam = conj(A^-1 conj(rhs)):
 * the forward solver with conjugated input and output. */
int helm_adjoint_batch(helm_ctx* ctx, int B, const helm_c32* rhs, helm_c32* lam, helm_stats* stats_host);

/* Refractive-index gradient of a real loss through Prop. 1 (Sec. V):
 *   grad_n[i] = sum_q 2 k0^2 eta_i Re(conj(u_q,i) lam_q,i) on Omega,
 * with u_q = u_in,q + u_sc,q the TOTAL field and lam_q the adjoint states;
 * for the quadratic data term 1/2 ||S u_sc,q - y_q||^2 on receiver samples S,
 * lam_q = A^-H S^T (S u_sc,q - y_q).  u_in may be NULL (u_sc is then taken
 * as the total field).  grad_n: device float[n^dim] (overwritten, Omega). */
int helm_grad_n(helm_ctx* ctx, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* lam,
                float* grad_n);

/* Receiver sampling S of the data term (Sec. V, eq. DataFidelityExplicit,
 * with on-grid receivers): y[q][i] = u[q][idx[i]] for M receiver flat indices
 * idx_dev (device int[M], on the extended grid).  The indices are checked on
 * the host first: HELM_EINVAL (nothing launched) for one outside the grid. */
int helm_sample(helm_ctx* ctx, int B, int M, const int* idx_dev, const helm_c32* u, helm_c32* y);

/* S^T: u = 0 except u[q][idx[i]] = y[q][i].  HELM_EINVAL (nothing launched) for
 * an index outside the grid or a repeated index (S^T of repeated receivers would
 * need a sum, and this form writes each point once). */
int helm_sample_adjoint(helm_ctx* ctx, int B, int M, const int* idx_dev, const helm_c32* y, helm_c32* u);

/* Smoothed isotropic total variation of an interior map (the regulariser of
 * Sec. V, smoothed so that it is differentiable):
 *   TV = sum_i sqrt(sum_axis (n_{i+e_axis} - n_i)^2 + eps^2), forward
 * differences, zero difference across the last row/column/plane.
 * grad_dev (device float[n^dim], overwritten) = scale * dTV/dn;
 * value_host = TV (FP64 sum of FP32 per-block partial sums). */
int helm_tv(helm_ctx* ctx, const float* n_map_dev, double eps, double scale, float* grad_dev, double* value_host);

/* ---- building blocks, exposed for verification and custom solvers ---- */

/* y = A_Hel x (unscaled), complex64 arithmetic. */
int helm_apply_A(helm_ctx* ctx, int B, const helm_c32* x, helm_c32* y);

/* r = rhs - A_Hel x evaluated in float-float (compensated FP32) with x
 * given as x_hi + x_lo (x_lo may be NULL). */
int helm_residual(helm_ctx* ctx, int B, const helm_c32* rhs, const helm_c32* x_hi, const helm_c32* x_lo,
                  helm_c32* r);

/* y = K'_level x: the h_level^2-scaled shifted operator of multigrid level
 * `level` (0 = finest), fields on that level's grid [B][n_l]^dim. */
int helm_apply_K(helm_ctx* ctx, int level, int B, const helm_c32* x, helm_c32* y);

/* coarse = 4 R fine (full weighting, scaled coarse right-hand side) from
 * level `level` to level+1. */
int helm_restrict(helm_ctx* ctx, int level, int B, const helm_c32* fine, helm_c32* coarse);

/* fine += P coarse (bilinear/trilinear prolongation) from level+1 to level. */
int helm_prolong_add(helm_ctx* ctx, int level, int B, const helm_c32* coarse, helm_c32* fine);

/* z = K'_coarsest^-1 r on the coarsest grid (explicit inverse). */
int helm_coarse_solve(helm_ctx* ctx, int B, const helm_c32* r, helm_c32* z);

/* z = M^-1 r: one multigrid cycle from a zero initial guess for the
 * h^2-scaled fine system K'_0 z = r (the FGMRES preconditioner). */
int helm_precondition(helm_ctx* ctx, int B, const helm_c32* r, helm_c32* z);

/* ---- inverse problem (Sec. V, eq. MAPInverse with on-grid receivers S) ----
 * Unknown: the scattering potential f = k0^2 (eta^2 - eta_b^2) on Omega
 * (device float [n^dim], x fastest; k0 as given to helm_setup), f >= lo. */

/* Medium from f: eta = sqrt(eta_b^2 + f / k0^2) (0 where the radicand is
 * negative), then exactly helm_update_n. */
int helm_update_f(helm_ctx* ctx, const float* f_dev);

/* Data-fidelity gradient with respect to f through Prop. 1:
 *   grad_f[i] = sum_q Re(conj(u_q,i) lam_q,i) on Omega   (helm_grad_n without the
 * chain factor 2 k0^2 eta_i); arguments as for helm_grad_n. */
int helm_grad_f(helm_ctx* ctx, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* lam,
                float* grad_f);

/* Several frequencies (the paper's experimental reconstructions use four, Sec. VI-C) share
 * one frequency-independent unknown, the contrast chi = eta^2 - eta_b^2 on Omega, with
 * f = k0^2 chi in the context of each frequency (its own k0).
 * helm_update_contrast: medium eta = sqrt(eta_b^2 + chi) (0 where the radicand is
 * negative), then exactly helm_update_n.  chi: device float [n^dim]. */
int helm_update_contrast(helm_ctx* ctx, const float* chi_dev);
/* Data-fidelity gradient with respect to chi through Prop. 1 and df/dchi = k0^2:
 *   g[i] = k0^2 sum_q Re(conj(u_q,i) lam_q,i) on Omega,
 * written to grad (accumulate = 0) or added to it (accumulate = 1), so that the contexts
 * of several frequencies sum their gradients in one buffer; arguments as helm_grad_f. */
int helm_grad_contrast(helm_ctx* ctx, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* lam,
                       int accumulate, float* grad);

/* Residual of the quadratic data term (eq. DataFidelityExplicit) at M on-grid
 * receivers: res[q][i] = u[q][idx[i]] - y[q][i] for q < B (u: device [B][grid],
 * y, res: device [B][M]); *loss_host = 1/2 sum |res|^2 (FP64) when non-NULL.
 * idx (device int [M]) is checked on the host: HELM_EINVAL for an index
 * outside the grid. */
int helm_data_residual(helm_ctx* ctx, int B, int M, const int* idx_dev, const helm_c32* u, const helm_c32* y,
                       helm_c32* res, double* loss_host);

/* Allocation-free variant of helm_data_residual, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and arithmetic: res is identical and
 * *loss_host equal to helm_data_residual's (the same block partial sums, added in the
 * same order in FP64).  Its scratch (block partial sums, the total and an index-error
 * flag) is a fixed device array of 4128 doubles (33 KB) that each GPU holds from the
 * first context created on it until the process ends; no hipMalloc, hipFree or other
 * allocating call is made and no error message is copied.  The receiver indices are
 * checked on the device before any read through them: HELM_EINVAL for one outside the
 * grid (res then unwritten).  Limit: B * M <= HELM_STATIC_MAX_SAMPLES (one partial sum
 * per 256 samples), else HELM_EINVAL.  Every call on one GPU shares that GPU's array and
 * keeps the last call's contents: calls that overlap on one GPU (other streams, other
 * threads or contexts) race and must be serialised by the caller. */
#define HELM_STATIC_MAX_SAMPLES 1048576
int helm_data_residual_static(helm_ctx* ctx, int B, int M, const int* idx_dev, const helm_c32* u, const helm_c32* y,
                              helm_c32* res, double* loss_host);

/* Proximal operator of eq. proximalOpt with isotropic TV (forward
 * differences, zero across the last index of each axis) and a lower bound:
 *   w = argmin_{w >= lo} 1/2 ||w - v||^2 + lam TV(w),
 * by `iters` steps of fast gradient projection on the dual (the method the
 * paper names).  v, w: device float [n^dim], must not alias.  lam = 0 or
 * iters = 0 gives max(v, lo). */
int helm_tv_prox(helm_ctx* ctx, const float* v_dev, double lam, double lo, int iters, float* w_dev);

/* One update of Alg. 4 (accelerated forward-backward splitting) after its
 * gradient grad = sum over the selected illuminations of grad_f at fbar:
 *   f' = prox_{gamma tau}(fbar - gamma grad)  (helm_tv_prox with lower bound lo)
 *   alpha' = (1 + sqrt(1 + 4 alpha^2)) / 2
 *   fbar' = f' + (alpha - 1) / alpha' (f' - f)
 * f and fbar (device float [n^dim]) are updated in place; *alpha_host (>= 1,
 * 1 at the start) is advanced. */
int helm_fbs_step(helm_ctx* ctx, float* f_dev, float* fbar_dev, const float* grad_dev, double gamma, double tau,
                  double lo, int prox_iters, double* alpha_host);

/* ---- sensor operator G~ (eq. DiscreteForward / DiscreteForwardHelm) ----
 * Sensors outside Omega record the scattered field of the induced source
 * s = f u (u = u_in + u_sc the total field) through the Lippmann-Schwinger
 * integral (eq. LSIntegral) with the free-space Green's function (eq. green):
 *   y_m = sum_{z in Omega} g(x_m - z) f(z) u(z) h^d,
 *   g(x) = (j/4) H0^(1)(k0 eta_b |x|) in 2D,  e^{j k0 eta_b |x|} / (4 pi |x|) in 3D.
 * With these sensors the data term of eq. MAPInverse has the gradient (Prop. 1)
 *   grad_f = sum_q Re(conj(u_q) (s_q + lam_q)),  s_q = G~^H r_q,  lam_q = A^-H (f s_q),
 * r_q = y_q(f) - y_q^meas: helm_farfield_adjoint gives s_q and f s_q, helm_adjoint_batch
 * lam_q, helm_grad_f_farfield the sum. */

/* Sensor positions sensors_host[M][dim] (x, y[, z]) in grid cells relative to the
 * centre of Omega; each must lie at least one cell outside Omega (HELM_EINVAL).
 * Builds G~ [M][n^dim] on the device (2D: H0^(1) by cubic Hermite interpolation
 * in a host FP64 table of H0^(1) and H0^(1)' at spacing 1/256 in k_b r). */
int helm_farfield_set(helm_ctx* ctx, int M, const double* sensors_host);
/* y[q][m] (device [B][M]) for fields u_in, u_sc (device [B][grid]; u_in may be NULL:
 * u_sc is then the total field).  HELM_ESTATE without sensors. */
int helm_farfield(helm_ctx* ctx, int B, const helm_c32* u_in, const helm_c32* u_sc, helm_c32* y);
/* y = G~ f (u_in + u_sc) as helm_farfield, res = y - y_meas (device [B][M]) and
 * *loss_host = 1/2 sum |res|^2 (FP64) when non-NULL. */
int helm_farfield_residual(helm_ctx* ctx, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* y_meas,
                           helm_c32* y, helm_c32* res, double* loss_host);
/* s_ext = G~^H r on Omega, 0 in the layer (device [B][grid], overwritten); rhs_ext
 * (or NULL) = f s_ext, the right-hand side of the adjoint solve. r: device [B][M]. */
int helm_farfield_adjoint(helm_ctx* ctx, int B, const helm_c32* r, helm_c32* s_ext, helm_c32* rhs_ext);
/* grad_f[i] = sum_q Re(conj(u_in + u_sc) (lam + s_ext)) on Omega. */
int helm_grad_f_farfield(helm_ctx* ctx, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* lam,
                         const helm_c32* s_ext, float* grad_f);

/* ---- learned preconditioner (not part of the paper's method) ----
 * A 2D convolutional U-Net used as the FGMRES preconditioner in place of the
 * V-cycle: 4 levels with 16/32/64/64 channels, 3x3 convolutions (zero
 * padding), ReLU after every convolution but the last, 2x2 average pooling
 * (zero padding, output ceil(n/2)), nearest-neighbour upsampling and skip
 * concatenation; layers A0..A3 (encoder), B2, B1, B0 (decoder), O (output).
 * BF16 weights and activations with FP32 accumulation on the matrix cores,
 * FP32 master weights and Adam.  Inputs: 4 channels (Re, Im of the
 * normalised residual, Re, Im of the coefficient contrast (c - c_b) / c_b);
 * outputs: 2 channels (Re, Im of the normalised correction).
 * Tensors are FP32 NHWC [nimg][H][W][channels] device arrays. */

int helm_net_layers(void);                                 /* 8 */
int helm_net_layer_shape(int layer, int* cin, int* cout);  /* real channel counts of the 2D network */
/* He-normal initial weights from `seed`, zero biases; work runs on hip_stream. */
int helm_net_create(unsigned long long seed, void* hip_stream, helm_net** out);
/* The 3D network for 3D contexts: the same eight layers with 3x3x3 convolutions, channels
 * 16/16/32/32 (encoder A0..A3: 4->16, 16->16, 16->32, 32->32; decoder B2 64->32, B1 48->16,
 * B0 32->16; O 16->2), 2x2x2 average pooling (zero padding, output ceil(n/2) per axis),
 * nearest-neighbour upsampling; tensors NDHWC [nimg][D][H][W][channels].  Weights as host
 * float[3][3][3][cin][cout] (tap (dz+1, dy+1, dx+1)).  Not part of the paper (Sec. VII
 * names 3D as future work). */
int helm_net_create3(unsigned long long seed, void* hip_stream, helm_net** out);
int helm_net_dim(const helm_net* net);                                      /* 2 or 3 */
/* Convolution kernels: generic = 0 (default) runs each layer that has one on a kernel
 * specialised for its input channel count (the 2D network's forward layers but the
 * pooled 16-channel one; the 3D network's layers but A3 and B2), generic = 1
 * every layer on the channel-generic kernels.  Both compute the same sums in the same
 * order, so outputs agree bit for bit; the switch is for tests and measurements.
 * HELM_EINVAL for a generic value other than 0 or 1. */
int helm_net_set_conv_kernels(helm_net* net, int generic);
int helm_net_shape(const helm_net* net, int layer, int* cin, int* cout);   /* this network's channels */
void helm_net_destroy(helm_net* net);
const char* helm_net_last_error(const helm_net* net);
/* Weights as host float[3][3][cin][cout] (tap (dy+1, dx+1)) and bias float[cout]. */
int helm_net_set_layer(helm_net* net, int layer, const float* w_host, const float* b_host);
int helm_net_get_layer(helm_net* net, int layer, float* w_host, float* b_host);
/* Gradient of the last helm_net_backward, same layout. */
int helm_net_get_grad(helm_net* net, int layer, float* dw_host, float* db_host);
/* y = network(x): x [nimg][H][W][4], y [nimg][H][W][2]. */
int helm_net_forward(helm_net* net, int nimg, int H, int W, const float* x_dev, float* y_dev);
/* Loss 1/2 sum (y - target)^2 / nimg and its parameter gradients. */
int helm_net_backward(helm_net* net, int nimg, int H, int W, const float* x_dev, const float* target_dev,
                      double* loss_host);
/* The same three calls for a 3D network on volumes of D x H x W (HELM_EINVAL for a 2D network,
 * and the 2D calls refuse a 3D one); the residual term uses the 7-point operator
 * (6 - c) y - (sum of the 6 neighbours) with the one-voxel border left out. */
int helm_net_forward3(helm_net* net, int nimg, int D, int H, int W, const float* x_dev, float* y_dev);
int helm_net_backward3(helm_net* net, int nimg, int D, int H, int W, const float* x_dev, const float* target_dev,
                       double* loss_host);
int helm_net_residual_ratio3(helm_net* net, int nimg, int D, int H, int W, const float* x_dev, double gamma,
                             double cb, double* ratio_host);
/* Training loss of helm_net_backward, per image:
 *   err_weight / 2 sum (y - target)^2
 * + res_weight / 2 sum over the image interior |r - gamma A' y|^2,
 * with r = x[..0] + j x[..1], y read as complex, and A' the scaled 5-point
 * operator (4 - c) y - (sum of the 4 neighbours), c = cb (1 + x[..2] + j x[..3])
 * (the coefficient the features encode; cb = (k_b h)^2).  The one-pixel border
 * of every image is left out of the residual term.  Defaults: 1, 0.
 * Errors: HELM_EINVAL for negative weights or gamma, cb <= 0. */
int helm_net_set_loss(helm_net* net, double err_weight, double res_weight, double gamma, double cb);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the gradients of the last backward. */
int helm_net_adam_step(helm_net* net, double lr);

/* Learned preconditioner modes. */
#define HELM_NET_REPLACE 0 /* z_j = net(v_j); multigrid cycle where rejected */
#define HELM_NET_THEN_MG 1 /* z_j = net(v_j) + MG(v_j - A' net(v_j)); net term dropped where rejected */

/* Use `net` (NULL: multigrid only) in the preconditioner of ctx.  For basis
 * vector v_j (unit norm) the network sees sqrt(N) v_j and its output, times
 * gamma / sqrt(N), is z_net.  A right-hand side whose ||v_j - A' z_net|| >
 * accept_tol (or is not finite) drops the network output for that step and
 * uses the multigrid cycle alone (FGMRES allows a different preconditioner per
 * step; the per-RHS count is helm_stats.fallbacks).  HELM_NET_THEN_MG follows
 * the network with a multigrid cycle of its residual and needs two extra
 * [max_batch][N] work vectors, allocated here on first use.  The context
 * keeps the pointer (not owned); the activation buffers of its applications belong
 * to the context, so one network may serve several contexts.  Errors: HELM_EINVAL for
 * a network of another dimension than the grid, an unknown mode or gamma <= 0. */
int helm_set_preconditioner(helm_ctx* ctx, helm_net* net, double accept_tol, double gamma, int mode);

/* helm_solve_batch that also copies the iterate x_hi after every
 * `every_cycles` restart cycles into snaps_dev[k] (device [max_snaps][B][grid]);
 * *n_snaps = snapshots taken.  Used to build training pairs from the method's
 * own solves: the error of snapshot k is x_final - x_k, its residual b - A x_k. */
int helm_solve_snapshots(helm_ctx* ctx, int B, const helm_c32* rhs, helm_c32* x, helm_stats* stats_host,
                         int every_cycles, int max_snaps, helm_c32* snaps_dev, int* n_snaps);

/* Training examples from (residual r = b - A x_k, x_final, x_k) fields [B][grid]:
 * crop i = (rhs, y0, x0) from crops_host[3 i ..] (3D: (rhs, z0, y0, x0) from
 * crops_host[4 i ..]), S^dim points; features feat [ncrop][S]^dim[4] = (h^2 r / rms,
 * Re and Im of (c - c_b) / c_b), targets tgt [ncrop][S]^dim[2] = (x_final - x_k) / rms
 * / gamma, where rms is the root
 * mean square of h^2 r over the whole grid of that right-hand side (the scale
 * the solver gives the network: sqrt(N) times a unit-norm vector). */
int helm_net_examples(helm_ctx* ctx, int B, const helm_c32* r, const helm_c32* x_final, const helm_c32* x_k, int ncrop,
                      const int* crops_host, int S, double gamma, float* feat_dev, float* tgt_dev);

/* Root mean square of count FP32 values (device), sum of squares in FP64: the
 * normalisation of the training targets (gamma of helm_set_preconditioner). */
int helm_examples_rms(helm_ctx* ctx, const float* x_dev, long long count, double* rms_host);
/* x *= factor in place for count FP32 values (device): rescaling of example targets. */
int helm_examples_scale(helm_ctx* ctx, float* x_dev, long long count, double factor);

/* Per-image residual ratio of the network on examples x [nimg][H][W][4] (H, W >= 3):
 *   ratio_host[i] = ||r - gamma A' y||_2 / ||r||_2 over the image interior,
 * y = network(x), with r, c (from cb = (k_b h)^2) and A' as in the residual term of
 * helm_net_set_loss.  1 = no better than a zero correction.  Sums in FP64. */
int helm_net_residual_ratio(helm_net* net, int nimg, int H, int W, const float* x_dev, double gamma, double cb,
                            double* ratio_host);

/* Launch shapes chosen by helm_autotune. */
#define HELM_TUNE_MAX_LEVELS 12
typedef struct {
  int from_cache;                       /* 1: taken from the cache file, not re-timed */
  int levels;
  int down[HELM_TUNE_MAX_LEVELS][2];    /* fused down-leg tile per level: coarse TCX x TCY points */
  int up[HELM_TUNE_MAX_LEVELS][3];      /* fused up-leg tile per level: fine TX x TY, PY points per thread
                                           (PY 0: one column per lane, every fourth row) */
  long long coarse_max;                 /* levels with at most this many points run in one launch */
  double vcycle_ms;                     /* one preconditioner cycle for B right-hand sides, chosen shapes */
  double vcycle_default_ms;             /* ... with the default shapes (0 when from_cache) */
  int up_mv_rows;                       /* tile height of the fused finest up-leg + basis matvec (s-step form) */
  int up_mv_rhs_per_block;              /* ... and the right-hand sides one of its workgroups walks */
} helm_tune;

/* Autotuner of the batched multigrid cycle (the batching / launch-shape part of
 * the method's many-right-hand-side solves): times every tile shape of the
 * fused 2D down- and up-legs on each level with B right-hand sides, the tile
 * height of the s-step form's fused finest up-leg + basis matvec, then the
 * threshold below which the coarse levels run as one launch, and keeps the
 * fastest for the following solves of this context (results do not depend on
 * the shapes: every point is computed by the same arithmetic).  cache_path
 * (nullable) is a JSON-lines file keyed by GPU architecture, dimension, grid,
 * levels, B, smoothing steps and cycle type: a matching entry is applied
 * without timing, a new result is appended.  Uses the Krylov workspace as
 * scratch (do not call during a solve on the same context); invalidates the
 * captured graph.  Errors: HELM_EINVAL (B outside [1, max_batch]), HELM_EHIP. */
int helm_autotune(helm_ctx* ctx, int B, const char* cache_path, helm_tune* out_host);

/* ---- per-launch profiler (measurement support) ----
 * While enabled, every kernel launch of the context is bracketed by HIP events
 * on the context's stream (restart cycles are then launched one kernel at a
 * time instead of from the captured graph).  Entries are grouped by kernel
 * name (multigrid kernels per level, e.g. "up_fused_l0"); `bytes` is the
 * algorithmic HBM traffic of the launches (minimum reads + writes of the
 * fields and coefficients they touch, counted for the right-hand sides still
 * iterating at the start of each restart cycle). */
int helm_profile_enable(helm_ctx* ctx, int on);
int helm_profile_reset(helm_ctx* ctx);
int helm_profile_count(const helm_ctx* ctx);
int helm_profile_get(const helm_ctx* ctx, int i, char* name, int name_len, double* total_ms, long long* launches,
                     double* bytes);

/* Last error message of ctx (or of the last failed helm_setup if ctx is NULL). */
const char* helm_last_error(const helm_ctx* ctx);

void helm_destroy(helm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H */
