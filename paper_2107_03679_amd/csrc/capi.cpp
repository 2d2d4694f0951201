// C ABI of libhelm (declared in include/helm.h) and the host side of the
// batched solver: level hierarchy, multigrid-cycle orchestration (Alg. 2),
// the restarted FGMRES driver with a float-float outer iterate, and the
// per-restart-cycle hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/helm.h"
#include "kernels.h"
#include "net_internal.h"
#include "setup_host.h"

using helm_host::cd;

namespace {

thread_local std::string g_setup_error;

struct Level {
  int n = 0;
  long long N = 0;
  c32* kc = nullptr;    // kappa * c_l
  c32* kclo = nullptr;  // low part of kappa * c_l as float-float (the set-up's coarse chain)
  c32* wd = nullptr;    // omega / diag(K_kappa,l)
  c32 ghost{};
  c32* rc = nullptr;  // [maxB][N] right-hand side (levels >= 1)
  c32* e = nullptr;   // [maxB][N] solution (levels >= 1)
  c32* t = nullptr;   // [maxB][N] scratch of the generic path
  c32* rr = nullptr;  // [maxB][N] right-hand side of a repeated visit (b - K e)
  c32* d = nullptr;   // [maxB][N] correction of a repeated visit
};

struct HipError {
  hipError_t code;
  const char* what;
};

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{e, what};
}

c32 to_c32(cd v) { return make_float2((float)v.real(), (float)v.imag()); }

}  // namespace

struct helm_ctx {
  helm_grid grid{};
  helm_abl abl{};
  helm_opts o{};
  helm_host::Geometry geo{};
  int dim = 2, n = 0, w = 0, ne = 0, L = 0;
  double h = 0, k0 = 0, k0h = 0, kbh = 0;
  long long N0 = 0;
  hipStream_t s = nullptr;       // the context's own stream (graphs cannot capture the null stream)
  hipStream_t user_s = nullptr;  // the caller's stream: work starts after it
  std::string err;
  const char* err_lit = nullptr;  // message of the allocation-free entry point (no string copy)

  // fine-level data
  float* d_nmap = nullptr;   // interior index (for the gradient)
  float* d_f = nullptr;      // f = k0^2 (eta^2 - eta_b^2) on Omega_e (0 in the layer), unscaled
  c32* d_chi = nullptr;      // c = (k0 h)^2 eta^2 alpha, hi part
  c32* d_dhi = nullptr;      // diagonal of A' (with the Sommerfeld terms), float-float hi ...
  c32* d_dlo = nullptr;      // ... and lo part (the true residual)
  c32 g0_hi{};               // fine ghost factor 1 + j k_b h
  float h2_hi = 0, h2_lo = 0;
  std::vector<Level> lv;
  c32* d_minvT = nullptr;
  c32* d_cs_part = nullptr;  // slice partials of the coarsest solve as a matrix product
  int Nc = 0;

  // Krylov workspace
  KrylovArgs k{};
  c32* d_xhi = nullptr;  // internal x (hi), [maxB][N0]
  c32* d_xlo = nullptr;  // internal x (lo)
  c32* d_xhi2 = nullptr;  // the second buffer of the iterate pair (2D: the fused update alternates)
  c32* d_xlo2 = nullptr;
  int* d_xpar = nullptr;  // [maxB] which buffer holds each right-hand side's x
  c32* d_rhs = nullptr;  // internal copy of the right-hand sides
  c32* d_T0 = nullptr;   // generic-path scratch on the fine level
  c32* d_tables = nullptr;
  int* d_ones = nullptr;
  int* d_zero_ints = nullptr;
  float* d_tv_mag = nullptr;   // [n^dim] TV magnitudes
  float* d_tv_part = nullptr;  // per-block TV partial sums
  double2* d_gram = nullptr;   // [maxB][nblk][(m+1)(m+2)/2] Gram partials of the s-step form
  // inverse-problem workspace (allocated on first use): FGP dual p and its
  // extrapolation r [dim][n^dim], primal w, prox input v, index map from f
  float* d_inv_p = nullptr;
  float* d_inv_r = nullptr;
  float* d_inv_w = nullptr;
  float* d_inv_v = nullptr;
  float* d_inv_n = nullptr;
  double* d_inv_part = nullptr;
  int inv_part_len = 0;
  // sensor operator G~ [M][n^dim] and its work buffers (helm_farfield_set)
  int ff_M = 0;
  c32* d_ffG = nullptr;
  c32* d_ff_src = nullptr;   // [maxB][n^dim] induced source
  c32* d_ff_part = nullptr;  // [splits][maxB][M]
  int ff_active_M = 0;       // sensors of the current set
  int* d_ff_iota = nullptr;  // 0 .. M-1 (the data residual of helm_farfield_residual)
  int* h_status = nullptr;  // pinned
  int* h_iters = nullptr;
  double* h_relres = nullptr;
  size_t bytes = 0;
  std::vector<void*> allocs;

  hipGraphExec_t graph = nullptr;
  int graph_B = 0;
  hipEvent_t ev_solve[2] = {nullptr, nullptr};  // bracket of a solve call (helm_stats.ms)

  // launch shapes (helm_autotune): fused-leg tile per level, single-launch coarse threshold
  int tune_down[HELM_MAX_LEVELS] = {0};
  int tune_up[HELM_MAX_LEVELS] = {0};
  int tune_mv = 0;  // launch-shape variant (rows, right-hand sides per block) of the fused finest up-leg + matvec
  long long coarse_max = -1;  // points; -1: default (48^2 in 2D, 16^3 in 3D), 0: never

  // learned preconditioner (NULL: multigrid only)
  helm_net* net = nullptr;
  NetSolveBufs* net_bufs = nullptr;  // this context's activation buffers of the network (owned)
  double accept_tol = 0.9;
  double net_gamma = 1.0;
  int net_mode = HELM_NET_REPLACE;
  c32* d_net_res = nullptr;    // [maxB][N0] v_j - A' z_net (HELM_NET_THEN_MG)
  c32* d_net_cor = nullptr;    // [maxB][N0] multigrid correction of that residual
  int* d_mg_mask = nullptr;    // [maxB] RHS whose learned output was rejected
  int* d_fallbacks = nullptr;  // [maxB] rejections during the current solve
  int* h_fallbacks = nullptr;  // pinned

  // opt-in per-launch profiler (HIP events on the context stream, no graph replay while on)
  struct ProfEntry {
    std::string name;
    double ms = 0.0, bytes = 0.0;
    long long launches = 0;
  };
  struct Pending {
    int idx;
    hipEvent_t e0, e1;
    double bytes;
  };
  bool prof_on = false;
  int prof_B = 0;  // right-hand sides still iterating (algorithmic byte model)
  std::vector<ProfEntry> prof;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  int last_B = 0;
  int last_conj = 0;

  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    check(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)), "hipMalloc");
    allocs.push_back(p);
    bytes += count * sizeof(T);
    return (T*)p;
  }
};

namespace {

LevelArgs fine_A(const helm_ctx* c) { return LevelArgs{c->ne, c->N0, c->d_chi, c->g0_hi, nullptr}; }
LevelArgs level_K(const helm_ctx* c, int l) {
  return LevelArgs{c->lv[l].n, c->lv[l].N, c->lv[l].kc, c->lv[l].ghost, c->lv[l].wd};
}

long long npts(int n, int dim) { return dim == 2 ? (long long)n * n : (long long)n * n * n; }

hipEvent_t prof_event(helm_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

// Times the launches made in its scope when profiling is on.
struct ProfScope {
  helm_ctx* c;
  int idx = -1;
  hipEvent_t e0 = nullptr;
  double bytes;
  ProfScope(helm_ctx* ctx, const std::string& name, double b) : c(ctx), bytes(b) {
    if (!c->prof_on) return;
    for (size_t i = 0; i < c->prof.size(); ++i)
      if (c->prof[i].name == name) idx = (int)i;
    if (idx < 0) {
      c->prof.push_back({name});
      idx = (int)c->prof.size() - 1;
    }
    e0 = prof_event(c);
    check(hipEventRecord(e0, c->s), "hipEventRecord");
  }
  ~ProfScope() {
    if (idx < 0) return;
    hipEvent_t e1 = prof_event(c);
    if (hipEventRecord(e1, c->s) == hipSuccess) c->pending.push_back({idx, e0, e1, bytes});
  }
};

// Accumulate the finished event pairs (after a stream synchronisation).
void prof_resolve(helm_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      c->prof[p.idx].ms += ms;
      c->prof[p.idx].bytes += p.bytes;
      c->prof[p.idx].launches += 1;
    }
    c->event_pool.push_back(p.e0);
    c->event_pool.push_back(p.e1);
  }
  c->pending.clear();
}

std::string lvl_name(const char* base, int l) { return std::string(base) + "_l" + std::to_string(l); }

// Copy B vectors of N elements between two strided vector sets.
void copy_set(helm_ctx* c, int B, VecSet src, VecSet dst, long long N) {
  check(hipMemcpy2DAsync(dst.p, dst.stride * sizeof(c32), src.p, src.stride * sizeof(c32), N * sizeof(c32), B,
                         hipMemcpyDeviceToDevice, c->s),
        "hipMemcpy2DAsync");
}

// nu Jacobi sweeps on level l: v <- v + w D^-1 (r - K v), ping-ponging through the level scratch.
void relax(helm_ctx* c, int B, int l, VecSet r, ScaleSet rs, VecSet v, int sweeps, const int* act) {
  const Level& L = c->lv[l];
  VecSet t{l == 0 ? c->d_T0 : L.t, L.N};
  for (int i = 0; i < sweeps; ++i) {
    {
      ProfScope ps(c, lvl_name("jacobi", l), c->prof_B * 24.0 * L.N + 8.0 * L.N);
      launch_jacobi(c->s, c->dim, B, r, rs, level_K(c, l), (float)c->o.omega_jac, v, t, act);
    }
    ProfScope ps(c, lvl_name("copy", l), c->prof_B * 16.0 * L.N);
    copy_set(c, B, t, v, L.N);
  }
}

long long coarse_small(const helm_ctx* c) {
  return c->coarse_max >= 0 ? c->coarse_max : (c->dim == 2 ? 48LL * 48 : 16LL * 16 * 16);
}

// True when a zero-guess visit of level l on the level's own (unscaled) buffers
// runs the fused 2D legs (not the coarsest solve, not the single-launch coarse
// cycle); repeated visits from a nonzero start use them.  The fused 3D legs take
// zero-guess visits only.
bool legs_fused(const helm_ctx* c, int l) {
  if (l >= c->L - 1 || !c->o.fused || c->dim != 2 || c->o.nu1 != 1 || c->o.nu2 != 1) return false;
  const bool v_below = c->o.cycle == 1 || c->o.cycle == 3;
  const bool single = v_below && l >= 1 && c->o.coarse_single_launch && c->lv[l].N <= coarse_small(c);
  return !single;
}

// True when a zero-guess visit of level l on the level's own buffers runs the fused
// 3D legs (not the coarsest solve, not the single-launch coarse cycle), whose up-leg
// can add its result to the output (a repeated visit without a separate add pass).
bool legs3_fused(const helm_ctx* c, int l) {
  if (l >= c->L - 1 || !c->o.fused || c->dim != 3 || c->o.nu1 != 1 || c->o.nu2 != 1) return false;
  const bool v_below = c->o.cycle == 1 || c->o.cycle == 3;
  return !(v_below && l >= 1 && c->o.coarse_single_launch && c->lv[l].N <= coarse_small(c));
}

void mg_cycle(helm_ctx* c, int B, int l, VecSet r, ScaleSet rs, VecSet out, bool zero_guess, const int* act,
              VecSet eres = VecSet{nullptr, 0}, bool accumulate = false);

// The coarse-grid corrections of one visit of level l (Alg. 2's CycleType; for
// cycle = 3 two on the finest level and one below), from the right-hand side
// already restricted into level l + 1's rc.  Returns the buffer that holds the
// coarse solution afterwards (e or d of level l + 1).
VecSet coarse_visits(helm_ctx* c, int B, int l, const int* act) {
  const int gamma = c->o.cycle == 3 ? (l == 0 ? 2 : 1) : c->o.cycle;
  Level& crs = c->lv[l + 1];
  VecSet rc{crs.rc, crs.N}, ec{crs.e, crs.N};
  const double Nc1 = (double)crs.N, Bp = c->prof_B;
  const bool next_is_coarsest = (l + 1 == c->L - 1);
  VecSet ecur = ec;
  for (int cyc = 0; cyc < gamma; ++cyc) {
    if (cyc == 0) {
      mg_cycle(c, B, l + 1, rc, ScaleSet{nullptr, 0}, ec, true, act);
      continue;
    }
    if (next_is_coarsest) break;  // a repeated exact solve of the same system is idempotent
    // repeated visit from the current e: MG(rc, e) = e + MG(rc - K e, 0)
    VecSet other{ecur.p == crs.e ? crs.d : crs.e, crs.N};
    if (legs_fused(c, l + 1)) {
      mg_cycle(c, B, l + 1, rc, ScaleSet{nullptr, 0}, other, true, act, ecur);
      ecur = other;
      continue;
    }
    VecSet rr{crs.rr, crs.N};
    {
      ProfScope ps(c, lvl_name("level_residual", l + 1), Bp * 24.0 * Nc1 + 8.0 * Nc1);
      launch_level_residual(c->s, c->dim, B, rc, ecur, level_K(c, l + 1), rr, act);
    }
    if (legs3_fused(c, l + 1)) {  // the up-leg adds MG(r - K e, 0) to e in place
      mg_cycle(c, B, l + 1, rr, ScaleSet{nullptr, 0}, ecur, true, act, VecSet{nullptr, 0}, true);
      continue;
    }
    mg_cycle(c, B, l + 1, rr, ScaleSet{nullptr, 0}, other, true, act);
    ProfScope ps(c, lvl_name("add", l + 1), Bp * 24.0 * Nc1);
    launch_add(c->s, B, other, ecur, crs.N, act);
  }
  return ecur;
}

// Alg. 2 on level l for K'_l v = r, result in `out` (which holds the initial
// guess when zero_guess is false).  Fused 2D legs serve the common case.
// With eres.p set (only where legs_fused(l)), the visit starts from the
// solution eres instead: out = eres + MG(r - K eres, 0), the residual formed
// inside the legs; out must not alias eres.  With accumulate (only where
// legs3_fused(l)), out += MG(r, 0).
void mg_cycle(helm_ctx* c, int B, int l, VecSet r, ScaleSet rs, VecSet out, bool zero_guess, const int* act,
              VecSet eres, bool accumulate) {
  const int dim = c->dim;
  if (l == c->L - 1) {  // coarsest: exact solve (the guess is irrelevant)
    ProfScope ps(c, "coarse_solve", 8.0 * c->Nc * c->Nc + c->prof_B * 16.0 * c->Nc);
    launch_coarse_solve(c->s, B, c->d_minvT, c->Nc, r, out, act, c->d_cs_part);
    return;
  }
  Level& fine = c->lv[l];
  const bool v_below = c->o.cycle == 1 || c->o.cycle == 3;
  const bool vcycle11 = c->o.fused && zero_guess && v_below && c->o.nu1 == 1 && c->o.nu2 == 1;
  const long long small = coarse_small(c);
  if (vcycle11 && l >= 1 && c->o.coarse_single_launch && fine.N <= small && rs.p == nullptr && r.stride == fine.N &&
      out.stride == fine.N && eres.p == nullptr && !accumulate) {
    // levels l .. L-1 in one launch, one workgroup per right-hand side
    CoarseCycleArgs a{};
    a.dim = dim;
    a.lp = l;
    a.L = c->L;
    a.omega = (float)c->o.omega_jac;
    a.minvT = c->d_minvT;
    a.active = act;
    double by = 8.0 * c->Nc * c->Nc;
    for (int q = l; q < c->L; ++q) {
      const Level& Lq = c->lv[q];
      a.lv[q] = CoarseLevel{Lq.n, Lq.N, Lq.wd, Lq.rc, Lq.e, Lq.t};
      by += c->prof_B * 40.0 * Lq.N + 8.0 * Lq.N;
    }
    a.lv[l].rc = r.p;  // this visit's right-hand side and result buffers
    a.lv[l].e = out.p;
    ProfScope ps(c, lvl_name("coarse_cycle", l), by);
    launch_coarse_cycle(c->s, B, a);
    return;
  }
  Level& crs = c->lv[l + 1];
  VecSet rc{crs.rc, crs.N}, ec{crs.e, crs.N};
  const float om = (float)c->o.omega_jac;
  const bool fused = c->o.fused && zero_guess && c->o.nu1 == 1 && c->o.nu2 == 1;
  const double Nf = (double)fine.N, Nc1 = (double)crs.N, Bp = c->prof_B;
  if (eres.p && (!fused || dim != 2)) throw HipError{hipErrorInvalidValue, "repeated visit outside the fused 2D legs"};
  if (accumulate && !(fused && dim == 3))
    throw HipError{hipErrorInvalidValue, "accumulating visit outside the fused 3D legs"};
  if (fused && dim == 3) {
    ProfScope ps(c, lvl_name("down_fused", l), Bp * 8.0 * (Nf + Nc1) + 8.0 * Nf);
    launch_down_fused3(c->s, B, r, rs, level_K(c, l), om, rc, crs.n, act);
  } else if (fused && eres.p) {
    ProfScope ps(c, lvl_name("down_fused_res", l), Bp * 8.0 * (2.0 * Nf + Nc1) + 16.0 * Nf);
    launch_down_fused2(c->s, B, r, rs, level_K(c, l), om, rc, crs.n, act, c->tune_down[l], eres);
  } else if (fused) {
    ProfScope ps(c, lvl_name("down_fused", l), Bp * 8.0 * (Nf + Nc1) + 8.0 * Nf);
    launch_down_fused2(c->s, B, r, rs, level_K(c, l), om, rc, crs.n, act, c->tune_down[l]);
  } else {
    int sweeps = c->o.nu1;
    if (zero_guess) {
      ProfScope ps(c, lvl_name("jacobi_zero", l), Bp * 16.0 * Nf + 8.0 * Nf);
      if (sweeps > 0) {
        launch_jacobi_zero(c->s, dim, B, r, rs, level_K(c, l), om, out, act);
        --sweeps;
      } else {
        launch_jacobi_zero(c->s, dim, B, r, rs, level_K(c, l), 0.0f, out, act);  // out = 0
      }
    }
    relax(c, B, l, r, rs, out, sweeps, act);
    // residual once per fine point into the level scratch, then a plain full weighting
    const VecSet t{l == 0 ? c->d_T0 : fine.t, fine.N};
    {
      ProfScope ps(c, lvl_name("level_residual", l), Bp * 24.0 * Nf + 8.0 * Nf);
      launch_level_residual(c->s, dim, B, r, out, level_K(c, l), t, act, rs);
    }
    ProfScope ps(c, lvl_name("restrict", l), Bp * (8.0 * Nf + 8.0 * Nc1));
    launch_restrict_residual(c->s, dim, B, t, ScaleSet{nullptr, 0}, VecSet{nullptr, 0}, level_K(c, l), rc, crs.n,
                             act);
  }
  const VecSet ecur = coarse_visits(c, B, l, act);
  if (fused && dim == 3) {
    ProfScope ps(c, lvl_name(accumulate ? "up_fused_acc" : "up_fused", l),
                 Bp * 8.0 * ((accumulate ? 3.0 : 2.0) * Nf + Nc1) + 8.0 * Nf);
    launch_up_fused3(c->s, B, r, rs, level_K(c, l), om, ecur, crs.n, out, act, accumulate ? 1 : 0);
  } else if (fused && eres.p) {
    ProfScope ps(c, lvl_name("up_fused_res", l), Bp * 8.0 * (3.0 * Nf + Nc1) + 16.0 * Nf);
    launch_up_fused2(c->s, B, r, rs, level_K(c, l), om, ecur, crs.n, out, act, c->tune_up[l], eres);
  } else if (fused) {
    ProfScope ps(c, lvl_name("up_fused", l), Bp * 8.0 * (2.0 * Nf + Nc1) + 8.0 * Nf);
    launch_up_fused2(c->s, B, r, rs, level_K(c, l), om, ecur, crs.n, out, act, c->tune_up[l]);
  } else if (c->o.nu2 > 0) {
    // prolongation into the scratch, so that the first post-smoothing sweep writes `out` directly
    const VecSet t{l == 0 ? c->d_T0 : fine.t, fine.N};
    {
      ProfScope ps(c, lvl_name("prolong_add", l), Bp * (16.0 * Nf + 8.0 * Nc1));
      launch_prolong_add(c->s, dim, B, ecur, crs.n, out, fine.n, act, t);
    }
    {
      ProfScope ps(c, lvl_name("jacobi", l), Bp * 24.0 * Nf + 8.0 * Nf);
      launch_jacobi(c->s, dim, B, r, rs, level_K(c, l), (float)c->o.omega_jac, t, out, act);
    }
    relax(c, B, l, r, rs, out, c->o.nu2 - 1, act);
  } else {
    ProfScope ps(c, lvl_name("prolong_add", l), Bp * (16.0 * Nf + 8.0 * Nc1));
    launch_prolong_add(c->s, dim, B, ecur, crs.n, out, fine.n, act);
  }
}

// One Arnoldi step j for all active right-hand sides.
void arnoldi_step(helm_ctx* c, int B, int j) {
  KrylovArgs& k = c->k;
  const long long N0 = c->N0;
  VecSet vj{k.V + (long long)j * N0, (long long)(k.m + 1) * N0};
  VecSet zj{k.Z + (long long)j * N0, (long long)k.m * N0};
  ScaleSet sj{k.vs + j, k.m + 1};
  const LevelArgs A = fine_A(c);
  if (c->net) {
    // z_j = network(v_j); RHS whose output fails ||v_j - A z_j|| <= tol ||v_j|| fall back to the V-cycle
    const double rootN = std::sqrt((double)N0);
    const c32 cb = make_float2((float)(c->kbh * c->kbh), 0.0f);
    {
      ProfScope ps(c, "net_apply", 0.0);
      check(net_apply(c->net, c->net_bufs, c->s, B, c->ne, vj.p, vj.stride, sj.p, sj.stride, (float)rootN,
                      c->d_chi, cb, (float)(c->net_gamma / rootN), zj.p, zj.stride, k.active),
            "network buffers do not fit this batch");
    }
    if (c->net_mode == HELM_NET_REPLACE) {
      {
        ProfScope ps(c, "accept", c->prof_B * 16.0 * N0);
        launch_accept(c->s, B, k, j, A, c->accept_tol, c->d_mg_mask, c->d_fallbacks, VecSet{nullptr, 0});
      }
      mg_cycle(c, B, 0, vj, sj, zj, true, c->d_mg_mask);
    } else {
      // z_j = z_net + MG(v_j - A' z_net), with z_net = 0 where the network output was rejected
      const VecSet res{c->d_net_res, N0}, cor{c->d_net_cor, N0};
      {
        ProfScope ps(c, "accept", c->prof_B * 24.0 * N0);
        launch_accept(c->s, B, k, j, A, c->accept_tol, c->d_mg_mask, c->d_fallbacks, res);
      }
      launch_reject_reset(c->s, B, k, j, c->d_mg_mask, res);
      mg_cycle(c, B, 0, res, ScaleSet{nullptr, 0}, cor, true, k.active);
      ProfScope ps(c, "add", c->prof_B * 24.0 * N0);
      launch_add(c->s, B, cor, zj, N0, k.active);
    }
  } else {
    mg_cycle(c, B, 0, vj, sj, zj, true, k.active);
  }
  const double Bp = c->prof_B, N = (double)N0, nv = j + 1.0;
  const double red_bytes = Bp * k.nblk * nv * 8.0;
  {
    ProfScope ps(c, "arnoldi_matvec_dots", Bp * (16.0 + 8.0 * nv) * N + 8.0 * N);
    launch_arnoldi_dots(c->s, B, k, j, &A, 1);
  }
  {
    ProfScope ps(c, "arnoldi_reduce", red_bytes);
    launch_arnoldi_reduce(c->s, B, k, j, 0);
  }
  {
    ProfScope ps(c, "arnoldi_update", Bp * (16.0 + 8.0 * nv) * N);
    launch_arnoldi_update(c->s, B, k, j);
  }
  if (c->o.reorth) {
    {
      ProfScope ps(c, "arnoldi_dots_reorth", Bp * (8.0 + 8.0 * nv) * N);
      launch_arnoldi_dots(c->s, B, k, j, &A, 0);
    }
    {
      ProfScope ps(c, "arnoldi_reduce", red_bytes);
      launch_arnoldi_reduce(c->s, B, k, j, 1);
    }
    ProfScope ps(c, "arnoldi_update", Bp * (16.0 + 8.0 * nv) * N);
    launch_arnoldi_update(c->s, B, k, j);
  }
  ProfScope ps(c, "givens", Bp * k.nblk * 4.0);
  launch_givens(c->s, B, k, j);
}

bool use_bicg(const helm_ctx* c) { return c->o.krylov == HELM_KRYLOV_BICGSTAB && c->net == nullptr; }

// The true residual of x (with fused_update on a 2D grid: the x update of the
// cycle and the residual in one pass), then the convergence decision.
void true_residual(helm_ctx* c, int B, int first, int conj_rhs, bool fused_update = false) {
  KrylovArgs& k = c->k;
  k.bicg = use_bicg(c) ? 1 : 0;
  if (fused_update) {
    ProfScope ps(c, "x_update_residual", c->prof_B * (8.0 * k.m + 48.0) * c->N0 + 16.0 * c->N0);
    launch_x_update_residual(c->s, B, k, XPair{c->d_xhi, c->d_xlo}, XPair{c->d_xhi2, c->d_xlo2}, c->d_rhs, c->N0,
                             conj_rhs, c->d_dhi, c->d_dlo, c->h2_hi, c->h2_lo, k.V, (long long)(k.m + 1) * c->N0);
    k.nres = krylov_xres_tiles(k.n);
    k.flip_x = 1;
  } else {
    ProfScope ps(c, "residual_ff", c->prof_B * (first ? 16.0 : 32.0) * c->N0 + (first ? 0.0 : 16.0 * c->N0));
    launch_residual_ff(c->s, B, k, c->d_rhs, c->N0, conj_rhs, c->d_xhi, c->d_xlo, first, c->d_dhi, c->d_dlo,
                       c->h2_hi, c->h2_lo, k.V, (long long)(k.m + 1) * c->N0, 1.0f);
    k.nres = krylov_residual_partials(k, first);
  }
  {
    ProfScope ps(c, "finalize", c->prof_B * k.nres * 4.0);
    if (k.bicg) launch_bicg_finalize(c->s, B, k, first);
    else launch_finalize(c->s, B, k, first);
  }
  k.nres = k.nblk;
  k.flip_x = 0;
}

// `restart` Bi-CGSTAB iterations (Alg. 3), two multigrid cycles each; the
// solution is updated inside the iteration.
void bicg_iterations(helm_ctx* c, int B) {
  KrylovArgs& k = c->k;
  const long long N0 = c->N0;
  const LevelArgs A = fine_A(c);
  const double Bp = c->prof_B, N = (double)N0;
  const long long vst = (long long)(k.m + 1) * N0, zst = (long long)k.m * N0;
  for (int it = 0; it < k.m; ++it) {
    {
      ProfScope ps(c, "bicg_dir", Bp * 32.0 * N);
      launch_bicg_dir(c->s, B, k);
    }
    mg_cycle(c, B, 0, VecSet{k.V + 2 * N0, vst}, ScaleSet{nullptr, 0}, VecSet{k.Z, zst}, true, k.active);
    {
      ProfScope ps(c, "bicg_apply", Bp * 24.0 * N + 8.0 * N);
      launch_bicg_apply(c->s, B, k, 0, 3, A, 0);
    }
    launch_bicg_alpha(c->s, B, k);
    {
      ProfScope ps(c, "bicg_s", Bp * 24.0 * N);
      launch_bicg_s(c->s, B, k);
    }
    mg_cycle(c, B, 0, VecSet{k.V, vst}, ScaleSet{nullptr, 0}, VecSet{k.Z + N0, zst}, true, k.active);
    {
      ProfScope ps(c, "bicg_apply", Bp * 24.0 * N + 8.0 * N);
      launch_bicg_apply(c->s, B, k, 1, 4, A, 1);
    }
    launch_bicg_sigma(c->s, B, k);
    {
      ProfScope ps(c, "bicg_update", Bp * 72.0 * N);
      launch_bicg_update(c->s, B, k, c->d_xhi, c->d_xlo);
    }
    launch_bicg_rho(c->s, B, k);
  }
}

// One cycle of GMRES(m) in s-step form: m multigrid cycles and matvecs build
// the basis, one Gram pass and a per-RHS Cholesky-QR least squares replace
// the Arnoldi orthogonalisation.
void sstep_basis(helm_ctx* c, int B) {
  KrylovArgs& k = c->k;
  const long long N0 = c->N0;
  const LevelArgs A = fine_A(c);
  const double Bp = c->prof_B, N = (double)N0;
  if (c->o.fused_step == 2 && c->dim == 2 && legs_fused(c, 0)) {
    // finest level: per step a down-leg, the coarse visits and the up-leg of Z_j
    // fused with W_{j+1} = A Z_j (the last matvec is the Gram kernel's)
    const Level& L1 = c->lv[1];
    const VecSet rc{L1.rc, L1.N};
    const float om = (float)c->o.omega_jac;
    const double Nc1 = (double)L1.N;
    for (int j = 0; j < k.m; ++j) {
      const VecSet vj{k.V + (long long)j * N0, (long long)(k.m + 1) * N0};
      const VecSet zj{k.Z + (long long)j * N0, (long long)k.m * N0};
      const ScaleSet sj{k.vs + j, k.m + 1};
      {
        ProfScope ps(c, "down_fused_l0", Bp * 8.0 * (N + Nc1) + 8.0 * N);
        launch_down_fused2(c->s, B, vj, sj, level_K(c, 0), om, rc, L1.n, k.active, c->tune_down[0]);
      }
      const VecSet ecur = coarse_visits(c, B, 0, k.active);
      if (j + 1 < k.m) {
        const VecSet vn{k.V + (long long)(j + 1) * N0, (long long)(k.m + 1) * N0};
        ProfScope ps(c, "up_mv_l0", Bp * 8.0 * (3.0 * N + Nc1) + 16.0 * N);
        launch_up_mv2(c->s, B, vj, sj, level_K(c, 0), A, om, ecur, L1.n, zj, vn, k.active, c->tune_mv);
      } else {
        ProfScope ps(c, "up_fused_l0", Bp * 8.0 * (2.0 * N + Nc1) + 8.0 * N);
        launch_up_fused2(c->s, B, vj, sj, level_K(c, 0), om, ecur, L1.n, zj, k.active, c->tune_up[0]);
      }
    }
    ProfScope ps(c, "sstep_gram", Bp * 8.0 * (k.m + 1.0) * N + 8.0 * N);
    launch_sstep_gram_solve(c->s, B, k, A, c->d_gram);
    return;
  }
  if (c->o.fused_step == 1 && c->dim == 2 && legs_fused(c, 0)) {
    // finest level: one down-leg, then per step the coarse visits and one fused
    // kernel (up-leg of Z_j, W_{j+1} = A Z_j, down-leg of W_{j+1}); the last up-leg alone
    const Level& L1 = c->lv[1];
    const VecSet rc{L1.rc, L1.N};
    const float om = (float)c->o.omega_jac;
    const double Nc1 = (double)L1.N;
    const VecSet v0{k.V, (long long)(k.m + 1) * N0};
    {
      ProfScope ps(c, "down_fused_l0", Bp * 8.0 * (N + Nc1) + 8.0 * N);
      launch_down_fused2(c->s, B, v0, ScaleSet{k.vs, k.m + 1}, level_K(c, 0), om, rc, L1.n, k.active,
                         c->tune_down[0]);
    }
    for (int j = 0; j < k.m; ++j) {
      const VecSet vj{k.V + (long long)j * N0, (long long)(k.m + 1) * N0};
      const VecSet zj{k.Z + (long long)j * N0, (long long)k.m * N0};
      const ScaleSet sj{k.vs + j, k.m + 1};
      const VecSet ecur = coarse_visits(c, B, 0, k.active);
      if (j + 1 < k.m) {
        const VecSet vn{k.V + (long long)(j + 1) * N0, (long long)(k.m + 1) * N0};
        ProfScope ps(c, "step_fused_l0", Bp * (28.0 * N + 4.0 * Nc1) + 16.0 * N);
        launch_step_fused2(c->s, B, vj, sj, level_K(c, 0), A, om, ecur, L1.n, zj, vn, rc, k.active);
      } else {
        ProfScope ps(c, "up_fused_l0", Bp * 8.0 * (2.0 * N + Nc1) + 8.0 * N);
        launch_up_fused2(c->s, B, vj, sj, level_K(c, 0), om, ecur, L1.n, zj, k.active, c->tune_up[0]);
      }
    }
    ProfScope ps(c, "sstep_gram", Bp * 8.0 * (k.m + 1.0) * N + 8.0 * N);
    launch_sstep_gram_solve(c->s, B, k, A, c->d_gram);
    return;
  }
  for (int j = 0; j < k.m; ++j) {
    VecSet vj{k.V + (long long)j * N0, (long long)(k.m + 1) * N0};
    VecSet zj{k.Z + (long long)j * N0, (long long)k.m * N0};
    mg_cycle(c, B, 0, vj, ScaleSet{k.vs + j, k.m + 1}, zj, true, k.active);
    if (j + 1 < k.m) {
      ProfScope ps(c, "sstep_matvec", Bp * 16.0 * N + 8.0 * N);
      launch_sstep_matvec(c->s, B, k, j, A);
    }
  }
  ProfScope ps(c, "sstep_gram", Bp * 8.0 * (k.m + 1.0) * N + 8.0 * N);
  launch_sstep_gram_solve(c->s, B, k, A, c->d_gram);
}

bool use_sstep(const helm_ctx* c) { return c->o.krylov == HELM_KRYLOV_SSTEP && c->net == nullptr; }

// The body of one restart cycle: m Arnoldi steps (or the s-step basis and its
// least squares), x update, true residual, decision.
void restart_cycle(helm_ctx* c, int B, int conj_rhs) {
  if (use_bicg(c)) {
    bicg_iterations(c, B);
    true_residual(c, B, 0, conj_rhs);
    return;
  }
  if (use_sstep(c)) sstep_basis(c, B);
  else
    for (int j = 0; j < c->k.m; ++j) arnoldi_step(c, B, j);
  if (c->dim == 2) {
    true_residual(c, B, 0, conj_rhs, true);
    return;
  }
  {
    ProfScope ps(c, "x_update", c->prof_B * (8.0 * c->k.m + 32.0) * c->N0);
    launch_x_update(c->s, B, c->k, c->d_xhi, c->d_xlo);
  }
  true_residual(c, B, 0, conj_rhs);
}

int fail(helm_ctx* c, int code, const std::string& msg) {
  if (c) {
    c->err = msg;
    c->err_lit = nullptr;
  } else {
    g_setup_error = msg;
  }
  return code;
}

// error return that copies no string (the allocation-free entry point)
int fail_lit(helm_ctx* c, int code, const char* msg) {
  c->err_lit = msg;
  return code;
}

int run_solve(helm_ctx* c, int B, const helm_c32* rhs, helm_c32* x, helm_stats* stats, int conj, int snap_every = 0,
              int max_snaps = 0, helm_c32* snaps = nullptr, int* n_snaps = nullptr) {
  if (!c) return fail(nullptr, HELM_EINVAL, "null context");
  if (B < 1 || B > c->o.max_batch) return fail(c, HELM_EINVAL, "B must be in [1, max_batch]");
  if (!rhs || !x) return fail(c, HELM_EINVAL, "null field pointer");
  const long long N0 = c->N0;
  float call_ms = 0.f;
  try {
    check(hipStreamSynchronize(c->user_s), "caller stream");
    for (hipEvent_t& e : c->ev_solve)
      if (!e) check(hipEventCreate(&e), "hipEventCreate");
    check(hipEventRecord(c->ev_solve[0], c->s), "hipEventRecord");
    check(hipMemcpyAsync(c->d_rhs, rhs, (size_t)B * N0 * sizeof(c32), hipMemcpyDeviceToDevice, c->s), "copy rhs");
    launch_status_init(c->s, B, c->k);
    check(hipMemcpyAsync(c->d_fallbacks, c->d_zero_ints, B * sizeof(int), hipMemcpyDeviceToDevice, c->s), "reset");
    check(hipMemcpyAsync(c->d_xpar, c->d_zero_ints, B * sizeof(int), hipMemcpyDeviceToDevice, c->s), "reset");
    launch_zero(c->s, (long long)B * N0, c->d_xhi);
    launch_zero(c->s, (long long)B * N0, c->d_xlo);
    c->prof_B = B;
    true_residual(c, B, 1, conj);
    const int max_cycles = c->o.max_iters / std::max(1, c->k.m) + 4;
    // restart cycles, replayed from a graph captured on first use per (B, conj)
    const bool use_graph = c->o.use_graph != 0 && !c->prof_on;
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
      if (use_graph) {
        if (c->graph == nullptr || c->graph_B != B * 2 + conj) {
          if (c->graph) {
            hipGraphExecDestroy(c->graph);
            c->graph = nullptr;
          }
          hipGraph_t g;
          check(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
          restart_cycle(c, B, conj);
          check(hipStreamEndCapture(c->s, &g), "hipStreamEndCapture");
          check(hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0), "hipGraphInstantiate");
          hipGraphDestroy(g);
          c->graph_B = B * 2 + conj;
        }
        check(hipGraphLaunch(c->graph, c->s), "hipGraphLaunch");
      } else {
        restart_cycle(c, B, conj);
      }
      check(hipGetLastError(), "kernel launch");
      check(hipMemcpyAsync(c->h_status, c->k.status, B * sizeof(int), hipMemcpyDeviceToHost, c->s), "status D2H");
      check(hipStreamSynchronize(c->s), "hipStreamSynchronize");
      int running = 0;
      for (int b = 0; b < B; ++b) running += c->h_status[b] == HELM_RUNNING;
      if (snaps && running && (cyc + 1) % snap_every == 0 && *n_snaps < max_snaps) {
        launch_x_select(c->s, B, N0, c->d_xpar, c->d_xhi, c->d_xhi2, (c32*)(snaps + (size_t)(*n_snaps) * B * N0),
                        0);
        ++*n_snaps;
      }
      if (c->prof_on) prof_resolve(c);
      c->prof_B = running;
      if (!running) break;
    }
    c->last_B = B;
    c->last_conj = conj;
    launch_x_select(c->s, B, N0, c->d_xpar, c->d_xhi, c->d_xhi2, (c32*)x, conj);
    check(hipMemcpyAsync(c->h_status, c->k.status, B * sizeof(int), hipMemcpyDeviceToHost, c->s), "status");
    check(hipMemcpyAsync(c->h_iters, c->k.iters, B * sizeof(int), hipMemcpyDeviceToHost, c->s), "iters");
    check(hipMemcpyAsync(c->h_relres, c->k.relres, B * sizeof(double), hipMemcpyDeviceToHost, c->s), "relres");
    check(hipMemcpyAsync(c->h_fallbacks, c->d_fallbacks, B * sizeof(int), hipMemcpyDeviceToHost, c->s), "fallbacks");
    check(hipEventRecord(c->ev_solve[1], c->s), "hipEventRecord");
    check(hipStreamSynchronize(c->s), "hipStreamSynchronize");
    check(hipGetLastError(), "kernel launch");
    check(hipEventElapsedTime(&call_ms, c->ev_solve[0], c->ev_solve[1]), "hipEventElapsedTime");
  } catch (const HipError& e) {
    return fail(c, HELM_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.code));
  }
  int rc = HELM_OK;
  for (int b = 0; b < B; ++b) {
    int st = c->h_status[b];
    if (st == HELM_RUNNING) st = HELM_STATUS_NOT_CONVERGED;
    if (st != HELM_STATUS_CONVERGED) rc = HELM_NOT_CONVERGED;
    if (stats) {
      stats[b].iters = c->h_iters[b];
      stats[b].status = st;
      stats[b].rel_res_true = c->h_relres[b];
      stats[b].fallbacks = c->net ? c->h_fallbacks[b] : 0;
      stats[b].ms = call_ms;
    }
  }
  return rc;
}

// Medium-independent planes, once per context (host FP64): every level's coefficient with the
// background index everywhere.  The absorbing layer, the float-float diagonal there and the
// outermost coarse rings keep these values for every medium; the Omega values and the coarse
// interiors are rewritten by update_medium.
void upload_static(helm_ctx* c) {
  const helm_host::Geometry& g = c->geo;
  std::vector<double> nm(npts(c->n, c->dim), c->o.n_b);
  std::vector<cd> cf = helm_host::fine_coefficient(g, nm);
  const long long N0 = c->N0;
  std::vector<c32> hi(N0), dhi(N0), dlo(N0);
  const cd gh(1.0, c->kbh);
  for (long long p = 0; p < N0; ++p) {
    hi[p] = to_c32(cf[p]);
    // diagonal of A' (2d - c - #ghosts (1 + j k_b h)) in FP64, split into float-float
    const int x = (int)(p % c->ne), y = (int)((p / c->ne) % c->ne), z = c->dim == 3 ? (int)(p / ((long long)c->ne * c->ne)) : 0;
    int ng = (x == 0) + (x == c->ne - 1) + (y == 0) + (y == c->ne - 1);
    if (c->dim == 3) ng += (z == 0) + (z == c->ne - 1);
    const cd D = 2.0 * c->dim - cf[p] - (double)ng * gh;
    const float dr = (float)D.real(), dm = (float)D.imag();
    dhi[p] = make_float2(dr, dm);
    dlo[p] = make_float2((float)(D.real() - dr), (float)(D.imag() - dm));
  }
  check(hipMemcpy(c->d_chi, hi.data(), N0 * sizeof(c32), hipMemcpyHostToDevice), "upload c");
  check(hipMemcpy(c->d_dhi, dhi.data(), N0 * sizeof(c32), hipMemcpyHostToDevice), "upload D");
  check(hipMemcpy(c->d_dlo, dlo.data(), N0 * sizeof(c32), hipMemcpyHostToDevice), "upload D");
  std::vector<float> fpl(N0, 0.0f);  // f = 0 for the background medium
  check(hipMemcpy(c->d_f, fpl.data(), N0 * sizeof(float), hipMemcpyHostToDevice), "upload f");
  const cd kappa(c->o.kappa_re, c->o.kappa_im);
  std::vector<cd> cl = cf;
  for (int l = 0; l < c->L; ++l) {
    if (l > 0) cl = helm_host::coarse_coefficient(g, cl, c->lv[l - 1].n, l);
    std::vector<c32> kc(cl.size()), kclo(cl.size()), wd(cl.size());
    const int nl = c->lv[l].n;
    const cd gl(1.0, c->kbh * std::ldexp(1.0, l));
    for (size_t p = 0; p < cl.size(); ++p) {
      const cd v = kappa * cl[p];
      kc[p] = to_c32(v);
      kclo[p] = make_float2((float)(v.real() - (double)kc[p].x), (float)(v.imag() - (double)kc[p].y));
      const int x = (int)(p % nl), y = (int)((p / nl) % nl), z = c->dim == 3 ? (int)(p / ((size_t)nl * nl)) : 0;
      int ng = (x == 0) + (x == nl - 1) + (y == 0) + (y == nl - 1);
      if (c->dim == 3) ng += (z == 0) + (z == nl - 1);
      const cd D = 2.0 * c->dim - kappa * cl[p] - (double)ng * gl;
      wd[p] = to_c32(c->o.omega_jac / D);
    }
    check(hipMemcpy(c->lv[l].kc, kc.data(), kc.size() * sizeof(c32), hipMemcpyHostToDevice), "upload kc");
    check(hipMemcpy(c->lv[l].kclo, kclo.data(), kclo.size() * sizeof(c32), hipMemcpyHostToDevice), "upload kc");
    check(hipMemcpy(c->lv[l].wd, wd.data(), wd.size() * sizeof(c32), hipMemcpyHostToDevice), "upload wd");
  }
}

std::pair<float, float> split_ff(double v) {
  const float hi = (float)v;
  return {hi, (float)(v - (double)hi)};
}

// Per medium: the Omega values of the fine planes and the coarse interiors on the GPU
// (k_setup.hip), then the exact inverse of the coarsest shifted operator from that level's
// coefficients (host FP64, a few hundred to a few thousand unknowns), uploaded.
void update_medium(helm_ctx* c, const float* n_map_dev) {
  const long long Ni = npts(c->n, c->dim);
  check(hipMemcpyAsync(c->d_nmap, n_map_dev, Ni * sizeof(float), hipMemcpyDeviceToDevice, c->s), "copy n_map");
  SetupFineArgs a{};
  a.dim = c->dim;
  a.n = c->n;
  a.w = c->w;
  a.ne = c->ne;
  a.nmap = c->d_nmap;
  std::tie(a.k2_hi, a.k2_lo) = split_ff(c->k0h * c->k0h);
  std::tie(a.kbh_hi, a.kbh_lo) = split_ff(c->kbh);
  std::tie(a.k02_hi, a.k02_lo) = split_ff(c->k0 * c->k0);
  std::tie(a.nb2_hi, a.nb2_lo) = split_ff(c->o.n_b * c->o.n_b);
  a.kappa = make_float2((float)c->o.kappa_re, (float)c->o.kappa_im);
  a.g0 = c->lv[0].ghost;
  a.omega = (float)c->o.omega_jac;
  a.chi = c->d_chi;
  a.dhi = c->d_dhi;
  a.dlo = c->d_dlo;
  a.kc0 = c->lv[0].kc;
  a.kc0lo = c->lv[0].kclo;
  a.wd0 = c->lv[0].wd;
  a.f = c->d_f;
  launch_setup_fine(c->s, a);
  for (int l = 1; l < c->L; ++l)
    launch_setup_coarse(c->s, c->dim, c->lv[l - 1].n, c->lv[l].n, c->lv[l - 1].kc, c->lv[l - 1].kclo,
                        (float)c->o.omega_jac, c->lv[l].kc, c->lv[l].kclo, c->lv[l].wd);
  check(hipGetLastError(), "set-up kernels");
  const Level& cl = c->lv[c->L - 1];
  std::vector<c32> kc32(cl.N), kclo32(cl.N);
  check(hipMemcpyAsync(kc32.data(), cl.kc, cl.N * sizeof(c32), hipMemcpyDeviceToHost, c->s), "coarsest kc");
  check(hipMemcpyAsync(kclo32.data(), cl.kclo, cl.N * sizeof(c32), hipMemcpyDeviceToHost, c->s), "coarsest kc");
  check(hipStreamSynchronize(c->s), "set-up");
  std::vector<cd> kc(cl.N);
  for (long long p = 0; p < cl.N; ++p)
    kc[p] = cd((double)kc32[p].x + kclo32[p].x, (double)kc32[p].y + kclo32[p].y);
  std::vector<cd> inv;
  if (!helm_host::dense_inverse_transposed(c->geo, kc, cl.n, c->L - 1, inv))
    throw HipError{hipErrorInvalidValue, "coarsest operator is singular"};
  std::vector<c32> inv32(inv.size());
  for (size_t p = 0; p < inv.size(); ++p) inv32[p] = to_c32(inv[p]);
  check(hipMemcpyAsync(c->d_minvT, inv32.data(), inv32.size() * sizeof(c32), hipMemcpyHostToDevice, c->s),
        "upload inverse");
  check(hipStreamSynchronize(c->s), "set-up");
}

void free_ctx(helm_ctx* c) {
  if (!c) return;
  if (c->graph) hipGraphExecDestroy(c->graph);
  net_bufs_destroy(c->net_bufs);
  for (hipEvent_t e : c->ev_solve)
    if (e) hipEventDestroy(e);
  for (auto& p : c->pending) {
    hipEventDestroy(p.e0);
    hipEventDestroy(p.e1);
  }
  for (hipEvent_t e : c->event_pool) hipEventDestroy(e);
  for (void* p : c->allocs) hipFree(p);
  if (c->h_status) hipHostFree(c->h_status);
  if (c->h_iters) hipHostFree(c->h_iters);
  if (c->h_relres) hipHostFree(c->h_relres);
  if (c->h_fallbacks) hipHostFree(c->h_fallbacks);
  if (c->s) hipStreamDestroy(c->s);
  delete c;
}

}  // namespace

#define HELM_GUARD_BEGIN \
  try {                  \
    check(hipStreamSynchronize(c->user_s), "caller stream");
#define HELM_GUARD_END(name)                                                       \
  check(hipGetLastError(), name);                                                  \
  check(hipStreamSynchronize(c->s), "sync");                                       \
  if (c->prof_on) prof_resolve(c);                                                 \
  }                                                                                \
  catch (const HipError& e) {                                                      \
    return fail(c, HELM_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.code)); \
  }                                                                                \
  return HELM_OK;

// ---------------------------------------------------------------- autotuner
namespace {

std::string tune_key(const helm_ctx* c, int B) {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) prop.gcnArchName[0] = 0;
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s d%d n%d L%d B%d nu%d%d cycle%d", arch.c_str(), c->dim, c->ne, c->L, B,
                c->o.nu1, c->o.nu2, c->o.cycle);
  return buf;
}

// one cache entry per line: {"key": "...", "down": [..], "up": [..], "coarse_max": N}
bool tune_load(helm_ctx* c, const char* path, const std::string& key) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  const std::string tag = "\"key\": \"" + key + "\"";
  while (!found && std::fgets(line, sizeof line, f)) {
    if (!std::strstr(line, tag.c_str())) continue;
    int down[HELM_MAX_LEVELS] = {0}, up[HELM_MAX_LEVELS] = {0};
    long long cm = -1;
    const char* p = std::strstr(line, "\"down\": [");
    const char* q = std::strstr(line, "\"up\": [");
    const char* m = std::strstr(line, "\"coarse_max\": ");
    if (!p || !q || !m || std::sscanf(m + 14, "%lld", &cm) != 1) break;
    p += 9;
    q += 7;
    bool ok = true;
    for (int l = 0; l < c->L && ok; ++l) {
      int nd = 0, nu = 0;
      ok = std::sscanf(p, "%d%n", &down[l], &nd) == 1 && std::sscanf(q, "%d%n", &up[l], &nu) == 1 && down[l] >= 0 &&
           down[l] < mg_down_variants() && up[l] >= 0 && up[l] < mg_up_variants();
      p += nd;
      q += nu;
      while (*p == ',' || *p == ' ') ++p;
      while (*q == ',' || *q == ' ') ++q;
    }
    if (!ok) break;
    std::memcpy(c->tune_down, down, sizeof down);
    std::memcpy(c->tune_up, up, sizeof up);
    c->coarse_max = cm;
    int mv = 0;
    const char* pm = std::strstr(line, "\"mv\": ");
    if (pm && std::sscanf(pm + 6, "%d", &mv) == 1 && mv >= 0 && mv < mg_up_mv_variants()) c->tune_mv = mv;
    found = true;
  }
  std::fclose(f);
  return found;
}

void tune_save(const helm_ctx* c, const char* path, const std::string& key) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;  // the cache is an optimisation: an unwritable path only costs a re-tune
  std::fprintf(f, "{\"key\": \"%s\", \"down\": [", key.c_str());
  for (int l = 0; l < c->L; ++l) std::fprintf(f, "%s%d", l ? ", " : "", c->tune_down[l]);
  std::fprintf(f, "], \"up\": [");
  for (int l = 0; l < c->L; ++l) std::fprintf(f, "%s%d", l ? ", " : "", c->tune_up[l]);
  std::fprintf(f, "], \"coarse_max\": %lld, \"mv\": %d}\n", c->coarse_max, c->tune_mv);
  std::fclose(f);
}

// mean duration (ms) of `reps` back-to-back calls of f on the context stream, after one warm-up call
template <class F>
double time_ms(helm_ctx* c, F&& f, int reps) {
  f();
  hipEvent_t e0, e1;
  check(hipEventCreate(&e0), "event");
  check(hipEventCreate(&e1), "event");
  check(hipEventRecord(e0, c->s), "event");
  for (int i = 0; i < reps; ++i) f();
  check(hipEventRecord(e1, c->s), "event");
  check(hipEventSynchronize(e1), "event");
  float ms = 0.f;
  check(hipEventElapsedTime(&ms, e0, e1), "event");
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  check(hipGetLastError(), "tuning launch");
  return ms / reps;
}

// The fastest of nv launch variants: three interleaved rounds (clock ramps and drift
// reach every variant alike), each variant's best mean over `reps` launches; ties go
// to the lower index.  With a margin, variant 0 (the default) is kept unless another
// is faster by more than that fraction.
template <class F>
int fastest_variant(helm_ctx* c, int nv, F&& launch, int reps, double keep_default_within = 0.0) {
  std::vector<double> best((size_t)nv, 1e30);
  for (int round = 0; round < 3; ++round)
    for (int v = 0; v < nv; ++v) best[v] = std::min(best[v], time_ms(c, [&] { launch(v); }, reps));
  const int v = (int)(std::min_element(best.begin(), best.end()) - best.begin());
  return best[v] < best[0] * (1.0 - keep_default_within) ? v : 0;
}

}  // namespace

extern "C" {

void helm_default_opts(helm_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->n_b = 1.333;
  o->kappa_re = 1.0;
  o->kappa_im = 0.5;
  o->omega_jac = 0.8;
  o->rtol = 1e-6;
  o->levels = 4;
  o->nu1 = 1;
  o->nu2 = 1;
  o->cycle = 1;
  o->restart = 10;
  o->max_iters = 4000;
  o->max_batch = 64;
  o->reorth = 0;
  o->fused = 1;
  o->use_graph = 1;
  o->coarse_single_launch = 1;
  o->krylov = HELM_KRYLOV_SSTEP;
  o->fused_step = 2;
}

int helm_extended_size(int n, int abl_width, int levels) { return helm_host::extended_size(n, abl_width, levels); }

int helm_setup(const helm_grid* grid, const float* n_map_dev, double k0, const helm_abl* abl, const helm_opts* opts,
               void* hip_stream, helm_ctx** out) {
  if (!out) return fail(nullptr, HELM_EINVAL, "null output pointer");
  *out = nullptr;
  if (!grid || !n_map_dev) return fail(nullptr, HELM_EINVAL, "null grid or n_map");
  if (grid->dim != 2 && grid->dim != 3) return fail(nullptr, HELM_EINVAL, "dim must be 2 or 3");
  if (grid->n < 1 || grid->abl_width < 0) return fail(nullptr, HELM_EINVAL, "bad interior size or layer width");
  if (!(k0 > 0.0) || !std::isfinite(k0)) return fail(nullptr, HELM_EINVAL, "k0 must be positive");
  helm_opts o;
  helm_default_opts(&o);
  if (opts) o = *opts;
  if (o.levels < 2 || o.levels > 12) return fail(nullptr, HELM_EINVAL, "levels must be in [2, 12]");
  if (o.restart < 1 || o.restart > krylov_max_restart()) return fail(nullptr, HELM_EINVAL, "restart must be in [1, 64]");
  if (o.krylov != HELM_KRYLOV_FGMRES && o.krylov != HELM_KRYLOV_SSTEP && o.krylov != HELM_KRYLOV_BICGSTAB)
    return fail(nullptr, HELM_EINVAL, "krylov must be HELM_KRYLOV_FGMRES, _SSTEP or _BICGSTAB");
  if (o.krylov == HELM_KRYLOV_BICGSTAB && o.restart < 4)
    return fail(nullptr, HELM_EINVAL, "Bi-CGSTAB takes restart >= 4 (iterations per status check)");
  if (o.krylov == HELM_KRYLOV_SSTEP && o.restart > sstep_max_restart())
    return fail(nullptr, HELM_EINVAL, "the s-step form takes restart <= 12");
  if (o.fused_step < 0 || o.fused_step > 2) return fail(nullptr, HELM_EINVAL, "fused_step must be 0, 1 or 2");
  if (o.max_batch < 1 || o.nu1 < 0 || o.nu2 < 0 || o.cycle < 1 || o.cycle > 3 || o.max_iters < 1 || !(o.rtol > 0))
    return fail(nullptr, HELM_EINVAL, "bad solver options");
  helm_abl a{0.15, 1, 0};
  if (abl) a = *abl;
  if (a.sign != 1 && a.sign != -1) return fail(nullptr, HELM_EINVAL, "abl sign must be +1 or -1");
  const int ne = helm_host::extended_size(grid->n, grid->abl_width, o.levels);
  if (ne < 3) return fail(nullptr, HELM_EINVAL, "grid too small");
  const int nc = (ne - 1) / (1 << (o.levels - 1)) + 1;
  if (nc < 2) return fail(nullptr, HELM_EINVAL, "too many levels for this grid");
  const long long Nc = npts(nc, grid->dim);
  if (Nc > 4096) return fail(nullptr, HELM_EINVAL, "coarsest grid too large for the dense inverse: add levels");

  helm_ctx* c = new (std::nothrow) helm_ctx();
  if (!c) return fail(nullptr, HELM_ENOMEM, "out of host memory");
  try {
    c->grid = *grid;
    c->abl = a;
    c->o = o;
    c->dim = grid->dim;
    c->n = grid->n;
    c->w = grid->abl_width;
    c->ne = ne;
    c->L = o.levels;
    c->h = grid->h > 0 ? grid->h : 1.0 / (ne - 1);
    c->k0 = k0;
    c->k0h = k0 * c->h;
    c->kbh = c->k0h * o.n_b;
    c->N0 = npts(ne, c->dim);
    c->user_s = (hipStream_t)hip_stream;
    check(hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking), "hipStreamCreate");
    c->geo = helm_host::Geometry{c->dim, c->n, c->w, ne, c->k0h, o.n_b, a.beta, a.sign, a.profile};
    const double h2 = c->h * c->h;
    c->h2_hi = (float)h2;
    c->h2_lo = (float)(h2 - (double)c->h2_hi);
    c->g0_hi = make_float2(1.0f, (float)c->kbh);
    const int maxB = o.max_batch, m = o.restart;
    const long long N0 = c->N0;
    c->lv.resize(c->L);
    for (int l = 0; l < c->L; ++l) {
      Level& L = c->lv[l];
      L.n = (ne - 1) / (1 << l) + 1;
      L.N = npts(L.n, c->dim);
      L.ghost = make_float2(1.0f, (float)(c->kbh * std::ldexp(1.0, l)));
      L.kc = c->alloc<c32>(L.N);
      L.kclo = c->alloc<c32>(L.N);
      L.wd = c->alloc<c32>(L.N);
      if (l > 0) {
        L.rc = c->alloc<c32>((size_t)maxB * L.N);
        L.e = c->alloc<c32>((size_t)maxB * L.N);
        L.t = c->alloc<c32>((size_t)maxB * L.N);
        if (o.cycle >= 2) {
          L.rr = c->alloc<c32>((size_t)maxB * L.N);
          L.d = c->alloc<c32>((size_t)maxB * L.N);
        }
      }
    }
    c->Nc = (int)c->lv[c->L - 1].N;
    c->d_minvT = c->alloc<c32>((size_t)c->Nc * c->Nc);
    c->d_cs_part = c->alloc<c32>(coarse_solve_part_size(maxB, c->Nc));
    c->d_nmap = c->alloc<float>(npts(c->n, c->dim));
    c->d_f = c->alloc<float>(N0);
    c->d_chi = c->alloc<c32>(N0);
    c->d_dhi = c->alloc<c32>(N0);
    c->d_dlo = c->alloc<c32>(N0);
    c->d_xhi = c->alloc<c32>((size_t)maxB * N0);
    c->d_xlo = c->alloc<c32>((size_t)maxB * N0);
    if (c->dim == 2) {
      c->d_xhi2 = c->alloc<c32>((size_t)maxB * N0);
      c->d_xlo2 = c->alloc<c32>((size_t)maxB * N0);
    }
    c->d_xpar = c->alloc<int>(maxB);
    c->d_rhs = c->alloc<c32>((size_t)maxB * N0);
    c->d_T0 = c->alloc<c32>((size_t)maxB * N0);
    c->d_tables = c->alloc<c32>((size_t)maxB * c->dim * ne);
    c->d_ones = c->alloc<int>(maxB);
    c->d_zero_ints = c->alloc<int>(maxB);
    c->d_mg_mask = c->alloc<int>(maxB);
    c->d_fallbacks = c->alloc<int>(maxB);
    c->d_tv_mag = c->alloc<float>(npts(c->n, c->dim));
    c->d_tv_part = c->alloc<float>(tv_partials(c->dim, c->n));
    KrylovArgs& k = c->k;
    k.dim = c->dim;
    k.n = ne;
    k.N = N0;
    k.m = m;
    k.nblk = krylov_blocks_per_rhs(N0);
    k.nres = k.nblk;
    k.xpar = c->d_xpar;
    k.flip_x = 0;
    k.V = c->alloc<c32>((size_t)maxB * (m + 1) * N0);
    k.Z = c->alloc<c32>((size_t)maxB * m * N0);
    k.vs = c->alloc<float>((size_t)maxB * (m + 1));
    k.P1 = c->alloc<c32>((size_t)maxB * k.nblk * (m + 1));
    k.P2 = c->alloc<float>((size_t)maxB * std::max(k.nblk, c->dim == 2 ? krylov_xres_tiles(ne) : 0));
    k.H = c->alloc<double2>((size_t)maxB * (m + 1) * m);
    k.cs = c->alloc<double>((size_t)maxB * m);
    k.sn = c->alloc<double2>((size_t)maxB * m);
    k.g = c->alloc<double2>((size_t)maxB * (m + 1));
    k.coef = c->alloc<c32>((size_t)maxB * (m + 1));
    k.y = c->alloc<c32>((size_t)maxB * m);
    if (o.krylov == HELM_KRYLOV_SSTEP)
      c->d_gram = c->alloc<double2>((size_t)maxB * k.nblk * sstep_gram_entries(m));
    k.active = c->alloc<int>(maxB);
    k.status = c->alloc<int>(maxB);
    k.jcount = c->alloc<int>(maxB);
    k.iters = c->alloc<int>(maxB);
    k.bnorm = c->alloc<double>(maxB);
    k.tol = c->alloc<double>(maxB);
    k.relres = c->alloc<double>(maxB);
    k.max_iters = o.max_iters;
    k.rtol = o.rtol;
    k.inner_factor = 0.5;
    check(hipHostMalloc((void**)&c->h_status, maxB * sizeof(int), hipHostMallocDefault), "hipHostMalloc");
    check(hipHostMalloc((void**)&c->h_iters, maxB * sizeof(int), hipHostMallocDefault), "hipHostMalloc");
    check(hipHostMalloc((void**)&c->h_relres, maxB * sizeof(double), hipHostMallocDefault), "hipHostMalloc");
    std::vector<int> ones(maxB, 1), zeros(maxB, 0);
    check(hipMemcpy(c->d_ones, ones.data(), maxB * sizeof(int), hipMemcpyHostToDevice), "upload ones");
    check(hipMemcpy(c->d_zero_ints, zeros.data(), maxB * sizeof(int), hipMemcpyHostToDevice), "upload zeros");
    check(hipMemcpy(c->d_xpar, zeros.data(), maxB * sizeof(int), hipMemcpyHostToDevice), "upload zeros");
    check(hipHostMalloc((void**)&c->h_fallbacks, maxB * sizeof(int), hipHostMallocDefault), "hipHostMalloc");
    upload_static(c);
    update_medium(c, n_map_dev);
    check(static_scratch_init(), "device scratch address");
    check(hipDeviceSynchronize(), "setup");
  } catch (const HipError& e) {
    std::string msg = std::string(e.what) + ": " + hipGetErrorString(e.code);
    free_ctx(c);
    return fail(nullptr, e.code == hipErrorOutOfMemory ? HELM_ENOMEM : HELM_EHIP, msg);
  } catch (const std::bad_alloc&) {
    free_ctx(c);
    return fail(nullptr, HELM_ENOMEM, "out of host memory");
  }
  *out = c;
  return HELM_OK;
}

int helm_update_n(helm_ctx* c, const float* n_map_dev) {
  if (!c || !n_map_dev) return fail(c, HELM_EINVAL, "null argument");
  try {
    check(hipStreamSynchronize(c->user_s), "caller stream");
    check(hipStreamSynchronize(c->s), "sync");
    update_medium(c, n_map_dev);
  } catch (const HipError& e) {
    return fail(c, HELM_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.code));
  } catch (const std::bad_alloc&) {
    return fail(c, HELM_ENOMEM, "out of host memory");
  }
  return HELM_OK;
}

int helm_get_info(const helm_ctx* c, helm_info* info) {
  if (!c || !info) return HELM_EINVAL;
  info->dim = c->dim;
  info->n = c->n;
  info->abl_width = c->w;
  info->n_e = c->ne;
  info->levels = c->L;
  info->coarsest_n = c->lv[c->L - 1].n;
  info->h = c->h;
  info->k0 = c->k0;
  info->n_b = c->o.n_b;
  info->workspace_bytes = c->bytes;
  return HELM_OK;
}

int helm_plane_wave_rhs(helm_ctx* c, int B, const double* dirs, helm_c32* rhs, helm_c32* u_in) {
  if (!c || !dirs || !rhs) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1 || B > c->o.max_batch) return fail(c, HELM_EINVAL, "B must be in [1, max_batch]");
  const int ne = c->ne, dim = c->dim;
  std::vector<c32> tab((size_t)B * dim * ne);
  const double centre = c->w + 0.5 * (c->n - 1);
  for (int b = 0; b < B; ++b)
    for (int a = 0; a < dim; ++a) {
      const double d = dirs[b * dim + a];
      for (int i = 0; i < ne; ++i) {
        const double ph = c->kbh * d * (i - centre);
        tab[((size_t)b * dim + a) * ne + i] = make_float2((float)std::cos(ph), (float)std::sin(ph));
      }
    }
  try {
    check(hipStreamSynchronize(c->user_s), "caller stream");
    check(hipMemcpyAsync(c->d_tables, tab.data(), tab.size() * sizeof(c32), hipMemcpyHostToDevice, c->s), "tables");
    launch_plane_wave(c->s, dim, B, ne, c->d_f, c->d_tables, (c32*)rhs, (c32*)u_in);
    check(hipGetLastError(), "plane wave");
    check(hipStreamSynchronize(c->s), "sync");
  } catch (const HipError& e) {
    return fail(c, HELM_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.code));
  }
  return HELM_OK;
}

int helm_solve_batch(helm_ctx* c, int B, const helm_c32* rhs, helm_c32* x, helm_stats* stats) {
  return run_solve(c, B, rhs, x, stats, 0);
}

int helm_solve_snapshots(helm_ctx* c, int B, const helm_c32* rhs, helm_c32* x, helm_stats* stats, int every_cycles,
                         int max_snaps, helm_c32* snaps, int* n_snaps) {
  if (!n_snaps || !snaps || every_cycles < 1 || max_snaps < 1) return fail(c, HELM_EINVAL, "bad snapshot arguments");
  *n_snaps = 0;
  return run_solve(c, B, rhs, x, stats, 0, every_cycles, max_snaps, snaps, n_snaps);
}

int helm_set_preconditioner(helm_ctx* c, helm_net* net, double accept_tol, double gamma, int mode) {
  if (!c) return HELM_EINVAL;
  if (net && net_dim(net) != c->dim) return fail(c, HELM_EINVAL, "the network's dimension differs from the grid's");
  if (mode != HELM_NET_REPLACE && mode != HELM_NET_THEN_MG) return fail(c, HELM_EINVAL, "unknown mode");
  if (!(gamma > 0.0)) return fail(c, HELM_EINVAL, "gamma must be positive");
  try {
    check(hipStreamSynchronize(c->s), "sync");
    if (c->graph) {  // the captured cycle refers to the old preconditioner and its buffers
      hipGraphExecDestroy(c->graph);
      c->graph = nullptr;
      c->graph_B = 0;
    }
    // fresh buffers for this context (a network may also serve other contexts, each with its own)
    c->net = nullptr;
    net_bufs_destroy(c->net_bufs);
    c->net_bufs = nullptr;
    if (net) c->net_bufs = net_bufs_create(net, c->o.max_batch, c->ne);
    if (net && mode == HELM_NET_THEN_MG && !c->d_net_res) {
      c->d_net_res = c->alloc<c32>((size_t)c->o.max_batch * c->N0);
      c->d_net_cor = c->alloc<c32>((size_t)c->o.max_batch * c->N0);
    }
  } catch (const HipError& e) {
    return fail(c, HELM_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.code));
  } catch (...) {
    return fail(c, HELM_ENOMEM, "could not reserve the network buffers");
  }
  c->net = net;
  c->accept_tol = accept_tol;
  c->net_gamma = gamma;
  c->net_mode = mode;
  return HELM_OK;
}

int helm_net_examples(helm_ctx* c, int B, const helm_c32* r, const helm_c32* x_final, const helm_c32* x_k, int ncrop,
                      const int* crops_host, int S, double gamma, float* feat, float* tgt) {
  if (!c || !r || !x_final || !x_k || !crops_host || !feat || !tgt || ncrop < 1 || S < 1 || S > c->ne)
    return fail(c, HELM_EINVAL, "bad argument");
  const int cw = 1 + c->dim;  // (rhs, (z0,) y0, x0)
  for (int i = 0; i < ncrop; ++i) {
    const int b = crops_host[cw * i];
    bool ok = b >= 0 && b < B;
    for (int a = 1; a < cw; ++a) ok = ok && crops_host[cw * i + a] >= 0 && crops_host[cw * i + a] + S <= c->ne;
    if (!ok) return fail(c, HELM_EINVAL, "crop outside the grid");
  }
  struct DevFree {
    void* p = nullptr;
    ~DevFree() {
      if (p) hipFree(p);
    }
  } crops_mem;
  HELM_GUARD_BEGIN
  const size_t crop_bytes = ((size_t)ncrop * cw * sizeof(int) + 255) / 256 * 256;
  check(hipMalloc(&crops_mem.p, crop_bytes + (size_t)B * sizeof(float)), "hipMalloc");
  int* d_crops = (int*)crops_mem.p;
  float* d_ss = (float*)((char*)crops_mem.p + crop_bytes);
  check(hipMemcpyAsync(d_crops, crops_host, (size_t)ncrop * cw * sizeof(int), hipMemcpyHostToDevice, c->s), "crops");
  launch_examples(c->s, c->dim, B, ncrop, S, c->ne, d_crops, d_ss, (const c32*)r, (const c32*)x_final, (const c32*)x_k, c->N0,
                  c->d_chi, make_float2((float)(c->kbh * c->kbh), 0.0f), (float)(c->h * c->h), (float)(1.0 / gamma),
                  feat, tgt);
  HELM_GUARD_END("net_examples")
}

int helm_examples_rms(helm_ctx* c, const float* x_dev, long long count, double* rms_host) {
  if (!c || !x_dev || !rms_host || count < 1) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  const int nbk = sumsq_blocks(count);
  if (nbk > c->inv_part_len) {
    c->d_inv_part = c->alloc<double>(nbk);
    c->inv_part_len = nbk;
  }
  launch_sumsq(c->s, count, x_dev, c->d_inv_part);
  std::vector<double> part(nbk);
  check(hipMemcpyAsync(part.data(), c->d_inv_part, nbk * sizeof(double), hipMemcpyDeviceToHost, c->s), "sumsq");
  check(hipStreamSynchronize(c->s), "sync");
  double sum = 0.0;
  for (double v : part) sum += v;
  *rms_host = std::sqrt(sum / (double)count);
  HELM_GUARD_END("examples_rms")
}

int helm_examples_scale(helm_ctx* c, float* x_dev, long long count, double factor) {
  if (!c || !x_dev || count < 1 || !std::isfinite(factor)) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  launch_scale(c->s, count, x_dev, (float)factor);
  HELM_GUARD_END("examples_scale")
}

int helm_adjoint_batch(helm_ctx* c, int B, const helm_c32* rhs, helm_c32* lam, helm_stats* stats) {
  return run_solve(c, B, rhs, lam, stats, 1);
}

int helm_solution_lo(helm_ctx* c, int B, helm_c32* x_lo) {
  if (!c || !x_lo) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1 || B > c->last_B) return fail(c, HELM_EINVAL, "B must be in [1, B of the last solve]");
  HELM_GUARD_BEGIN
  launch_x_select(c->s, B, c->N0, c->d_xpar, c->d_xlo, c->d_xlo2, (c32*)x_lo, c->last_conj);
  HELM_GUARD_END("solution_lo")
}

int helm_grad_n(helm_ctx* c, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* lam,
                float* grad_n) {
  if (!c || !u_sc || !lam || !grad_n) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1) return fail(c, HELM_EINVAL, "B must be >= 1");
  try {
    check(hipStreamSynchronize(c->user_s), "caller stream");
    launch_grad_n(c->s, c->dim, B, c->ne, c->w, c->n, (const c32*)u_in, (const c32*)u_sc, (const c32*)lam,
                  c->d_nmap, (float)(2.0 * c->k0 * c->k0), grad_n);
    check(hipGetLastError(), "grad_n");
    check(hipStreamSynchronize(c->s), "sync");
  } catch (const HipError& e) {
    return fail(c, HELM_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.code));
  }
  return HELM_OK;
}


int helm_apply_A(helm_ctx* c, int B, const helm_c32* x, helm_c32* y) {
  if (!c || !x || !y || B < 1) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  launch_apply(c->s, c->dim, B, VecSet{(c32*)x, c->N0}, ScaleSet{nullptr, 0}, fine_A(c), (float)(1.0 / (c->h * c->h)),
               VecSet{(c32*)y, c->N0}, nullptr);
  HELM_GUARD_END("apply_A")
}

int helm_residual(helm_ctx* c, int B, const helm_c32* rhs, const helm_c32* x_hi, const helm_c32* x_lo, helm_c32* r) {
  if (!c || !rhs || !x_hi || !r || B < 1) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  KrylovArgs k = c->k;
  k.status = nullptr;
  k.P2 = nullptr;
  launch_residual_ff(c->s, B, k, (const c32*)rhs, c->N0, 0, (const c32*)x_hi, (const c32*)x_lo, 0, c->d_dhi,
                     c->d_dlo, c->h2_hi, c->h2_lo, (c32*)r, c->N0, (float)(1.0 / (c->h * c->h)));
  HELM_GUARD_END("residual")
}

int helm_apply_K(helm_ctx* c, int level, int B, const helm_c32* x, helm_c32* y) {
  if (!c || !x || !y || B < 1 || level < 0 || level >= c->L) return fail(c, HELM_EINVAL, "bad argument");
  const long long N = c->lv[level].N;
  HELM_GUARD_BEGIN
  launch_apply(c->s, c->dim, B, VecSet{(c32*)x, N}, ScaleSet{nullptr, 0}, level_K(c, level), 1.0f, VecSet{(c32*)y, N},
               nullptr);
  HELM_GUARD_END("apply_K")
}

int helm_restrict(helm_ctx* c, int level, int B, const helm_c32* fine, helm_c32* coarse) {
  if (!c || !fine || !coarse || B < 1 || level < 0 || level >= c->L - 1) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  launch_restrict_residual(c->s, c->dim, B, VecSet{(c32*)fine, c->lv[level].N}, ScaleSet{nullptr, 0},
                           VecSet{nullptr, 0}, level_K(c, level), VecSet{(c32*)coarse, c->lv[level + 1].N},
                           c->lv[level + 1].n, nullptr);
  HELM_GUARD_END("restrict")
}

int helm_prolong_add(helm_ctx* c, int level, int B, const helm_c32* coarse, helm_c32* fine) {
  if (!c || !fine || !coarse || B < 1 || level < 0 || level >= c->L - 1) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  launch_prolong_add(c->s, c->dim, B, VecSet{(c32*)coarse, c->lv[level + 1].N}, c->lv[level + 1].n,
                     VecSet{(c32*)fine, c->lv[level].N}, c->lv[level].n, nullptr);
  HELM_GUARD_END("prolong")
}

int helm_coarse_solve(helm_ctx* c, int B, const helm_c32* r, helm_c32* z) {
  if (!c || !r || !z || B < 1) return fail(c, HELM_EINVAL, "bad argument");
  const long long N = c->lv[c->L - 1].N;
  HELM_GUARD_BEGIN
  launch_coarse_solve(c->s, B, c->d_minvT, c->Nc, VecSet{(c32*)r, N}, VecSet{(c32*)z, N}, nullptr);
  HELM_GUARD_END("coarse_solve")
}

int helm_precondition(helm_ctx* c, int B, const helm_c32* r, helm_c32* z) {
  if (!c || !r || !z || B < 1 || B > c->o.max_batch) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  mg_cycle(c, B, 0, VecSet{(c32*)r, c->N0}, ScaleSet{nullptr, 0}, VecSet{(c32*)z, c->N0}, true, c->d_ones);
  HELM_GUARD_END("precondition")
}

int helm_autotune(helm_ctx* c, int B, const char* cache_path, helm_tune* out) {
  if (!c) return HELM_EINVAL;
  if (B < 1 || B > c->o.max_batch) return fail(c, HELM_EINVAL, "B must be in [1, max_batch]");
  HELM_GUARD_BEGIN
  const std::string key = tune_key(c, B);
  if (c->graph) {  // a captured graph holds the old launch shapes
    hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_B = 0;
  }
  struct ProfOff {  // no per-launch events while timing; restored on every exit
    helm_ctx* c;
    bool was;
    ~ProfOff() { c->prof_on = was; }
  } prof_off{c, c->prof_on};
  c->prof_on = false;
  helm_tune t{};
  t.from_cache = cache_path && tune_load(c, cache_path, key);
  // the default shapes' V-cycle time, for the report
  const long long N0 = c->N0;
  const VecSet r0{c->k.V, N0}, z0{c->k.Z, N0};
  check(hipMemsetAsync(c->k.V, 0, (size_t)B * N0 * sizeof(c32), c->s), "memset");
  auto vcycle = [&] { mg_cycle(c, B, 0, r0, ScaleSet{nullptr, 0}, z0, true, nullptr); };
  if (!t.from_cache) {
    for (int l = 0; l < HELM_MAX_LEVELS; ++l) c->tune_down[l] = c->tune_up[l] = 0;
    c->coarse_max = -1;
    t.vcycle_default_ms = time_ms(c, vcycle, 3);
    // 1. fused-leg tiles, level by level, on the level's own buffers
    if (c->dim == 2 && c->o.fused) {
      const float om = (float)c->o.omega_jac;
      for (int l = 0; l + 1 < c->L; ++l) {
        Level& f = c->lv[l];
        Level& cr = c->lv[l + 1];
        const VecSet r = l == 0 ? r0 : VecSet{f.rc, f.N};
        const VecSet out = l == 0 ? z0 : VecSet{f.t, f.N};
        const LevelArgs K = level_K(c, l);
        if (l > 0) check(hipMemsetAsync(f.rc, 0, (size_t)B * f.N * sizeof(c32), c->s), "memset");
        check(hipMemsetAsync(cr.e, 0, (size_t)B * cr.N * sizeof(c32), c->s), "memset");
        c->tune_down[l] = fastest_variant(
            c, mg_down_variants(),
            [&](int v) {
              launch_down_fused2(c->s, B, r, ScaleSet{nullptr, 0}, K, om, VecSet{cr.rc, cr.N}, cr.n, nullptr, v);
            },
            5);
        c->tune_up[l] = fastest_variant(
            c, mg_up_variants(),
            [&](int v) {
              launch_up_fused2(c->s, B, r, ScaleSet{nullptr, 0}, K, om, VecSet{cr.e, cr.N}, cr.n, out, nullptr, v);
            },
            5);
      }
    }
    // 2. the launch shape of the fused finest up-leg + basis matvec (the s-step form's finest
    // step).  Timed alone (every right-hand side active, no graph) it ranks shapes within a
    // few percent differently from inside the solve, where the default (16 rows, 4 right-hand
    // sides per workgroup) measured fastest on MI355X at 512^2 x 60; the default is kept
    // unless a variant is clearly faster.
    c->tune_mv = 0;
    if (c->dim == 2 && c->o.fused && c->o.krylov == HELM_KRYLOV_SSTEP && c->o.fused_step == 2 && c->L >= 2) {
      const float om = (float)c->o.omega_jac;
      const Level& L1 = c->lv[1];
      check(hipMemsetAsync(L1.e, 0, (size_t)B * L1.N * sizeof(c32), c->s), "memset");
      c->tune_mv = fastest_variant(
          c, mg_up_mv_variants(),
          [&](int v) {
            launch_up_mv2(c->s, B, r0, ScaleSet{nullptr, 0}, level_K(c, 0), fine_A(c), om, VecSet{L1.e, L1.N}, L1.n,
                          z0, VecSet{c->d_T0, N0}, nullptr, v);
          },
          5, 0.02);
    }
    // 3. the single-launch threshold for the coarse levels, on whole V-cycles
    if (c->o.coarse_single_launch) {
      const long long cand2[] = {0, 24LL * 24, 48LL * 48, 96LL * 96};
      const long long cand3[] = {0, 8LL * 8 * 8, 16LL * 16 * 16, 24LL * 24 * 24};
      const long long* cand = c->dim == 2 ? cand2 : cand3;
      const int pick = fastest_variant(
          c, 4,
          [&](int i) {
            c->coarse_max = cand[i];
            vcycle();
          },
          3);
      c->coarse_max = cand[pick];
    }
    if (cache_path) tune_save(c, cache_path, key);
  }
  t.vcycle_ms = time_ms(c, vcycle, 3);
  t.levels = c->L;
  for (int l = 0; l < c->L && l < HELM_TUNE_MAX_LEVELS; ++l) {
    mg_down_shape(c->tune_down[l], &t.down[l][0], &t.down[l][1]);
    mg_up_shape(c->tune_up[l], &t.up[l][0], &t.up[l][1], &t.up[l][2]);
  }
  t.coarse_max = c->coarse_max >= 0 ? c->coarse_max : (c->dim == 2 ? 48LL * 48 : 16LL * 16 * 16);
  t.up_mv_rows = mg_up_mv_rows(c->tune_mv);
  t.up_mv_rhs_per_block = mg_up_mv_rhs_per_block(c->tune_mv);
  if (out) *out = t;
  HELM_GUARD_END("autotune")
}

int helm_profile_enable(helm_ctx* c, int on) {
  if (!c) return HELM_EINVAL;
  c->prof_on = on != 0;
  return HELM_OK;
}

int helm_profile_reset(helm_ctx* c) {
  if (!c) return HELM_EINVAL;
  c->prof.clear();
  return HELM_OK;
}

int helm_profile_count(const helm_ctx* c) { return c ? (int)c->prof.size() : HELM_EINVAL; }

int helm_profile_get(const helm_ctx* c, int i, char* name, int name_len, double* total_ms, long long* launches,
                     double* bytes) {
  if (!c || i < 0 || i >= (int)c->prof.size()) return HELM_EINVAL;
  const auto& e = c->prof[i];
  if (name && name_len > 0) {
    std::strncpy(name, e.name.c_str(), name_len - 1);
    name[name_len - 1] = 0;
  }
  if (total_ms) *total_ms = e.ms;
  if (launches) *launches = e.launches;
  if (bytes) *bytes = e.bytes;
  return HELM_OK;
}

namespace {
// Receiver indices (device int[M]) checked on the host: each inside the extended grid and,
// where S^T scatters into them, distinct.  Returns an empty string when they are valid.
std::string receiver_error(helm_ctx* c, int M, const int* idx_dev, bool distinct) {
  std::vector<int> idx(M);
  check(hipMemcpy(idx.data(), idx_dev, (size_t)M * sizeof(int), hipMemcpyDeviceToHost), "copy idx");
  for (int i : idx)
    if (i < 0 || (long long)i >= c->N0) return "receiver index outside the grid";
  if (distinct) {
    std::sort(idx.begin(), idx.end());
    if (std::adjacent_find(idx.begin(), idx.end()) != idx.end()) return "receiver indices must be distinct";
  }
  return std::string();
}
}  // namespace

int helm_sample(helm_ctx* c, int B, int M, const int* idx, const helm_c32* u, helm_c32* y) {
  if (!c || !idx || !u || !y || B < 1 || M < 1) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  const std::string bad = receiver_error(c, M, idx, false);
  if (!bad.empty()) return fail(c, HELM_EINVAL, bad);
  launch_gather(c->s, B, M, c->N0, idx, (const c32*)u, (c32*)y);
  HELM_GUARD_END("sample")
}

int helm_sample_adjoint(helm_ctx* c, int B, int M, const int* idx, const helm_c32* y, helm_c32* u) {
  if (!c || !idx || !u || !y || B < 1 || M < 1) return fail(c, HELM_EINVAL, "bad argument");
  HELM_GUARD_BEGIN
  const std::string bad = receiver_error(c, M, idx, true);
  if (!bad.empty()) return fail(c, HELM_EINVAL, bad);
  launch_zero(c->s, (long long)B * c->N0, (c32*)u);
  launch_scatter(c->s, B, M, c->N0, idx, (const c32*)y, (c32*)u);
  HELM_GUARD_END("sample_adjoint")
}

int helm_tv(helm_ctx* c, const float* n_map, double eps, double scale, float* grad, double* value) {
  if (!c || !n_map || !grad) return fail(c, HELM_EINVAL, "bad argument");
  const int np = tv_partials(c->dim, c->n);
  HELM_GUARD_BEGIN
  launch_tv(c->s, c->dim, c->n, n_map, (float)eps, (float)scale, c->d_tv_mag, c->d_tv_part, grad);
  if (value) {
    std::vector<float> part(np);
    check(hipMemcpyAsync(part.data(), c->d_tv_part, np * sizeof(float), hipMemcpyDeviceToHost, c->s), "tv");
    check(hipStreamSynchronize(c->s), "sync");
    double v = 0.0;
    for (float x : part) v += x;
    *value = v;
  }
  HELM_GUARD_END("tv")
}

// ---------------------------------------------------------------- inverse problem (Sec. V, Alg. 4)
namespace {
void inv_reserve(helm_ctx* c) {
  if (c->d_inv_p) return;
  const long long Ni = npts(c->n, c->dim);
  c->d_inv_p = c->alloc<float>((size_t)c->dim * Ni);
  c->d_inv_r = c->alloc<float>((size_t)c->dim * Ni);
  c->d_inv_w = c->alloc<float>(Ni);
  c->d_inv_v = c->alloc<float>(Ni);
  c->d_inv_n = c->alloc<float>(Ni);
}
}  // namespace

int helm_update_f(helm_ctx* c, const float* f_dev) {
  if (!c || !f_dev) return fail(c, HELM_EINVAL, "null argument");
  try {
    check(hipStreamSynchronize(c->user_s), "caller stream");
    inv_reserve(c);
    launch_index_from_f(c->s, npts(c->n, c->dim), f_dev, 1.0 / (c->k0 * c->k0), c->o.n_b * c->o.n_b, c->d_inv_n);
    check(hipGetLastError(), "index_from_f");
    check(hipStreamSynchronize(c->s), "sync");
    update_medium(c, c->d_inv_n);
  } catch (const HipError& e) {
    return fail(c, HELM_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.code));
  } catch (const std::bad_alloc&) {
    return fail(c, HELM_ENOMEM, "out of host memory");
  }
  return HELM_OK;
}

int helm_update_contrast(helm_ctx* c, const float* chi_dev) {
  if (!c || !chi_dev) return fail(c, HELM_EINVAL, "null argument");
  try {
    check(hipStreamSynchronize(c->user_s), "caller stream");
    inv_reserve(c);
    // eta = sqrt(eta_b^2 + chi): the map of helm_update_f with k0^2 = 1
    launch_index_from_f(c->s, npts(c->n, c->dim), chi_dev, 1.0, c->o.n_b * c->o.n_b, c->d_inv_n);
    check(hipGetLastError(), "index_from_contrast");
    check(hipStreamSynchronize(c->s), "sync");
    update_medium(c, c->d_inv_n);
  } catch (const HipError& e) {
    return fail(c, HELM_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.code));
  } catch (const std::bad_alloc&) {
    return fail(c, HELM_ENOMEM, "out of host memory");
  }
  return HELM_OK;
}

int helm_grad_contrast(helm_ctx* c, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* lam,
                       int accumulate, float* grad) {
  if (!c || !u_sc || !lam || !grad) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1) return fail(c, HELM_EINVAL, "B must be >= 1");
  HELM_GUARD_BEGIN
  launch_grad_n(c->s, c->dim, B, c->ne, c->w, c->n, (const c32*)u_in, (const c32*)u_sc, (const c32*)lam, nullptr,
                (float)(c->k0 * c->k0), grad, nullptr, accumulate ? 1 : 0);
  HELM_GUARD_END("grad_contrast")
}

int helm_grad_f(helm_ctx* c, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* lam, float* grad_f) {
  if (!c || !u_sc || !lam || !grad_f) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1) return fail(c, HELM_EINVAL, "B must be >= 1");
  HELM_GUARD_BEGIN
  launch_grad_n(c->s, c->dim, B, c->ne, c->w, c->n, (const c32*)u_in, (const c32*)u_sc, (const c32*)lam, nullptr,
                1.0f, grad_f);
  HELM_GUARD_END("grad_f")
}

int helm_data_residual(helm_ctx* c, int B, int M, const int* idx_dev, const helm_c32* u, const helm_c32* y,
                       helm_c32* res, double* loss_host) {
  if (!c || !idx_dev || !u || !y || !res) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1 || M < 1) return fail(c, HELM_EINVAL, "B and M must be >= 1");
  HELM_GUARD_BEGIN
  const std::string bad = receiver_error(c, M, idx_dev, false);
  if (!bad.empty()) return fail(c, HELM_EINVAL, bad);
  const int nbk = data_residual_blocks(B, M);
  if (nbk > c->inv_part_len) {
    c->d_inv_part = c->alloc<double>(nbk);
    c->inv_part_len = nbk;
  }
  launch_data_residual(c->s, B, M, c->N0, idx_dev, (const c32*)u, (const c32*)y, (c32*)res, c->d_inv_part);
  if (loss_host) {
    std::vector<double> part(nbk);
    check(hipMemcpyAsync(part.data(), c->d_inv_part, nbk * sizeof(double), hipMemcpyDeviceToHost, c->s), "loss");
    check(hipStreamSynchronize(c->s), "sync");
    double sum = 0.0;
    for (double v : part) sum += v;
    *loss_host = 0.5 * sum;
  }
  HELM_GUARD_END("data_residual")
}

int helm_data_residual_static(helm_ctx* c, int B, int M, const int* idx_dev, const helm_c32* u, const helm_c32* y,
                              helm_c32* res, double* loss_host) {
  if (!c) return HELM_EINVAL;
  if (!idx_dev || !u || !y || !res) return fail_lit(c, HELM_EINVAL, "null argument");
  if (B < 1 || M < 1) return fail_lit(c, HELM_EINVAL, "B and M must be >= 1");
  if ((long long)B * M > HELM_STATIC_MAX_SAMPLES)
    return fail_lit(c, HELM_EINVAL, "B * M exceeds the fixed scratch of helm_data_residual_static (1048576 samples)");
  const int nbk = data_residual_blocks(B, M);
  if (nbk > static_scratch_partials()) return fail_lit(c, HELM_EINVAL, "too many partial sums for the fixed scratch");
  hipError_t e = hipStreamSynchronize(c->user_s);
  double* scr = static_scratch();
  if (!scr && e == hipSuccess) {  // first call on this device
    e = static_scratch_init();
    scr = static_scratch();
  }
  if (e != hipSuccess || !scr) return fail_lit(c, HELM_EHIP, "device scratch address unavailable");
  // receiver indices checked on the device (flag in the scratch), before any read through them
  double flag = 0.0, total = 0.0;
  launch_static_check(c->s, M, c->N0, idx_dev, scr);
  e = hipMemcpyAsync(&flag, static_flag(scr), sizeof(double), hipMemcpyDeviceToHost, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return fail_lit(c, HELM_EHIP, "receiver index check failed");
  if (flag != 0.0) return fail_lit(c, HELM_EINVAL, "receiver index outside the grid");
  launch_data_residual(c->s, B, M, c->N0, idx_dev, (const c32*)u, (const c32*)y, (c32*)res, scr);
  if (loss_host) {
    launch_static_total(c->s, nbk, scr);
    e = hipMemcpyAsync(&total, static_total(scr), sizeof(double), hipMemcpyDeviceToHost, c->s);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return fail_lit(c, HELM_EHIP, "data residual failed");
  if (loss_host) *loss_host = 0.5 * total;
  return HELM_OK;
}


int helm_tv_prox(helm_ctx* c, const float* v_dev, double lam, double lo, int iters, float* w_dev) {
  if (!c || !v_dev || !w_dev) return fail(c, HELM_EINVAL, "null argument");
  if (iters < 0 || !(lam >= 0.0) || !std::isfinite(lam)) return fail(c, HELM_EINVAL, "bad lam or iters");
  HELM_GUARD_BEGIN
  inv_reserve(c);
  launch_tv_prox(c->s, c->dim, c->n, v_dev, (float)lam, (float)lo, iters, c->d_inv_p, c->d_inv_r, c->d_inv_w);
  check(hipMemcpyAsync(w_dev, c->d_inv_w, (size_t)npts(c->n, c->dim) * sizeof(float), hipMemcpyDeviceToDevice, c->s),
        "copy w");
  HELM_GUARD_END("tv_prox")
}

int helm_fbs_step(helm_ctx* c, float* f_dev, float* fbar_dev, const float* grad_dev, double gamma, double tau,
                  double lo, int prox_iters, double* alpha_host) {
  if (!c || !f_dev || !fbar_dev || !grad_dev || !alpha_host) return fail(c, HELM_EINVAL, "null argument");
  if (!(gamma > 0.0) || !(tau >= 0.0) || prox_iters < 0 || !(*alpha_host >= 1.0))
    return fail(c, HELM_EINVAL, "bad gamma, tau, prox_iters or alpha");
  HELM_GUARD_BEGIN
  inv_reserve(c);
  const long long Ni = npts(c->n, c->dim);
  launch_axmy(c->s, Ni, fbar_dev, (float)gamma, grad_dev, c->d_inv_v);
  launch_tv_prox(c->s, c->dim, c->n, c->d_inv_v, (float)(gamma * tau), (float)lo, prox_iters, c->d_inv_p, c->d_inv_r,
                 c->d_inv_w);
  const double a = *alpha_host, an = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * a * a));
  launch_fbs_momentum(c->s, Ni, c->d_inv_w, (float)((a - 1.0) / an), f_dev, fbar_dev);
  *alpha_host = an;
  HELM_GUARD_END("fbs_step")
}

// ---------------------------------------------------------------- sensor operator (eq. DiscreteForwardHelm)
int helm_farfield_set(helm_ctx* c, int M, const double* sensors_host) {
  if (!c || !sensors_host || M < 1) return fail(c, HELM_EINVAL, "bad argument");
  const int dim = c->dim;
  const double half = 0.5 * (c->n - 1);
  double rmin = 1e300, rmax = 0.0;
  for (int m = 0; m < M; ++m) {
    double d2 = 0.0, far2 = 0.0;
    for (int a = 0; a < dim; ++a) {
      const double x = sensors_host[m * dim + a];
      if (!std::isfinite(x)) return fail(c, HELM_EINVAL, "non-finite sensor coordinate");
      const double out = std::fabs(x) - half;
      if (out > 0) d2 += out * out;
      far2 += (std::fabs(x) + half) * (std::fabs(x) + half);
    }
    if (d2 < 1.0) return fail(c, HELM_EINVAL, "a sensor lies within one cell of Omega");
    rmin = std::min(rmin, std::sqrt(d2));
    rmax = std::max(rmax, std::sqrt(far2));
  }
  HELM_GUARD_BEGIN
  const long long Ni = npts(c->n, dim);
  if (M > c->ff_M) {
    c->d_ffG = c->alloc<c32>((size_t)M * Ni);
    c->d_ff_part = c->alloc<c32>((size_t)ff_splits(Ni) * c->o.max_batch * M);
    c->d_ff_iota = c->alloc<int>(M);
    std::vector<int> iota(M);
    for (int m = 0; m < M; ++m) iota[m] = m;
    check(hipMemcpy(c->d_ff_iota, iota.data(), (size_t)M * sizeof(int), hipMemcpyHostToDevice), "iota");
    c->ff_M = M;
  }
  if (!c->d_ff_src) c->d_ff_src = c->alloc<c32>((size_t)c->o.max_batch * Ni);
  // 2D: table of H0^(1) and its derivative -H1^(1) (FP64, host) on the argument range
  std::vector<double2> tab;
  double x0 = 0.0, dx = 1.0;
  int ntab = 2;
  if (dim == 2) {
    dx = 1.0 / 256.0;
    x0 = std::max(1e-3, c->kbh * rmin - 4 * dx);
    ntab = (int)std::ceil((c->kbh * rmax + 4 * dx - x0) / dx) + 2;
    tab.resize(2 * (size_t)ntab);
    for (int k = 0; k < ntab; ++k) {
      const double x = x0 + k * dx;
      tab[2 * k] = make_double2(std::cyl_bessel_j(0.0, x), std::cyl_neumann(0.0, x));
      tab[2 * k + 1] = make_double2(-std::cyl_bessel_j(1.0, x), -std::cyl_neumann(1.0, x));
    }
  } else {
    tab.assign(4, make_double2(0.0, 0.0));
  }
  void* d_tab = nullptr;
  void* d_sens = nullptr;
  check(hipMalloc(&d_tab, tab.size() * sizeof(double2)), "hipMalloc");
  if (hipMalloc(&d_sens, (size_t)M * dim * sizeof(double)) != hipSuccess) {
    hipFree(d_tab);
    throw HipError{hipErrorOutOfMemory, "hipMalloc"};
  }
  hipError_t e = hipMemcpyAsync(d_tab, tab.data(), tab.size() * sizeof(double2), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_sens, sensors_host, (size_t)M * dim * sizeof(double), hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) {
    launch_ff_matrix(c->s, dim, c->n, M, (const double*)d_sens, c->kbh, c->h, (const double2*)d_tab, x0, dx, ntab,
                     c->d_ffG);
    e = hipStreamSynchronize(c->s);
  }
  hipFree(d_tab);
  hipFree(d_sens);
  check(e, "farfield matrix");
  c->ff_M = std::max(c->ff_M, M);
  c->ff_active_M = M;
  HELM_GUARD_END("farfield_set")
}

int helm_farfield(helm_ctx* c, int B, const helm_c32* u_in, const helm_c32* u_sc, helm_c32* y) {
  if (!c || !u_sc || !y) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1 || B > c->o.max_batch) return fail(c, HELM_EINVAL, "B must be in [1, max_batch]");
  if (!c->ff_active_M) return fail(c, HELM_ESTATE, "no sensors: call helm_farfield_set first");
  HELM_GUARD_BEGIN
  launch_ff_forward(c->s, c->dim, B, c->ff_active_M, c->ne, c->w, c->n, c->d_f, (const c32*)u_in, (const c32*)u_sc,
                    c->d_ffG, c->d_ff_src, c->d_ff_part, (c32*)y);
  HELM_GUARD_END("farfield")
}

int helm_farfield_residual(helm_ctx* c, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* y_meas,
                           helm_c32* y, helm_c32* res, double* loss_host) {
  if (!c || !u_sc || !y_meas || !y || !res) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1 || B > c->o.max_batch) return fail(c, HELM_EINVAL, "B must be in [1, max_batch]");
  if (!c->ff_active_M) return fail(c, HELM_ESTATE, "no sensors: call helm_farfield_set first");
  const int M = c->ff_active_M;
  HELM_GUARD_BEGIN
  launch_ff_forward(c->s, c->dim, B, M, c->ne, c->w, c->n, c->d_f, (const c32*)u_in, (const c32*)u_sc, c->d_ffG,
                    c->d_ff_src, c->d_ff_part, (c32*)y);
  const int nbk = data_residual_blocks(B, M);
  if (nbk > c->inv_part_len) {
    c->d_inv_part = c->alloc<double>(nbk);
    c->inv_part_len = nbk;
  }
  // res = y - y_meas as the data residual of the identity "receivers" 0 .. M-1 of y
  launch_data_residual(c->s, B, M, M, c->d_ff_iota, (const c32*)y, (const c32*)y_meas, (c32*)res, c->d_inv_part);
  if (loss_host) {
    std::vector<double> part(nbk);
    check(hipMemcpyAsync(part.data(), c->d_inv_part, nbk * sizeof(double), hipMemcpyDeviceToHost, c->s), "loss");
    check(hipStreamSynchronize(c->s), "sync");
    double sum = 0.0;
    for (double v : part) sum += v;
    *loss_host = 0.5 * sum;
  }
  HELM_GUARD_END("farfield_residual")
}

int helm_farfield_adjoint(helm_ctx* c, int B, const helm_c32* r, helm_c32* s_ext, helm_c32* rhs_ext) {
  if (!c || !r || !s_ext) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1) return fail(c, HELM_EINVAL, "B must be >= 1");
  if (!c->ff_active_M) return fail(c, HELM_ESTATE, "no sensors: call helm_farfield_set first");
  HELM_GUARD_BEGIN
  launch_zero(c->s, (long long)B * c->N0, (c32*)s_ext);
  if (rhs_ext) launch_zero(c->s, (long long)B * c->N0, (c32*)rhs_ext);
  launch_ff_adjoint(c->s, c->dim, B, c->ff_active_M, c->ne, c->w, c->n, c->d_ffG, (const c32*)r, c->d_f, (c32*)s_ext,
                    (c32*)rhs_ext);
  HELM_GUARD_END("farfield_adjoint")
}

int helm_grad_f_farfield(helm_ctx* c, int B, const helm_c32* u_in, const helm_c32* u_sc, const helm_c32* lam,
                         const helm_c32* s_ext, float* grad_f) {
  if (!c || !u_sc || !lam || !s_ext || !grad_f) return fail(c, HELM_EINVAL, "null argument");
  if (B < 1) return fail(c, HELM_EINVAL, "B must be >= 1");
  HELM_GUARD_BEGIN
  launch_grad_n(c->s, c->dim, B, c->ne, c->w, c->n, (const c32*)u_in, (const c32*)u_sc, (const c32*)lam, nullptr,
                1.0f, grad_f, (const c32*)s_ext);
  HELM_GUARD_END("grad_f_farfield")
}

const char* helm_last_error(const helm_ctx* c) {
  if (!c) return g_setup_error.c_str();
  return c->err_lit ? c->err_lit : c->err.c_str();
}

void helm_destroy(helm_ctx* c) {
  if (!c) return;
  hipStreamSynchronize(c->s);
  free_ctx(c);
}

}  // extern "C"
