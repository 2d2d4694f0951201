"""GPU parity: every building block and the full batched solve against the FP64 oracle.

All calls go through the C ABI (libhelm.so via the ctypes binding).  Sizes
span several LDS tiles with ragged tails (the fused kernels use 64 x 16 fine
tiles); tolerances follow from complex64 arithmetic (unit roundoff 6e-8)
and, for solves, from the 1e-6 residual target (the field-parity target 1e-5).
"""
import numpy as np
import pytest

import synth
from oracle import model
from oracle.discretization import helmholtz_matrix
from oracle.multigrid import Hierarchy

from .helpers import gpu_context, medium, oracle_problem, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = {
    # name: (interior n, layer w, levels) -> n_e spans 1..4 tiles with ragged tails
    "small": (40, 8, 3),
    "ragged": (150, 20, 4),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    n, w, levels = CASES[request.param]
    print(f"\n[case {request.param}: n={n} w={w} levels={levels}]", flush=True)
    nmap = medium(n)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=8)
    assert ctx.n_e == prob.n_e
    yield prob, ctx, Hierarchy(prob)
    ctx.close()


def fields(shape, B, seed):
    return synth.complex_field((B, *shape), seed)


def test_apply_A(pair):
    prob, ctx, _ = pair
    x = fields(prob.shape, 3, 1)
    y = to_np(ctx.apply_A(to_dev(x)))
    a = helmholtz_matrix(prob, scaled=False)
    ref = np.stack([(a @ xi.ravel()).reshape(prob.shape) for xi in x])
    assert rel(y, ref) < 2e-6


def test_apply_K_every_level(pair):
    prob, ctx, hier = pair
    for l in range(hier.levels):
        shape = (hier.sizes[l],) * prob.d
        x = fields(shape, 2, 10 + l)
        y = to_np(ctx.apply_K(l, to_dev(x)))
        ref = np.stack([(hier.K[l] @ xi.ravel()).reshape(shape) for xi in x])
        assert rel(y, ref) < 2e-6, l


def test_restrict_and_prolong(pair):
    prob, ctx, hier = pair
    for l in range(hier.levels - 1):
        fshape = (hier.sizes[l],) * prob.d
        cshape = (hier.sizes[l + 1],) * prob.d
        f = fields(fshape, 2, 20 + l)
        rc = to_np(ctx.restrict(l, to_dev(f)))
        ref = np.stack([4.0 * (hier.R[l] @ fi.ravel()).reshape(cshape) for fi in f])
        assert rel(rc, ref) < 1e-6
        e = fields(cshape, 2, 30 + l)
        base = fields(fshape, 2, 40 + l)
        out = to_np(ctx.prolong_add(l, to_dev(e), to_dev(base)))
        ref = np.stack([bi + (hier.P[l] @ ei.ravel()).reshape(fshape) for bi, ei in zip(base, e)])
        assert rel(out, ref) < 1e-6


def test_coarse_solve(pair):
    prob, ctx, hier = pair
    shape = (hier.sizes[-1],) * prob.d
    r = fields(shape, 5, 50)
    z = to_np(ctx.coarse_solve(to_dev(r)))
    ref = np.stack([hier.coarse_lu.solve(ri.ravel()).reshape(shape) for ri in r])
    assert rel(z, ref) < 1e-5


def test_vcycle_fused_matches_oracle(pair):
    prob, ctx, hier = pair
    r = fields(prob.shape, 3, 60)
    z = to_np(ctx.precondition(to_dev(r)))
    ref = np.stack([hier.vcycle(ri.ravel()).reshape(prob.shape) for ri in r])
    assert rel(z, ref) < 1e-5


@pytest.mark.parametrize("variant", ["generic_v", "generic_nu2", "w_cycle", "per_level_launch", "per_level_launch_b5",
                                     "top_w", "generic_w"])
def test_cycle_variants_match_oracle(variant):
    """Cycle variants against the oracle's Alg. 2; per_level_launch_b5 runs the coarsest solve
    as one matrix product over its 5 right-hand sides."""
    n, w, levels = CASES["ragged"]
    nmap = medium(n, seed=3)
    nu = 2 if variant == "generic_nu2" else 1
    cyc = {"w_cycle": 2, "generic_w": 2, "top_w": 3}.get(variant, 1)
    print(f"\n[cycle variant {variant}]", flush=True)
    prob = oracle_problem(nmap, w=w, levels=levels, nu=nu)
    hier = Hierarchy(prob)
    ctx = gpu_context(nmap, w=w, levels=levels, nu=nu, cycle=cyc, fused=0 if variant.startswith("generic") else 1,
                      coarse_single_launch=0 if variant.startswith("per_level_launch") else 1,
                      max_batch=5 if variant.endswith("b5") else 2)
    r = fields(prob.shape, 5 if variant.endswith("b5") else 2, 61)
    z = to_np(ctx.precondition(to_dev(r)))
    oracle_ct = [2] + [1] * (levels - 2) if cyc == 3 else cyc
    ref = np.stack([hier.cycle(ri.ravel(), None, 0, oracle_ct).reshape(prob.shape) for ri in r])
    ctx.close()
    assert rel(z, ref) < 1e-5


def test_plane_wave_rhs(pair):
    prob, ctx, _ = pair
    dirs = synth.directions_2d(5)
    rhs, uin = ctx.plane_wave_rhs(dirs, with_uin=True)
    rhs, uin = to_np(rhs), to_np(uin)
    for q, d in enumerate(dirs):
        assert rel(uin[q], model.plane_wave(prob, d)) < 1e-6
        assert rel(rhs[q], model.rhs(prob, d)) < 1e-6


def test_float_float_residual(pair):
    # r = b - A (x_hi + x_lo) to far below complex64 resolution
    prob, ctx, _ = pair
    ex = model.ExactSolver(prob)
    b = np.stack([model.rhs(prob, d) for d in synth.directions_2d(2)])
    u = np.stack([ex.solve(bi) for bi in b])
    x_hi = u.astype(np.complex64)
    x_lo = (u - x_hi.astype(np.complex128)).astype(np.complex64)
    b32 = b.astype(np.complex64)
    r = to_np(ctx.residual(to_dev(b32), to_dev(x_hi), to_dev(x_lo)))
    a = ex.A
    xs = x_hi.astype(np.complex128) + x_lo.astype(np.complex128)
    ref = np.stack([b32[q].astype(np.complex128).ravel() - a @ xs[q].ravel() for q in range(2)]).reshape(r.shape)
    bn = np.linalg.norm(b32.ravel())
    assert np.linalg.norm((r - ref).ravel()) / bn < 1e-9
    # x_hi + x_lo solves A x = b to ~1e-14; what remains is the complex64 rounding of b itself
    assert np.linalg.norm(ref.ravel()) / bn < 1e-7
    # with x_hi alone the complex64 floor shows up
    r32 = to_np(ctx.residual(to_dev(b32), to_dev(x_hi)))
    assert np.linalg.norm(r32.ravel()) / bn > 1e-8


def test_batched_solve_matches_exact_solution(pair):
    prob, ctx, _ = pair
    dirs = synth.directions_2d(4)
    rhs = ctx.plane_wave_rhs(dirs)
    x, st = ctx.solve(rhs)
    assert st.converged, st
    assert np.all(st.rel_res_true <= 1e-6)
    ex = model.ExactSolver(prob)
    b = to_np(rhs)
    u = np.stack([ex.solve(bi) for bi in b])
    xh = to_np(x)
    lo = to_np(ctx.solution_lo(4))
    for q in range(4):
        assert rel(xh[q], u[q]) < 1e-5, q
        # host FP64 residual of the float-float iterate certifies the 1e-6 claim
        xs = xh[q] + lo[q]
        rq = np.linalg.norm(b[q].ravel() - ex.A @ xs.ravel()) / np.linalg.norm(b[q].ravel())
        assert rq <= 1.05e-6
        assert rq == pytest.approx(st.rel_res_true[q], rel=0.05, abs=1e-9)
    # restart cycles within one of the oracle's FP64 FGMRES(m) at equal parameters (the s-step
    # form spends whole cycles: its count is m per cycle)
    m = ctx.opts.restart
    _, info = model.mg_fgmres_solve(prob, model.rhs(prob, dirs[0]), rtol=1e-6, restart=m)
    assert st.iters[0] % m == 0
    assert abs(st.iters[0] // m - -(-info.iters // m)) <= 1


@pytest.mark.parametrize("case,m", [("small", 3), ("small", 5), ("small", 8), ("small", 12), ("ragged", 5)])
def test_sstep_and_fgmres_reach_the_same_solution(case, m):
    """GMRES(m) in s-step form and as FGMRES(m) minimise over the same Krylov space: same
    solution, same number of restart cycles (up to one) as the oracle's FP64 FGMRES(m)."""
    from paper_2107_03679_amd import helm

    n, w, levels = CASES[case]
    print(f"\n[s-step vs FGMRES: {case} m={m}]", flush=True)
    nmap = medium(n, seed=3)
    prob = oracle_problem(nmap, w=w, levels=levels)
    dirs = synth.directions_2d(3)
    ex = model.ExactSolver(prob)
    out = {}
    for kry in (helm.KRYLOV_FGMRES, helm.KRYLOV_SSTEP):
        ctx = gpu_context(nmap, w=w, levels=levels, max_batch=3, restart=m, krylov=kry)
        rhs = ctx.plane_wave_rhs(dirs)
        x, st = ctx.solve(rhs)
        assert st.converged and np.all(st.rel_res_true <= 1e-6), (kry, st)
        b = to_np(rhs)
        for q in range(3):
            assert rel(to_np(x)[q], ex.solve(b[q])) < 1e-5, (kry, q)
        out[kry] = st
        ctx.close()
    _, info = model.mg_fgmres_solve(prob, model.rhs(prob, dirs[0]), rtol=1e-6, restart=m)
    cycles = -(-info.iters // m)
    assert np.all(out[helm.KRYLOV_SSTEP].iters % m == 0)
    assert abs(out[helm.KRYLOV_SSTEP].iters[0] // m - cycles) <= 1
    assert abs(-(-out[helm.KRYLOV_FGMRES].iters[0] // m) - cycles) <= 1


@pytest.mark.parametrize("case,cycle", [("small", 3), ("ragged", 3), ("ragged", 1)])
def test_fused_finest_step_matches_separate_kernels(case, cycle):
    """The s-step basis with its finest-level work fused into one kernel per step (up-leg,
    basis matvec, next down-leg; or the up-leg and basis matvec only) against the same basis
    from the separate kernels: the same exact solution and the same restart cycles (up to
    one: the matvec's sum order differs)."""
    n, w, levels = CASES[case]
    print(f"\n[fused finest step: {case} cycle={cycle}]", flush=True)
    nmap = medium(n, seed=23)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ex = model.ExactSolver(prob)
    dirs = synth.directions_2d(3)
    out = {}
    for fs in (1, 2, 0):
        ctx = gpu_context(nmap, w=w, levels=levels, max_batch=3, restart=5, cycle=cycle, fused_step=fs)
        rhs = ctx.plane_wave_rhs(dirs)
        x, st = ctx.solve(rhs)
        assert st.converged and np.all(st.rel_res_true <= 1e-6), (fs, st)
        b = to_np(rhs)
        for q in range(3):
            assert rel(to_np(x)[q], ex.solve(b[q])) < 1e-5, (fs, q)
        out[fs] = (to_np(x), st)
        ctx.close()
    for fs in (1, 2):
        assert rel(out[fs][0], out[0][0]) < 2e-5, fs
        assert np.all(np.abs(out[fs][1].iters - out[0][1].iters) <= 5), (fs, out[fs][1].iters, out[0][1].iters)


@pytest.mark.parametrize("case", ["small", "ragged"])
def test_bicgstab_alg3_matches_exact_solution(case):
    """The paper's Alg. 3 (batched Bi-CGSTAB, two cycles per iteration): the exact solution to
    the 1e-5 field bar, a certified true residual, and about the oracle's FP64 iteration count."""
    from paper_2107_03679_amd import helm

    n, w, levels = CASES[case]
    print(f"\n[Bi-CGSTAB: {case}]", flush=True)
    nmap = medium(n, seed=5)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=3, krylov=helm.KRYLOV_BICGSTAB, restart=8)
    dirs = synth.directions_2d(3)
    rhs = ctx.plane_wave_rhs(dirs)
    x, st = ctx.solve(rhs)
    assert st.converged and np.all(st.rel_res_true <= 1e-6), st
    assert np.all(st.iters % 2 == 0)
    ex = model.ExactSolver(prob)
    b = to_np(rhs)
    lo = to_np(ctx.solution_lo(3))
    for q in range(3):
        u = ex.solve(b[q])
        assert rel(to_np(x)[q], u) < 1e-5, q
        xs = to_np(x)[q] + lo[q]
        rq = np.linalg.norm(b[q].ravel() - ex.A @ xs.ravel()) / np.linalg.norm(b[q].ravel())
        assert rq <= 1.05e-6
    _, info = model.mg_bicgstab_solve(prob, model.rhs(prob, dirs[0]), rtol=1e-6)
    assert info.converged
    assert abs(st.iters[0] - info.iters) <= max(6, 0.2 * info.iters), (st.iters, info.iters)
    ctx.close()


def test_adjoint_solve(pair):
    prob, ctx, _ = pair
    g = fields(prob.shape, 2, 70).astype(np.complex64)
    lam, st = ctx.adjoint(to_dev(g))
    assert st.converged
    ex = model.ExactSolver(prob)
    ref = np.stack([ex.solve_adjoint(gi.astype(np.complex128)) for gi in g])
    assert rel(to_np(lam), ref) < 1e-5


def test_grad_n_kernel(pair):
    prob, ctx, _ = pair
    u = fields(prob.shape, 3, 80).astype(np.complex64)
    lam = fields(prob.shape, 3, 81).astype(np.complex64)
    uin = fields(prob.shape, 3, 82).astype(np.complex64)
    g = ctx.grad_n(to_dev(u), to_dev(lam)).cpu().numpy().astype(np.float64)
    ref = model.scalar_field_gradient(prob, u.astype(np.complex128), lam.astype(np.complex128))
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-5
    g2 = ctx.grad_n(to_dev(u), to_dev(lam), u_in=to_dev(uin)).cpu().numpy().astype(np.float64)
    ref2 = model.scalar_field_gradient(prob, u.astype(np.complex128) + uin, lam.astype(np.complex128))
    assert np.linalg.norm(g2 - ref2) / np.linalg.norm(ref2) < 1e-5


def test_solve_is_deterministic(pair):
    _, ctx, _ = pair
    rhs = ctx.plane_wave_rhs(synth.directions_2d(2))
    x1, _ = ctx.solve(rhs)
    x2, _ = ctx.solve(rhs)
    assert bool((x1 == x2).all())


def test_edge_cases_zero_nan_and_iteration_cap():
    n, w, levels = CASES["small"]
    nmap = medium(n, seed=9)
    print("\n[edge cases]", flush=True)
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=4)
    rhs = ctx.plane_wave_rhs(synth.directions_2d(3))
    rhs[1].zero_()
    rhs[2, 5, 5] = complex(float("nan"), 0.0)
    x, st = ctx.solve(rhs)
    assert st.status[0] == 0 and st.rel_res_true[0] <= 1e-6
    assert st.status[1] == 0 and st.iters[1] == 0 and float(x[1].abs().max()) == 0.0
    assert st.status[2] == 2  # breakdown flagged only for the poisoned right-hand side
    ctx.close()
    # the iteration cap is checked per step (FGMRES) or per restart cycle (s-step form)
    for kry, expect in ((0, 1), (1, 10)):
        ctx = gpu_context(nmap, w=w, levels=levels, max_batch=2, max_iters=1, krylov=kry, restart=10)
        x, st = ctx.solve(ctx.plane_wave_rhs(synth.directions_2d(2)))
        assert np.all(st.status == 1) and np.all(st.iters == expect), (kry, st)
        assert np.all((st.rel_res_true > 0) & (st.rel_res_true < 1))
        ctx.close()


def test_options_restart_levels_and_no_graph():
    n, w, levels = CASES["small"]
    nmap = medium(n, seed=11)
    print("\n[options]", flush=True)
    prob = oracle_problem(nmap, w=w, levels=2)
    ex = model.ExactSolver(prob)
    for opts in (dict(levels=2, restart=1), dict(levels=2, restart=1, krylov=0),
                 dict(levels=2, restart=30, use_graph=0, krylov=0), dict(levels=2, restart=12, use_graph=0),
                 dict(levels=2, reorth=1, krylov=0)):
        ctx = gpu_context(nmap, w=w, max_batch=1, **opts)
        rhs = ctx.plane_wave_rhs(synth.directions_2d(1))
        x, st = ctx.solve(rhs)
        assert st.converged, opts
        assert rel(to_np(x)[0], ex.solve(to_np(rhs)[0])) < 1e-5, opts
        ctx.close()


def test_graph_replays_match_eager_launches():
    """One hipGraph per restart cycle, replayed every cycle: two solves in a row with the
    graph (the second replays the first's capture) against the same solves launched eagerly,
    with eager work (right-hand sides, a residual) and synchronisations in between.  The
    kernels are the same, so the results must agree bit for bit after every replay."""
    n, w, levels = CASES["ragged"]
    nmap = medium(n, seed=29)
    print("\n[graph replays vs eager]", flush=True)
    dirs = synth.directions_2d(3)
    out = {}
    for graph in (1, 0):
        ctx = gpu_context(nmap, w=w, levels=levels, max_batch=3, cycle=3, use_graph=graph)
        res = []
        for rep in range(2):
            rhs = ctx.plane_wave_rhs(dirs if rep == 0 else dirs[::-1].copy())
            x, st = ctx.solve(rhs)
            assert st.converged, (graph, rep, st)
            import torch

            ctx.residual(rhs, x)  # eager work between the solves
            torch.cuda.synchronize()
            res.append((to_np(x), st.iters.copy()))
        out[graph] = res
        ctx.close()
    for rep in range(2):
        assert np.array_equal(out[1][rep][0], out[0][rep][0]), rep
        assert np.array_equal(out[1][rep][1], out[0][rep][1]), rep
