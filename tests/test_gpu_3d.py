"""3D parity (7-point stencil, 27-point full weighting, trilinear prolongation) against the oracle.

Beyond the paper (its conclusion names 3D as future work): every 2D rule is
extended axis by axis; the oracle assembles the same operators with
Kronecker products of the 1D ghost-row second difference.
"""
import numpy as np
import pytest

import synth
from oracle import model
from oracle.discretization import helmholtz_matrix
from oracle.multigrid import Hierarchy

from .helpers import gpu_context, medium, oracle_problem, rel, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cube():
    n, w, levels = 16, 4, 3
    print(f"\n[3D case n={n} w={w} levels={levels}]", flush=True)
    nmap = medium(n, d=3, seed=4)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=4)
    assert ctx.n_e == prob.n_e and ctx.dim == 3
    yield prob, ctx, Hierarchy(prob)
    ctx.close()


def test_operators_3d(cube):
    prob, ctx, hier = cube
    x = synth.complex_field((2, *prob.shape), 1)
    y = to_np(ctx.apply_A(to_dev(x)))
    a = helmholtz_matrix(prob, scaled=False)
    assert rel(y, np.stack([(a @ xi.ravel()).reshape(prob.shape) for xi in x])) < 2e-6
    for l in range(hier.levels):
        shape = (hier.sizes[l],) * 3
        xl = synth.complex_field((2, *shape), 2 + l)
        yl = to_np(ctx.apply_K(l, to_dev(xl)))
        assert rel(yl, np.stack([(hier.K[l] @ xi.ravel()).reshape(shape) for xi in xl])) < 2e-6
    for l in range(hier.levels - 1):
        f = synth.complex_field((2, *(hier.sizes[l],) * 3), 10 + l)
        cshape = (hier.sizes[l + 1],) * 3
        rc = to_np(ctx.restrict(l, to_dev(f)))
        assert rel(rc, np.stack([4 * (hier.R[l] @ fi.ravel()).reshape(cshape) for fi in f])) < 1e-6
        e = synth.complex_field((2, *cshape), 20 + l)
        base = np.zeros_like(f)
        out = to_np(ctx.prolong_add(l, to_dev(e), to_dev(base)))
        assert rel(out, np.stack([(hier.P[l] @ ei.ravel()).reshape(f.shape[1:]) for ei in e])) < 1e-6


def test_vcycle_3d(cube):
    prob, ctx, hier = cube
    r = synth.complex_field((2, *prob.shape), 30)
    z = to_np(ctx.precondition(to_dev(r)))
    assert rel(z, np.stack([hier.vcycle(ri.ravel()).reshape(prob.shape) for ri in r])) < 1e-5


def test_solve_adjoint_and_gradient_3d(cube):
    prob, ctx, _ = cube
    dirs = synth.directions_cone(3)
    rhs, uin = ctx.plane_wave_rhs(dirs, with_uin=True)
    b = to_np(rhs)
    for q, d in enumerate(dirs):
        assert rel(b[q], model.rhs(prob, d)) < 1e-6
    x, st = ctx.solve(rhs)
    assert st.converged and np.all(st.rel_res_true <= 1e-6)
    ex = model.ExactSolver(prob)
    u = np.stack([ex.solve(bi) for bi in b])
    assert rel(to_np(x), u) < 1e-5
    g = synth.complex_field((3, *prob.shape), 40).astype(np.complex64)
    lam, st = ctx.adjoint(to_dev(g))
    assert st.converged
    lam_ref = np.stack([ex.solve_adjoint(gi.astype(np.complex128)) for gi in g])
    assert rel(to_np(lam), lam_ref) < 1e-5
    grad = ctx.grad_n(x, lam, u_in=uin).cpu().numpy().astype(np.float64)
    ref = model.scalar_field_gradient(prob, u + to_np(uin), lam_ref)
    assert np.linalg.norm(grad - ref) / np.linalg.norm(ref) < 1e-4


@pytest.mark.parametrize("cycle", [1, 3])
def test_fused_3d_legs_match_oracle_over_several_tiles(cycle):
    """The fused 3D legs on three levels (the single-launch coarse cycle off), on a 49^3 grid:
    down-leg tiles of 8x4x4 coarse points and up-leg tiles of 16x8x8 fine points, both ragged
    at every level; the cycle equals the oracle's and the generic kernels' (fused off)."""
    n, w, levels = 40, 4, 4
    print(f"\n[3D fused legs n={n} levels={levels} cycle={cycle}]", flush=True)
    nmap = medium(n, d=3, seed=9)
    prob = oracle_problem(nmap, w=w, levels=levels)
    hier = Hierarchy(prob)
    r = synth.complex_field((3, *prob.shape), 31)
    gamma = [2] + [1] * (levels - 1) if cycle == 3 else 1
    ref = np.stack([hier.cycle(ri.ravel(), None, 0, gamma).reshape(prob.shape) for ri in r])
    out = {}
    for fused in (1, 0):
        ctx = gpu_context(nmap, w=w, levels=levels, max_batch=3, cycle=cycle, fused=fused, coarse_single_launch=0)
        assert ctx.n_e == prob.n_e == 49
        out[fused] = to_np(ctx.precondition(to_dev(r)))
        ctx.close()
    assert rel(out[1], ref) < 1e-5
    assert rel(out[1], out[0]) < 1e-5


def test_float_float_residual_3d(cube):
    """The 3D float-float true residual (z-marching kernel: 64 x 8 columns over 16 planes, here
    ragged in x and y and split 16 + 9 in z on the 25^3 grid) against FP64: r = b - A (x_hi + x_lo)
    to far below complex64 resolution."""
    prob, ctx, _ = cube
    ex = model.ExactSolver(prob)
    b = np.stack([model.rhs(prob, d) for d in synth.directions_cone(2)])
    u = np.stack([ex.solve(bi) for bi in b])
    x_hi = u.astype(np.complex64)
    x_lo = (u - x_hi.astype(np.complex128)).astype(np.complex64)
    b32 = b.astype(np.complex64)
    r = to_np(ctx.residual(to_dev(b32), to_dev(x_hi), to_dev(x_lo)))
    xs = x_hi.astype(np.complex128) + x_lo.astype(np.complex128)
    ref = np.stack([b32[q].astype(np.complex128).ravel() - ex.A @ xs[q].ravel() for q in range(2)]).reshape(r.shape)
    bn = np.linalg.norm(b32.ravel())
    assert np.linalg.norm((r - ref).ravel()) / bn < 1e-9
    assert np.linalg.norm(ref.ravel()) / bn < 1e-7
    r32 = to_np(ctx.residual(to_dev(b32), to_dev(x_hi)))
    assert np.linalg.norm(r32.ravel()) / bn > 1e-8


def test_bicgstab_3d(cube):
    """The paper's Alg. 3 in 3D (its decision kernel sums the marching residual's per-tile partial
    norms): converged, certified by the oracle's FP64 operator, and the exact solution."""
    from paper_2107_03679_amd import helm

    prob, _, _ = cube
    nmap = medium(16, d=3, seed=4)
    ctx = gpu_context(nmap, w=4, levels=3, max_batch=2, krylov=helm.KRYLOV_BICGSTAB, restart=8)
    rhs = ctx.plane_wave_rhs(synth.directions_cone(2))
    x, st = ctx.solve(rhs)
    assert st.converged and np.all(st.rel_res_true <= 1e-6), st
    lo = to_np(ctx.solution_lo(2))
    b = to_np(rhs)
    ex = model.ExactSolver(prob)
    for q in range(2):
        rq = np.linalg.norm(b[q].ravel() - ex.A @ (to_np(x)[q] + lo[q]).ravel()) / np.linalg.norm(b[q].ravel())
        assert rq <= 1.05e-6, (q, rq)
        assert rel(to_np(x)[q], ex.solve(b[q])) < 1e-5, q
    ctx.close()
