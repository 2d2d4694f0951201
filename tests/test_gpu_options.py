"""GPU parity for the solver options beside the defaults: the shift kappa (Sec. IV-B; kappa = 1 is
the paper's operator), the printed layer sign and the second layer profile (Sec. IV-A), with
max-abs checks on the boundary ring and corners (where the ghost and layer terms live), plus
argument checks of the binding and one network shared by two contexts."""
import numpy as np
import pytest

import synth
from oracle import model
from oracle.multigrid import Hierarchy

from .helpers import gpu_context, medium, oracle_problem, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

N, W, LEVELS = 40, 8, 3
KAPPAS = [1.0 + 0.0j, 1.0 + 0.5j, 1.0 - 0.5j]
OPTION_CASES = [(k, s, p) for k in KAPPAS for s in (1, -1) for p in (0, 1)]


def ring_mask(shape, width=2):
    """Points within `width` of the edge of the grid (boundary rows, corners, outer layer)."""
    m = np.zeros(shape, dtype=bool)
    for ax in range(len(shape)):
        sl = [slice(None)] * len(shape)
        sl[ax] = slice(0, width)
        m[tuple(sl)] = True
        sl[ax] = slice(shape[ax] - width, shape[ax])
        m[tuple(sl)] = True
    return m


def ring_err(y, ref):
    """max |y - ref| on the boundary ring of every field, relative to max |ref| of that field."""
    m = ring_mask(ref.shape[1:])
    return max(float(np.abs(y[q] - ref[q])[m].max() / np.abs(ref[q]).max()) for q in range(ref.shape[0]))


@pytest.mark.parametrize("kappa,sign,profile", OPTION_CASES)
def test_operators_and_cycle_for_options(kappa, sign, profile):
    print(f"\n[options kappa={kappa} sign={sign} profile={profile}]", flush=True)
    nmap = medium(N, seed=11)
    prob = oracle_problem(nmap, w=W, levels=LEVELS, kappa=kappa, sign=sign, profile=profile, beta=0.6)
    hier = Hierarchy(prob)
    ctx = gpu_context(nmap, w=W, levels=LEVELS, kappa=kappa, sign=sign, profile=profile, beta=0.6, max_batch=2)
    try:
        for l in range(hier.levels):
            shape = (hier.sizes[l],) * prob.d
            x = synth.complex_field((2, *shape), 100 + l)
            y = to_np(ctx.apply_K(l, to_dev(x)))
            ref = np.stack([(hier.K[l] @ xi.ravel()).reshape(shape) for xi in x])
            assert rel(y, ref) < 2e-6, l
            assert ring_err(y, ref) < 2e-6, l
        r = synth.complex_field((2, *prob.shape), 7)
        z = to_np(ctx.precondition(to_dev(r)))
        ref = np.stack([hier.vcycle(ri.ravel()).reshape(prob.shape) for ri in r])
        assert rel(z, ref) < 1e-5
        assert ring_err(z, ref) < 1e-5
    finally:
        ctx.close()


@pytest.mark.parametrize("sign,profile", [(-1, 0), (1, 1)])
def test_converged_solve_for_layer_options(sign, profile):
    # the printed layer sign and the second profile: converged batched solves against sparse LU
    print(f"\n[layer option solve sign={sign} profile={profile}]", flush=True)
    n, w, levels, B = 64, 16, 4, 3
    nmap = medium(n, seed=12)
    prob = oracle_problem(nmap, w=w, levels=levels, sign=sign, profile=profile)
    ctx = gpu_context(nmap, w=w, levels=levels, sign=sign, profile=profile, max_batch=B, rtol=1e-7)
    try:
        rhs = ctx.plane_wave_rhs(synth.directions_2d(B))
        x, st = ctx.solve(rhs)
        assert st.converged and np.all(st.rel_res_true <= 1e-7)
        lo = to_np(ctx.solution_lo(B))
        ex = model.ExactSolver(prob)
        b = to_np(rhs)
        for q in range(B):
            u = ex.solve(b[q])
            xq = to_np(x)[q] + lo[q]
            assert rel(xq, u) < 1e-5, q
            assert ring_err(xq[None], u[None]) < 1e-5, q
    finally:
        ctx.close()


def test_apply_A_ring_and_corners():
    n, w, levels = 40, 8, 3
    nmap = medium(n, seed=13)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=2)
    try:
        from oracle.discretization import helmholtz_matrix

        x = synth.complex_field((2, *prob.shape), 14)
        y = to_np(ctx.apply_A(to_dev(x)))
        a = helmholtz_matrix(prob, scaled=False)
        ref = np.stack([(a @ xi.ravel()).reshape(prob.shape) for xi in x])
        assert ring_err(y, ref) < 2e-6
        ne = prob.n_e
        for (i, j) in ((0, 0), (0, ne - 1), (ne - 1, 0), (ne - 1, ne - 1)):  # corners: two ghosts each
            assert abs(y[0, i, j] - ref[0, i, j]) <= 2e-6 * np.abs(ref[0]).max()
    finally:
        ctx.close()


def test_receiver_indices_are_checked():
    import torch

    from paper_2107_03679_amd import helm

    nmap = medium(24, seed=1)
    ctx = gpu_context(nmap, w=4, levels=2, max_batch=2)
    try:
        ne = ctx.n_e
        u = to_dev(synth.complex_field((2, ne, ne), 3))
        good = torch.tensor([0, 5, ne * ne - 1], dtype=torch.int32, device="cuda")
        assert ctx.sample(good, u).shape == (2, 3)
        for bad in ([0, ne * ne], [-1, 2]):
            with pytest.raises(helm.HelmError, match="outside the grid"):
                ctx.sample(torch.tensor(bad, dtype=torch.int32, device="cuda"), u)
        y = to_dev(synth.complex_field((2, 3), 4))
        with pytest.raises(helm.HelmError, match="distinct"):
            ctx.sample_adjoint(torch.tensor([4, 9, 4], dtype=torch.int32, device="cuda"), y)
        with pytest.raises(helm.HelmError, match="int32"):
            ctx.sample(good.to(torch.int64), u)
        with pytest.raises(helm.HelmError, match="complex64"):
            ctx.solve(u.to(torch.complex128))
        with pytest.raises(helm.HelmError, match="shape"):
            ctx.solve(u[:, 1:, :].contiguous())
    finally:
        ctx.close()


def test_one_network_serves_two_contexts_of_different_size():
    # each context owns the activation buffers of its network applications
    from paper_2107_03679_amd import learned

    net = learned.new_network(3)
    p = net.params()
    rng = np.random.default_rng(0)
    p["O.w"][:] = 1e-3 * rng.standard_normal(p["O.w"].shape)
    net.set_params(p)
    ctxs = []
    try:
        for n, w, B in ((40, 8, 2), (72, 12, 3)):
            ctx = gpu_context(medium(n, seed=n), w=w, levels=3, max_batch=B, restart=5, krylov=0)
            ctx.set_preconditioner(net, accept_tol=1.0, gamma=1.0, mode="then_mg")
            ctxs.append((ctx, B))
        for _ in range(2):  # alternate between the contexts: buffers must not be shared
            for ctx, B in ctxs:
                rhs = ctx.plane_wave_rhs(synth.directions_2d(B))
                _, st = ctx.solve(rhs)
                assert st.converged and np.all(st.rel_res_true <= 1e-6)
    finally:
        for ctx, _ in ctxs:
            ctx.close()
        net.close()
