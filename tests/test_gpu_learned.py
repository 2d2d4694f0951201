"""Learned preconditioner on the GPU: BF16-MFMA network kernels vs the FP64 reference network,
training, and its use inside FGMRES with the multigrid fallback.

The network is not part of the paper: parity with the paper is unpinned; the
expected values come from oracle.learned (FP64 NumPy, pinned by finite
differences).  BF16 storage of weights and activations bounds the agreement
to about 1e-2 relative.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import learned, model

from .helpers import gpu_context, medium, oracle_problem, rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def bf16_round(a):
    return torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)


@pytest.fixture(scope="module")
def net_and_params():
    from paper_2107_03679_amd import helm

    print("\n[network]", flush=True)
    p = learned.init_params(5)
    rng = np.random.default_rng(6)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    net = helm.Net(seed=1)
    net.set_params(p)
    # what the kernels see: BF16 weights (biases stay FP32)
    pq = {k: (bf16_round(v) if k.endswith(".w") else v) for k, v in p.items()}
    yield net, pq
    net.close()


def test_weights_roundtrip(net_and_params):
    net, pq = net_and_params
    got = net.params()
    for k, v in got.items():
        assert np.allclose(v, pq[k], rtol=1e-2, atol=1e-3), k


@pytest.mark.parametrize("shape", [(3, 37, 45), (2, 64, 64)])
def test_forward_matches_reference(net_and_params, shape):
    net, pq = net_and_params
    n, h, w = shape
    x = bf16_round(np.random.default_rng(7).standard_normal((n, h, w, 4)))
    y = net.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    ref, _ = learned.forward(pq, x)
    assert rel(y, ref) < 3e-2


@pytest.mark.parametrize("shape", [(3, 37, 45), (2, 130, 97), (1, 577, 577)])
def test_specialised_convolutions_match_generic(net_and_params, shape):
    """The channel-specialised 2D convolution kernels form the generic kernel's sums in the
    same order, so the forward outputs agree bit for bit (ragged tiles on every level)."""
    net, _ = net_and_params
    n, h, w = shape
    print(f"[specialised vs generic convolutions {shape}]", flush=True)
    x = torch.tensor(np.random.default_rng(11).standard_normal((n, h, w, 4)), dtype=torch.float32, device="cuda")
    net.set_conv_kernels(generic=True)
    try:
        y_gen = net.forward(x)
    finally:
        net.set_conv_kernels(generic=False)
    y = net.forward(x)
    assert torch.isfinite(y).all()
    assert torch.equal(y, y_gen), float((y - y_gen).abs().max())
    assert net.lib.helm_net_set_conv_kernels(net._h, 2) == -1  # only 0 and 1


@pytest.mark.parametrize("weights", [(1.0, 0.0), (0.5, 2.0)])
def test_gradients_match_reference(net_and_params, weights):
    net, pq = net_and_params
    err_w, res_w = weights
    rng = np.random.default_rng(8)
    x = bf16_round(rng.standard_normal((2, 40, 36, 4)) * [1, 1, 0.1, 0.05])
    tgt = rng.standard_normal((2, 40, 36, 2))
    kw = dict(err_w=err_w, res_w=res_w, gamma=0.3, cb=0.39)
    net.set_loss(err_w, res_w, gamma=0.3, cb=0.39)
    loss = net.backward(torch.tensor(x, dtype=torch.float32, device="cuda"),
                        torch.tensor(tgt, dtype=torch.float32, device="cuda"))
    net.set_loss()
    ref_loss, ref_grads, _ = learned.loss_and_grads(pq, x, tgt, **kw)
    assert loss == pytest.approx(ref_loss, rel=2e-2)
    g = net.grads()
    for name in ref_grads:
        a, b = g[name].ravel().astype(np.float64), ref_grads[name].ravel()
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        assert cos > 0.995, (name, cos)
        assert rel(a, b) < 0.1, name


def test_adam_training_reduces_loss():
    from paper_2107_03679_amd import helm

    net = helm.Net(seed=2)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((8, 32, 32, 4)).astype(np.float32)
    # a smooth linear target the network can fit: a blurred copy of the first two input channels
    tgt = 0.25 * (x[..., :2] + np.roll(x[..., :2], 1, axis=1) + np.roll(x[..., :2], 1, axis=2)
                  + np.roll(x[..., :2], (1, 1), axis=(1, 2)))
    xt = torch.tensor(x, device="cuda")
    tt = torch.tensor(tgt.astype(np.float32), device="cuda")
    losses = []
    for _ in range(60):
        losses.append(net.backward(xt, tt))
        net.adam_step(2e-3)
    net.close()
    assert losses[-1] < 0.5 * losses[0], losses[::10]


def test_fgmres_with_network_and_fallback():
    from paper_2107_03679_amd import helm

    n, w, levels = 40, 8, 3
    nmap = medium(n, seed=13)
    prob = oracle_problem(nmap, w=w, levels=levels)
    # FGMRES throughout, so that the multigrid-only solve is comparable step for step
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=3, krylov=helm.KRYLOV_FGMRES)
    net = helm.Net(seed=3)  # untrained: its outputs fail the acceptance test and the V-cycle takes over
    ctx.set_preconditioner(net, accept_tol=0.5, gamma=1.0)
    rhs = ctx.plane_wave_rhs(synth.directions_2d(3))
    x, st = ctx.solve(rhs)
    assert st.converged and np.all(st.rel_res_true <= 1e-6)
    assert np.all(st.fallbacks > 0)
    ex = model.ExactSolver(prob)
    b = to_np(rhs)
    u = np.stack([ex.solve(bi) for bi in b])
    assert rel(to_np(x), u) < 1e-5
    ctx.set_preconditioner(None)
    x2, st2 = ctx.solve(rhs)
    assert st2.converged and np.all(st2.fallbacks == 0)
    # network followed by a V-cycle of its residual: accepting every output still converges to u
    ctx.set_preconditioner(net, accept_tol=1e30, gamma=0.1, mode="then_mg")
    x3, st3 = ctx.solve(rhs)
    assert st3.converged and np.all(st3.fallbacks == 0) and np.all(st3.rel_res_true <= 1e-6)
    assert rel(to_np(x3), u) < 1e-5
    # ... and rejecting every output is the plain multigrid cycle, step for step
    ctx.set_preconditioner(net, accept_tol=0.0, gamma=1.0, mode="then_mg")
    x4, st4 = ctx.solve(rhs)
    assert np.all(st4.fallbacks == st4.iters) and np.all(np.abs(st4.iters - st2.iters) <= 1)
    assert rel(to_np(x4), to_np(x2)) < 1e-6
    ctx.close()
    net.close()


def test_snapshots_and_examples():
    n, w, levels = 40, 8, 3
    nmap = medium(n, seed=14)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=2, restart=5)
    rhs = ctx.plane_wave_rhs(synth.directions_2d(2))
    x, st, snaps = ctx.solve_snapshots(rhs, every_cycles=2, max_snaps=4)
    assert st.converged and 1 <= snaps.shape[0] <= 4
    xk = snaps[0].contiguous()
    r = ctx.residual(rhs, xk)
    crops = np.array([[0, 3, 5], [1, 10, 2]])
    S = 24
    feat, tgt = ctx.net_examples(r, x, xk, crops, S, gamma=2.0)
    feat, tgt = feat.cpu().numpy(), tgt.cpu().numpy()
    rr, xx, kk = to_np(r), to_np(x), to_np(xk)
    c = prob.coefficient()
    cb = prob.kbh ** 2
    for i, (b, y0, x0) in enumerate(crops):
        win = (slice(y0, y0 + S), slice(x0, x0 + S))
        rs = prob.h ** 2 * rr[b][win]
        rms = np.sqrt(np.mean(np.abs(prob.h ** 2 * rr[b]) ** 2))  # over the whole grid
        assert np.allclose(feat[i, ..., 0] + 1j * feat[i, ..., 1], rs / rms, atol=1e-5)
        assert np.allclose(feat[i, ..., 2] + 1j * feat[i, ..., 3], (c[win] - cb) / cb, atol=1e-5)
        e = (xx[b][win] - kk[b][win]) / rms / 2.0
        assert np.allclose(tgt[i, ..., 0] + 1j * tgt[i, ..., 1], e, rtol=1e-4, atol=1e-4 * np.abs(e).max())
    ctx.close()


def test_trained_network_gain():
    """Train on pairs from the solver's own solves on training media, evaluate on a held-out medium.

    What the network gains is measured, not assumed: the test prints the
    iteration counts of multigrid-FGMRES with and without the network and
    asserts that (i) on held-out examples the trained network's output
    reduces the residual (||r - A' y|| < ||r||, the zero output gives 1),
    (ii) with the network (acceptance-gated, multigrid cycle after it) some
    outputs are accepted and the solve still reaches the exact solution, and
    (iii) it needs fewer preconditioner applications than multigrid alone in the
    same Krylov method (FGMRES(5) for both).  The time per application is
    another matter: the network costs about ten multigrid cycles at this size
    (the benchmark reports both).
    """
    import torch

    from paper_2107_03679_amd import learned as train_lib

    n, w, levels, B = 96, 20, 4, 16
    from paper_2107_03679_amd import helm

    ctx = gpu_context(medium(n, seed=1000), w=w, levels=levels, max_batch=B, restart=5, cycle=3,
                      krylov=helm.KRYLOV_FGMRES)
    rng = np.random.default_rng(21)
    ex = None
    for seed in (1000, 1001, 1002):
        ctx.update_n(torch.tensor(medium(n, seed=seed), dtype=torch.float32, device="cuda"))
        th = np.radians(rng.uniform(-60, 60, B))
        rhs = ctx.plane_wave_rhs(np.stack([np.sin(th), np.cos(th)], 1))
        ex = train_lib.collect(ctx, [rhs], size=64, crops_per_snapshot=4, every_cycles=4, max_snaps=8, seed=seed,
                               out=ex)
    # held-out examples from a medium the network never sees in training
    nmap = medium(n, seed=7)
    ctx.update_n(torch.tensor(nmap, dtype=torch.float32, device="cuda"))
    rhs = ctx.plane_wave_rhs(synth.directions_2d(B))
    val = train_lib.collect(ctx, [rhs], size=64, crops_per_snapshot=2, every_cycles=4, max_snaps=4, seed=5)
    val = train_lib.rescaled(ctx, val, ex.gamma)
    net = train_lib.new_network(4)
    train_lib.train(net, ex, steps=1500, batch=16, lr=1e-4, seed=6, err_weight=0.0, res_weight=1.0)
    ratio = train_lib.residual_ratio(ctx, net, val)
    x_mg, st_mg = ctx.solve(rhs)
    ctx.set_preconditioner(net, accept_tol=1.0, gamma=ex.gamma, mode="then_mg")
    x_nn, st_nn = ctx.solve(rhs)
    accepted = 1.0 - st_nn.fallbacks.sum() / st_nn.iters.sum()
    print(f"\n[learned gain] pairs {ex.feat.shape[0]}, held-out residual ratio {ratio:.3f}; "
          f"iterations MG {st_mg.iters.mean():.1f}, MG+net {st_nn.iters.mean():.1f}; "
          f"network outputs accepted {100 * accepted:.0f}%", flush=True)
    assert ratio < 0.95
    assert accepted > 0.0
    assert st_nn.converged and np.all(st_nn.rel_res_true <= 1e-6)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ex_solver = model.ExactSolver(prob)
    b = to_np(rhs)
    for q in (0, B // 2, B - 1):
        assert rel(to_np(x_nn)[q], ex_solver.solve(b[q])) < 1e-5
    assert st_nn.iters.mean() < st_mg.iters.mean(), (st_nn.iters, st_mg.iters)
    ctx.close()
    net.close()
