"""GPU parity of the sensor operator G~ (eq. DiscreteForwardHelm with eq. green) and of the
far-field data gradient (Prop. 1) against the FP64 oracle (direct Hankel/exponential kernels,
exact LU solves)."""
import numpy as np
import pytest
import torch

import synth
from oracle import farfield as off
from oracle import model

from .helpers import gpu_context, medium, oracle_problem, rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def circle(m, radius):
    t = 2 * np.pi * np.arange(m) / m + 0.1
    return np.stack([radius * np.cos(t), radius * np.sin(t)], axis=1)


@pytest.fixture(scope="module")
def ff2d():
    n, w, levels = 40, 8, 3
    print("\n[far field 2D n=40, 48 sensors]", flush=True)
    nmap = medium(n, seed=17)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=4, rtol=1e-7)
    sens = circle(48, 0.75 * n)
    ctx.farfield_set(sens)
    yield prob, ctx, sens
    ctx.close()


def test_forward_and_adjoint_match_oracle(ff2d):
    prob, ctx, sens = ff2d
    G = off.sensor_matrix(prob, sens)
    B = 3
    usc = synth.complex_field((B, *prob.shape), 51).astype(np.complex64)
    uin = synth.complex_field((B, *prob.shape), 52).astype(np.complex64)
    y = to_np(ctx.farfield(to_dev(usc), u_in=to_dev(uin)))
    ref = np.stack([off.farfield(prob, G, usc[q].astype(np.complex128) + uin[q]) for q in range(B)])
    assert rel(y, ref) < 1e-5
    r = synth.complex_field((B, len(sens)), 53).astype(np.complex64)
    s, rhs = ctx.farfield_adjoint(to_dev(r))
    s, rhs = to_np(s), to_np(rhs)
    sref = np.zeros((B, *prob.shape), dtype=np.complex128)
    for q in range(B):
        sref[q][prob.interior_slices()] = (G.conj().T @ r[q]).reshape(prob.n, prob.n)
    assert rel(s, sref) < 1e-5
    assert rel(rhs, model.scattering_potential(prob) * sref) < 1e-5
    # no sensors inside Omega
    from paper_2107_03679_amd.helm import HelmError

    with pytest.raises(HelmError):
        ctx.farfield_set(np.array([[0.0, 3.0]]))
    ctx.farfield_set(sens)


def test_far_field_gradient_matches_oracle(ff2d):
    prob, ctx, sens = ff2d
    dirs = synth.directions_2d(3)
    y_meas = (synth.complex_field((3, len(sens)), 61) * 1e-3).astype(np.complex64)
    loss_ref, grad_ref = off.farfield_loss_and_gradient(prob, sens, dirs, y_meas.astype(np.complex128))
    rhs, uin = ctx.plane_wave_rhs(dirs, with_uin=True)
    usc, st = ctx.solve(rhs)
    assert st.converged
    y = ctx.farfield(usc, u_in=uin)
    r = y - torch.tensor(y_meas, device="cuda")
    loss = 0.5 * float((r.abs() ** 2).sum())
    s, arhs = ctx.farfield_adjoint(r)
    lam, st_a = ctx.adjoint(arhs)
    assert st_a.converged
    g = ctx.grad_f_farfield(usc, lam, s, u_in=uin).cpu().numpy().astype(np.float64)
    assert loss == pytest.approx(loss_ref, rel=1e-4)
    assert rel(g, grad_ref) < 1e-3


def test_forward_3d_matches_oracle():
    n, w, levels = 10, 4, 2
    print("\n[far field 3D n=10]", flush=True)
    nmap = medium(n, d=3, seed=5)
    prob = oracle_problem(nmap, w=w, levels=levels)
    ctx = gpu_context(nmap, w=w, levels=levels, max_batch=2)
    rng = np.random.default_rng(4)
    v = rng.standard_normal((20, 3))
    sens = 12.0 * v / np.linalg.norm(v, axis=1, keepdims=True)
    ctx.farfield_set(sens)
    usc = synth.complex_field((2, *prob.shape), 71).astype(np.complex64)
    y = to_np(ctx.farfield(to_dev(usc)))
    G = off.sensor_matrix(prob, sens)
    ref = np.stack([off.farfield(prob, G, usc[q].astype(np.complex128)) for q in range(2)])
    assert rel(y, ref) < 1e-5
    ctx.close()


def test_fbs_with_far_field_sensors_reduces_the_data_term():
    """Alg. 4 with the sensor operator: data from exact LU solves of a blob medium at 64
    sensors on a circle around Omega; a few accelerated FBS iterations on the GPU must cut
    the data term and keep f >= 0."""
    from paper_2107_03679_amd.inverse import FBSReconstruction

    n, w, levels, Q = 40, 8, 3, 8
    print("\n[FBS with far-field sensors 40^2 x 8]", flush=True)
    n_true = synth.blob_map(n, 2, (4.0, 7.0), 0.05, 41).astype(np.float32).astype(np.float64)
    dirs = synth.directions_2d(Q, -180.0, 135.0)
    sens = circle(64, 0.8 * n)
    p_true = oracle_problem(n_true, w=w, levels=levels)
    G = off.sensor_matrix(p_true, sens)
    ex = model.ExactSolver(p_true)
    y = np.stack([off.farfield(p_true, G, model.plane_wave(p_true, d) + ex.solve(model.rhs(p_true, d)))
                  for d in dirs]).astype(np.complex64)
    nb = np.full((n, n), p_true.n_b)
    ctx = gpu_context(nb, w=w, levels=levels, max_batch=Q, rtol=1e-7)
    ctx.farfield_set(sens)
    rec = FBSReconstruction(ctx, dirs, None, torch.tensor(y, device="cuda"), gamma=1.0, tau=0.0, prox_iters=30)
    g0, loss0, _ = rec.gradient(rec.f, np.arange(Q))
    f_true = p_true.k0 ** 2 * (n_true ** 2 - p_true.n_b ** 2)
    rec.gamma = 0.3 * f_true.max() / float(g0.abs().max())
    rec.tau = 1e-4 * float(g0.abs().max())
    for _ in range(6):
        rec.step()
    f = rec.f.cpu().numpy()
    print(f"[FBS far field] data term {np.array(rec.log.loss) / loss0}", flush=True)
    assert np.all(f >= 0.0) and rec.log.loss[-1] < 0.5 * loss0
    ctx.close()
