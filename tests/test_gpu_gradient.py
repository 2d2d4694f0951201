"""GPU parity of the differentiation path (Sec. V, Prop. 1): receivers, TV, adjoint gradient.

Workload: 256^2 interior (inverse step), 32 plane waves in [-60, 60] degrees,
layer strength 0 (the paper's inverse setting), 256 receivers on the last
interior row, data from a seeded blob map with 1% complex Gaussian noise,
gradient evaluated at n_b + (n_true - n_b) / 2.  Expected values come from
the FP64 oracle (exact LU solves).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import model
from oracle.discretization import Problem

from .helpers import KBH, N_B, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

N, W, LEVELS, NQ = 256, 20, 5, 32


@pytest.fixture(scope="module")
def inverse_case():
    from paper_2107_03679_amd import helm
    from paper_2107_03679_amd.autograd import receiver_line

    print("\n[inverse step 256^2 x 32]", flush=True)
    n_true = synth.workload_medium("inverse256x32").astype(np.float32).astype(np.float64)
    n_eval = (N_B + 0.5 * (n_true - N_B)).astype(np.float32).astype(np.float64)
    dirs = synth.workload_directions("inverse256x32")
    p_true = Problem(n_true, k0h=KBH / N_B, w=W, levels=LEVELS, beta=0.0)
    ex = model.ExactSolver(p_true)
    clean = np.stack([model.sample(p_true, ex.solve(model.rhs(p_true, d))) for d in dirs])
    rng = np.random.default_rng(11)
    scale = 0.01 * np.linalg.norm(clean, axis=1, keepdims=True) / np.sqrt(clean.shape[1])
    data = clean + scale * (rng.standard_normal(clean.shape) + 1j * rng.standard_normal(clean.shape)) / np.sqrt(2)
    data = data.astype(np.complex64).astype(np.complex128)
    p_eval = Problem(n_eval, k0h=KBH / N_B, w=W, levels=LEVELS, beta=0.0)
    ne = p_eval.n_e
    hctx = helm.Context(torch.tensor(n_eval, dtype=torch.float32, device="cuda"), (KBH / N_B) * (ne - 1),
                        abl_width=W, beta=0.0, levels=LEVELS, max_batch=NQ, rtol=1e-7)
    rx = receiver_line(hctx)
    yield dict(n_eval=n_eval, dirs=dirs, data=data, p_eval=p_eval, hctx=hctx, rx=rx)
    hctx.close()


def test_receivers_match_oracle_sampling(inverse_case):
    c = inverse_case
    prob, hctx = c["p_eval"], c["hctx"]
    u = synth.complex_field((3, *prob.shape), 5).astype(np.complex64)
    y = to_np(hctx.sample(c["rx"], to_dev(u)))
    assert np.array_equal(y, np.stack([model.sample(prob, ui) for ui in u.astype(np.complex128)]))
    back = to_np(hctx.sample_adjoint(c["rx"], to_dev(y.astype(np.complex64))))
    assert np.array_equal(back, np.stack([model.sample_adjoint(prob, yi) for yi in y]))


def test_tv_matches_oracle(inverse_case):
    c = inverse_case
    for eps in (1e-4, 0.05):
        val, grad = c["hctx"].tv(torch.tensor(c["n_eval"], dtype=torch.float32, device="cuda"), eps)
        ref_val, ref_grad = model.tv_smoothed(c["n_eval"], eps)
        assert val == pytest.approx(ref_val, rel=1e-5)
        assert np.linalg.norm(grad.cpu().numpy() - ref_grad) / np.linalg.norm(ref_grad) < 1e-4


def test_adjoint_gradient_matches_oracle(inverse_case):
    from paper_2107_03679_amd.autograd import data_loss

    c = inverse_case
    n_t = torch.tensor(c["n_eval"], dtype=torch.float32, device="cuda", requires_grad=True)
    data = torch.tensor(c["data"], dtype=torch.complex64, device="cuda")
    loss = data_loss(n_t, c["hctx"], c["dirs"], c["rx"], data, tau=1e-3, tv_eps=1e-4)
    loss.backward()
    g = n_t.grad.detach().cpu().numpy().astype(np.float64)
    ref_loss, ref_grad = model.loss_and_gradient(c["p_eval"], c["dirs"], c["data"], tau=1e-3, tv_eps=1e-4)
    assert float(loss.detach()) == pytest.approx(ref_loss, rel=1e-4)
    assert np.linalg.norm(g - ref_grad) / np.linalg.norm(ref_grad) < 1e-3


def test_gradient_central_differences_on_gpu(inverse_case):
    # complex64 FD through the GPU forward model on 16 seeded pixels (reading A22: informational, loose)
    from paper_2107_03679_amd.autograd import data_loss

    c = inverse_case
    data = torch.tensor(c["data"], dtype=torch.complex64, device="cuda")
    n0 = torch.tensor(c["n_eval"], dtype=torch.float32, device="cuda", requires_grad=True)
    loss = data_loss(n0, c["hctx"], c["dirs"], c["rx"], data, tau=0.0)
    loss.backward()
    g = n0.grad.detach().cpu().numpy()
    rng = np.random.default_rng(12)
    pix = rng.integers(0, N, size=(16, 2))
    delta = 1e-3
    errs = []
    for i, j in pix:
        vals = []
        for sgn in (1, -1):
            nm = c["n_eval"].copy()
            nm[i, j] += sgn * delta
            with torch.no_grad():
                vals.append(float(data_loss(torch.tensor(nm, dtype=torch.float32, device="cuda"), c["hctx"],
                                            c["dirs"], c["rx"], data, tau=0.0)))
        fd = (vals[0] - vals[1]) / (2 * delta)
        errs.append(abs(fd - g[i, j]) / max(abs(g[i, j]), 1e-3 * np.abs(g).max()))
    assert np.median(errs) < 0.05, errs
