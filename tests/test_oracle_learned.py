"""Pins of the FP64 reference network of the learned preconditioner (not in the paper: parity unpinned;
pinned here by finite differences and closed-form special cases)."""
import numpy as np
import pytest

from oracle import learned


def test_conv_identity_and_shift_kernels():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6, 3))
    w = np.zeros((3, 3, 3, 3))
    w[1, 1] = np.eye(3)
    assert np.allclose(learned.conv3x3(x, w, np.zeros(3)), x)
    w = np.zeros((3, 3, 3, 3))
    w[1, 2] = np.eye(3)  # tap (dy, dx) = (0, +1): out[y, x] = in[y, x + 1], zero past the edge
    out = learned.conv3x3(x, w, np.zeros(3))
    assert np.allclose(out[:, :, :-1], x[:, :, 1:]) and np.allclose(out[:, :, -1], 0)


def test_pool_up_adjoints():
    rng = np.random.default_rng(1)
    for h, wd in ((6, 8), (7, 5)):
        x = rng.standard_normal((2, h, wd, 3))
        px = learned.pool(x)
        assert px.shape == (2, (h + 1) // 2, (wd + 1) // 2, 3)
        g = rng.standard_normal(px.shape)
        assert np.sum(px * g) == pytest.approx(np.sum(x * learned.pool_backward(g, x.shape)))
        u = learned.upsample(g, x.shape)
        assert np.sum(u * x) == pytest.approx(np.sum(g * learned.upsample_backward(x, g.shape)))


def test_network_gradients_match_finite_differences():
    p = learned.init_params(3)
    rng = np.random.default_rng(4)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((2, 9, 11, 4))
    tgt = rng.standard_normal((2, 9, 11, 2))
    loss, grads, _ = learned.loss_and_grads(p, x, tgt)
    for name in ("A0.w", "A3.w", "B2.w", "B0.b", "O.w", "A1.b"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=3, replace=False):
            old = flat[idx]
            flat[idx] = old + 1e-6
            lp = learned.loss_and_grads(p, x, tgt)[0]
            flat[idx] = old - 1e-6
            lm = learned.loss_and_grads(p, x, tgt)[0]
            flat[idx] = old
            fd = (lp - lm) / 2e-6
            assert grads[name].reshape(-1)[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), (name, idx)


def test_residual_term_annihilates_discrete_plane_wave():
    # interior rows of A' y vanish for y = exp(j(kx X + ky Y)) when 4 - 2 cos kx - 2 cos ky = c (closed form)
    kx, ky = 0.4, 0.25
    c = 4 - 2 * np.cos(kx) - 2 * np.cos(ky)
    cb = 0.39
    Y, X = np.mgrid[0:9, 0:12]
    yc = np.exp(1j * (kx * X + ky * Y))[None]
    x = np.zeros((1, 9, 12, 4))
    x[..., 2] = c / cb - 1.0  # c = cb (1 + f)
    y = np.stack([yc.real, yc.imag], -1)
    loss, _ = learned.residual_term(x, y, gamma=1.0, cb=cb)
    assert loss < 1e-24
    # and the point stencil: A' of a unit impulse is 4 - c at the centre, -1 at the 4 neighbours
    imp = np.zeros((1, 5, 5), complex)
    imp[0, 2, 2] = 1.0
    a = learned.scaled_operator(imp, np.full((1, 5, 5), 0.3 + 0.1j))
    assert a[0, 2, 2] == pytest.approx(3.7 - 0.1j)
    assert all(a[0, i, j] == -1 for i, j in ((1, 2), (3, 2), (2, 1), (2, 3))) and np.count_nonzero(a) == 5


def test_residual_term_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 6, 7, 4)) * [1, 1, 0.1, 0.05]
    y = rng.standard_normal((2, 6, 7, 2))
    loss, g = learned.residual_term(x, y, gamma=1.7, cb=0.39)
    for _ in range(8):
        idx = tuple(rng.integers(0, s) for s in y.shape)
        yp, ym = y.copy(), y.copy()
        yp[idx] += 1e-6
        ym[idx] -= 1e-6
        fd = (learned.residual_term(x, yp, 1.7, 0.39)[0] - learned.residual_term(x, ym, 1.7, 0.39)[0]) / 2e-6
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_combined_loss_parameter_gradient():
    p = learned.init_params(8)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((1, 8, 8, 4)) * [1, 1, 0.1, 0.05]
    tgt = rng.standard_normal((1, 8, 8, 2))
    kw = dict(err_w=0.5, res_w=2.0, gamma=1.3, cb=0.39)
    loss, grads, _ = learned.loss_and_grads(p, x, tgt, **kw)
    for name in ("O.w", "B0.w", "A0.b"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=2, replace=False):
            old = flat[idx]
            flat[idx] = old + 1e-6
            lp = learned.loss_and_grads(p, x, tgt, **kw)[0]
            flat[idx] = old - 1e-6
            lm = learned.loss_and_grads(p, x, tgt, **kw)[0]
            flat[idx] = old
            assert grads[name].reshape(-1)[idx] == pytest.approx((lp - lm) / 2e-6, rel=1e-5, abs=1e-8)
