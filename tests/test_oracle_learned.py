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
