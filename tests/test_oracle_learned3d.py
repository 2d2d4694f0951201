"""Pins of the FP64 reference of the 3D learned-preconditioner network (not in the paper: parity
unpinned; pinned here by finite differences, adjoint identities and closed-form special cases)."""
import numpy as np
import pytest

from oracle import learned, learned3d


def test_conv_identity_shift_and_planar_kernels():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 5, 6, 3))
    w = np.zeros((3, 3, 3, 3, 3))
    w[1, 1, 1] = np.eye(3)
    assert np.allclose(learned3d.conv(x, w, np.zeros(3)), x)
    w = np.zeros((3, 3, 3, 3, 3))
    w[2, 1, 1] = np.eye(3)  # tap (dz, dy, dx) = (+1, 0, 0): out[z] = in[z + 1], zero past the edge
    out = learned3d.conv(x, w, np.zeros(3))
    assert np.allclose(out[:, :-1], x[:, 1:]) and np.allclose(out[:, -1], 0)
    # weights only in the dz = 0 plane act as the 2D convolution of the 2D reference on every plane
    w2 = rng.standard_normal((3, 3, 3, 4))
    w = np.zeros((3, 3, 3, 3, 4))
    w[1] = w2
    b = rng.standard_normal(4)
    out = learned3d.conv(x, w, b)
    for z in range(4):
        assert np.allclose(out[:, z], learned.conv3x3(x[:, z], w2, b))


def test_pool_up_adjoints_and_constants():
    rng = np.random.default_rng(1)
    for d, h, wd in ((4, 6, 8), (5, 7, 3)):
        x = rng.standard_normal((2, d, h, wd, 3))
        px = learned3d.pool(x)
        assert px.shape == (2, (d + 1) // 2, (h + 1) // 2, (wd + 1) // 2, 3)
        g = rng.standard_normal(px.shape)
        assert np.sum(px * g) == pytest.approx(np.sum(x * learned3d.pool_backward(g, x.shape)))
        u = learned3d.upsample(g, x.shape)
        assert u.shape == x.shape
        assert np.sum(u * x) == pytest.approx(np.sum(g * learned3d.upsample_backward(x, g.shape)))
    # the average of a constant is the constant away from the padded high faces
    ones = np.ones((1, 5, 5, 5, 1))
    p = learned3d.pool(ones)
    assert np.allclose(p[:, :2, :2, :2], 1.0) and p[0, 2, 2, 2, 0] == pytest.approx(1.0 / 8.0)


def test_network_gradients_match_finite_differences():
    p = learned3d.init_params(3)
    rng = np.random.default_rng(4)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((1, 5, 6, 7, 4))
    tgt = rng.standard_normal((1, 5, 6, 7, 2))
    loss, grads, _ = learned3d.loss_and_grads(p, x, tgt)
    for name in ("A0.w", "A3.w", "B2.w", "B0.b", "O.w", "A1.b"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=3, replace=False):
            old = flat[idx]
            flat[idx] = old + 1e-6
            lp = learned3d.loss_and_grads(p, x, tgt)[0]
            flat[idx] = old - 1e-6
            lm = learned3d.loss_and_grads(p, x, tgt)[0]
            flat[idx] = old
            fd = (lp - lm) / 2e-6
            assert grads[name].reshape(-1)[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), (name, idx)


def test_residual_term_annihilates_discrete_plane_wave_in_3d():
    # interior rows of A' y vanish for y = exp(j(kx X + ky Y + kz Z)) when 6 - 2 cos kx - 2 cos ky - 2 cos kz = c
    kx, ky, kz = 0.4, 0.25, 0.3
    c = 6 - 2 * np.cos(kx) - 2 * np.cos(ky) - 2 * np.cos(kz)
    cb = 0.39
    Z, Y, X = np.mgrid[0:6, 0:7, 0:8]
    yc = np.exp(1j * (kx * X + ky * Y + kz * Z))[None]
    x = np.zeros((1, 6, 7, 8, 4))
    x[..., 2] = c / cb - 1.0
    y = np.stack([yc.real, yc.imag], -1)
    loss, _ = learned3d.residual_term(x, y, gamma=1.0, cb=cb)
    assert loss < 1e-24
    imp = np.zeros((1, 5, 5, 5), complex)
    imp[0, 2, 2, 2] = 1.0
    a = learned3d.scaled_operator(imp, np.full((1, 5, 5, 5), 0.3 + 0.1j))
    assert a[0, 2, 2, 2] == pytest.approx(5.7 - 0.1j)
    nbrs = ((1, 2, 2), (3, 2, 2), (2, 1, 2), (2, 3, 2), (2, 2, 1), (2, 2, 3))
    assert all(a[(0, *i)] == -1 for i in nbrs) and np.count_nonzero(a) == 7


def test_residual_and_combined_loss_gradients():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((1, 4, 5, 6, 4)) * [1, 1, 0.1, 0.05]
    y = rng.standard_normal((1, 4, 5, 6, 2))
    loss, g = learned3d.residual_term(x, y, gamma=1.7, cb=0.39)
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in y.shape)
        yp, ym = y.copy(), y.copy()
        yp[idx] += 1e-6
        ym[idx] -= 1e-6
        fd = (learned3d.residual_term(x, yp, 1.7, 0.39)[0] - learned3d.residual_term(x, ym, 1.7, 0.39)[0]) / 2e-6
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    p = learned3d.init_params(8)
    tgt = rng.standard_normal((1, 4, 5, 6, 2))
    kw = dict(err_w=0.5, res_w=2.0, gamma=1.3, cb=0.39)
    _, grads, _ = learned3d.loss_and_grads(p, x, tgt, **kw)
    for name in ("O.w", "B0.w", "A0.b"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=2, replace=False):
            old = flat[idx]
            flat[idx] = old + 1e-6
            lp = learned3d.loss_and_grads(p, x, tgt, **kw)[0]
            flat[idx] = old - 1e-6
            lm = learned3d.loss_and_grads(p, x, tgt, **kw)[0]
            flat[idx] = old
            assert grads[name].reshape(-1)[idx] == pytest.approx((lp - lm) / 2e-6, rel=1e-5, abs=1e-8)
