"""FP64 reference of the three-dimensional learned preconditioner network.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it.  Not part of the paper (its method uses multigrid
only, and Sec. VII names 3D as future work); this is the reference the 3D
BF16-MFMA kernels are checked against.  Parity with the paper is unpinned for
this part; its pins are finite differences and closed-form special cases.

Network (3D U-Net, 4 levels, channels 16/16/32/32, 3x3x3 convolutions, zero
padding, ReLU after every convolution but the last):
    e0 = relu(conv(x, A0))                         4 -> 16   level 0
    e1 = relu(conv(pool(e0), A1))                 16 -> 16   level 1
    e2 = relu(conv(pool(e1), A2))                 16 -> 32   level 2
    e3 = relu(conv(pool(e2), A3))                 32 -> 32   level 3
    d2 = relu(conv(cat(up(e3), e2), B2))          64 -> 32
    d1 = relu(conv(cat(up(d2), e1), B1))          48 -> 16
    d0 = relu(conv(cat(up(d1), e0), B0))          32 -> 16
    y  = conv(d0, O)                              16 -> 2
(16 output channels fill one 16-wide matrix-core tile, so the finest level
is no cheaper with 8.)
pool: 2x2x2 sum / 8 with zero padding (output ceil(D/2) per axis); up: nearest
neighbour back to the skip's size; cat: channel concatenation (up first).
Arrays are [image][z][y][x][channel]; weights [3][3][3][cin][cout], tap
(dz+1, dy+1, dx+1).  The residual term uses the h^2-scaled 7-point operator
A' y = (6 - c) y - (sum of the 6 neighbours), neighbours outside the image 0.
"""
from __future__ import annotations

import numpy as np

CH = (16, 16, 32, 32)
LAYERS = [  # name, cin, cout, relu
    ("A0", 4, 16, True), ("A1", 16, 16, True), ("A2", 16, 32, True), ("A3", 32, 32, True),
    ("B2", 64, 32, True), ("B1", 48, 16, True), ("B0", 32, 16, True), ("O", 16, 2, False),
]


def init_params(seed: int = 0, dtype=np.float64) -> dict:
    """He-normal weights (fan-in 27 cin), zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, cin, cout, _ in LAYERS:
        std = np.sqrt(2.0 / (27 * cin))
        p[name + ".w"] = (rng.standard_normal((3, 3, 3, cin, cout)) * std).astype(dtype)
        p[name + ".b"] = np.zeros(cout, dtype=dtype)
    return p


def conv(x, w, b):
    """out[i, z, y, x, o] = b[o] + sum_{dz, dy, dx, c} x[i, z+dz, y+dy, x+dx, c] w[dz+1, dy+1, dx+1, c, o],
    zero padding."""
    n, d, h, wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((n, d, h, wd, w.shape[4]), dtype=np.result_type(x, w))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                out += xp[:, kz:kz + d, ky:ky + h, kx:kx + wd, :] @ w[kz, ky, kx]
    return out + b


def conv_backward(x, w, g):
    """Gradients of sum(g * conv(x, w, b)) with respect to x, w and b."""
    n, d, h, wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    gx_p = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                patch = xp[:, kz:kz + d, ky:ky + h, kx:kx + wd, :]
                gw[kz, ky, kx] = np.einsum("nzyxc,nzyxo->co", patch, g)
                gx_p[:, kz:kz + d, ky:ky + h, kx:kx + wd, :] += g @ w[kz, ky, kx].T
    return gx_p[:, 1:d + 1, 1:h + 1, 1:wd + 1, :], gw, g.sum(axis=(0, 1, 2, 3))


def _pad_even(x):
    n, d, h, w, c = x.shape
    xp = np.zeros((n, d + d % 2, h + h % 2, w + w % 2, c), dtype=x.dtype)
    xp[:, :d, :h, :w] = x
    return xp


def pool(x):
    """2x2x2 average with zero padding: the eight children summed, divided by 8."""
    xp = _pad_even(x)
    s = 0.0
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                s = s + xp[:, a::2, b::2, c::2]
    return s / 8.0


def pool_backward(g, shape):
    n, d, h, w, c = shape
    up = np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3)[:, :d, :h, :w]
    return up / 8.0


def upsample(x, shape):
    """Nearest neighbour to spatial size shape[1:4]: out[z, y, x] = in[z // 2, y // 2, x // 2]."""
    d, h, w = shape[1], shape[2], shape[3]
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)[:, :d, :h, :w]


def upsample_backward(g, shape):
    """Adjoint of upsample: each coarse voxel collects the gradient of its (up to) eight children."""
    gp = _pad_even(g)
    s = 0.0
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                s = s + gp[:, a::2, b::2, c::2]
    return s[:, :shape[1], :shape[2], :shape[3]]


def forward(p: dict, x: np.ndarray):
    """Returns the output and the activations the backward pass needs."""
    t = {}

    def layer(name, inp, relu):
        z = conv(inp, p[name + ".w"], p[name + ".b"])
        t[name + ".in"] = inp
        out = np.maximum(z, 0) if relu else z
        t[name + ".out"] = out
        return out

    e0 = layer("A0", x, True)
    e1 = layer("A1", pool(e0), True)
    e2 = layer("A2", pool(e1), True)
    e3 = layer("A3", pool(e2), True)
    d2 = layer("B2", np.concatenate([upsample(e3, e2.shape), e2], axis=4), True)
    d1 = layer("B1", np.concatenate([upsample(d2, e1.shape), e1], axis=4), True)
    d0 = layer("B0", np.concatenate([upsample(d1, e0.shape), e0], axis=4), True)
    y = layer("O", d0, False)
    t.update(e0=e0, e1=e1, e2=e2, e3=e3, d2=d2, d1=d1, d0=d0)
    return y, t


def backward(p: dict, t: dict, gy: np.ndarray) -> dict:
    """Gradients of sum(gy * y) with respect to every parameter."""
    grads = {}

    def layer_back(name, gout, relu):
        if relu:
            gout = gout * (t[name + ".out"] > 0)
        gin, gw, gb = conv_backward(t[name + ".in"], p[name + ".w"], gout)
        grads[name + ".w"], grads[name + ".b"] = gw, gb
        return gin

    c = CH
    g_d0 = layer_back("O", gy, False)
    g_cat0 = layer_back("B0", g_d0, True)
    g_d1 = upsample_backward(g_cat0[..., :c[1]], t["d1"].shape)
    g_e0 = g_cat0[..., c[1]:].copy()
    g_cat1 = layer_back("B1", g_d1, True)
    g_d2 = upsample_backward(g_cat1[..., :c[2]], t["d2"].shape)
    g_e1 = g_cat1[..., c[2]:].copy()
    g_cat2 = layer_back("B2", g_d2, True)
    g_e3 = upsample_backward(g_cat2[..., :c[3]], t["e3"].shape)
    g_e2 = g_cat2[..., c[3]:].copy()
    g_e2 += pool_backward(layer_back("A3", g_e3, True), t["e2"].shape)
    g_e1 += pool_backward(layer_back("A2", g_e2, True), t["e1"].shape)
    g_e0 += pool_backward(layer_back("A1", g_e1, True), t["e0"].shape)
    layer_back("A0", g_e0, True)
    return grads


def scaled_operator(y: np.ndarray, c: np.ndarray) -> np.ndarray:
    """A' y = (6 - c) y - (sum of the 6 neighbours) per image, neighbours outside the image = 0."""
    out = (6.0 - c) * y
    for ax in (1, 2, 3):
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        out[tuple(hi)] -= y[tuple(lo)]
        out[tuple(lo)] -= y[tuple(hi)]
    return out


def residual_term(x: np.ndarray, y: np.ndarray, gamma: float, cb: float):
    """1/2 sum over image interiors of |r - gamma A' y|^2 and its gradient w.r.t. y (real pairs);
    r = x[..., 0] + j x[..., 1], c = cb (1 + x[..., 2] + j x[..., 3]), the one-voxel border left out."""
    r = x[..., 0] + 1j * x[..., 1]
    c = cb * (1.0 + x[..., 2] + 1j * x[..., 3])
    yc = y[..., 0] + 1j * y[..., 1]
    q = r - gamma * scaled_operator(yc, c)
    mask = np.zeros(q.shape, dtype=bool)
    mask[:, 1:-1, 1:-1, 1:-1] = True
    q = np.where(mask, q, 0.0)
    loss = 0.5 * float(np.sum(np.abs(q) ** 2))
    g = -gamma * scaled_operator(q, np.conj(c))
    return loss, np.stack([g.real, g.imag], axis=-1)


def loss_and_grads(p: dict, x: np.ndarray, target: np.ndarray, err_w: float = 1.0, res_w: float = 0.0,
                   gamma: float = 1.0, cb: float = 1.0):
    """L = (err_w/2 sum (y - target)^2 + res_w/2 sum_interior |r - gamma A' y|^2) / n_images
    and its parameter gradients."""
    y, t = forward(p, x)
    nimg = x.shape[0]
    gy = err_w * (y - target) / nimg
    loss = err_w * 0.5 * float(np.sum((y - target) ** 2)) / nimg
    if res_w:
        lr, gr = residual_term(x, y, gamma, cb)
        loss += res_w * lr / nimg
        gy = gy + res_w * gr / nimg
    return loss, backward(p, t, gy), y
