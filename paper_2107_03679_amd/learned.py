"""Training of the learned FGMRES preconditioner on the solver's own residual/error pairs.

The pairs come from multigrid-preconditioned FGMRES solves on training media:
the iterate x_k is kept every few restart cycles, and with the converged x*
each snapshot gives r = b - A x_k and e = x* - x_k, so that A e = r exactly
(up to the solve tolerance).  Crops of (r, e) together with the medium
contrast are the examples; the network learns r -> e on them with the
library's own BF16-MFMA forward/backward kernels and Adam (every arithmetic
step runs in libhelm; torch only holds the tensors and draws minibatches).

Scaling: features are the h^2-scaled residual divided by its rms over the
crop (the solver feeds sqrt(N) v_j, v_j of unit norm, so the rms is 1 in
both cases); targets are e / rms / gamma with gamma chosen so that the
targets have unit rms over the training set.  The same gamma is handed to
Context.set_preconditioner.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import helm


@dataclass
class Examples:
    feat: torch.Tensor  # [n][S]^dim[4] float32: Re r, Im r, Re and Im of (c - c_b) / c_b
    tgt: torch.Tensor   # [n][S]^dim[2] float32: Re e, Im e (divided by gamma)
    gamma: float
    cb: float  # (k_b h)^2: the background coefficient the contrast features are relative to
    solve_iters: list = field(default_factory=list)


def collect(ctx: helm.Context, rhs_batches, size: int, crops_per_snapshot: int, every_cycles: int,
            max_snaps: int, seed: int, out: Examples | None = None) -> Examples:
    """Solve each batch in `rhs_batches` (device tensors [B][n_e]^dim) with snapshots and
    cut `crops_per_snapshot` random crops of size^dim from every (snapshot, RHS)."""
    rng = np.random.default_rng(seed)
    ne = ctx.info.n_e
    feats, tgts, iters = [], [], []
    for rhs in rhs_batches:
        B = rhs.shape[0]
        x, st, snaps = ctx.solve_snapshots(rhs, every_cycles=every_cycles, max_snaps=max_snaps)
        iters.extend(st.iters.tolist())
        for k in range(snaps.shape[0]):
            xk = snaps[k].contiguous()
            r = ctx.residual(rhs, xk)
            ncrop = B * crops_per_snapshot
            crops = np.stack([np.repeat(np.arange(B), crops_per_snapshot)]
                             + [rng.integers(0, ne - size + 1, ncrop) for _ in range(ctx.dim)], axis=1)
            f, t = ctx.net_examples(r, x, xk, crops, size, gamma=1.0)
            feats.append(f)
            tgts.append(t)
        del snaps
    feat = torch.cat(feats) if out is None else torch.cat([out.feat] + feats)
    tgt = torch.cat(tgts) if out is None else torch.cat([ctx.examples_scale(out.tgt, out.gamma)] + tgts)
    keep = torch.isfinite(feat).flatten(1).all(1) & torch.isfinite(tgt).flatten(1).all(1)
    feat, tgt = feat[keep].contiguous(), tgt[keep].contiguous()
    gamma = ctx.examples_rms(tgt)
    ctx.examples_scale(tgt, 1.0 / gamma)
    prev = out.solve_iters if out is not None else []
    cb = (ctx.info.k0 * ctx.info.n_b * ctx.info.h) ** 2
    return Examples(feat, tgt, gamma, cb, prev + iters)


def rescaled(ctx: helm.Context, ex: Examples, gamma: float) -> Examples:
    """The examples with targets expressed for another scale gamma (targets times ex.gamma / gamma, in
    place, by the library), e.g. a validation set for a network trained at the training set's gamma."""
    ctx.examples_scale(ex.tgt, ex.gamma / gamma)
    return Examples(ex.feat, ex.tgt, gamma, ex.cb, ex.solve_iters)


def _augment(x: torch.Tensor, y: torch.Tensor, k: int):
    """One of 8 symmetries of the grid: in 2D the flips and the transposition of the two image axes,
    in 3D the flips of the three axes."""
    if k & 1:
        x, y = x.flip(1), y.flip(1)
    if k & 2:
        x, y = x.flip(2), y.flip(2)
    if k & 4:
        if x.dim() == 5:
            x, y = x.flip(3), y.flip(3)
        else:
            x, y = x.transpose(1, 2), y.transpose(1, 2)
    return x.contiguous(), y.contiguous()


LAYERS = (("A0", 4, 16, 0), ("A1", 16, 32, 1), ("A2", 32, 64, 2), ("A3", 64, 64, 3),
          ("B2", 128, 64, 2), ("B1", 96, 32, 1), ("B0", 48, 16, 0), ("O", 16, 2, 0))
LAYERS3 = (("A0", 4, 16, 0), ("A1", 16, 16, 1), ("A2", 16, 32, 2), ("A3", 32, 32, 3),
           ("B2", 64, 32, 2), ("B1", 48, 16, 1), ("B0", 32, 16, 0), ("O", 16, 2, 0))


def flops_per_image(H: int, W: int, D: int | None = None) -> float:
    """Multiply-adds x 2 of the eight 3x3 (3x3x3 with depth D) convolutions for one image (no
    padding counted)."""
    shape = [(H, W) if D is None else (D, H, W)]
    for _ in range(3):
        shape.append(tuple((s + 1) // 2 for s in shape[-1]))
    taps, layers = (9, LAYERS) if D is None else (27, LAYERS3)
    return float(sum(2 * taps * ci * co * int(np.prod(shape[lvl])) for _, ci, co, lvl in layers))


def new_network(seed: int, dim: int = 2) -> helm.Net:
    """He-initialised network whose output layer starts at zero (the network first outputs 0,
    the zero correction, and training moves it from there)."""
    net = helm.Net(seed=seed, dim=dim)
    p = net.params()
    p["O.w"][:] = 0.0
    p["O.b"][:] = 0.0
    net.set_params(p)
    return net


@dataclass
class TrainLog:
    losses: list
    seconds: float
    steps: int
    pixels_per_step: int


def train(net: helm.Net, ex: Examples, steps: int, batch: int, lr: float, seed: int, lr_final: float | None = None,
          err_weight: float = 1.0, res_weight: float = 0.0, log_every: int = 0, log=print) -> TrainLog:
    """Adam on minibatches of `batch` examples; the learning rate decays by cosine to lr_final.

    Loss per example: err_weight/2 |y - e|^2 + res_weight/2 |r - gamma A' y|^2 (the second
    term asks the network output to reduce the residual, the quantity the solver's
    acceptance test measures)."""
    net.set_loss(err_weight, res_weight, gamma=ex.gamma, cb=ex.cb)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = ex.feat.shape[0]
    lr_final = lr * 0.05 if lr_final is None else lr_final
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(ex.feat.device)
        k = int(torch.randint(0, 8, (1,), generator=g))
        x, y = _augment(ex.feat.index_select(0, idx), ex.tgt.index_select(0, idx), k)
        losses.append(net.backward(x, y))
        a = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * it / max(1, steps - 1)))
        net.adam_step(a)
        if log_every and (it % log_every == 0 or it == steps - 1):
            log(f"[train] step {it} loss {losses[-1]:.4f}")
    torch.cuda.synchronize()
    return TrainLog(losses, time.perf_counter() - t0, steps, batch * int(np.prod(ex.feat.shape[1:-1])))


def residual_ratio(ctx: helm.Context, net: helm.Net, ex: Examples, count: int = 64) -> float:
    """Median over examples of ||r - gamma A' net(r)|| / ||r|| on crop interiors (1 = no better than zero);
    the ratios come from the library's kernel."""
    return float(np.median(net.residual_ratio(ex.feat[:count], ex.gamma, ex.cb)))
