"""Accelerated forward-backward splitting (Alg. 4) for the inverse problem of
Sec. V (eq. MAPInverse) with on-grid receivers S:

    f* = argmin_{f >= 0} sum_q 1/2 ||S u_sc,q(f) - y_q||^2 + tau TV(f),

f = k0^2 (n^2 - n_b^2) the scattering potential on Omega.  Per iteration:
a (random) subset of the illuminations (Alg. 4's stochastic selection), the
medium from fbar, the batched forward solves, the data residual, the batched
adjoint solves on S^T r, the gradient of Prop. 1 (grad_f), and the library's
FBS update (TV prox by fast gradient projection, momentum).  Every step runs
in libhelm; this module orders the calls and draws the subsets.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from .helm import Context


@dataclass
class FBSLog:
    loss: list = field(default_factory=list)       # data term of the selected subset at fbar
    iters: list = field(default_factory=list)      # mean multigrid cycles per forward solve
    subsets: list = field(default_factory=list)


class FBSReconstruction:
    """State of Alg. 4: f, fbar, alpha; the data y [Q, M] either at on-grid receivers rx_idx
    (flat grid indices) or, with rx_idx None, at the far-field sensors of ctx.farfield_set
    (the sensor operator G~ of eq. DiscreteForwardHelm)."""

    def __init__(self, ctx: Context, dirs: np.ndarray, rx_idx: torch.Tensor | None, y: torch.Tensor, gamma: float,
                 tau: float, prox_iters: int = 50, subset: int | None = None, seed: int = 0,
                 f0: torch.Tensor | None = None):
        self.ctx, self.dirs, self.rx, self.y = ctx, np.asarray(dirs, dtype=np.float64), rx_idx, y
        self.gamma, self.tau, self.prox_iters = gamma, tau, prox_iters
        self.subset = subset
        self.rng = np.random.default_rng(seed)
        shape = (ctx.info.n,) * ctx.dim
        self.f = (torch.zeros(shape, dtype=torch.float32, device=ctx.device) if f0 is None
                  else f0.to(torch.float32).contiguous().clone())
        self.fbar = self.f.clone()
        self.alpha = 1.0
        self.log = FBSLog()

    def gradient(self, f: torch.Tensor, sel: np.ndarray):
        """(sum over the selection of grad_f D_q at f, data term, mean iterations)."""
        ctx = self.ctx
        ctx.update_f(f)
        rhs, uin = ctx.plane_wave_rhs(self.dirs[sel], with_uin=True)
        usc, st = ctx.solve(rhs)
        if not st.converged:
            raise RuntimeError(f"forward solves did not converge: {st}")
        sel_t = torch.as_tensor(sel, device=self.y.device)
        y_sel = self.y.index_select(0, sel_t).contiguous()
        if self.rx is None:  # far-field sensors: grad = Re(conj(u) (s + A^-H f s)), s = G~^H r
            _, res, loss = ctx.farfield_residual(usc, y_sel, u_in=uin)
            s, arhs = ctx.farfield_adjoint(res)
            lam, st_a = ctx.adjoint(arhs)
            if not st_a.converged:
                raise RuntimeError(f"adjoint solves did not converge: {st_a}")
            return ctx.grad_f_farfield(usc, lam, s, u_in=uin), loss, float(st.iters.mean())
        res, loss = ctx.data_residual(self.rx, usc, y_sel)
        lam, st_a = ctx.adjoint(ctx.sample_adjoint(self.rx, res))
        if not st_a.converged:
            raise RuntimeError(f"adjoint solves did not converge: {st_a}")
        return ctx.grad_f(usc, lam, u_in=uin), loss, float(st.iters.mean())

    def step(self):
        Q = self.dirs.shape[0]
        if self.subset is None or self.subset >= Q:
            sel = np.arange(Q)
        else:
            sel = np.sort(self.rng.choice(Q, size=self.subset, replace=False))
        grad, loss, its = self.gradient(self.fbar, sel)
        self.alpha = self.ctx.fbs_step(self.f, self.fbar, grad, self.gamma, self.tau, self.alpha, lo=0.0,
                                       prox_iters=self.prox_iters)
        self.log.loss.append(loss)
        self.log.iters.append(its)
        self.log.subsets.append(sel)
        return loss

    def run(self, iterations: int):
        for _ in range(iterations):
            self.step()
        return self.f
