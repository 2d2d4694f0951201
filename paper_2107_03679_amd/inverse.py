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


@dataclass
class MultiFrequencyLog:
    loss: list = field(default_factory=list)       # data term over all frequencies (selected subsets) at chibar
    subsets: list = field(default_factory=list)    # per iteration: the selected plane waves of every frequency


class MultiFrequencyFBS:
    """Alg. 4 over several frequencies, as in the paper's experimental reconstructions (Sec. VI-C: four
    frequencies, a subset of the sources per iteration).  One Context per frequency (its own k0, the same
    grid), each with its plane waves, on-grid receivers and data.  The unknown is the
    frequency-independent contrast chi = n^2 - n_b^2 >= 0 on Omega (f = k0^2 chi at each frequency); the
    gradient is the sum over frequencies of k0^2 sum_q Re(conj(u_q) lam_q), accumulated in one buffer by
    the library, and the update is the library's FBS step (TV prox, momentum) on chi."""

    def __init__(self, ctxs, dirs, rx_idx, ys, gamma: float, tau: float, prox_iters: int = 50,
                 subset: int | None = None, seed: int = 0, chi0: torch.Tensor | None = None):
        assert len(ctxs) == len(dirs) == len(rx_idx) == len(ys) and len(ctxs) >= 1
        self.ctxs, self.rx, self.ys = list(ctxs), list(rx_idx), list(ys)
        self.dirs = [np.asarray(d, dtype=np.float64) for d in dirs]
        self.gamma, self.tau, self.prox_iters, self.subset = gamma, tau, prox_iters, subset
        self.rng = np.random.default_rng(seed)
        c0 = self.ctxs[0]
        shape = (c0.info.n,) * c0.dim
        self.chi = (torch.zeros(shape, dtype=torch.float32, device=c0.device) if chi0 is None
                    else chi0.to(torch.float32).contiguous().clone())
        self.chibar = self.chi.clone()
        self.grad = torch.empty_like(self.chi)
        self.alpha = 1.0
        self.log = MultiFrequencyLog()

    def select(self):
        """Alg. 4's stochastic selection, drawn per frequency (all plane waves when subset is None)."""
        out = []
        for d in self.dirs:
            Q = d.shape[0]
            if self.subset is None or self.subset >= Q:
                out.append(np.arange(Q))
            else:
                out.append(np.sort(self.rng.choice(Q, size=self.subset, replace=False)))
        return out

    def gradient(self, chi: torch.Tensor, sels):
        """(gradient with respect to chi summed over frequencies into self.grad, data term)."""
        loss = 0.0
        for i, (ctx, sel) in enumerate(zip(self.ctxs, sels)):
            ctx.update_contrast(chi)
            rhs, uin = ctx.plane_wave_rhs(self.dirs[i][sel], with_uin=True)
            usc, st = ctx.solve(rhs)
            if not st.converged:
                raise RuntimeError(f"forward solves of frequency {i} did not converge: {st}")
            y_sel = self.ys[i].index_select(0, torch.as_tensor(sel, device=self.ys[i].device)).contiguous()
            res, li = ctx.data_residual(self.rx[i], usc, y_sel)
            lam, st_a = ctx.adjoint(ctx.sample_adjoint(self.rx[i], res))
            if not st_a.converged:
                raise RuntimeError(f"adjoint solves of frequency {i} did not converge: {st_a}")
            ctx.grad_contrast(usc, lam, u_in=uin, out=self.grad, accumulate=i > 0)
            loss += li
        return self.grad, loss

    def step(self):
        sels = self.select()
        grad, loss = self.gradient(self.chibar, sels)
        self.alpha = self.ctxs[0].fbs_step(self.chi, self.chibar, grad, self.gamma, self.tau, self.alpha, lo=0.0,
                                           prox_iters=self.prox_iters)
        self.log.loss.append(loss)
        self.log.subsets.append(sels)
        return loss

    def run(self, iterations: int):
        for _ in range(iterations):
            self.step()
        return self.chi
