"""torch.autograd.Function for the Helmholtz forward model and its adjoint gradient.

Forward (Sec. V, eq. DiscreteForwardHelm with on-grid receivers S):
    y_q = S u_sc,q(n),   A_Hel(n) u_sc,q = f(n) u_in,q,   f = k0^2 (n^2 - n_b^2)
Backward (Prop. 1): with the incoming gradient g_q = dL/dy_q (torch's
convention for complex outputs, so g_q = S u_sc,q - y_q for a quadratic data
term), the adjoint states lam_q = A^-H S^T g_q come from the batched adjoint
solve and
    dL/dn = sum_q 2 k0^2 n Re(conj(u_in,q + u_sc,q) lam_q)
is one gradient kernel.  Every step runs in libhelm; this module only orders
the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from .helm import Context


class HelmholtzScattering(torch.autograd.Function):
    """y = S u_sc(n) for all plane waves of a scan; backward = adjoint solve + grad_n kernel."""

    @staticmethod
    def forward(fctx, n_map: torch.Tensor, hctx: Context, dirs: np.ndarray, rx_idx: torch.Tensor):
        nm = n_map.detach().to(torch.float32).contiguous()
        hctx.update_n(nm)
        rhs, uin = hctx.plane_wave_rhs(dirs, with_uin=True)
        usc, st = hctx.solve(rhs)
        if not st.converged:
            raise RuntimeError(f"forward solve did not converge: {st}")
        fctx.hctx, fctx.rx_idx, fctx.n_map, fctx.version = hctx, rx_idx, nm, hctx.medium_version
        fctx.save_for_backward(uin, usc)
        return hctx.sample(rx_idx, usc)

    @staticmethod
    def backward(fctx, grad_y: torch.Tensor):
        uin, usc = fctx.saved_tensors
        hctx = fctx.hctx
        if hctx.medium_version != fctx.version:  # the context saw another medium since the forward pass
            hctx.update_n(fctx.n_map)
        g = hctx.sample_adjoint(fctx.rx_idx, grad_y.to(torch.complex64).contiguous())
        lam, st = hctx.adjoint(g)
        if not st.converged:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        grad_n = hctx.grad_n(usc, lam, u_in=uin)
        return grad_n, None, None, None


class HelmholtzDataTerm(torch.autograd.Function):
    """L = sum_q 1/2 ||S u_sc,q(n) - y_q||^2 (eq. DataFidelityExplicit with on-grid receivers).

    Forward: medium update, batched forward solves, and the data residual r_q = S u_sc,q - y_q
    with L from the library (helm_data_residual).  Backward (Prop. 1): lam_q = A^-H S^T r_q by the
    batched adjoint solve, dL/dn = sum_q 2 k0^2 n Re(conj(u_in,q + u_sc,q) lam_q) (helm_grad_n);
    the residual that seeds the adjoint comes from the library, not from torch."""

    @staticmethod
    def forward(fctx, n_map: torch.Tensor, hctx: Context, dirs: np.ndarray, rx_idx: torch.Tensor,
                data: torch.Tensor):
        nm = n_map.detach().to(torch.float32).contiguous()
        hctx.update_n(nm)
        rhs, uin = hctx.plane_wave_rhs(dirs, with_uin=True)
        usc, st = hctx.solve(rhs)
        if not st.converged:
            raise RuntimeError(f"forward solve did not converge: {st}")
        res, loss = hctx.data_residual(rx_idx, usc, data.to(torch.complex64).contiguous())
        fctx.hctx, fctx.rx_idx, fctx.n_map, fctx.version = hctx, rx_idx, nm, hctx.medium_version
        fctx.save_for_backward(uin, usc, res)
        return torch.tensor(loss, dtype=torch.float64, device=n_map.device)

    @staticmethod
    def backward(fctx, g):
        uin, usc, res = fctx.saved_tensors
        hctx = fctx.hctx
        if hctx.medium_version != fctx.version:  # the context saw another medium since the forward pass
            hctx.update_n(fctx.n_map)
        lam, st = hctx.adjoint(hctx.sample_adjoint(fctx.rx_idx, res))
        if not st.converged:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        grad_n = hctx.grad_n(usc, lam, u_in=uin)
        # chain rule through the scalar output (g = 1 for loss.backward())
        return grad_n * g.to(grad_n.dtype), None, None, None, None


class SmoothedTV(torch.autograd.Function):
    """Smoothed isotropic TV of the interior map (value and gradient from libhelm)."""

    @staticmethod
    def forward(fctx, n_map: torch.Tensor, hctx: Context, eps: float):
        val, grad = hctx.tv(n_map.detach(), eps)
        fctx.save_for_backward(grad)
        return torch.tensor(val, dtype=torch.float64, device=n_map.device)

    @staticmethod
    def backward(fctx, g):
        (grad,) = fctx.saved_tensors
        return grad * g.to(grad.dtype), None, None


def receiver_line(hctx: Context, row: int | None = None) -> torch.Tensor:
    """Flat indices of an on-grid receiver line: one interior row of Omega (default: the last,
    on the transmission side of waves travelling toward +y)."""
    info = hctx.info
    w, n, ne = info.abl_width, info.n, info.n_e
    row = w + n - 1 if row is None else row
    idx = row * ne + w + np.arange(n)
    return torch.tensor(idx, dtype=torch.int32, device=hctx.device)


def data_loss(n_map: torch.Tensor, hctx: Context, dirs, rx_idx, data: torch.Tensor, tau: float = 1e-3,
              tv_eps: float = 1e-4) -> torch.Tensor:
    """sum_q 1/2 ||S u_sc,q(n) - y_q||^2 + tau TV_eps(n) (eq. MAPInverse with the quadratic data term);
    the data term and its gradient seed come from the library (HelmholtzDataTerm)."""
    loss = HelmholtzDataTerm.apply(n_map, hctx, dirs, rx_idx, data)
    if tau:
        loss = loss + tau * SmoothedTV.apply(n_map, hctx, tv_eps)
    return loss
