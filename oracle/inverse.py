"""Inverse-problem steps of Sec. V: the TV proximal operator with
nonnegativity (eq. proximalOpt) and the accelerated forward-backward
splitting of Alg. 4.  Plain NumPy, FP64.

TEST INFRASTRUCTURE (see the package doc): only tests, the smoke check and
the CPU-baseline leg of the benchmark use it.

TV (isotropic, forward differences, zero difference across the last index of
each axis):  TV(w) = sum_i ||(D w)_i||_2,  (D w)_{a,i} = w_{i+e_a} - w_i.

prox: argmin_{w >= lo} 1/2 ||w - v||^2 + lam TV(w), computed as the paper
does, by the fast gradient projection on the dual (Beck and Teboulle 2009):
with the dual field p (one vector per point, ||p_i|| <= 1),
    w(p) = P_C(v - lam D^T p),        P_C = clip to [lo, inf)
the dual objective is concave with gradient lam D w(p) and Lipschitz
constant lam^2 ||D||^2 <= 4 d lam^2, so the projected ascent step is
    p <- P_B(r + D w(r) / (4 d lam))
with Nesterov extrapolation r of the dual iterates (t' = (1 + sqrt(1 + 4 t^2)) / 2,
r = p + (t - 1) / t' (p - p_prev)); the primal answer is w(p) after the last step.
"""
from __future__ import annotations

import numpy as np


def tv_value(w: np.ndarray) -> float:
    """Isotropic TV with forward differences (zero across the last index)."""
    return float(np.sum(np.sqrt(np.sum(forward_diff(w) ** 2, axis=0))))


def forward_diff(w: np.ndarray) -> np.ndarray:
    """D w: array [d][shape], component a = w(x + e_a) - w(x), 0 at the last index along a."""
    out = np.zeros((w.ndim, *w.shape))
    for a in range(w.ndim):
        sl_lo = [slice(None)] * w.ndim
        sl_hi = [slice(None)] * w.ndim
        sl_lo[a] = slice(0, -1)
        sl_hi[a] = slice(1, None)
        out[(a, *sl_lo)] = w[tuple(sl_hi)] - w[tuple(sl_lo)]
    return out


def forward_diff_adjoint(p: np.ndarray) -> np.ndarray:
    """D^T p, written out from <D w, p> = <w, D^T p>."""
    d = p.shape[0]
    out = np.zeros(p.shape[1:])
    for a in range(d):
        pa = p[a].copy()
        sl_last = [slice(None)] * d
        sl_last[a] = -1
        pa[tuple(sl_last)] = 0.0  # no difference across the last index
        out -= pa
        sl_lo = [slice(None)] * d
        sl_hi = [slice(None)] * d
        sl_lo[a] = slice(0, -1)
        sl_hi[a] = slice(1, None)
        out[tuple(sl_hi)] += pa[tuple(sl_lo)]
    return out


def tv_prox(v: np.ndarray, lam: float, lo: float = 0.0, iters: int = 100) -> np.ndarray:
    """argmin_{w >= lo} 1/2 ||w - v||^2 + lam TV(w) by FGP on the dual (module doc)."""
    if lam <= 0.0:
        return np.maximum(v, lo)
    d = v.ndim
    p = np.zeros((d, *v.shape))
    r = p.copy()
    t = 1.0
    for _ in range(iters):
        w = np.maximum(v - lam * forward_diff_adjoint(r), lo)
        q = r + forward_diff(w) / (4.0 * d * lam)
        q /= np.maximum(1.0, np.sqrt(np.sum(q ** 2, axis=0)))
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        r = q + ((t - 1.0) / t_next) * (q - p)
        p, t = q, t_next
    return np.maximum(v - lam * forward_diff_adjoint(p), lo)


def fbs_update(f: np.ndarray, fbar: np.ndarray, grad: np.ndarray, gamma: float, tau: float, alpha: float,
               prox_iters: int = 100, lo: float = 0.0):
    """One iteration of Alg. 4 after its gradient: f' = prox_{gamma tau}(fbar - gamma grad),
    alpha' = (1 + sqrt(1 + 4 alpha^2)) / 2, fbar' = f' + (alpha - 1) / alpha' (f' - f).
    Returns (f', fbar', alpha')."""
    f_new = tv_prox(fbar - gamma * grad, gamma * tau, lo=lo, iters=prox_iters)
    alpha_next = (1.0 + np.sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0
    fbar_new = f_new + ((alpha - 1.0) / alpha_next) * (f_new - f)
    return f_new, fbar_new, alpha_next
