"""Krylov solvers for A u = b, preconditioned on the right by a multigrid cycle.

* ``fgmres``   restarted flexible GMRES(m) with right preconditioning
               (Saad 1993): z_j = M(v_j), w = A z_j, modified Gram-Schmidt,
               complex Givens rotations, x += Z y at the end of each cycle and
               a true residual at every restart.  FGMRES is used because the
               paper's idea (Sec. IV-C: a Krylov method corrects the
               deviations of an MG preconditioner) must also admit a
               nonlinear preconditioner.
* ``sstep_gmres`` the same GMRES(m) iterates computed in s-step form: per
               cycle the basis W_0 = r/||r||, W_{j+1} = A M W_j is built
               without orthogonalisation; its Gram matrix G = W^H W gives a
               Cholesky factor R (G = R^H R, i.e. W = Q R), and the cycle's
               least-squares problem min ||r - A M W_{0:m} y|| is
               min || ||r|| R_00 e_0 - R[:, 1:] y ||, solved here with a
               library least-squares routine.  In exact arithmetic this is
               GMRES(m) (the Krylov space and the minimised norm are the same).
* ``bicgstab`` Alg. 3 of the paper (MG-preconditioned Bi-CGSTAB).  Readings:
               the printed sigma plays the role of van der Vorst's omega, the
               stop test is relative, ||r|| <= eps ||b|| (Sec. VI states
               relative), and u_0 = 0.  Convergence is judged on the true
               residual b - A u; where the recurrence's residual meets the
               tolerance and the true one does not, the recurrence restarts
               from the true residual.

Inner product <a, b> = a^H b (reading A14: the paper defines real inner
products only).  Iteration counts are preconditioner applications.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SolveInfo:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    rel_res_true: float = np.inf
    history: list = field(default_factory=list)   # estimated relative residual per iteration


def _norm(v):
    return float(np.sqrt(np.vdot(v, v).real))


def givens(a: complex, b: complex):
    """Rotation G = [[c, s], [-conj(s), c]] (c real) with G [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    rho = np.hypot(abs(a), abs(b))
    c = abs(a) / rho
    s = (a / abs(a)) * np.conj(b) / rho
    return c, s


def fgmres(apply_a, precond, b: np.ndarray, rtol: float = 1e-6, restart: int = 20, max_iters: int = 2000,
           x0: np.ndarray | None = None) -> tuple[np.ndarray, SolveInfo]:
    """Right-preconditioned FGMRES(restart) until ||b - A x|| <= rtol ||b|| (true residual)."""
    info = SolveInfo()
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = _norm(b)
    if bnorm == 0.0:
        info.converged, info.rel_res_true = True, 0.0
        return x, info
    r = b - apply_a(x) if x0 is not None else b.copy()
    while True:
        beta = _norm(r)
        info.rel_res_true = beta / bnorm
        if info.rel_res_true <= rtol:
            info.converged = True
            return x, info
        if info.iters >= max_iters:
            return x, info
        m = restart
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        Z = np.zeros((m, b.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r.ravel() / beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j].reshape(b.shape)).ravel()
            w = apply_a(Z[j].reshape(b.shape)).ravel()
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = _norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            info.iters += 1
            k = j + 1
            info.history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or info.iters >= max_iters:
                break
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + (y @ Z[:k]).reshape(b.shape)
        r = b - apply_a(x)
        info.restarts += 1


def sstep_gmres(apply_a, precond, b: np.ndarray, rtol: float = 1e-6, restart: int = 5, max_iters: int = 2000,
                x0: np.ndarray | None = None) -> tuple[np.ndarray, SolveInfo]:
    """GMRES(restart) in s-step form (module doc) until ||b - A x|| <= rtol ||b||.

    Every cycle performs `restart` preconditioner applications (info.iters
    counts them); the update uses the smallest leading basis whose residual
    estimate meets the tolerance.  history holds the estimate after each
    basis size of each cycle.
    """
    info = SolveInfo()
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = _norm(b)
    if bnorm == 0.0:
        info.converged, info.rel_res_true = True, 0.0
        return x, info
    r = b - apply_a(x) if x0 is not None else b.copy()
    m = restart
    while True:
        beta = _norm(r)
        info.rel_res_true = beta / bnorm
        if info.rel_res_true <= rtol:
            info.converged = True
            return x, info
        if info.iters >= max_iters:
            return x, info
        W = [r.ravel() / beta]
        Z = []
        for _ in range(m):
            Z.append(precond(W[-1].reshape(b.shape)).ravel())
            W.append(apply_a(Z[-1].reshape(b.shape)).ravel())
        Wm = np.array(W)
        G = Wm.conj() @ Wm.T
        R = np.linalg.cholesky(G).conj().T  # G = R^H R, R upper triangular
        info.iters += m
        k_use = m
        for k in range(1, m + 1):
            g = np.zeros(k + 1, dtype=np.complex128)
            g[0] = beta * R[0, 0]
            y, *_ = np.linalg.lstsq(R[:k + 1, 1:k + 1], g, rcond=None)
            est = np.linalg.norm(g - R[:k + 1, 1:k + 1] @ y)
            info.history.append(est / bnorm)
            if est <= rtol * bnorm:
                k_use = k
                break
        g = np.zeros(k_use + 1, dtype=np.complex128)
        g[0] = beta * R[0, 0]
        y, *_ = np.linalg.lstsq(R[:k_use + 1, 1:k_use + 1], g, rcond=None)
        x = x + (y @ np.array(Z[:k_use])).reshape(b.shape)
        r = b - apply_a(x)
        info.restarts += 1


def bicgstab(apply_a, precond, b: np.ndarray, rtol: float = 1e-6, max_iters: int = 2000,
             x0: np.ndarray | None = None) -> tuple[np.ndarray, SolveInfo]:
    """Alg. 3: Bi-CGSTAB with a multigrid cycle as right preconditioner (two cycles per iteration)."""
    info = SolveInfo()
    u = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = _norm(b)
    r = b - apply_a(u) if x0 is not None else b.copy()
    r_hat = r.copy()
    rho_prev, alpha, sigma = 1.0 + 0j, 1.0 + 0j, 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    if bnorm == 0.0:
        info.converged, info.rel_res_true = True, 0.0
        return u, info
    for it in range(1, max_iters + 1):
        if it > 1 and info.history[-1] <= rtol:
            # the recurrence met the tolerance but the true residual did not: restart from it
            r = b - apply_a(u)
            r_hat = r.copy()
            rho_prev, alpha, sigma = 1.0 + 0j, 1.0 + 0j, 1.0 + 0j
            v = np.zeros_like(b)
            p = np.zeros_like(b)
        rho = np.vdot(r_hat, r)
        beta = (rho / rho_prev) * (alpha / sigma)
        p = r + beta * (p - sigma * v)
        y = precond(p)
        v = apply_a(y)
        alpha = rho / np.vdot(r_hat, v)
        hvec = u + alpha * y
        s = r - alpha * v
        z = precond(s)
        t = apply_a(z)
        sigma = np.vdot(t, s) / np.vdot(t, t)
        u = hvec + sigma * z
        r = s - sigma * t
        rho_prev = rho
        info.iters += 2
        rel = _norm(r) / bnorm
        info.history.append(rel)
        if rel <= rtol and _norm(b - apply_a(u)) <= rtol * bnorm:
            break
    info.rel_res_true = _norm(b - apply_a(u)) / bnorm
    info.converged = info.rel_res_true <= rtol
    return u, info
