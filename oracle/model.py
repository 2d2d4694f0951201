"""Forward model, adjoint and gradient (Sec. II-A, Sec. IV-A, Sec. V, Prop. 1).

Unscaled semantics: ``A`` below is A_Hel of eq. (discretizedHelm) (the
1/h^2 form), ``b = f u_in`` with f = k0^2 (eta^2 - eta_b^2) (zero in the
absorbing layer), and u_sc = A^-1 b (eq. HelmScatterRightIncident:discrete).
The multigrid solver works on the h^2-scaled system A' = h^2 A,
b' = h^2 b, which has the same solution.

Readings:
* A17 plane wave u_in(x) = exp(j k_b <d, x - x_c>), u_0 = 1, with x_c the
      centre of Omega and k_b = k0 eta_b the background wavenumber.
* A16 Prop. 1 omits the sensor operator; for the on-grid receivers used
      here, H(f) = S u_sc(f) and du_sc = A^-1 diag(u) df with the TOTAL field
      u = u_in + u_sc.  For L = 1/2 ||S u_sc - y||^2 and real f,
      grad_f L = Re(conj(u) * lambda) with lambda = A^-H S^T (S u_sc - y),
      and grad_n L = 2 k0^2 n grad_f L on Omega (chain rule through f).
* A23 smoothed isotropic TV: sum sqrt(dx^2 + dy^2 + eps^2), forward
      differences, zero difference across the last row/column.
* F6  A is complex symmetric (the Sommerfeld terms are diagonal), hence
      A^-H g = conj(A^-1 conj(g)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import Problem, helmholtz_matrix
from .krylov import bicgstab, fgmres
from .multigrid import Hierarchy


def plane_wave(prob: Problem, direction) -> np.ndarray:
    """u_in on Omega_e for a unit direction (x, y[, z]) (reading A17)."""
    d = prob.d
    direction = np.asarray(direction, dtype=np.float64)
    centre = prob.w + (prob.n - 1) / 2.0
    axes = np.meshgrid(*([np.arange(prob.n_e, dtype=np.float64)] * d), indexing="ij")
    # C-order axes are (y, x) / (z, y, x); the direction is given as (x, y[, z])
    phase = 0.0
    for a in range(d):
        comp = direction[d - 1 - a]
        phase = phase + comp * (axes[a] - centre)
    return np.exp(1j * prob.kbh * phase)


def scattering_potential(prob: Problem) -> np.ndarray:
    """f = k0^2 (eta^2 - eta_b^2) on Omega_e (zero in the layer), unscaled units."""
    f = np.zeros(prob.shape)
    f[prob.interior_slices()] = prob.k0 ** 2 * (prob.n_map ** 2 - prob.n_b ** 2)
    return f


def rhs(prob: Problem, direction) -> np.ndarray:
    """b = f u_in (eq. HelmScatterRightIncident), unscaled."""
    return scattering_potential(prob) * plane_wave(prob, direction)


class ExactSolver:
    """Sparse LU of A (unscaled); the reference answer u_sc = A^-1 b (plain definition)."""

    def __init__(self, prob: Problem):
        self.prob = prob
        self.A = helmholtz_matrix(prob, scaled=False)
        self.lu = spla.splu(self.A.tocsc())

    def solve(self, b: np.ndarray) -> np.ndarray:
        return self.lu.solve(b.ravel().astype(np.complex128)).reshape(b.shape)

    def solve_adjoint(self, g: np.ndarray) -> np.ndarray:
        """A^-H g via the factorisation of A (trans='H')."""
        return self.lu.solve(g.ravel().astype(np.complex128), trans="H").reshape(g.shape)


def mg_fgmres_solve(prob: Problem, b: np.ndarray, rtol: float = 1e-6, restart: int = 20,
                    max_iters: int = 4000, hierarchy: Hierarchy | None = None):
    """u = A^-1 b by FGMRES(restart) preconditioned with one V-cycle on K_kappa (unscaled in/out)."""
    hier = Hierarchy(prob) if hierarchy is None else hierarchy
    a_scaled = helmholtz_matrix(prob, scaled=True)
    shape = b.shape
    bs = (prob.h ** 2) * b.ravel()
    x, info = fgmres(lambda v: a_scaled @ v, hier.vcycle, bs, rtol=rtol, restart=restart, max_iters=max_iters)
    return x.reshape(shape), info


def mg_bicgstab_solve(prob: Problem, b: np.ndarray, rtol: float = 1e-6, max_iters: int = 4000,
                      hierarchy: Hierarchy | None = None):
    """u = A^-1 b by Alg. 3 (Bi-CGSTAB, one V-cycle on K_kappa per preconditioner application)."""
    hier = Hierarchy(prob) if hierarchy is None else hierarchy
    a_scaled = helmholtz_matrix(prob, scaled=True)
    shape = b.shape
    bs = (prob.h ** 2) * b.ravel()
    x, info = bicgstab(lambda v: a_scaled @ v, hier.vcycle, bs, rtol=rtol, max_iters=max_iters)
    return x.reshape(shape), info


def adjoint_by_conjugation(solve, g: np.ndarray) -> np.ndarray:
    """lambda = A^-H g = conj(A^-1 conj(g)) (A = A^T)."""
    return np.conj(solve(np.conj(g)))


# -- data term, receivers and gradient --------------------------------------

def receiver_row(prob: Problem) -> tuple:
    """Index of the receiver line S: the last interior row of Omega on the transmission side (reading A21)."""
    assert prob.d == 2
    return (prob.w + prob.n - 1, slice(prob.w, prob.w + prob.n))


def sample(prob: Problem, u: np.ndarray) -> np.ndarray:
    """S u: values of u on the receiver line."""
    return u[receiver_row(prob)].copy()


def sample_adjoint(prob: Problem, r: np.ndarray) -> np.ndarray:
    """S^T r: receiver values scattered back onto Omega_e (zeros elsewhere)."""
    out = np.zeros(prob.shape, dtype=np.complex128)
    out[receiver_row(prob)] = r
    return out


def tv_smoothed(n_map: np.ndarray, eps: float = 1e-4):
    """Value and gradient of sum sqrt((D_x n)^2 + (D_y n)^2 + eps^2) (reading A23)."""
    dx = np.zeros_like(n_map)
    dy = np.zeros_like(n_map)
    dx[:, :-1] = n_map[:, 1:] - n_map[:, :-1]
    dy[:-1, :] = n_map[1:, :] - n_map[:-1, :]
    mag = np.sqrt(dx * dx + dy * dy + eps * eps)
    val = float(mag.sum())
    px = dx / mag
    py = dy / mag
    grad = np.zeros_like(n_map)
    # d/dn of dx[i,j] = n[i,j+1] - n[i,j]
    grad[:, :-1] -= px[:, :-1]
    grad[:, 1:] += px[:, :-1]
    grad[:-1, :] -= py[:-1, :]
    grad[1:, :] += py[:-1, :]
    return val, grad


def loss_and_gradient(prob: Problem, directions, data, tau: float = 1e-3, tv_eps: float = 1e-4,
                      solver: ExactSolver | None = None):
    """L(n) = sum_q 1/2 ||S u_sc,q - y_q||^2 + tau TV_eps(n) and grad_n L on Omega (exact LU solves)."""
    solver = ExactSolver(prob) if solver is None else solver
    grad_f = np.zeros(prob.shape)
    loss = 0.0
    for q, dvec in enumerate(directions):
        uin = plane_wave(prob, dvec)
        b = scattering_potential(prob) * uin
        usc = solver.solve(b)
        res = sample(prob, usc) - data[q]
        loss += 0.5 * float(np.vdot(res, res).real)
        lam = solver.solve_adjoint(sample_adjoint(prob, res))
        grad_f += np.real(np.conj(uin + usc) * lam)
    grad_n = 2.0 * prob.k0 ** 2 * prob.n_map * grad_f[prob.interior_slices()]
    tv, tvg = tv_smoothed(prob.n_map, tv_eps)
    return loss + tau * tv, grad_n + tau * tvg


def loss_only(prob: Problem, directions, data, tau: float = 1e-3, tv_eps: float = 1e-4) -> float:
    solver = ExactSolver(prob)
    loss = 0.0
    for q, dvec in enumerate(directions):
        usc = solver.solve(rhs(prob, dvec))
        res = sample(prob, usc) - data[q]
        loss += 0.5 * float(np.vdot(res, res).real)
    return loss + tau * tv_smoothed(prob.n_map, tv_eps)[0]


def scalar_field_gradient(prob: Problem, u_total: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """grad_n = sum_q 2 k0^2 n Re(conj(u_q) lambda_q) on Omega for stacked fields [B, ...]."""
    s = np.real(np.conj(u_total) * lam).sum(axis=0)
    return 2.0 * prob.k0 ** 2 * prob.n_map * s[prob.interior_slices()]
