"""Sensor operator G~ of eq. DiscreteForwardHelm: the scattered field at
sensors outside Omega from the induced source f u on Omega, by the
Lippmann-Schwinger integral (eq. LSIntegral) with the free-space Green's
function (eq. green) and the rectangle rule.  Plain NumPy/SciPy, FP64.

TEST INFRASTRUCTURE (see the package doc).

    y_m = sum_{z in Omega} g(x_m - z) f(z) u(z) h^d
    g(x) = (j/4) H0^(1)(k_b |x|) (2D),  exp(j k_b |x|) / (4 pi |x|) (3D)

Sensor positions are in grid cells relative to the centre of Omega.
Gradient of 1/2 ||y(f) - y_meas||^2 through Prop. 1:
    dy = G~ (I + diag(f) A^-1) diag(u) df
    grad_f = Re(conj(u) (s + A^-H (f s))),  s = G~^H (y - y_meas)   on Omega.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from .discretization import Problem
from .model import ExactSolver, plane_wave, rhs, scattering_potential


def interior_coords(prob: Problem) -> np.ndarray:
    """[n^d, d] coordinates (x, y[, z]) in cells relative to the centre of Omega, x fastest."""
    ax = np.arange(prob.n) - (prob.n - 1) / 2.0
    grids = np.meshgrid(*([ax] * prob.d), indexing="ij")  # C order: (y, x) / (z, y, x)
    return np.stack([g.ravel() for g in grids[::-1]], axis=1)


def sensor_matrix(prob: Problem, sensors: np.ndarray) -> np.ndarray:
    sensors = np.asarray(sensors, dtype=np.float64).reshape(-1, prob.d)
    z = interior_coords(prob)
    r = np.sqrt(((sensors[:, None, :] - z[None, :, :]) ** 2).sum(axis=2)) * prob.h
    kb = prob.kbh / prob.h
    if prob.d == 2:
        g = 0.25j * special.hankel1(0, kb * r)
    else:
        g = np.exp(1j * kb * r) / (4.0 * np.pi * r)
    return g * prob.h ** prob.d


def farfield(prob: Problem, G: np.ndarray, u_total: np.ndarray) -> np.ndarray:
    """y = G~ (f u) for one total field on Omega_e."""
    f = scattering_potential(prob)[prob.interior_slices()]
    return G @ (f * u_total[prob.interior_slices()]).ravel()


def farfield_loss_and_gradient(prob: Problem, sensors, directions, y_meas):
    """(1/2 sum_q ||y_q - y_meas,q||^2, grad_f on Omega) with exact LU solves."""
    G = sensor_matrix(prob, sensors)
    ex = ExactSolver(prob)
    f = scattering_potential(prob)
    grad = np.zeros((prob.n,) * prob.d)
    loss = 0.0
    for q, d in enumerate(directions):
        u = plane_wave(prob, d) + ex.solve(rhs(prob, d))
        r = farfield(prob, G, u) - y_meas[q]
        loss += 0.5 * float(np.vdot(r, r).real)
        s = np.zeros(prob.shape, dtype=np.complex128)
        s[prob.interior_slices()] = (G.conj().T @ r).reshape((prob.n,) * prob.d)
        lam = ex.solve_adjoint(f * s)
        grad += np.real(np.conj(u) * (s + lam))[prob.interior_slices()]
    return loss, grad
