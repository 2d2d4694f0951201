"""Local Fourier analysis symbols of Sec. IV-B (constant k, periodic boundaries).

Grid function v(theta, x) = exp(j theta_1 x_1 / h) exp(j theta_2 x_2 / h).
These are closed forms used only as pins for the assembled operators.
"""
from __future__ import annotations

import numpy as np


def symbol_a(theta1, theta2, kh: complex, h: float = 1.0):
    """Eigenvalue of A^h on the mode theta: (4 - 2 cos t1 - 2 cos t2 - k^2 h^2) / h^2."""
    return (4.0 - 2.0 * (np.cos(theta1) + np.cos(theta2)) - kh * kh) / (h * h)


def symbol_jacobi(theta1, theta2, kh: complex, omega: float):
    """Eigenvalue of S^h = I - omega D^-1 A^h: 1 - omega + 2 omega (cos t1 + cos t2) / (4 - k^2 h^2)."""
    return 1.0 - omega + 2.0 * omega * (np.cos(theta1) + np.cos(theta2)) / (4.0 - kh * kh)


def jacobi_max_amplification(kh: float, omega: float) -> float:
    """max_theta |s^h(theta)| = 1 - omega + 4 omega / (4 - k^2 h^2) for 4 - k^2 h^2 > 0."""
    return 1.0 - omega + 4.0 * omega / (4.0 - kh * kh)


def cgc_ratio(theta1, theta2, kh: complex, kappa: complex = 1.0):
    """a^h(theta) / a^{2h}(2 theta) of the operator -Lap - kappa k^2 (kappa = 1: A itself; a
    complex kappa: the shifted operator of Sec. IV-B); the coarse-grid-correction factor is
    1 minus this ratio."""
    kh_eff = np.sqrt(complex(kappa)) * kh
    return symbol_a(theta1, theta2, kh_eff, 1.0) / symbol_a(2 * theta1, 2 * theta2, 2 * kh_eff, 2.0)
