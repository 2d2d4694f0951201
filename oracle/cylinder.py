"""Analytic total field of a dielectric cylinder under plane-wave illumination.

Used to pin the discretisation against the paper's disk experiment
(Sec. VI-A, Fig. 4): a disk of index eta_d = 2.2 in air, radius 1.25
wavelengths, wavelength 10 cm, 256^2 samples over a 3.2-wavelength square
(h = 0.125 cm), for which the paper reports a squared-norm relative error
of 7.5e-3 for its Helmholtz solver.

Textbook separation of variables (e^{-j w t}, outgoing H^(1)):
  u_in  = sum_n j^n J_n(k_b r) e^{j n (phi - phi_d)}
  u_sc  = sum_n j^n a_n H_n(k_b r) e^{j n (phi - phi_d)}      (r > R)
  u     = sum_n j^n c_n J_n(k_d r) e^{j n (phi - phi_d)}      (r < R)
with continuity of u and du/dr at r = R.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def cylinder_total_field(x: np.ndarray, y: np.ndarray, radius: float, k_b: float, k_d: float,
                         phi_d: float, n_terms: int | None = None) -> np.ndarray:
    """Total field at points (x, y) (cylinder centred at the origin), incident direction angle phi_d."""
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    if n_terms is None:
        kr = max(k_d * radius, k_b * float(np.max(r)))
        n_terms = int(kr + 4.0 * kr ** (1.0 / 3.0) + 15)
    out = np.zeros(r.shape, dtype=np.complex128)
    kbR, kdR = k_b * radius, k_d * radius
    inside = r < radius
    for n in range(-n_terms, n_terms + 1):
        jb, jbp = special.jv(n, kbR), special.jvp(n, kbR)
        jd, jdp = special.jv(n, kdR), special.jvp(n, kdR)
        hb, hbp = special.hankel1(n, kbR), special.h1vp(n, kbR)
        a_n = (k_d * jdp * jb - k_b * jd * jbp) / (k_b * jd * hbp - k_d * jdp * hb)
        c_n = (jb + a_n * hb) / jd
        ang = (1j ** n) * np.exp(1j * n * (phi - phi_d))
        out_out = (special.jv(n, k_b * r) + a_n * special.hankel1(n, k_b * r)) * ang
        out_in = c_n * special.jv(n, k_d * r) * ang
        out += np.where(inside, out_in, out_out)
    return out
