"""Golden pin: the paper's disk experiment (Sec. VI-A, Fig. 4) against the analytic cylinder field.

The paper reports a squared-norm relative total-field error of 7.5e-3 for its
Helmholtz discretisation (256^2 samples, 80 points per wavelength, 32-point
layer with beta = 0.15, first-order Sommerfeld rows).  The oracle's
discretisation of the same setup must land at the same order of magnitude;
this pins the operator, the ghost rows, the layer and the plane-wave
conventions as a whole against physics.
"""
import json
import os

import numpy as np
import pytest

from oracle.cylinder import cylinder_total_field
from oracle.discretization import Problem
from oracle.model import ExactSolver, plane_wave, rhs

HERE = os.path.dirname(os.path.abspath(__file__))


def test_cylinder_series_satisfies_interface_conditions():
    # the textbook series: continuity of u and du/dr across r = R
    k_b, k_d, R = 2 * np.pi, 2 * np.pi * 2.2, 1.25
    phi = np.linspace(0, 2 * np.pi, 7)
    eps = 1e-6
    ui = cylinder_total_field((R - eps) * np.cos(phi), (R - eps) * np.sin(phi), R, k_b, k_d, 0.3)
    uo = cylinder_total_field((R + eps) * np.cos(phi), (R + eps) * np.sin(phi), R, k_b, k_d, 0.3)
    assert np.allclose(ui, uo, atol=1e-4)
    # far from the cylinder with k_d = k_b the field is the plane wave itself
    x, y = np.array([3.0, -2.0]), np.array([0.5, 4.0])
    u = cylinder_total_field(x, y, R, k_b, k_b, 0.3)
    assert np.allclose(u, np.exp(1j * k_b * (np.cos(0.3) * x + np.sin(0.3) * y)), atol=1e-10)


@pytest.mark.slow
def test_disk_in_air_total_field_error_matches_paper_order():
    g = json.load(open(os.path.join(HERE, "golden", "disk_in_air.json")))
    lam, hphys, n = g["wavelength_cm"], g["h_cm"], g["N_side"]
    k0h = 2 * np.pi / lam * hphys
    radius_cells = g["radius_wavelengths"] * lam / hphys
    ax = np.arange(n) - (n - 1) / 2
    yy, xx = np.meshgrid(ax, ax, indexing="ij")
    nmap = np.where(xx ** 2 + yy ** 2 <= radius_cells ** 2, g["eta_disk"], g["eta_b"])
    prob = Problem(nmap, k0h=k0h, n_b=g["eta_b"], w=g["abl_points_per_side"], beta=g["abl_beta"], levels=1)
    d = [0.0, -1.0]  # from the top of the image toward decreasing row index
    u_sc = ExactSolver(prob).solve(rhs(prob, d))
    u = (u_sc + plane_wave(prob, d))[prob.interior_slices()]
    k_b = 2 * np.pi / lam
    u_gt = cylinder_total_field(xx * hphys, yy * hphys, g["radius_wavelengths"] * lam, k_b, k_b * g["eta_disk"],
                                np.arctan2(d[1], d[0]))
    eps = np.linalg.norm(u - u_gt) ** 2 / np.linalg.norm(u_gt) ** 2
    ref = g["reported_error_helmholtz"]
    assert ref / 4 < eps < 2 * ref, eps
