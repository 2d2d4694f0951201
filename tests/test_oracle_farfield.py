"""Pins of the oracle's sensor operator (eq. DiscreteForwardHelm, eq. LSIntegral, eq. green, Prop. 1)."""
import numpy as np
import pytest

import synth
from oracle.cylinder import cylinder_total_field
from oracle.discretization import Problem
from oracle.farfield import farfield, farfield_loss_and_gradient, interior_coords, sensor_matrix
from oracle.model import ExactSolver, plane_wave, rhs


def circle(m, radius):
    t = 2 * np.pi * np.arange(m) / m
    return np.stack([radius * np.cos(t), radius * np.sin(t)], axis=1)


def disk_far_field_error(ppw):
    """Relative error of the Lippmann-Schwinger far field of the discrete total field of a
    dielectric disk (index 1.2 in air, radius 0.75 wavelength, 3.2-wavelength square, layer
    1.5 wavelengths) at 48 sensors on a circle, against the analytic cylinder series."""
    n, w = int(3.2 * ppw), int(1.5 * ppw)
    k0h = 2 * np.pi / ppw
    radius = 0.75 * ppw  # cells
    prob = Problem(synth.disk_map(n, radius, 0.2, n_b=1.0), k0h=k0h, n_b=1.0, w=w, beta=0.15, levels=1)
    d = np.array([0.0, 1.0])
    u = plane_wave(prob, d) + ExactSolver(prob).solve(rhs(prob, d))
    sens = circle(48, 1.3 * n / 2)
    y = farfield(prob, sensor_matrix(prob, sens), u)
    kb = k0h / prob.h
    xs, ys = sens[:, 0] * prob.h, sens[:, 1] * prob.h
    ref = cylinder_total_field(xs, ys, radius * prob.h, kb, 1.2 * kb, np.arctan2(d[1], d[0]))
    ref -= np.exp(1j * kb * (d[0] * xs + d[1] * ys))
    return np.linalg.norm(y - ref) / np.linalg.norm(ref)


@pytest.mark.slow
def test_far_field_of_a_disk_converges_to_the_cylinder_series():
    """Physics pin: the Green's function normalisation, its sign convention and the
    quadrature weight all enter; the error is a few percent and falls at first order in h
    (the staircased disk boundary), as it must for a correct operator (measured: 8.6% at 20,
    4.4% at 40 points per wavelength)."""
    e20, e40 = disk_far_field_error(20), disk_far_field_error(40)
    assert e40 < 0.05 and e40 < 0.6 * e20, (e20, e40)


def test_interior_coordinates_are_x_fastest_and_centred():
    prob = Problem(np.ones((4, 4)), k0h=0.3, w=2, levels=1)
    z = interior_coords(prob)
    assert np.allclose(z[:2], [[-1.5, -1.5], [-0.5, -1.5]]) and np.allclose(z.mean(axis=0), 0.0)
    prob3 = Problem(np.ones((3, 3, 3)), k0h=0.3, w=2, levels=1)
    z3 = interior_coords(prob3)
    assert np.allclose(z3[1], [0.0, -1.0, -1.0]) and np.allclose(z3[3], [-1.0, 0.0, -1.0])


def test_farfield_gradient_matches_finite_differences():
    n, w = 12, 6
    k0h = 2 * np.pi / 10 / 1.333
    nmap = synth.blob_map(n, 2, (2.0, 3.0), 0.08, 8)
    sens = circle(8, 12.0)
    dirs = synth.directions_2d(2)
    y_meas = synth.complex_field((2, 8), 9) * 1e-3
    prob = Problem(nmap, k0h=k0h, w=w, levels=1)
    loss, grad = farfield_loss_and_gradient(prob, sens, dirs, y_meas)
    k02 = prob.k0 ** 2
    f = k02 * (nmap ** 2 - prob.n_b ** 2)
    rng = np.random.default_rng(3)
    for flat in rng.choice(n * n, 5, replace=False):
        iy, ix = divmod(int(flat), n)
        df = 1e-4 * max(1.0, abs(f[iy, ix]))
        vals = []
        for sgn in (1, -1):
            fp = f.copy()
            fp[iy, ix] += sgn * df
            pp = Problem(np.sqrt(prob.n_b ** 2 + fp / k02), k0h=k0h, w=w, levels=1)
            vals.append(farfield_loss_and_gradient(pp, sens, dirs, y_meas)[0])
        fd = (vals[0] - vals[1]) / (2 * df)
        assert fd == pytest.approx(grad[iy, ix], rel=1e-5, abs=1e-9 * abs(loss) / df)
