"""Pins of the oracle's discretisation (Sec. IV-A) against closed forms and brute force."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import lfa
from oracle.discretization import (Problem, extended_size, helmholtz_matrix, helmholtz_matrix_rowwise,
                                   laplacian)

KBH = 2 * np.pi / 10  # 10 points per background wavelength


def small_problem(n=12, w=4, levels=2, beta=0.15, sign=+1, seed=5, d=2):
    nmap = synth.blob_map(n, 3, (1.5, 3.0), 0.2, seed, d=d)
    return Problem(nmap, k0h=KBH / 1.333, w=w, levels=levels, beta=beta, abl_sign=sign)


def test_extended_size_rule():
    # smallest odd n_e >= n + 2w with (n_e - 1) divisible by 2^(L-1) (reading A5)
    assert extended_size(128, 20, 4) == 169
    assert extended_size(512, 20, 5) == 561
    assert extended_size(256, 20, 4) == 297
    assert extended_size(128, 20, 5) == 177
    for n, w, L in [(30, 3, 3), (100, 7, 4), (64, 20, 6)]:
        ne = extended_size(n, w, L)
        assert ne % 2 == 1 and (ne - 1) % 2 ** (L - 1) == 0 and ne >= n + 2 * w
        assert not any(((m - 1) % 2 ** (L - 1) == 0 and m % 2 == 1) for m in range(n + 2 * w, ne))


def test_rowwise_assembly_matches_matrix():
    # brute-force row-by-row assembly of eq. (discretizedHelm) with the ghost rules
    prob = small_problem()
    a = helmholtz_matrix(prob).toarray()
    b = helmholtz_matrix_rowwise(prob).toarray()
    assert np.abs(a - b).max() < 1e-14  # equal up to the order of the diagonal sums


def test_unscaled_is_scaled_over_h2():
    prob = small_problem()
    a = helmholtz_matrix(prob, scaled=False)
    a2 = helmholtz_matrix(prob, scaled=True)
    assert abs(a - a2 / prob.h ** 2).max() < 1e-9 * abs(a).max()
    # off-diagonals are -1/h^2 (the 1/h^2 Laplacian of eq. discretizedHelm)
    off = a.toarray()[0, 1]
    assert off == pytest.approx(-1.0 / prob.h ** 2)


def test_symmetric_not_hermitian():
    # the Sommerfeld terms only touch the diagonal: A = A^T, but A != A^H
    prob = small_problem()
    a = helmholtz_matrix(prob)
    assert abs(a - a.T).max() == 0.0
    assert abs(a - a.conj().T).max() > 1e-3


@pytest.mark.parametrize("theta", [(0.3, -1.1), (2.0, 0.7), (-2.9, 3.0)])
def test_lfa_symbol_on_interior_rows(theta):
    # a^h(theta) of Sec. IV-B: constant k, interior rows see a Fourier mode as an eigenvector
    nmap = np.full((16, 16), 1.333)
    prob = Problem(nmap, k0h=KBH / 1.333, w=4, levels=1, beta=0.0)
    a = helmholtz_matrix(prob, scaled=False)
    ne = prob.n_e
    yy, xx = np.meshgrid(np.arange(ne), np.arange(ne), indexing="ij")
    v = np.exp(1j * (theta[0] * xx + theta[1] * yy))
    av = (a @ v.ravel()).reshape(v.shape)
    sym = lfa.symbol_a(theta[0], theta[1], KBH, prob.h)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(av[inner], sym * v[inner], rtol=1e-12, atol=1e-9 * abs(sym))


def test_jacobi_symbol_and_divergence():
    # s^h(theta) and max|s| = 1 - w + 4w/(4 - k^2h^2) > 1 (Sec. IV-B), checked on a periodic grid
    omega = 0.8
    n = 16
    kh = KBH
    t = laplacian(n, 1, 1.0).toarray()
    t[0, -1] = t[-1, 0] = -1.0  # periodic wrap
    t[0, 0] = t[-1, -1] = 2.0
    eye = np.eye(n)
    a = np.kron(t, eye) + np.kron(eye, t) - kh * kh * np.eye(n * n)
    s = np.eye(n * n) - omega * a / np.diag(a)[:, None]
    eig = np.linalg.eigvals(s)
    assert np.max(np.abs(eig)) == pytest.approx(lfa.jacobi_max_amplification(kh, omega), rel=1e-10)
    assert lfa.jacobi_max_amplification(kh, omega) == pytest.approx(1.0876, abs=1e-4)
    th = 2 * np.pi * np.arange(n) / n
    predicted = np.sort_complex(np.array([lfa.symbol_jacobi(a1, a2, kh, omega) for a1 in th for a2 in th]))
    assert np.allclose(np.sort_complex(eig.astype(complex)), predicted, atol=1e-10)


def test_cgc_ratio_negative_without_shift():
    # Sec. IV-B: a^h(theta)/a^{2h}(2 theta) is negative for some smooth modes at 10 ppw
    th = np.linspace(-np.pi / 2, np.pi / 2, 81)
    t1, t2 = np.meshgrid(th, th)
    ratio = lfa.cgc_ratio(t1, t2, KBH)
    assert np.any(np.real(ratio) < 0)


def test_discrete_plane_wave_annihilated():
    # homogeneous medium, no layer: exp(j(kx m + ky n)) solves the interior rows iff
    # 4 - 2 cos kx - 2 cos ky = c exactly
    nmap = np.full((20, 20), 1.0)
    th = 0.4
    kx, ky = KBH * np.sin(th), KBH * np.cos(th)
    c = 4 - 2 * np.cos(kx) - 2 * np.cos(ky)
    prob = Problem(nmap, k0h=np.sqrt(c), n_b=1.0, w=4, levels=1, beta=0.0)
    a = helmholtz_matrix(prob)
    ne = prob.n_e
    yy, xx = np.meshgrid(np.arange(ne), np.arange(ne), indexing="ij")
    u = np.exp(1j * (kx * xx + ky * yy))
    r = (a @ u.ravel()).reshape(u.shape)
    assert np.abs(r[1:-1, 1:-1]).max() < 1e-12
    # with the continuous wavenumber the interior residual is O((kh)^4): second-order consistency
    prob2 = Problem(nmap, k0h=KBH, n_b=1.0, w=4, levels=1, beta=0.0)
    u2 = np.exp(1j * KBH * (np.sin(th) * xx + np.cos(th) * yy))
    r2 = (helmholtz_matrix(prob2) @ u2.ravel()).reshape(u2.shape)
    assert np.abs(r2[1:-1, 1:-1]).max() < 0.2 * KBH ** 4


def test_layer_energy_identity_and_sign():
    # Im(u^H A' u) = -sum (k0h)^2 n^2 Im(alpha)|u|^2 - sum_ghosts k_b h |u_b|^2 (reading A3)
    for sign in (+1, -1):
        prob = small_problem(beta=3.0, sign=sign)
        a = helmholtz_matrix(prob)
        u = synth.complex_field(prob.shape, 9).ravel()
        lhs = np.vdot(u, a @ u).imag
        c = prob.coefficient().ravel()
        ne = prob.n_e
        yy, xx = np.meshgrid(np.arange(ne), np.arange(ne), indexing="ij")
        nghost = ((xx == 0).astype(int) + (xx == ne - 1) + (yy == 0) + (yy == ne - 1)).ravel()
        rhs = -np.sum(c.imag * np.abs(u) ** 2) - prob.kbh * np.sum(nghost * np.abs(u) ** 2)
        assert lhs == pytest.approx(rhs, rel=1e-12)
        layer_term = -np.sum(c.imag * np.abs(u) ** 2)
        assert (layer_term < 0) == (sign > 0)


def test_second_order_manufactured_solution():
    # u = gaussian bump * exp(j k x) supported well inside Omega; error ratio -> 4 as h halves
    k = 40.0
    s, cx, cy = 0.08, 0.5, 0.47
    errs = []
    for n_int in (25, 57, 121):
        w = 4
        prob = Problem(np.full((n_int, n_int), 1.0), k0h=0.0, n_b=1.0, w=w, levels=1, beta=0.0)
        prob.k0h = k * prob.h
        h = prob.h
        ax = np.arange(prob.n_e) * h
        yy, xx = np.meshgrid(ax, ax, indexing="ij")
        r2 = (xx - cx) ** 2 + (yy - cy) ** 2
        g = np.exp(-r2 / (2 * s * s))
        phase = np.exp(1j * k * xx)
        u = g * phase
        lap_g = g * (r2 / s ** 4 - 2 / s ** 2)
        gx = -(xx - cx) / s ** 2 * g
        f = -phase * (lap_g + 2j * k * gx)          # -Lap u - k^2 u
        a = helmholtz_matrix(prob, scaled=False)
        uh = spla.spsolve(a.tocsc(), f.ravel()).reshape(u.shape)
        step = (prob.n_e - 1) // 32
        errs.append(np.abs(uh - u)[::step, ::step].max())
    r1, r2_ = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r2_ < 4.7, errs
    assert r1 > 3.0, errs


# ---- the absorbing-layer profile (Sec. IV-A, readings A3/A4), pinned by values worked out by hand ----
#
# Grid used below: n = 12 interior points, w = 4 layer cells, 2 levels, so n_e = 21 (the smallest odd
# n_e >= 20 with n_e - 1 even), Omega = indices [4, 16) per axis, high-side layer indices 16..20
# (5 cells), and the unit-square normalisation gives 1/(n_e - 1) = 1/20.  With d the distance in cells
# from a point to its projection on Omega:
#   profile 0: gamma = beta (d/20)^2 / (4/20) = beta d^2 / 80
#   profile 1: gamma = beta (d/4)^2 = beta d^2 / 16
# beta = 0.15.  Points are (y, x) index pairs; (y, x) = (8, 0) sits 4 cells left of Omega (d^2 = 16),
# (8, 20) 5 cells right of it (d^2 = 25), (0, 0) is a layer corner (d^2 = 4^2 + 4^2 = 32), (20, 20)
# the far corner (d^2 = 5^2 + 5^2 = 50), (15, 4) lies on the edge of Omega (d = 0).
ALPHA_PINS_FINE = {
    0: {(8, 0): 0.15 * 16 / 80, (8, 20): 0.15 * 25 / 80, (0, 0): 0.15 * 32 / 80, (20, 20): 0.15 * 50 / 80,
        (15, 4): 0.0, (2, 9): 0.15 * 4 / 80},
    1: {(8, 0): 0.15 * 16 / 16, (8, 20): 0.15 * 25 / 16, (0, 0): 0.15 * 32 / 16, (20, 20): 0.15 * 50 / 16,
        (15, 4): 0.0, (2, 9): 0.15 * 4 / 16},
}
# Level 1 (stride 2, 11 points per axis): coarse (y, x) sits at fine (2y, 2x); coarse (4, 1) is fine
# (8, 2) (d^2 = 4), coarse (10, 10) is fine (20, 20) (d^2 = 50), coarse (0, 5) is fine (0, 10) (d^2 = 16).
ALPHA_PINS_COARSE = {
    0: {(4, 1): 0.15 * 4 / 80, (10, 10): 0.15 * 50 / 80, (0, 5): 0.15 * 16 / 80},
    1: {(4, 1): 0.15 * 4 / 16, (10, 10): 0.15 * 50 / 16, (0, 5): 0.15 * 16 / 16},
}


def _alpha_pin_failures(make_problem):
    """Every (profile, sign, point) where alpha_at disagrees with the hand-worked value."""
    bad = []
    for profile in (0, 1):
        for sign in (+1, -1):
            prob = make_problem(profile, sign)
            assert prob.n_e == 21
            for pins, stride in ((ALPHA_PINS_FINE, 1), (ALPHA_PINS_COARSE, 2)):
                for (y, x), gamma in pins[profile].items():
                    got = complex(prob.alpha_at([np.array(y), np.array(x)], stride=stride))
                    if abs(got - (1.0 + 1j * sign * gamma)) > 1e-14:
                        bad.append((profile, sign, stride, (y, x), got, gamma))
    return bad


def _pin_problem(profile, sign, cls=Problem):
    return cls(np.full((12, 12), 1.4), k0h=KBH / 1.333, w=4, levels=2, beta=0.15, abl_sign=sign,
               abl_profile=profile)


def test_layer_profile_matches_hand_worked_values():
    assert _alpha_pin_failures(_pin_problem) == []


def _planted(mistake):
    """A Problem whose layer profile carries one planted mistake (for the test below only)."""

    class Planted(Problem):
        def alpha_at(self, idx_axes, stride=1):
            lo, hi = self.w, self.w + self.n - 1
            if mistake == "high side as wide as the low side":
                hi = self.n_e - 1 - self.w
            step = 1 if mistake == "coarse indices not scaled" else stride
            d2 = 0.0
            for ia in idx_axes:
                x = np.asarray(ia, dtype=np.float64) * step
                d2 = d2 + np.maximum(0.0, np.maximum(lo - x, x - hi)) ** 2
            unit = 1.0 / (self.n_e - 1)
            if mistake == "distance not squared":
                d2 = np.sqrt(d2)
            if mistake == "layer length in cells":
                g = self.beta * d2 * unit * unit / self.w
            elif self.abl_profile == 1:
                g = self.beta * d2 / self.w ** 2
            else:
                g = self.beta * d2 * unit / self.w
            sign = -self.abl_sign if mistake == "sign" else self.abl_sign
            return 1.0 + 1j * sign * g

    return Planted


PLANTED = ("distance not squared", "layer length in cells", "coarse indices not scaled", "sign",
           "high side as wide as the low side")


def test_layer_profile_pins_catch_plausible_mistakes():
    # the same pins fail for each planted mistake, and pass for the planted class without one
    assert _alpha_pin_failures(lambda p, s: _pin_problem(p, s, _planted("none"))) == []
    for mistake in PLANTED:
        assert _alpha_pin_failures(lambda p, s: _pin_problem(p, s, _planted(mistake))), mistake


def test_coefficient_in_the_layer_is_background_times_alpha():
    # c = (k0 h)^2 n_b^2 (1 + j gamma) in the layer, (k0 h)^2 n^2 on Omega (Sec. IV-A)
    for profile in (0, 1):
        prob = _pin_problem(profile, +1)
        c = prob.coefficient()
        k0h2 = (KBH / 1.333) ** 2
        for (y, x), gamma in ALPHA_PINS_FINE[profile].items():
            inside = 4 <= y < 16 and 4 <= x < 16
            nn = 1.4 if inside else 1.333
            assert c[y, x] == pytest.approx(k0h2 * nn * nn * (1 + 1j * gamma), rel=1e-14, abs=1e-16)


def test_cgc_ratio_positive_with_the_shift():
    # Sec. IV-B: with kappa = 1 the ratio a^h(theta) / a^2h(2 theta) changes sign for smooth modes near
    # the wavenumber (above); with the dissipative shift kappa = 1 + 0.5j both symbols share the
    # imaginary part -0.5 (kh)^2 and the real part of the ratio stays positive everywhere
    th = np.linspace(-np.pi / 2, np.pi / 2, 161)
    t1, t2 = np.meshgrid(th, th)
    ratio = lfa.cgc_ratio(t1, t2, KBH, kappa=1 + 0.5j)
    assert np.all(np.real(ratio) > 0)
    # the printed operator (kappa = 1) seen through the same function keeps its negative ratios
    assert np.any(np.real(lfa.cgc_ratio(t1, t2, KBH, kappa=1.0)) < 0)
    # closed form at the mode theta = (kh, 0), where the fine symbol of A vanishes to leading order:
    # a^h = 2 - 2 cos(kh) - kappa (kh)^2, a^2h = (2 - 2 cos(2 kh) - 4 kappa (kh)^2) / 4
    kh = KBH
    for kappa in (1.0, 1 + 0.5j):
        a1 = 2 - 2 * np.cos(kh) - kappa * kh * kh
        a2 = (2 - 2 * np.cos(2 * kh) - 4 * kappa * kh * kh) / 4
        assert lfa.cgc_ratio(kh, 0.0, KBH, kappa=kappa) == pytest.approx(a1 / a2, rel=1e-12)
