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
