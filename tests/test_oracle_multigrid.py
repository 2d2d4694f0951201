"""Pins of the oracle's multigrid (Sec. III Alg. 1-2, Sec. IV-C transfer operators)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.discretization import Problem
from oracle.multigrid import Hierarchy, prolongation, restriction

KBH = 2 * np.pi / 10


def prob2d(n=9, w=4, levels=3, kappa=1 + 0.5j, seed=3, nu=1):
    nmap = synth.blob_map(n, 2, (1.0, 2.0), 0.2, seed)
    return Problem(nmap, k0h=KBH / 1.333, w=w, levels=levels, kappa=kappa, nu1=nu, nu2=nu)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_prolongation_is_2d_restriction_transpose(d):
    # the printed P weights equal 2^d R^T (reading A7)
    n_f = 9
    r = restriction(n_f, d).toarray()
    p = prolongation((n_f - 1) // 2 + 1, d).toarray()
    assert np.abs(p - (2 ** d) * r.T).max() < 1e-15


def test_restriction_printed_weights():
    # r^{2h}_{m,n} = (4 r_c + 2 (edges) + corners) / 16 at an interior coarse point
    n_f = 9
    r = restriction(n_f, 2)
    fine = np.zeros((n_f, n_f))
    fine[3:6, 1:4] = np.arange(9).reshape(3, 3) + 1.0  # around fine (4, 2) = coarse (2, 1)
    out = (r @ fine.ravel()).reshape(5, 5)
    blk = fine[3:6, 1:4]
    expected = (4 * blk[1, 1] + 2 * (blk[0, 1] + blk[2, 1] + blk[1, 0] + blk[1, 2])
                + blk[0, 0] + blk[0, 2] + blk[2, 0] + blk[2, 2]) / 16
    assert out[2, 1] == pytest.approx(expected)
    # boundary coarse point: neighbours outside the grid count as zero (reading A6)
    ones = np.ones(n_f * n_f)
    rc = (r @ ones).reshape(5, 5)
    assert rc[2, 2] == pytest.approx(1.0)
    assert rc[0, 2] == pytest.approx(12 / 16)
    assert rc[0, 0] == pytest.approx(9 / 16)


def test_prolongation_reproduces_linear_functions():
    n_c = 5
    p = prolongation(n_c, 2)
    yc, xc = np.meshgrid(np.arange(n_c) * 2.0, np.arange(n_c) * 2.0, indexing="ij")
    yf, xf = np.meshgrid(np.arange(9) * 1.0, np.arange(9) * 1.0, indexing="ij")
    lin_c = 3 * xc - 2 * yc + 1
    out = (p @ lin_c.ravel()).reshape(9, 9)
    assert np.allclose(out, 3 * xf - 2 * yf + 1)


def test_coarse_coefficient_rule():
    # c_{l+1} = 4 FW(c_l) at interior coarse points; background k_b^2 h_l^2 alpha on the ring (reading A8)
    prob = prob2d(levels=3)
    hier = Hierarchy(prob)
    c0, c1 = hier.coef[0], hier.coef[1]
    n1 = c1.shape[0]
    i, j = 3, 2
    blk = c0[2 * i - 1:2 * i + 2, 2 * j - 1:2 * j + 2]
    wts = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    assert c1[i, j] == pytest.approx(4.0 * np.sum(wts * blk))
    # ring values by hand: n = 9, w = 4, 3 levels give n_e = 17, Omega = [4, 13) and the unit-square
    # factor 1/16, so gamma = beta d^2 / (w 16) = 0.15 d^2 / 64.  Coarse (0, 4) is fine (0, 8): d = 4;
    # coarse (8, 0) is fine (16, 0): d^2 = 4^2 + 4^2.  Level-1 background (k_b 2h)^2
    assert prob.n_e == 17 and n1 == 9
    cb1 = (KBH * 2) ** 2
    assert c1[0, 4] == pytest.approx(cb1 * (1 + 1j * 0.15 * 16 / 64), rel=1e-13)
    assert c1[n1 - 1, 0] == pytest.approx(cb1 * (1 + 1j * 0.15 * 32 / 64), rel=1e-13)
    c2 = hier.coef[2]  # level 2: coarse (2, 0) is fine (8, 0), d = 4; (0, 0) is fine (0, 0), d^2 = 32
    assert c2[2, 0] == pytest.approx((KBH * 4) ** 2 * (1 + 1j * 0.15 * 16 / 64), rel=1e-13)
    assert c2[0, 0] == pytest.approx((KBH * 4) ** 2 * (1 + 1j * 0.15 * 32 / 64), rel=1e-13)


def test_scaled_cycle_equals_unscaled_two_grid_matrix():
    # eq. (itererror): e_new = S^nu2 C S^nu1 e with S = I - w D^-1 A^h and
    # C = I - P (A^{2h})^-1 R A^h, written with the UNSCALED level matrices
    for nu in (1, 2):
        prob = prob2d(n=9, w=4, levels=2, nu=nu)
        hier = Hierarchy(prob)
        h = prob.h
        k0 = hier.K[0].toarray() / h ** 2
        k1 = hier.K[1].toarray() / (2 * h) ** 2
        r = hier.R[0].toarray()
        p = hier.P[0].toarray()
        n = k0.shape[0]
        s = np.eye(n) - prob.omega_jac * k0 / np.diag(k0)[:, None]
        c = np.eye(n) - p @ np.linalg.solve(k1, r @ k0)
        e_mat = np.linalg.matrix_power(s, nu) @ c @ np.linalg.matrix_power(s, nu)
        u_star = synth.complex_field(n, 1)
        v0 = synth.complex_field(n, 2)
        b = hier.K[0] @ u_star  # scaled right-hand side of the scaled system
        v1 = hier.cycle(b, v0.copy())
        assert np.allclose(u_star - v1, e_mat @ (u_star - v0), atol=1e-10)
        v2 = hier.two_grid(b, v0.copy())
        assert np.allclose(v1, v2, atol=1e-12)


def test_one_level_cycle_is_exact_solve_and_cycle_linear():
    prob = prob2d(levels=3)
    hier1 = Hierarchy(prob, levels=1)
    b = synth.complex_field(prob.size, 4)
    x = hier1.vcycle(b)
    assert np.abs(hier1.K[0] @ x - b).max() < 1e-10
    hier = Hierarchy(prob)
    b2 = synth.complex_field(prob.size, 5)
    assert np.abs(hier.vcycle(np.zeros_like(b))).max() == 0.0
    lin = hier.vcycle(2.0 * b - 1j * b2) - (2.0 * hier.vcycle(b) - 1j * hier.vcycle(b2))
    assert np.abs(lin).max() < 1e-12 * np.abs(hier.vcycle(b)).max()


def test_w_cycle_recursion_counts():
    # Alg. 2 with CycleType = 2 calls the coarsest solve 2^(L-1) times; the two calls made
    # from one visit of the next-to-coarsest level solve the same system exactly, so Fig. 3
    # draws 2^(L-2) coarsest nodes for a W-cycle
    prob = prob2d(levels=4)
    hier = Hierarchy(prob)
    calls = []
    lu = hier.coarse_lu

    class Counting:
        def solve(self, b):
            calls.append(1)
            return lu.solve(b)

    hier.coarse_lu = Counting()
    hier.cycle(synth.complex_field(prob.size, 7), None, 0, 2)
    assert len(calls) == 8
    calls.clear()
    hier.cycle(synth.complex_field(prob.size, 7), None, 0, 1)
    assert len(calls) == 1


def test_shifted_vcycle_is_a_contraction_for_the_shifted_operator():
    # with kappa = 1 + 0.5j the V-cycle used as a stationary iteration on K_kappa converges
    prob = prob2d(n=40, w=8, levels=4)
    hier = Hierarchy(prob)
    u_star = synth.complex_field(prob.size, 8)
    b = hier.K[0] @ u_star
    v = np.zeros_like(b)
    errs = []
    for _ in range(6):
        v = hier.cycle(b, v)
        errs.append(np.linalg.norm(u_star - v))
    assert errs[-1] < 0.5 * errs[0]
    assert errs[-1] < 0.2 * np.linalg.norm(u_star)


def test_coarsest_lu_residual():
    prob = prob2d(levels=3)
    hier = Hierarchy(prob)
    b = synth.complex_field(hier.K[-1].shape[0], 6)
    x = hier.coarse_lu.solve(b)
    assert np.linalg.norm(hier.K[-1] @ x - b) < 1e-13 * np.linalg.norm(b)
    x2 = spla.spsolve(hier.K[-1].tocsc(), b)
    assert np.allclose(x, x2, atol=1e-12)


def test_cycle_from_a_guess_is_guess_plus_zero_guess_cycle():
    # every step of Alg. 2 is affine and consistent: MG(b, v0) = v0 + MG(b - K v0, 0)
    prob = prob2d(n=12, w=4, levels=3)
    hier = Hierarchy(prob)
    b = synth.complex_field(prob.size, 12)
    v0 = synth.complex_field(prob.size, 13)
    for ct in (1, 2, [2, 1, 1]):
        lhs = hier.cycle(b, v0.copy(), 0, ct)
        rhs = v0 + hier.cycle(b - hier.K[0] @ v0, None, 0, ct)
        assert np.allclose(lhs, rhs, atol=1e-12 * np.abs(lhs).max())


def test_per_level_cycle_type_sits_between_v_and_w():
    prob = prob2d(n=12, w=4, levels=4)
    hier = Hierarchy(prob)
    calls = []
    lu = hier.coarse_lu

    class Counting:
        def solve(self, b):
            calls.append(1)
            return lu.solve(b)

    hier.coarse_lu = Counting()
    hier.cycle(synth.complex_field(prob.size, 7), None, 0, [2, 1, 1])
    assert len(calls) == 2
