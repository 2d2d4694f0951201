"""Pins of the oracle's Krylov solvers (FGMRES, Alg. 3 Bi-CGSTAB) and model (Sec. V, Prop. 1)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import model
from oracle.discretization import Problem, helmholtz_matrix
from oracle.krylov import bicgstab, fgmres, givens, sstep_gmres
from oracle.multigrid import Hierarchy

KBH = 2 * np.pi / 10


def problem(n=24, w=6, levels=3, seed=2, beta=0.15):
    nmap = synth.blob_map(n, 3, (2.0, 4.0), 0.1, seed)
    return Problem(nmap, k0h=KBH / 1.333, w=w, levels=levels, beta=beta)


def test_givens_zeroes_second_entry():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a, b = rng.standard_normal(2) @ [1, 1j], abs(rng.standard_normal())
        c, s = givens(a, b)
        assert abs(-np.conj(s) * a + c * b) < 1e-14
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-14


def test_fgmres_residuals_match_brute_force_krylov_minimisation():
    # unrestarted right-preconditioned GMRES: the k-th residual is min ||r0 - A M K_k c||
    # over the Krylov space span{r0, (AM) r0, ...}; built here by brute force (dense lstsq)
    prob = problem(n=10, w=4, levels=2)
    hier = Hierarchy(prob)
    a = helmholtz_matrix(prob).toarray()
    n = a.shape[0]
    mmat = np.column_stack([hier.vcycle(e) for e in np.eye(n)])
    b = synth.complex_field(n, 3)
    _, info = fgmres(lambda v: a @ v, hier.vcycle, b, rtol=1e-13, restart=400, max_iters=12)
    am = a @ mmat
    kry = [b]
    for _ in range(11):
        kry.append(am @ kry[-1])
    bn = np.linalg.norm(b)
    for k in range(1, 13):
        basis = np.column_stack(kry[:k])
        q, _ = np.linalg.qr(basis)
        coef, *_ = np.linalg.lstsq(am @ q, b, rcond=None)
        res = np.linalg.norm(b - am @ q @ coef) / bn
        assert info.history[k - 1] == pytest.approx(res, rel=1e-6, abs=1e-12)


def test_mg_fgmres_reaches_lu_solution():
    prob = problem()
    ex = model.ExactSolver(prob)
    b = model.rhs(prob, [0.3, np.sqrt(1 - 0.09)])
    u = ex.solve(b)
    assert np.linalg.norm(ex.A @ u.ravel() - b.ravel()) < 1e-13 * np.linalg.norm(b)
    for restart in (5, 20):
        x, info = model.mg_fgmres_solve(prob, b, rtol=1e-12, restart=restart)
        assert info.converged and info.rel_res_true <= 1e-12
        assert np.linalg.norm(x - u) < 1e-10 * np.linalg.norm(u)
    # the final Givens estimate agrees with the true residual to FP64 round-off
    assert info.history[-1] == pytest.approx(info.rel_res_true, rel=1e-2, abs=1e-14)


def test_fgmres_matches_library_gmres_solution():
    prob = problem(n=16, w=4)
    hier = Hierarchy(prob)
    a = helmholtz_matrix(prob)
    b = synth.complex_field(prob.size, 11)
    x, info = fgmres(lambda v: a @ v, hier.vcycle, b, rtol=1e-11, restart=30)
    m = spla.LinearOperator(a.shape, matvec=hier.vcycle, dtype=np.complex128)
    x_lib, flag = spla.gmres(a, b, M=m, rtol=1e-12, restart=60, maxiter=50)
    assert flag == 0
    assert np.linalg.norm(x - x_lib) < 1e-9 * np.linalg.norm(x_lib)


def test_sstep_gmres_iterates_equal_fgmres():
    """The s-step form minimises over the same Krylov space as FGMRES(m) with a fixed
    preconditioner: in FP64 the residual estimate after each basis size of each cycle
    and the iterate after each cycle agree with FGMRES(m) (brute force pins FGMRES)."""
    prob = problem(n=16, w=4)
    hier = Hierarchy(prob)
    a = helmholtz_matrix(prob)
    b = synth.complex_field(prob.size, 13)
    for m in (1, 3, 5):
        x_f, info_f = fgmres(lambda v: a @ v, hier.vcycle, b, rtol=1e-10, restart=m, max_iters=m * 6)
        x_s, info_s = sstep_gmres(lambda v: a @ v, hier.vcycle, b, rtol=1e-10, restart=m, max_iters=m * 6)
        assert info_s.iters == info_f.iters == m * 6
        np.testing.assert_allclose(info_s.history, info_f.history, rtol=1e-6, atol=1e-13)
        assert np.linalg.norm(x_s - x_f) < 1e-8 * np.linalg.norm(x_f)


def test_sstep_gmres_reaches_lu_solution_in_whole_cycles():
    prob = problem()
    ex = model.ExactSolver(prob)
    hier = Hierarchy(prob)
    b = prob.h ** 2 * model.rhs(prob, [0.0, 1.0]).ravel()
    a = helmholtz_matrix(prob, scaled=True)
    x, info = sstep_gmres(lambda v: a @ v, hier.vcycle, b, rtol=1e-9, restart=4)
    assert info.converged and info.rel_res_true <= 1e-9 and info.iters % 4 == 0
    u = ex.solve(model.rhs(prob, [0.0, 1.0]))
    assert np.linalg.norm(x - u.ravel()) < 1e-7 * np.linalg.norm(u)
    # whole cycles: the count is m times the cycles FGMRES(m) needs
    _, info_f = fgmres(lambda v: a @ v, hier.vcycle, b, rtol=1e-9, restart=4)
    assert info.iters == 4 * -(-info_f.iters // 4)


def test_bicgstab_alg3_converges_to_lu_solution():
    prob = problem()
    ex = model.ExactSolver(prob)
    b = model.rhs(prob, [0.0, 1.0])
    hier = Hierarchy(prob)
    a = helmholtz_matrix(prob)
    bs = prob.h ** 2 * b.ravel()
    x, info = bicgstab(lambda v: a @ v, hier.vcycle, bs, rtol=1e-10)
    assert info.rel_res_true < 2e-10
    assert np.linalg.norm(x.reshape(b.shape) - ex.solve(b)) < 1e-8 * np.linalg.norm(ex.solve(b))


def test_zero_contrast_gives_zero_scattered_field():
    prob = Problem(np.full((20, 20), 1.333), k0h=KBH / 1.333, w=6, levels=3)
    b = model.rhs(prob, [0.0, 1.0])
    assert np.abs(b).max() == 0.0
    x, info = model.mg_fgmres_solve(prob, b)
    assert info.converged and np.abs(x).max() == 0.0


def test_plane_wave_convention():
    # u_in = exp(j k_b <d, x - x_c>): unit modulus, phase 0 at the centre of Omega, wavelength 10 cells
    prob = Problem(np.full((21, 21), 1.333), k0h=KBH / 1.333, w=4, levels=1)
    u = model.plane_wave(prob, [0.0, 1.0])
    c = prob.w + 10
    assert u[c, c] == pytest.approx(1.0)
    assert u[c + 10, c] == pytest.approx(1.0)           # one wavelength along +y (row index)
    assert u[c + 5, c] == pytest.approx(-1.0)
    assert u[c, c + 7] == pytest.approx(1.0)             # constant along x for d = (0, 1)
    assert np.allclose(np.abs(u), 1.0)


def test_adjoint_identities():
    prob = problem(n=12, w=4)
    ex = model.ExactSolver(prob)
    a = ex.A
    u = synth.complex_field(prob.size, 1)
    v = synth.complex_field(prob.size, 2)
    # <A u, v> = <u, A^H v> and u^T A v = v^T A u
    assert np.vdot(a @ u, v) == pytest.approx(np.vdot(u, a.conj().T @ v), rel=1e-13)
    assert (u @ (a @ v)) == pytest.approx(v @ (a @ u), rel=1e-13)
    g = synth.complex_field(prob.shape, 3)
    lam1 = ex.solve_adjoint(g)
    lam2 = model.adjoint_by_conjugation(ex.solve, g)
    lam3 = spla.spsolve(a.conj().T.tocsc(), g.ravel()).reshape(g.shape)
    assert np.allclose(lam1, lam3, rtol=1e-10, atol=1e-14 * np.abs(lam3).max())
    assert np.allclose(lam2, lam3, rtol=1e-10, atol=1e-14 * np.abs(lam3).max())


def test_tv_gradient_finite_differences():
    rng = np.random.default_rng(4)
    n = rng.uniform(1.3, 1.4, size=(9, 9))
    val, grad = model.tv_smoothed(n, 1e-2)
    for _ in range(10):
        i, j = rng.integers(0, 9, size=2)
        e = np.zeros_like(n)
        e[i, j] = 1e-6
        fd = (model.tv_smoothed(n + e, 1e-2)[0] - model.tv_smoothed(n - e, 1e-2)[0]) / 2e-6
        assert grad[i, j] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_gradient_matches_central_differences():
    # Prop. 1 adjoint gradient vs FP64 central differences on random pixels (reading A22)
    n_true = synth.blob_map(16, 2, (2.0, 3.0), 0.15, 21)
    n_b = 1.333
    n_eval = n_b + 0.5 * (n_true - n_b)
    dirs = synth.directions_2d(3)
    p_true = Problem(n_true, k0h=KBH / n_b, w=4, levels=1, beta=0.0)
    ex_true = model.ExactSolver(p_true)
    data = [model.sample(p_true, ex_true.solve(model.rhs(p_true, d))) for d in dirs]
    p = Problem(n_eval, k0h=KBH / n_b, w=4, levels=1, beta=0.0)
    # tau = 0.1 with a TV smoothing well above the FD step keeps both terms differentiable at delta
    kw = dict(tau=0.1, tv_eps=0.05)
    loss, grad = model.loss_and_gradient(p, dirs, data, **kw)
    assert loss == pytest.approx(model.loss_only(p, dirs, data, **kw), rel=1e-12)
    rng = np.random.default_rng(12)
    delta = 1e-4
    for _ in range(8):
        i, j = rng.integers(0, 16, size=2)
        e = np.zeros_like(n_eval)
        e[i, j] = delta
        lp = model.loss_only(Problem(n_eval + e, k0h=KBH / n_b, w=4, levels=1, beta=0.0), dirs, data, **kw)
        lm = model.loss_only(Problem(n_eval - e, k0h=KBH / n_b, w=4, levels=1, beta=0.0), dirs, data, **kw)
        fd = (lp - lm) / (2 * delta)
        assert grad[i, j] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(grad).max())


def test_shift_needed_at_ten_points_per_wavelength():
    # Sec. IV-B: the paper preconditions with kappa = 1 and saw no benefit from a shift.  At 10 points
    # per wavelength (every workload here) the unshifted preconditioner leaves MG-FGMRES stalled, and
    # so does the shift of the other sign, while the dissipative shift kappa = 1 + 0.5j converges
    # (64^2 interior, 20-cell layer, disk of contrast 0.05, normal incidence, FGMRES(20))
    from oracle.discretization import Problem
    from oracle import model

    nmap = synth.disk_map(64, 10.0, 0.05)
    its = {}
    for kappa in (1.0, 1 - 0.5j, 1 + 0.5j):
        prob = Problem(nmap, k0h=KBH / 1.333, w=20, levels=4, kappa=kappa)
        b = prob.h ** 2 * model.rhs(prob, (0.0, 1.0)).ravel()
        _, info = model.mg_fgmres_solve(prob, b, rtol=1e-6, restart=20, max_iters=300)
        its[kappa] = info
    assert its[1 + 0.5j].converged and its[1 + 0.5j].iters < 200
    for kappa in (1.0, 1 - 0.5j):
        assert not its[kappa].converged and its[kappa].rel_res_true > 1e-2, (kappa, its[kappa].rel_res_true)
