"""Pins of the oracle's inverse-problem steps (Sec. V: eq. proximalOpt, Alg. 4)."""
import numpy as np
import pytest

from oracle.inverse import fbs_update, forward_diff, forward_diff_adjoint, tv_prox, tv_value


def test_difference_operator_and_its_adjoint():
    rng = np.random.default_rng(0)
    for shape in [(5, 7), (3, 4, 6)]:
        w = rng.standard_normal(shape)
        p = rng.standard_normal((len(shape), *shape))
        assert np.vdot(forward_diff(w), p) == pytest.approx(np.vdot(w, forward_diff_adjoint(p)), rel=1e-12)
    # a vertical edge of height 2 over 6 rows: TV = 2 * 6 (only the column before the edge differs)
    w = np.zeros((6, 9))
    w[:, 4:] = 2.0
    assert tv_value(w) == pytest.approx(12.0)
    assert tv_value(np.full((4, 4, 4), 3.0)) == 0.0


def test_prox_special_cases():
    rng = np.random.default_rng(1)
    v = rng.standard_normal((8, 8))
    assert np.array_equal(tv_prox(v, 0.0, lo=0.0), np.maximum(v, 0.0))
    c = np.full((6, 6), 1.5)
    assert np.allclose(tv_prox(c, 0.7, lo=0.0), c)
    # TV dominates: the minimiser tends to the constant closest to v, its mean
    v = 2.0 + 0.3 * rng.standard_normal((6, 6))
    w = tv_prox(v, 50.0, lo=0.0, iters=3000)
    assert np.allclose(w, v.mean(), atol=2e-3)


def test_prox_of_a_step_has_the_closed_form():
    # each row is an independent 1D TV denoising of a step: with m1 points at a and m2 at b > a,
    # the levels move toward each other by lam / m1 and lam / m2 (while the jump stays positive)
    a, b, m1, m2, lam = 1.0, 3.0, 5, 7, 1.2
    v = np.tile(np.r_[np.full(m1, a), np.full(m2, b)], (4, 1))
    w = tv_prox(v, lam, lo=0.0, iters=4000)
    ref = np.tile(np.r_[np.full(m1, a + lam / m1), np.full(m2, b - lam / m2)], (4, 1))
    assert np.allclose(w, ref, atol=1e-5)
    # the nonnegativity constraint is active where the unconstrained answer would be negative
    w0 = tv_prox(v - 2.0, lam, lo=0.0, iters=4000)
    assert np.all(w0 >= 0.0) and np.allclose(w0[:, :m1], 0.0, atol=1e-6)


def test_prox_duality_gap_closes():
    """Weak duality certifies the answer without retyping the algorithm: for every dual field
    p with ||p_i|| <= 1, h(p) = min_{w >= lo} 1/2||w - v||^2 + lam <p, D w> <= the primal value;
    the primal value of the prox output minus the best dual bound found must vanish."""
    rng = np.random.default_rng(2)
    v = np.abs(rng.standard_normal((10, 12))) + np.where(rng.random((10, 12)) < 0.3, 2.0, 0.0) - 0.5
    lam, lo = 0.4, 0.0
    w = tv_prox(v, lam, lo=lo, iters=3000)
    primal = 0.5 * np.sum((w - v) ** 2) + lam * tv_value(w)

    def dual(p):
        wp = np.maximum(v - lam * forward_diff_adjoint(p), lo)
        return 0.5 * np.sum((wp - v) ** 2) + lam * np.vdot(forward_diff(wp), p)

    # a dual field aligned with the primal's gradient field is (near) optimal
    g = forward_diff(w)
    p = g / np.maximum(1e-12, np.sqrt(np.sum(g ** 2, axis=0)))
    # where the gradient vanishes the dual is free: fill it by projected ascent from zero
    for _ in range(2000):
        q = p + forward_diff(np.maximum(v - lam * forward_diff_adjoint(p), lo)) / (8 * lam)
        p = q / np.maximum(1.0, np.sqrt(np.sum(q ** 2, axis=0)))
    assert dual(p) <= primal + 1e-9
    assert primal - dual(p) < 1e-6 * primal


def test_fbs_on_a_linear_model_decreases_the_objective_to_its_minimum():
    rng = np.random.default_rng(3)
    n = 8
    a = rng.standard_normal((40, n * n)) / 6.0
    f_true = np.zeros((n, n))
    f_true[2:6, 3:7] = 1.0
    y = a @ f_true.ravel()
    tau = 0.05
    lip = np.linalg.norm(a, 2) ** 2
    gamma = 1.0 / lip

    def obj(f):
        return 0.5 * np.sum((a @ f.ravel() - y) ** 2) + tau * tv_value(f)

    def run(iters, accelerated):
        f = np.zeros((n, n))
        fbar, alpha = f.copy(), 1.0
        vals = []
        for _ in range(iters):
            grad = (a.T @ (a @ fbar.ravel() - y)).reshape(n, n)
            f_new, fbar_new, alpha = fbs_update(f, fbar, grad, gamma, tau, alpha, prox_iters=200)
            fbar = fbar_new if accelerated else f_new
            f = f_new
            vals.append(obj(f))
        return f, np.array(vals)

    # reference minimum: the plain (non-accelerated) iteration run ten times longer
    _, ref = run(2000, accelerated=False)
    f, vals = run(200, accelerated=True)
    assert np.all(f >= 0.0)
    assert vals[-1] <= ref[-1] * (1 + 1e-4)
    _, slow = run(200, accelerated=False)
    assert vals[-1] < slow[-1]  # the acceleration of Alg. 4 pays off at equal iteration count
    assert np.linalg.norm(f - f_true) < 0.5 * np.linalg.norm(f_true)
