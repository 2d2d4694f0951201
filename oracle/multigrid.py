"""Multigrid preconditioner for the shifted operator K_kappa (Sec. III, Sec. IV-B/C).

* damped Jacobi, eq. (dampedJ), D = diag(K) including the ghost terms (A25)
* full-weighting restriction R as printed in Sec. IV-C; Sec. IV-C zeroes the
  values beyond the boundary, read here as fine neighbours outside Omega_e
  counting as 0 (zero padding, reading A6)
* prolongation P as printed in Sec. IV-C (the printed weights equal 2^d R^T;
  the text's "adjoint of R" is read as that printed formula, reading A7)
* coarse operators by re-discretisation with mesh size 2h; the coefficient
  k0^2 eta^2 (times alpha) is restricted by full weighting and the outermost
  ring of each coarse grid is reset to the background value (reading A8)
* the coarsest level is solved exactly (Alg. 2), here by sparse LU
* Alg. 1 (two-grid) and Alg. 2 (multigrid cycle, CycleType 1 = V, 2 = W)

All level operators are h_ell^2-scaled (K'_ell = h_ell^2 K_ell).  Because
(2h)^2 = 4 h^2, the scaled coarse right-hand side is 4 R r' (the factor that
keeps the scaled and unscaled hierarchies identical).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import Problem, laplacian


def restriction_1d_weights():
    return np.array([0.25, 0.5, 0.25])


def restriction(n_fine: int, d: int) -> sp.csr_matrix:
    """Full weighting R from the printed 9-point (2D) formula; 3D extends it axis-wise (27 points).

    Coarse point I sits on fine point 2I; weights (1/4, 1/2, 1/4) per axis,
    fine neighbours outside the grid contribute 0.
    """
    n_c = (n_fine - 1) // 2 + 1
    w1 = restriction_1d_weights()
    rows, cols, vals = [], [], []
    offsets = np.array(np.meshgrid(*([np.arange(-1, 2)] * d), indexing="ij")).reshape(d, -1).T
    coarse = np.array(np.meshgrid(*([np.arange(n_c)] * d), indexing="ij")).reshape(d, -1).T
    cflat = np.ravel_multi_index(tuple(coarse.T), (n_c,) * d)
    for off in offsets:
        fine = 2 * coarse + off
        ok = np.all((fine >= 0) & (fine < n_fine), axis=1)
        wgt = np.prod(w1[off + 1])
        rows.append(cflat[ok])
        cols.append(np.ravel_multi_index(tuple(fine[ok].T), (n_fine,) * d))
        vals.append(np.full(ok.sum(), wgt))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n_c ** d, n_fine ** d))


def prolongation(n_coarse: int, d: int) -> sp.csr_matrix:
    """Bilinear (trilinear) interpolation from the printed case formula of Sec. IV-C.

    Per axis: even fine index 2I copies coarse I; odd 2I+1 averages I and I+1.
    """
    n_f = 2 * (n_coarse - 1) + 1
    fine = np.array(np.meshgrid(*([np.arange(n_f)] * d), indexing="ij")).reshape(d, -1).T
    fflat = np.ravel_multi_index(tuple(fine.T), (n_f,) * d)
    # per axis: list of (coarse index, weight)
    rows, cols, vals = [], [], []
    for corner in np.array(np.meshgrid(*([np.arange(2)] * d), indexing="ij")).reshape(d, -1).T:
        ci = np.empty_like(fine)
        wgt = np.ones(len(fine))
        ok = np.ones(len(fine), dtype=bool)
        for a in range(d):
            f = fine[:, a]
            even = (f % 2 == 0)
            # even: only corner 0 contributes with weight 1
            # odd : corners 0 and 1 contribute (f-1)/2 and (f+1)/2 with weight 1/2
            ci[:, a] = np.where(even, f // 2, (f - 1) // 2 + corner[a])
            wgt *= np.where(even, 1.0 if corner[a] == 0 else 0.0, 0.5)
            ok &= ~(even & (corner[a] == 1))
        rows.append(fflat[ok])
        cols.append(np.ravel_multi_index(tuple(ci[ok].T), (n_coarse,) * d))
        vals.append(wgt[ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n_f ** d, n_coarse ** d))


class Hierarchy:
    """Level operators K'_ell = -Lap'_ell - kappa c_ell (h_ell^2-scaled), R, P and the coarsest LU."""

    def __init__(self, prob: Problem, kappa: complex | None = None, levels: int | None = None):
        self.prob = prob
        self.kappa = prob.kappa if kappa is None else kappa
        self.levels = prob.levels if levels is None else levels
        d = prob.d
        self.sizes = [(prob.n_e - 1) // (2 ** l) + 1 for l in range(self.levels)]
        self.coef = [prob.coefficient()]
        for l in range(1, self.levels):
            self.coef.append(self._coarse_coefficient(self.coef[-1], l))
        self.K = []
        self.Dinv = []
        for l, (nl, cl) in enumerate(zip(self.sizes, self.coef)):
            k = (laplacian(nl, d, prob.ghost(l)) - self.kappa * sp.diags(cl.ravel())).tocsr()
            self.K.append(k)
            self.Dinv.append(1.0 / k.diagonal())
        self.R = [restriction(self.sizes[l], d) for l in range(self.levels - 1)]
        self.P = [prolongation(self.sizes[l + 1], d) for l in range(self.levels - 1)]
        self.coarse_lu = spla.splu(self.K[-1].tocsc())

    def _coarse_coefficient(self, c_fine: np.ndarray, level: int) -> np.ndarray:
        """c_{ell} from c_{ell-1}: 4 x full weighting at interior points, background ring (reading A8)."""
        prob = self.prob
        d = prob.d
        n_f = c_fine.shape[0]
        n_c = (n_f - 1) // 2 + 1
        r = restriction(n_f, d)
        cc = 4.0 * (r @ c_fine.ravel()).reshape((n_c,) * d)
        # outermost coarse ring: background k_b^2 h_ell^2 alpha(x)
        axes = np.meshgrid(*([np.arange(n_c)] * d), indexing="ij")
        ring = np.zeros((n_c,) * d, dtype=bool)
        for a in axes:
            ring |= (a == 0) | (a == n_c - 1)
        alpha = prob.alpha_at(axes, stride=2 ** level)
        cb = (prob.kbh * 2 ** level) ** 2 * alpha
        cc[ring] = cb[ring]
        return cc

    # -- smoother / cycle --------------------------------------------------
    def jacobi(self, l: int, b: np.ndarray, v: np.ndarray, sweeps: int) -> np.ndarray:
        """eq. (dampedJ): v <- v - omega D^-1 (K v - b), ``sweeps`` times."""
        w = self.prob.omega_jac
        for _ in range(sweeps):
            v = v - w * self.Dinv[l] * (self.K[l] @ v - b)
        return v

    def cycle(self, b: np.ndarray, v: np.ndarray | None = None, l: int = 0, cycle_type=1) -> np.ndarray:
        """Alg. 2 on level l for the scaled system K'_l v = b (v = 0 when None).

        ``cycle_type`` is Alg. 2's CycleType (1 = V, 2 = W) or a per-level
        sequence of them (e.g. [2, 1, 1, ...]: two coarse-grid corrections on
        the finest level only, V-cycles below -- a per-level choice outside the
        paper, analogous to its per-level smoothing counts).
        """
        if v is None:
            v = np.zeros_like(b)
        if l == self.levels - 1:
            return self.coarse_lu.solve(b)
        gamma = cycle_type if np.isscalar(cycle_type) else cycle_type[l]
        v = self.jacobi(l, b, v, self.prob.nu1)
        r = b - self.K[l] @ v
        rc = 4.0 * (self.R[l] @ r)
        e = np.zeros_like(rc)
        for _ in range(gamma):
            e = self.cycle(rc, e, l + 1, cycle_type)
        v = v + self.P[l] @ e
        return self.jacobi(l, b, v, self.prob.nu2)

    def vcycle(self, r: np.ndarray) -> np.ndarray:
        """One V-cycle from a zero initial guess: the preconditioner application z = M^-1 r."""
        return self.cycle(r, None, 0, 1)

    def two_grid(self, b: np.ndarray, v: np.ndarray) -> np.ndarray:
        """Alg. 1 on levels 0/1 with an exact level-1 solve."""
        v = self.jacobi(0, b, v, self.prob.nu1)
        r = b - self.K[0] @ v
        rc = 4.0 * (self.R[0] @ r)
        e = spla.spsolve(self.K[1].tocsc(), rc)
        v = v + self.P[0] @ e
        return self.jacobi(0, b, v, self.prob.nu2)
