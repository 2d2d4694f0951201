"""Discretisation of the scattered-field Helmholtz equation (Sec. IV-A).

Everything is FP64 / complex128 and assembled as explicit scipy.sparse
matrices.  Arrays are C-ordered ``[y][x]`` (2D) or ``[z][y][x]`` (3D), so the
flat index of point (m, n) is ``n * n_e + m`` with x fastest, the row order of
eq. (discretizedHelm).

Readings (where the paper is silent, ambiguous or inconsistent):

* A3  absorbing-layer sign.  Under the e^{-j w t} time factor (Sec. II-A) and
      the outgoing Sommerfeld ghosts of Sec. IV-A, a layer absorbs only if
      Im(alpha) >= 0.  The printed alpha = 1 - j beta |x - P(x)|^2 / L is
      amplifying, so the default is alpha = 1 + j beta |x - P(x)|^2 / L;
      ``abl_sign=-1`` gives the printed sign.
* A4  the layer profile uses the paper's normalisation of Omega_e to the
      unit square literally (whatever the physical mesh size): distances
      d = d_cells / (n_e - 1) and L = w / (n_e - 1) with w the low-side layer
      width in cells, so gamma = beta d_cells^2 / (w (n_e - 1)) (profile 0).
      Profile 1 is the alternative beta (d / L)^2 = beta d_cells^2 / w^2.
* A5  vertex-centred coarsening needs n_e odd with (n_e - 1) divisible by
      2^(levels-1); n_e is the smallest such value >= n + 2 w and the extra
      cells go to the high-side layer.  Omega is indices [w, w + n).
* A10 the ghost factor (1 + j h eta) uses eta = k0 * n_b (the layer carries
      the background index), real, with no alpha.
* A24 scaled form: every operator here is h^2 times the paper's, i.e.
      A' = h^2 A_Hel, with off-diagonals -1 and diagonal 4 - c (2D),
      c = (k0 h)^2 n^2 alpha.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


def extended_size(n: int, w: int, levels: int) -> int:
    """Smallest odd n_e >= n + 2w with (n_e - 1) divisible by 2^(levels-1) (reading A5)."""
    step = 2 ** max(levels - 1, 1)
    ne = n + 2 * w
    while (ne - 1) % step != 0:
        ne += 1
    return ne


@dataclass
class Problem:
    """One medium on the extended grid Omega_e plus the solver parameters.

    n_map      interior refractive index, shape (n,)*d, on Omega
    k0h        free-space wavenumber times the fine mesh size, k0*h
    h          fine mesh size (Sec. IV-A normalises Omega_e to the unit square: h = 1/(n_e - 1))
    w          low-side absorbing-layer width in cells
    beta       absorbing-layer strength (Sec. IV-A)
    levels     number of multigrid levels
    kappa      complex shift of the preconditioner K_kappa (Sec. IV-B)
    """

    n_map: np.ndarray
    k0h: float
    n_b: float = 1.333
    w: int = 20
    beta: float = 0.15
    abl_sign: int = +1
    abl_profile: int = 0
    levels: int = 4
    kappa: complex = 1.0 + 0.5j
    omega_jac: float = 0.8
    nu1: int = 1
    nu2: int = 1
    h: float | None = None
    n_e: int = field(init=False)
    d: int = field(init=False)
    n: int = field(init=False)

    def __post_init__(self):
        self.n_map = np.asarray(self.n_map, dtype=np.float64)
        self.d = self.n_map.ndim
        self.n = self.n_map.shape[0]
        assert all(s == self.n for s in self.n_map.shape), "cubic interior expected"
        self.n_e = extended_size(self.n, self.w, self.levels)
        if self.h is None:
            self.h = 1.0 / (self.n_e - 1)

    # -- geometry -------------------------------------------------------
    @property
    def k0(self) -> float:
        return self.k0h / self.h

    @property
    def kbh(self) -> float:
        """Background wavenumber times h, k0 * n_b * h."""
        return self.k0h * self.n_b

    @property
    def shape(self):
        return (self.n_e,) * self.d

    @property
    def size(self) -> int:
        return self.n_e ** self.d

    def interior_slices(self):
        return tuple(slice(self.w, self.w + self.n) for _ in range(self.d))

    def interior_mask(self) -> np.ndarray:
        m = np.zeros(self.shape, dtype=bool)
        m[self.interior_slices()] = True
        return m

    def index_map(self) -> np.ndarray:
        """Refractive index on Omega_e: n_map on Omega, n_b in the layer."""
        out = np.full(self.shape, self.n_b)
        out[self.interior_slices()] = self.n_map
        return out

    def alpha_at(self, idx_axes, stride: int = 1) -> np.ndarray:
        """Layer factor alpha at fine-grid indices (times ``stride``) given per axis (reading A3/A4).

        ``idx_axes`` is a list of d index arrays broadcastable to a grid
        (level-ell indices are fine indices / 2^ell, so pass stride 2^ell).
        """
        lo = float(self.w)
        hi = float(self.w + self.n - 1)
        dist2 = 0.0
        for ia in idx_axes:
            x = np.asarray(ia, dtype=np.float64) * stride
            dx = np.maximum(0.0, np.maximum(lo - x, x - hi))
            dist2 = dist2 + dx * dx
        if self.w <= 0:
            gamma = 0.0 * dist2
        elif self.abl_profile == 1:
            gamma = self.beta * dist2 / float(self.w) ** 2
        else:
            unit = 1.0 / (self.n_e - 1)          # Omega_e normalised to [0, 1]
            gamma = self.beta * (dist2 * unit * unit) / (self.w * unit)
        return 1.0 + 1j * self.abl_sign * gamma

    def alpha(self) -> np.ndarray:
        axes = np.meshgrid(*([np.arange(self.n_e)] * self.d), indexing="ij")
        return self.alpha_at(axes)

    def coefficient(self) -> np.ndarray:
        """c = (k0 h)^2 n^2 alpha on Omega_e (complex, h^2-scaled k0^2 eta^2 alpha)."""
        return (self.k0h ** 2) * self.index_map() ** 2 * self.alpha()

    def ghost(self, level: int = 0) -> complex:
        """Sommerfeld ghost factor 1 + j k_b h_ell (Sec. IV-A, reading A10)."""
        return 1.0 + 1j * self.kbh * (2 ** level)


def second_difference_1d(n_pts: int, g: complex) -> sp.csr_matrix:
    """1D -d^2/dx^2 (times h^2) with first-order Sommerfeld ghosts u_{-1} = g u_0, u_n = g u_{n-1}."""
    main = np.full(n_pts, 2.0 + 0j)
    main[0] -= g
    main[-1] -= g
    off = -np.ones(n_pts - 1, dtype=np.complex128)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr", dtype=np.complex128)


def laplacian(n_pts: int, d: int, g: complex) -> sp.csr_matrix:
    """-Laplacian (times h^2) on an n_pts^d vertex grid with Sommerfeld ghosts, flat index x fastest."""
    t = second_difference_1d(n_pts, g)
    eye = sp.identity(n_pts, dtype=np.complex128, format="csr")
    out = None
    for axis in range(d):
        # axis 0 of the C-ordered array is the slowest (y in 2D, z in 3D)
        factors = [eye] * d
        factors[axis] = t
        term = factors[0]
        for f in factors[1:]:
            term = sp.kron(term, f, format="csr")
        out = term if out is None else out + term
    return out.tocsr()


def helmholtz_matrix(prob: Problem, scaled: bool = True) -> sp.csr_matrix:
    """A_Hel of eq. (discretizedHelm) with Sommerfeld rows; h^2 A_Hel if ``scaled``."""
    a = laplacian(prob.n_e, prob.d, prob.ghost(0)) - sp.diags(prob.coefficient().ravel())
    a = a.tocsr()
    if not scaled:
        a = a / (prob.h ** 2)
    return a


def helmholtz_matrix_rowwise(prob: Problem) -> sp.csr_matrix:
    """Brute-force 2D assembly straight from the printed row formula and ghost rules (tiny grids only)."""
    assert prob.d == 2
    ne = prob.n_e
    c = prob.coefficient()
    g = prob.ghost(0)
    rows, cols, vals = [], [], []
    for nn in range(ne):          # y index (row of the image)
        for m in range(ne):       # x index
            i = nn * ne + m
            diag = 4.0 - c[nn, m]
            for dm, dn in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                mm, nb = m + dm, nn + dn
                if 0 <= mm < ne and 0 <= nb < ne:
                    rows.append(i)
                    cols.append(nb * ne + mm)
                    vals.append(-1.0)
                else:
                    # ghost value replaced by g * u_{m,n}: -g u on the diagonal
                    diag -= g
            rows.append(i)
            cols.append(i)
            vals.append(diag)
    return sp.csr_matrix((np.array(vals, dtype=np.complex128), (rows, cols)), shape=(ne * ne, ne * ne))
