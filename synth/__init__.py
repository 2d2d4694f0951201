"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *defines inputs*: refractive-index maps, illumination
directions and random test vectors.  It holds none of the solver's arithmetic
(no grid geometry, no operator, no coefficient), so both the FP64 oracle and
the HIP path may draw their inputs from it without sharing method code.

Media (refractive-index maps on the interior domain Omega):
  * ``disk_map``  -- one disk inclusion (the paper's robustness experiments
    use disks, Sec. VI-A);
  * ``blob_map``  -- a background index plus a sum of seeded Gaussian blobs,
    standing in for the paper's simulated object and experimental targets
    (Sec. VI-B, VI-C), whose images and data are not available.

Blob recipe (per blob, in this draw order, ``numpy.random.default_rng(seed)``):
sigma ~ U[sigma_lo, sigma_hi]; amplitude ~ U[0, amp_hi]; centre ~
U[3 sigma, n - 1 - 3 sigma] per axis (clamped to the middle if the interval is
empty); n(x) = n_b + sum amplitude * exp(-|x - centre|^2 / (2 sigma^2)).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "disk_map",
    "blob_map",
    "directions_2d",
    "directions_cone",
    "complex_field",
    "WORKLOADS",
]


def disk_map(n: int, radius: float, dn: float, n_b: float = 1.333, d: int = 2) -> np.ndarray:
    """Index map ``n_b`` with ``n_b + dn`` at grid points within ``radius`` cells of the centre."""
    ax = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    grids = np.meshgrid(*([ax] * d), indexing="ij")
    r2 = sum(g * g for g in grids)
    out = np.full((n,) * d, n_b, dtype=np.float64)
    out[r2 <= radius * radius] = n_b + dn
    return out


def blob_map(n: int, n_blobs: int, sigma_range, amp_hi: float, seed: int,
             n_b: float = 1.333, d: int = 2, max_dn: float | None = None) -> np.ndarray:
    """Background ``n_b`` plus ``n_blobs`` seeded Gaussian blobs (recipe in the module doc)."""
    rng = np.random.default_rng(seed)
    ax = np.arange(n, dtype=np.float64)
    grids = np.meshgrid(*([ax] * d), indexing="ij")
    dn = np.zeros((n,) * d, dtype=np.float64)
    for _ in range(n_blobs):
        sigma = rng.uniform(sigma_range[0], sigma_range[1])
        amp = rng.uniform(0.0, amp_hi)
        lo, hi = 3.0 * sigma, (n - 1) - 3.0 * sigma
        if lo > hi:
            lo = hi = (n - 1) / 2.0
        centre = rng.uniform(lo, hi, size=d)
        r2 = sum((g - c) ** 2 for g, c in zip(grids, centre))
        dn += amp * np.exp(-r2 / (2.0 * sigma * sigma))
    if max_dn is not None and dn.max() > max_dn:
        dn *= max_dn / dn.max()
    return n_b + dn


def directions_2d(count: int, theta_lo_deg: float = -60.0, theta_hi_deg: float = 60.0) -> np.ndarray:
    """Unit vectors (d_x, d_y) = (sin t, cos t), t = linspace(lo, hi, count) inclusive.

    t = 0 is normal incidence, propagating toward increasing row index (+y).
    """
    if count == 1:
        th = np.array([0.5 * (theta_lo_deg + theta_hi_deg)])
    else:
        th = np.linspace(theta_lo_deg, theta_hi_deg, count)
    th = np.deg2rad(th)
    return np.stack([np.sin(th), np.cos(th)], axis=1)


def directions_cone(count: int, half_angle_deg: float = 45.0) -> np.ndarray:
    """Unit vectors (d_x, d_y, d_z) on a cone about +z: (sin a cos p, sin a sin p, cos a), p = 2 pi q / count."""
    a = np.deg2rad(half_angle_deg)
    p = 2.0 * np.pi * np.arange(count) / count
    return np.stack([np.sin(a) * np.cos(p), np.sin(a) * np.sin(p), np.full(count, np.cos(a))], axis=1)


def complex_field(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Standard complex Gaussian test vector (re, im ~ N(0, 1/2))."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    return z.astype(dtype)


# Named workloads: interior size, medium recipe, illuminations.  Every
# configuration samples the background wavelength with 10 grid points and
# uses a 20-cell absorbing layer on the low side of each axis.
WORKLOADS = {
    "disk128": dict(d=2, n=128, medium=("disk", dict(radius=20.0, dn=0.05)), rhs=1,
                    directions=("normal",), beta=0.15),
    "blobs512x60": dict(d=2, n=512, medium=("blobs", dict(n_blobs=8, sigma_range=(10.0, 40.0), amp_hi=0.1, seed=0)),
                        rhs=60, directions=("fan", -60.0, 60.0), beta=0.15),
    "inverse256x32": dict(d=2, n=256, medium=("blobs", dict(n_blobs=8, sigma_range=(5.0, 20.0), amp_hi=0.1, seed=1)),
                          rhs=32, directions=("fan", -60.0, 60.0), beta=0.0),
    "strong1024x120": dict(d=2, n=1024, medium=("blobs", dict(n_blobs=8, sigma_range=(20.0, 80.0), amp_hi=0.4, seed=2,
                                                              max_dn=0.4)),
                           rhs=120, directions=("fan", -60.0, 60.0), beta=0.15),
    "cube128x40": dict(d=3, n=128, medium=("blobs", dict(n_blobs=12, sigma_range=(4.0, 16.0), amp_hi=0.15, seed=3)),
                       rhs=40, directions=("cone", 45.0), beta=0.15),
}


def workload_medium(name: str, n_b: float = 1.333) -> np.ndarray:
    """Interior index map of a named workload."""
    wl = WORKLOADS[name]
    kind, kw = wl["medium"]
    if kind == "disk":
        return disk_map(wl["n"], kw["radius"], kw["dn"], n_b=n_b, d=wl["d"])
    return blob_map(wl["n"], kw["n_blobs"], kw["sigma_range"], kw["amp_hi"], kw["seed"], n_b=n_b, d=wl["d"],
                    max_dn=kw.get("max_dn"))


def workload_directions(name: str, count: int | None = None) -> np.ndarray:
    """Illumination directions of a named workload (optionally a different count)."""
    wl = WORKLOADS[name]
    count = wl["rhs"] if count is None else count
    kind = wl["directions"][0]
    if kind == "normal":
        return directions_2d(1, 0.0, 0.0) if count == 1 else directions_2d(count, 0.0, 0.0)
    if kind == "fan":
        return directions_2d(count, wl["directions"][1], wl["directions"][2])
    return directions_cone(count, wl["directions"][1])
