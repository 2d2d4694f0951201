"""Robustness experiments of Sec. VI-A on the GPU path, with this implementation's numbers.

* The disk of Fig. 4 (eta 2.2 in air, radius 1.25 wavelengths, 256^2 samples
  at 80 points per wavelength, 32-point layer with beta = 0.15): the GPU
  solution's squared-norm total-field error against the analytic cylinder
  series must land at the order of the 7.5e-3 the paper reports for its
  Helmholtz solver (the same bar as the oracle's golden test).
* Contrast and radius sweeps in the spirit of Figs. 5/6 (whose data files
  are not available): a disk in the 1.333 background at 10 points per
  wavelength, 256^2 interior, 8 plane waves, solved with the paper's
  Bi-CGSTAB (Alg. 3) and with GMRES(5).  Bi-CGSTAB must reach the certified
  1e-6 residual on every case and match the exact LU solution on the
  strongest; GMRES(5) must converge up to contrast 0.2 (on the strongest,
  resonant disk the restarted minimisation stagnates near 6e-6, exactly as
  the oracle's FP64 FGMRES(5) does).  The cycle counts are printed.
"""
import json
import os
import time

import numpy as np
import pytest

import synth
from oracle import model
from oracle.cylinder import cylinder_total_field

from .helpers import KBH, N_B, oracle_problem, rel, to_np

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def test_disk_in_air_matches_the_paper_error():
    import torch

    from paper_2107_03679_amd import helm

    g = json.load(open(os.path.join(HERE, "golden", "disk_in_air.json")))
    lam, hphys, n, w = g["wavelength_cm"], g["h_cm"], g["N_side"], g["abl_points_per_side"]
    print("\n[disk in air, 256^2 at 80 points per wavelength]", flush=True)
    k0h = 2 * np.pi / lam * hphys
    radius_cells = g["radius_wavelengths"] * lam / hphys
    ax = np.arange(n) - (n - 1) / 2
    yy, xx = np.meshgrid(ax, ax, indexing="ij")
    nmap = np.where(xx ** 2 + yy ** 2 <= radius_cells ** 2, g["eta_disk"], g["eta_b"]).astype(np.float32)
    levels = 6
    ne = helm.extended_size(n, w, levels)
    ctx = helm.Context(torch.tensor(nmap, device="cuda"), k0h * (ne - 1), abl_width=w, beta=g["abl_beta"],
                       levels=levels, n_b=g["eta_b"], max_batch=1, restart=5, cycle=3)
    d = np.array([[0.0, -1.0]])  # from the top of the image toward decreasing row index
    rhs, uin = ctx.plane_wave_rhs(d, with_uin=True)
    x, st = ctx.solve(rhs)
    assert st.converged, st
    u = to_np(x + uin)[0][w:w + n, w:w + n]
    k_b = 2 * np.pi / lam
    u_gt = cylinder_total_field(xx * hphys, yy * hphys, g["radius_wavelengths"] * lam, k_b, k_b * g["eta_disk"],
                                np.arctan2(d[0, 1], d[0, 0]))
    eps = np.linalg.norm(u - u_gt) ** 2 / np.linalg.norm(u_gt) ** 2
    ref = g["reported_error_helmholtz"]
    print(f"[disk in air] squared-norm error {eps:.2e} (paper: {ref:.1e}), {st.iters[0]} iterations", flush=True)
    assert ref / 4 < eps < 2 * ref, eps
    ctx.close()


def test_contrast_and_radius_sweep():
    import torch

    from paper_2107_03679_amd import helm

    n, w, levels, B = 256, 20, 5, 8
    ne = helm.extended_size(n, w, levels)
    dirs = synth.directions_2d(B)
    print("\n[contrast/radius sweep, 256^2 interior, 10 points per wavelength, 8 plane waves]", flush=True)
    t0 = torch.tensor(synth.disk_map(n, 16, 0.05), dtype=torch.float32, device="cuda")
    k0 = (KBH / N_B) * (ne - 1)
    kw = dict(abl_width=w, levels=levels, max_batch=B, cycle=3, max_iters=3000)
    solvers = {"Bi-CGSTAB": helm.Context(t0, k0, krylov=helm.KRYLOV_BICGSTAB, restart=8, **kw),
               "GMRES(5)": helm.Context(t0, k0, krylov=helm.KRYLOV_SSTEP, restart=5, **kw)}
    rows = []
    last = None
    for dn in (0.05, 0.1, 0.2, 0.4):
        for radius in (16, 32, 64):
            nmap = synth.disk_map(n, radius, dn).astype(np.float32).astype(np.float64)
            line = f"[sweep] dn={dn:.2f} radius={radius:3d}"
            for name, ctx in solvers.items():
                ctx.update_n(torch.tensor(nmap, dtype=torch.float32, device="cuda"))
                rhs = ctx.plane_wave_rhs(dirs)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                x, st = ctx.solve(rhs)
                torch.cuda.synchronize()
                el = time.perf_counter() - t1
                ok = bool(st.converged and np.all(st.rel_res_true <= 1e-6))
                rows.append((name, dn, radius, st.iters.mean(), ok))
                line += (f"  {name}: {st.iters.mean():6.1f} cycles{'' if ok else ' (stalled)'}, "
                         f"{1e3 * el:6.1f} ms")
                if name == "Bi-CGSTAB":
                    assert ok, (dn, radius, st)
                    last = (nmap, rhs, x)
                elif dn <= 0.2:
                    assert ok, (dn, radius, st)
            print(line, flush=True)
    # the strongest, largest scatterer against the exact discrete solution
    nmap, rhs, x = last
    prob = oracle_problem(nmap, w=w, levels=levels)
    ex = model.ExactSolver(prob)
    b = to_np(rhs)
    for q in (0, B - 1):
        assert rel(to_np(x)[q], ex.solve(b[q])) < 1e-5, q
    # robustness of the paper's method: its cycle count stays within a few times the weakest case
    it = np.array([r[3] for r in rows if r[0] == "Bi-CGSTAB"])
    assert it.max() < 6 * it.min(), rows
    for ctx in solvers.values():
        ctx.close()


SETTINGS = [  # (Im kappa, cycle, levels, omega): the shift of Sec. IV-B, Alg. 2's cycle type, the depth
    (0.3, 3, 4, 0.8), (0.5, 3, 4, 0.8), (0.7, 3, 4, 0.8), (0.5, 1, 4, 0.8), (0.5, 2, 4, 0.8), (0.5, 3, 5, 0.8),
    (0.4, 3, 4, 0.9),
]


def test_settings_sweep_beside_the_oracle():
    """Cycles per solve over the shift, the cycle type (V, W, two corrections on the finest level), the
    level count and the smoothing factor, on the GPU (s-step GMRES(8)) and in the FP64 oracle (FGMRES(8),
    same preconditioner): equal restart cycles up to one for every setting (128^2 blobs, 20-cell layer,
    normal incidence).  The full-size sweep (512^2 x 60) is bench.py --sweep."""
    from oracle.discretization import Problem

    from .helpers import gpu_context, medium

    n, w, m = 128, 20, 8
    nmap = medium(n, seed=9)
    print("\n[settings sweep 128^2 beside the oracle]", flush=True)
    rows = []
    for kim, cyc, L, om in SETTINGS:
        ctx = gpu_context(nmap, w=w, levels=L, kappa=1 + 1j * kim, max_batch=1, restart=m, cycle=cyc,
                          omega_jac=om)
        rhs = ctx.plane_wave_rhs(synth.directions_2d(1, 0.0, 0.0))
        _, st = ctx.solve(rhs)
        ctx.close()
        assert st.converged and st.rel_res_true[0] <= 1e-6
        prob = Problem(nmap, k0h=KBH / N_B, w=w, levels=L, kappa=1 + 1j * kim, omega_jac=om)
        b = model.rhs(prob, (0.0, 1.0))
        from oracle.krylov import fgmres
        from oracle.discretization import helmholtz_matrix
        from oracle.multigrid import Hierarchy

        hier = Hierarchy(prob)
        a = helmholtz_matrix(prob)
        ct = [2] + [1] * (L - 2) if cyc == 3 else cyc
        _, info = fgmres(lambda v: a @ v, lambda r: hier.cycle(r, None, 0, ct), (prob.h ** 2 * b).ravel(),
                         rtol=1e-6, restart=m, max_iters=4000)
        assert info.converged
        gpu_cycles, ora_cycles = int(st.iters[0]) // m, -(-info.iters // m)
        rows.append((kim, cyc, L, om, int(st.iters[0]), info.iters))
        assert abs(gpu_cycles - ora_cycles) <= 1, (kim, cyc, L, om, st.iters[0], info.iters)
    for r in rows:
        print(f"[sweep] Im kappa {r[0]} cycle {r[1]} levels {r[2]} omega {r[3]}: GPU {r[4]}, oracle {r[5]} "
              f"preconditioner applications", flush=True)
