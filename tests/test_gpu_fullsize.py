"""Parity at the benchmark's full size and launch configuration.

The 512^2 interior with 60 plane waves in [-60, 60] degrees (blob medium,
seed 0), 7 levels, GMRES(8) in s-step form, two coarse corrections on the
finest level, autotuned launch shapes, hipGraph replay: the whole batch is
solved as bench.py times it; the first, a middle and the last plane wave are
compared with exact sparse-LU solves of the FP64 oracle (field error <= 1e-5
over the extended grid), and their float-float iterates are certified by a
host FP64 residual <= 1.05e-6.
"""
import numpy as np
import pytest

import synth
from oracle import model
from oracle.discretization import Problem

from .helpers import KBH, N_B, rel, to_np

pytestmark = pytest.mark.gpu


def test_benchmark_workload_matches_exact_solutions(tmp_path):
    import torch

    from paper_2107_03679_amd import helm

    print("\n[full size: blobs512x60, 7 levels, GMRES(8) s-step, cycle 3]", flush=True)
    wl = synth.WORKLOADS["blobs512x60"]
    nmap = synth.workload_medium("blobs512x60").astype(np.float32).astype(np.float64)
    dirs = synth.workload_directions("blobs512x60")
    levels, w = 7, 20
    ne = helm.extended_size(wl["n"], w, levels)
    ctx = helm.Context(torch.tensor(nmap, dtype=torch.float32, device="cuda"), (KBH / N_B) * (ne - 1),
                       abl_width=w, beta=wl["beta"], levels=levels, restart=8, cycle=3, max_batch=60,
                       max_iters=20000)
    ctx.autotune(60, cache=str(tmp_path / "tune.jsonl"))
    rhs = ctx.plane_wave_rhs(dirs)
    x, st = ctx.solve(rhs)
    assert st.converged and np.all(st.rel_res_true <= 1e-6), st
    print(f"[full size] iterations mean {st.iters.mean():.1f} max {st.iters.max()}", flush=True)
    lo = to_np(ctx.solution_lo(60))
    xs, bs = to_np(x), to_np(rhs)
    prob = Problem(nmap, k0h=KBH / N_B, w=w, levels=levels, beta=wl["beta"])
    assert prob.n_e == ne
    ex = model.ExactSolver(prob)
    for q in (0, 30, 59):  # the first (-60 degrees), a middle and the last (60 degrees) plane wave
        u = ex.solve(bs[q])
        err = rel(xs[q], u)
        rq = np.linalg.norm(bs[q].ravel() - ex.A @ (xs[q] + lo[q]).ravel()) / np.linalg.norm(bs[q].ravel())
        print(f"[full size] plane wave {q}: field error {err:.2e}, FP64 residual {rq:.2e}", flush=True)
        assert err < 1e-5, (q, err)
        assert rq <= 1.05e-6, (q, rq)
    ctx.close()
