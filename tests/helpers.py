"""Shared set-up for the GPU parity tests: one medium, built identically for
the HIP library (through its C ABI) and for the FP64 oracle."""
from __future__ import annotations

import numpy as np

import synth
from oracle.discretization import Problem

KBH = 2 * np.pi / 10.0  # 10 points per background wavelength
N_B = 1.333


def medium(n: int, kind: str = "blobs", seed: int = 7, d: int = 2) -> np.ndarray:
    """Interior index map, rounded to float32 (the library's input precision)."""
    if kind == "disk":
        m = synth.disk_map(n, n / 6.4, 0.05, N_B, d=d)
    else:
        m = synth.blob_map(n, 4, (n / 20, n / 8), 0.1, seed, n_b=N_B, d=d)
    return m.astype(np.float32).astype(np.float64)


def oracle_problem(nmap, w=8, levels=3, beta=0.15, kappa=1 + 0.5j, nu=1, sign=1, profile=0) -> Problem:
    return Problem(nmap, k0h=KBH / N_B, w=w, levels=levels, beta=beta, kappa=kappa, nu1=nu, nu2=nu,
                   abl_sign=sign, abl_profile=profile)


def gpu_context(nmap, w=8, levels=3, beta=0.15, kappa=1 + 0.5j, nu=1, sign=1, profile=0, **opts):
    import torch

    from paper_2107_03679_amd import helm

    ne = helm.extended_size(nmap.shape[0], w, levels)
    k0 = (KBH / N_B) * (ne - 1)  # k0 in units of 1/h with h = 1/(n_e - 1)
    t = torch.tensor(nmap, dtype=torch.float32, device="cuda")
    return helm.Context(t, k0, abl_width=w, beta=beta, abl_sign=sign, abl_profile=profile, kappa=kappa, levels=levels,
                        nu1=nu, nu2=nu, **opts)


def to_np(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.complex128)


def to_dev(a: np.ndarray):
    import torch

    return torch.tensor(np.ascontiguousarray(a), dtype=torch.complex64, device="cuda")


def rel(a, b) -> float:
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
