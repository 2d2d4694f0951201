"""MI355X-native batched Helmholtz solver (multigrid-preconditioned FGMRES),
the hot path of Helmholtz diffraction tomography (arXiv 2107.03679).

The compute lives in the HIP library libhelm.so (C ABI in include/helm.h);
``paper_2107_03679_amd.helm`` is its ctypes binding.
"""
__all__ = ["helm"]
