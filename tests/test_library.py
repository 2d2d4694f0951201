"""The C-ABI library loads and exports every symbol include/helm.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2107_03679_amd", "lib", "libhelm.so")


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "helm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(helm_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("helm_setup", "helm_solve_batch", "helm_adjoint_batch", "helm_grad_n", "helm_destroy"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_host_only_entry_points():
    from paper_2107_03679_amd import helm

    assert helm.extended_size(128, 20, 4) == 169
    assert helm.extended_size(512, 20, 7) == 577
    assert helm.extended_size(-1, 20, 4) == -1
    o = helm.default_opts()
    assert (o.levels, o.nu1, o.nu2, o.cycle) == (4, 1, 1, 1)
    assert o.omega_jac == pytest.approx(0.8) and o.rtol == pytest.approx(1e-6)
    assert (o.kappa_re, o.kappa_im) == (1.0, 0.5)
    assert set(helm.EXPORTS) == set(declared_symbols()) | {"helm_default_opts"} - set()


def test_product_path_has_no_oracle_import():
    pkg = os.path.join(ROOT, "paper_2107_03679_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_binding_checks_dtypes_and_shapes_before_calling():
    # the binding refuses tensors the library would misread (wrong dtype, shape or device), on the CPU
    import torch

    from paper_2107_03679_amd import helm

    ctx = object.__new__(helm.Context)  # no device context: only the argument checks run
    ctx.dim, ctx.n_e, ctx.levels = 2, 21, 3
    ctx.info = helm.HelmInfo()
    ctx.info.n = 12
    ok = torch.zeros((2, 21, 21), dtype=torch.complex64)
    with pytest.raises(helm.HelmError, match="GPU"):
        ctx._f(ok, 2)  # right dtype and shape, but host memory
    with pytest.raises(helm.HelmError, match="complex64"):
        ctx._f(ok.to(torch.complex128), 2)
    with pytest.raises(helm.HelmError, match="shape"):
        ctx._f(ok[:, :20, :].contiguous(), 2)
    with pytest.raises(helm.HelmError, match="shape"):
        ctx._f(ok, 3)
    with pytest.raises(helm.HelmError, match="shape"):
        ctx._f(torch.zeros((2, 11, 11), dtype=torch.complex64), 2, level=0)
    with pytest.raises(helm.HelmError, match="int32"):
        ctx._idx(torch.zeros(4, dtype=torch.int64))
    with pytest.raises(helm.HelmError, match="float32"):
        ctx._interior(torch.zeros((12, 12), dtype=torch.float64))
    with pytest.raises(helm.HelmError, match="float32"):
        ctx._interior(torch.zeros((13, 12), dtype=torch.float32))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_null_arguments_return_einval_without_a_device():
    # argument errors are reported before any HIP call
    from paper_2107_03679_amd import helm

    lib = helm.load_library()
    assert lib.helm_sample(None, 1, 1, None, None, None) == -1
    assert lib.helm_sample_adjoint(None, 1, 1, None, None, None) == -1
    assert lib.helm_data_residual(None, 1, 1, None, None, None, None, None) == -1
    assert lib.helm_examples_rms(None, None, 1, None) == -1
    assert lib.helm_net_residual_ratio(None, 1, 8, 8, None, 1.0, 1.0, None) == -1
    assert lib.helm_net_set_conv_kernels(None, 0) == -1


def test_workgroup_order_maps_are_bijections(tmp_path):
    """The XCD-aware workgroup orders of the kernels (dev_common.h: xcd_stretch, xcd_tile) visit
    every (right-hand side, tile) exactly once: a host program built from the same header."""
    import shutil
    import subprocess

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "xcd_order_check")
    cmd = [hipcc if os.path.exists(hipcc) else "hipcc", "-O1", "-std=c++17", "--offload-arch=gfx950",
           "-I", os.path.join(root, "include"), "-I", os.path.join(root, "paper_2107_03679_amd", "csrc"),
           os.path.join(root, "tests", "xcd_order_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
