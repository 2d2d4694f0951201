"""The allocation-free data residual (fixed device scratch) against the allocating entry point it
mirrors, through the C ABI: equal outputs on two calls in a row, the second smaller, and the
argument checks that keep it from reading outside the grid or its scratch."""
import numpy as np
import pytest

import synth

from .helpers import gpu_context, medium, to_dev

pytestmark = pytest.mark.gpu


def _case(ctx, B, M, seed):
    import torch

    rng = np.random.default_rng(seed)
    N = ctx.n_e ** 2
    idx = torch.tensor(rng.choice(N, size=M, replace=False).astype(np.int32), device="cuda")
    u = to_dev(synth.complex_field((B, ctx.n_e, ctx.n_e), seed + 1))
    y = to_dev(synth.complex_field((B, M), seed + 2))
    return idx, u, y


def test_static_data_residual_matches_the_allocating_one():
    import torch

    from paper_2107_03679_amd import helm

    ctx = gpu_context(medium(40, seed=2), w=8, levels=3, max_batch=8)
    try:
        for B, M, seed in ((8, 700, 10), (3, 57, 20)):  # the second call smaller than the first
            print(f"\n[static data residual B={B} M={M}]", flush=True)
            idx, u, y = _case(ctx, B, M, seed)
            res_ref, loss_ref = ctx.data_residual(idx, u, y)
            res = torch.full((B, M), float("nan"), dtype=torch.complex64, device="cuda")
            res, loss = ctx.data_residual_static(idx, u, y, res)
            torch.cuda.synchronize()
            assert torch.equal(res, res_ref)
            assert loss == loss_ref  # same partial sums added in the same order
            ref = (to_np_c(u)[:, to_np_i(idx) // ctx.n_e, to_np_i(idx) % ctx.n_e] - to_np_c(y))
            assert np.allclose(to_np_c(res), ref, rtol=0, atol=1e-6)
        # an index outside the grid is refused before any read through it; the next call still works
        bad = idx.clone()
        bad[1] = ctx.n_e ** 2
        with pytest.raises(helm.HelmError, match="outside the grid"):
            ctx.data_residual_static(bad, u, y, torch.empty_like(y))
        res, loss = ctx.data_residual_static(idx, u, y, torch.empty_like(y))
        assert loss == ctx.data_residual(idx, u, y)[1]
        # sizes beyond the fixed scratch
        lib = helm.load_library()
        big_m = helm_max = 1048576
        rc = lib.helm_data_residual_static(ctx._h, 2, big_m // 2 + 1, idx.data_ptr(), u.data_ptr(), y.data_ptr(),
                                           y.data_ptr(), None)
        assert rc == -1 and b"exceeds" in lib.helm_last_error(ctx._h)
        assert helm_max == 1048576
    finally:
        ctx.close()


def to_np_c(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def to_np_i(t):
    return t.detach().cpu().numpy().astype(np.int64)
