"""Autotuner of the batched multigrid cycle (launch shapes of the fused legs,
single-launch threshold of the coarse levels).

Every tile shape computes each point with the same arithmetic, so the cycle
must be bit-identical whatever the tuner picks; the coarse-level threshold
switches between two kernels, which are compared with the FP64 oracle.  The
JSON-lines cache is checked by re-applying a stored choice, and every tile
variant is forced through an edited cache line.
"""
import json

import numpy as np
import pytest

import synth
from oracle.multigrid import Hierarchy

from .helpers import gpu_context, medium, oracle_problem, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

N, W, LEVELS, B = 150, 20, 4, 4
DEFAULT_COARSE_MAX = 48 * 48


@pytest.fixture(scope="module")
def case():
    print(f"\n[autotune n={N} w={W} levels={LEVELS} B={B}]", flush=True)
    nmap = medium(N, seed=3)
    prob = oracle_problem(nmap, w=W, levels=LEVELS)
    hier = Hierarchy(prob)
    r = synth.complex_field((B, *prob.shape), 91)
    ref = np.stack([hier.vcycle(ri.ravel()).reshape(prob.shape) for ri in r])
    return nmap, prob, r, ref


def _edit(line: str, levels: int, down: int, up: int, coarse_max: int, mv: int = 0) -> str:
    e = json.loads(line)
    e["down"] = [down] * levels
    e["up"] = [up] * levels
    e["coarse_max"] = coarse_max
    e["mv"] = mv
    return json.dumps(e) + "\n"


def test_autotune_keeps_results_and_caches(case, tmp_path):
    nmap, prob, r, ref = case
    cache = tmp_path / "tune.jsonl"
    ctx = gpu_context(nmap, w=W, levels=LEVELS, max_batch=B)
    rd = to_dev(r)
    z0 = ctx.precondition(rd)
    assert rel(to_np(z0), ref) < 1e-5
    t = ctx.autotune(B, cache=str(cache))
    print(f"[autotune] {t}", flush=True)
    assert not t["from_cache"]
    assert len(t["down_tiles"]) == LEVELS - 1 and len(t["up_tiles"]) == LEVELS - 1
    assert t["vcycle_ms"] > 0 and t["vcycle_default_ms"] > 0
    z1 = ctx.precondition(rd)
    assert rel(to_np(z1), ref) < 1e-5
    if t["coarse_single_launch_max_points"] == DEFAULT_COARSE_MAX:
        assert bool((z1 == z0).all())
    # the solve with the tuned shapes reaches the target and matches the untuned solve's accuracy
    rhs = ctx.plane_wave_rhs(synth.directions_2d(B))
    x, st = ctx.solve(rhs)
    assert st.converged and np.all(st.rel_res_true <= 1e-6)
    ctx.close()
    # a fresh context on the same problem takes the cached choice without timing
    ctx2 = gpu_context(nmap, w=W, levels=LEVELS, max_batch=B)
    t2 = ctx2.autotune(B, cache=str(cache))
    assert t2["from_cache"]
    for k in ("down_tiles", "up_tiles", "coarse_single_launch_max_points"):
        assert t2[k] == t[k]
    assert bool((ctx2.precondition(rd) == z1).all())
    x2, st2 = ctx2.solve(rhs)
    assert bool((x2 == x).all()) and np.array_equal(st2.iters, st.iters)
    ctx2.close()
    assert len(cache.read_text().splitlines()) == 1


@pytest.mark.parametrize("cycle", [1, 3])
@pytest.mark.parametrize("variant", range(7))
def test_every_tile_variant_is_bit_identical(case, tmp_path, variant, cycle):
    """Forced tile shapes against the defaults; cycle 3 adds the repeated visit of level 1
    (the legs that form r - K e themselves)."""
    nmap, prob, r, ref = case
    ctx = gpu_context(nmap, w=W, levels=LEVELS, max_batch=B, cycle=cycle)
    rd = to_dev(r)
    z0 = ctx.precondition(rd)
    first = tmp_path / "first.jsonl"
    ctx.autotune(B, cache=str(first))
    line = first.read_text().splitlines()[0]
    forced = tmp_path / "forced.jsonl"
    forced.write_text(_edit(line, LEVELS, variant, variant, DEFAULT_COARSE_MAX))
    t = ctx.autotune(B, cache=str(forced))
    assert t["from_cache"], "the forced cache line was not accepted"
    z = ctx.precondition(rd)
    assert bool((z == z0).all()), f"tile variant {variant} changed the cycle"
    ctx.close()


def test_up_mv_heights_are_bit_identical(case, tmp_path):
    """Every launch shape (tile height, right-hand sides per workgroup) of the s-step form's fused
    finest up-leg + basis matvec, forced through the cache: the same iterates (bit for bit) and cycle
    counts as the default shape."""
    nmap, prob, r, ref = case
    ctx = gpu_context(nmap, w=W, levels=LEVELS, max_batch=B, restart=6)
    first = tmp_path / "first.jsonl"
    t0 = ctx.autotune(B, cache=str(first))
    line = first.read_text().splitlines()[0]
    rhs = ctx.plane_wave_rhs(synth.directions_2d(B))
    e = json.loads(line)
    xs = []
    for mv in range(9):
        forced = tmp_path / f"mv{mv}.jsonl"
        forced.write_text(_edit(line, LEVELS, e["down"][0], e["up"][0], e["coarse_max"], mv))
        t = ctx.autotune(B, cache=str(forced))
        assert t["from_cache"] and t["up_mv_rows"] == (16, 12, 20, 28, 12, 12, 12, 20, 20)[mv]
        assert t["up_mv_rhs_per_block"] == (4, 1, 1, 1, 2, 4, 6, 2, 4)[mv]
        x, st = ctx.solve(rhs)
        assert st.converged
        xs.append((x, st.iters))
    for x, it in xs[1:]:
        assert bool((x == xs[0][0]).all()) and np.array_equal(it, xs[0][1])
    print(f"[autotune] up-mv shape chosen: {t0['up_mv_rows']} rows, {t0['up_mv_rhs_per_block']} per block", flush=True)
    ctx.close()


def test_up_mv_shapes_with_idle_right_hand_sides(tmp_path):
    """Seven right-hand sides (groups of four and three in the shapes that walk four per
    workgroup), the second and the fifth zero: inactive from the start and skipped inside
    their groups.  Every launch shape of the fused finest up-leg gives the same iterates bit
    for bit and the same cycle counts, and the zero right-hand sides keep a zero solution."""
    nb = 7
    print(f"\n[autotune up-mv shapes, B={nb} with two zero right-hand sides]", flush=True)
    nmap = medium(N, seed=3)
    ctx = gpu_context(nmap, w=W, levels=LEVELS, max_batch=nb, restart=6)
    first = tmp_path / "first.jsonl"
    ctx.autotune(nb, cache=str(first))
    line = first.read_text().splitlines()[0]
    e = json.loads(line)
    rhs = ctx.plane_wave_rhs(synth.directions_2d(nb))
    rhs[1].zero_()
    rhs[4].zero_()
    xs = []
    for mv in range(9):
        forced = tmp_path / f"mv{mv}.jsonl"
        forced.write_text(_edit(line, LEVELS, e["down"][0], e["up"][0], e["coarse_max"], mv))
        t = ctx.autotune(nb, cache=str(forced))
        assert t["from_cache"]
        x, st = ctx.solve(rhs)
        assert st.converged
        xs.append((x.clone(), np.array(st.iters)))
    x0, it0 = xs[0]
    assert bool((x0[1] == 0).all()) and bool((x0[4] == 0).all())
    assert it0[1] == 0 and it0[4] == 0 and np.all(np.delete(it0, [1, 4]) > 0)
    for x, it in xs[1:]:
        assert bool((x == x0).all()) and np.array_equal(it, it0)
    ctx.close()


def test_coarse_threshold_variants_match_oracle(case, tmp_path):
    nmap, prob, r, ref = case
    ctx = gpu_context(nmap, w=W, levels=LEVELS, max_batch=B)
    rd = to_dev(r)
    first = tmp_path / "first.jsonl"
    ctx.autotune(B, cache=str(first))
    line = first.read_text().splitlines()[0]
    for cm in (0, 24 * 24, 96 * 96):
        forced = tmp_path / f"cm{cm}.jsonl"
        forced.write_text(_edit(line, LEVELS, 0, 0, cm))
        t = ctx.autotune(B, cache=str(forced))
        assert t["from_cache"] and t["coarse_single_launch_max_points"] == cm
        assert rel(to_np(ctx.precondition(rd)), ref) < 1e-5, cm
    ctx.close()


def test_autotune_rejects_bad_batch(case):
    from paper_2107_03679_amd.helm import HelmError

    nmap = case[0]
    ctx = gpu_context(nmap, w=W, levels=LEVELS, max_batch=B)
    with pytest.raises(HelmError):
        ctx.autotune(B + 1)
    with pytest.raises(HelmError):
        ctx.autotune(0)
    ctx.close()
