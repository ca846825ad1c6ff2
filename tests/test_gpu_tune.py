"""Autotuner (bem_autotune): timed choice within the candidate sets, JSON cache
written and reused, and results unchanged beyond summation order."""

import json

import numpy as np
import pytest

from workloads import sphere_eval_points, sphere_problem

pytestmark = pytest.mark.gpu

CANDIDATES = {"far_rows": {32, 64, 128}, "gemv_rows": {2, 4, 8}, "gemm_blocks": {512, 1024, 2048},
              "eval_blocks": {1024, 2048, 4096}, "trace_tile": {64, 128, 256}, "trace_splitk": {2, 4, 8},
              "trace_split": {0, 32, 64, 128, 256}, "trace_few": {0, 2, 4, 8, 16}}


@pytest.fixture(scope="module")
def bem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    return bem


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_cache_and_results(bem, tmp_path, precision):
    import torch
    prec = bem.FP64 if precision == "fp64" else bem.MIXED
    p = sphere_problem(3, V0=1.0)
    pts = torch.tensor(sphere_eval_points(1000, seed=1), device="cuda")
    ctx = bem.Context.from_problem(p, precision=prec, eta=6.0)
    ctx.assemble()
    rows0 = ctx.copy_rows(0, ctx.n).cpu().numpy()
    sol0, _ = ctx.solve(p.body_V, tol=1e-12)
    _, E0 = ctx.eval_field(sol0, pts)
    cache = tmp_path / "tune.json"
    assert ctx.autotune(str(cache)) is False
    chosen = {k: ctx.get_tuning(k) for k in CANDIDATES}
    for k, v in chosen.items():
        assert v in CANDIDATES[k], (k, v)
    data = json.loads(cache.read_text())
    assert len(data) == 1
    (key, entry), = data.items()
    assert "gfx950" in key and f"N={p.n_tri}" in key
    assert entry == chosen
    # the re-assembled operator is the same matrix (tile shapes do not change an entry)
    rows1 = ctx.copy_rows(0, ctx.n).cpu().numpy()
    assert np.array_equal(rows0, rows1)
    sol1, _ = ctx.solve(p.body_V, tol=1e-12)
    _, E1 = ctx.eval_field(sol1, pts)
    tol = 1e-10 if prec == bem.FP64 else 1e-6
    assert float((sol1 - sol0).abs().max() / sol0.abs().max()) <= tol
    assert float((E1 - E0).abs().max() / E0.abs().max()) <= tol
    ctx.close()
    # a second context of the same problem takes the cached choice without timing
    ctx2 = bem.Context.from_problem(p, precision=prec, eta=6.0)
    ctx2.assemble()
    assert ctx2.autotune(str(cache)) is True
    assert {k: ctx2.get_tuning(k) for k in CANDIDATES} == chosen
    ctx2.close()


def test_tuning_knob_validation(bem):
    p = sphere_problem(1)
    ctx = bem.Context.from_problem(p)
    for key, bad in (("far_rows", 48), ("gemv_rows", 3), ("eval_blocks", 10), ("trace_split", -1),
                     ("trace_tile", 96), ("trace_groups", -1), ("trace_groups", 3), ("trace_fold", 2),
                     ("near_rule", 2), ("grad_batch", 8), ("nope", 1)):
        with pytest.raises(bem.BemError):
            ctx.set_tuning(key, bad)
    assert ctx.get_tuning("gemv_rows") == 4      # FP64 default
    assert ctx.get_tuning("trace_groups") == 0   # two line groups from 128 lines
    assert ctx.get_tuning("trace_fold") == 1 and ctx.get_tuning("near_rule") == 0
    ctx.set_tuning("gemv_rows", 8)
    assert ctx.get_tuning("gemv_rows") == 8
    with pytest.raises(bem.BemError):
        ctx.autotune(None)          # not assembled yet
    ctx.close()
    ctx = bem.Context.from_problem(p, precision=bem.MIXED)
    assert ctx.get_tuning("gemv_rows") == 8      # MIXED default (FP32 rows, FP64 x)
    ctx.close()
