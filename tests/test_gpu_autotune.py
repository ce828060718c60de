"""Launch-shape autotuner: picks one of the bitwise-neutral shapes, sets it,
caches it by key, and leaves results unchanged."""
import json

import numpy as np
import pytest

import synth
from oracle import deflation, wilson

pytestmark = pytest.mark.gpu

M_W = -1.6


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


def test_autotune_sets_cached_neutral_shape(env, tmp_path):
    sg, torch = env
    from paper_0704_3486_amd.autotune import DOT_COLS, UPDATE_BATCH, autotune

    dims, mu = (4, 4, 4, 4), 0.2
    links = synth.random_links(dims, 81)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    S, T, _, _ = deflation.critical_from_dense(A, 6)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_deflate_import(ctx, torch.from_numpy(S).cuda(), T)
        x = torch.from_numpy(synth.gaussian_source(dims, 8100)).cuda()
        y0, y1 = torch.empty_like(x), torch.empty_like(x)
        sg.sgn_apply_fixed(ctx, x, y0, 60)  # default shape
        cache = str(tmp_path / "tune.json")
        r1 = autotune(ctx, k=60, cache=cache, reps=1)
        print("autotune", r1, flush=True)
        assert not r1["cached"] and r1["update_batch"] in UPDATE_BATCH and r1["dot_cols"] in DOT_COLS
        assert sg.sgn_get_tuning(ctx) == (r1["update_batch"], r1["dot_cols"], 8)
        sg.sgn_apply_fixed(ctx, x, y1, 60)
        assert torch.equal(y0, y1)
        with open(cache) as f:
            table = json.load(f)
        assert len(table) == 1
        sg.sgn_set_tuning(ctx, 16, 2, 8)
        r2 = autotune(ctx, k=60, cache=cache)
        assert r2["cached"] and (r2["update_batch"], r2["dot_cols"]) == (r1["update_batch"], r1["dot_cols"])
        assert sg.sgn_get_tuning(ctx)[:2] == (r1["update_batch"], r1["dot_cols"])
        assert sg.sgn_get_precision(ctx) == sg.SGN_PREC_FP64
        r3 = autotune(ctx, k=40, cache=cache, reps=1)  # another key
        assert not r3["cached"]
        with open(cache) as f:
            assert len(json.load(f)) == 2
        del A
        assert np.isfinite(y1.abs().sum().item())
    finally:
        sg.sgn_destroy(ctx)
