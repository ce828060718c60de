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


def test_stencil_walks_bitwise_equal(env):
    sg, torch = env
    from paper_0704_3486_amd.autotune import autotune_stencil

    dims = (8, 8, 8, 16)
    ctx = sg.sgn_create(synth.random_links(dims, 82), dims, 0.3, M_W)
    try:
        x = torch.from_numpy(synth.gaussian_source(dims, 8200)).cuda()
        ref = torch.empty_like(x)
        sg.sgn_matvec(ctx, x, ref)  # default order (natural at this size)
        for blocks in ((4, 8, 4), (8, 4, 2), (4, 2, 16), (-1, 0, 0), (0, 0, 0)):
            sg.sgn_set_stencil_blocks(ctx, *blocks)
            y = torch.empty_like(x)
            sg.sgn_matvec(ctx, x, y)
            assert torch.equal(y, ref), blocks
        for bad in ((3, 1, 1), (2, 8, 4), (4, 3, 4), (4, 8, 0)):  # 8*2 not a multiple of 32; not divisors
            with pytest.raises(sg.SgnError) as e:
                sg.sgn_set_stencil_blocks(ctx, *bad)
            assert e.value.status == sg.SGN_EINVAL
        r = autotune_stencil(ctx, reps=2)
        print("stencil walk", r, flush=True)
        y = torch.empty_like(x)
        sg.sgn_matvec(ctx, x, y)
        assert torch.equal(y, ref)
        # an apply is unchanged by the walk
        sg.sgn_deflate(ctx, 0)
        y1, y2 = torch.empty_like(x), torch.empty_like(x)
        sg.sgn_apply_fixed(ctx, x, y1, 40)
        sg.sgn_set_stencil_blocks(ctx, -1)
        sg.sgn_apply_fixed(ctx, x, y2, 40)
        assert torch.equal(y1, y2)
    finally:
        sg.sgn_destroy(ctx)
