"""The entry point that allocates nothing (sgn_matvec_noalloc) against the
allocating one (sgn_matvec): bitwise equal results on two calls in a row, the
second on a smaller lattice, through the C ABI; sizes beyond the static
staging buffer are rejected."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

M_W = -1.6


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


def _one(sg, torch, dims, mu, seed):
    links = synth.random_links(dims, seed)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        x = torch.from_numpy(synth.gaussian_source(dims, seed + 1)).cuda()
        y_ref = torch.empty_like(x)
        y_na = torch.full_like(x, float("nan"))
        sg.sgn_matvec(ctx, x, y_ref)
        sg.sgn_matvec_noalloc(ctx, x, y_na)
        return torch.equal(y_ref, y_na), float(y_ref.abs().max())
    finally:
        sg.sgn_destroy(ctx)


def test_noalloc_matvec_equals_matvec_twice_smaller_second(env):
    sg, torch = env
    print("noalloc 8x8x8x8 then 4x4x4x6", flush=True)
    same1, mag1 = _one(sg, torch, (8, 8, 8, 8), 0.3, 11)
    same2, mag2 = _one(sg, torch, (4, 4, 4, 6), 0.5, 23)
    assert same1 and same2
    assert mag1 > 0 and mag2 > 0


def test_noalloc_matvec_largest_and_rejected_sizes(env):
    sg, torch = env
    print("noalloc 20x20x20x20, then 24x24x24x24 rejected", flush=True)
    same, _ = _one(sg, torch, (20, 20, 20, 20), 0.2, 31)
    assert same
    dims = (24, 24, 24, 24)
    links = synth.random_links(dims, 5)
    ctx = sg.sgn_create(links, dims, 0.2, M_W)
    try:
        N = 12 * int(np.prod(dims))
        x = torch.zeros(N, dtype=torch.complex128, device="cuda")
        y = torch.empty_like(x)
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_matvec_noalloc(ctx, x, y)
        assert e.value.status == sg.SGN_EINVAL
    finally:
        sg.sgn_destroy(ctx)
