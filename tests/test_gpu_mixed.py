"""Mixed precision (FP32 stencil and Krylov vectors, FP64 elsewhere) against
the FP64 oracle.  Bound: relative error <= 1e-6 (FP32 storage of the basis,
unit roundoff 6e-8, limits the attainable accuracy to about 1e-7)."""
import os

import numpy as np
import pytest

import synth
from oracle import arnoldi, deflation, matfunc, wilson

pytestmark = pytest.mark.gpu
M_W = -1.6
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def test_mixed_stencil_matches_oracle_to_fp32(env):
    # the FP32 stencil, seen through a k = 1 apply, agrees with FP64 to FP32 rounding
    sg, torch = env
    dims, mu = (4, 2, 6, 4), 0.3
    links = synth.random_links(dims, 5)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    x = synth.gaussian_source(dims, 9)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_set_precision(ctx, sg.SGN_PREC_MIXED)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        sg.sgn_apply_fixed(ctx, _dev(torch, x), y, 2)
        st = arnoldi.modified_arnoldi(lambda v: A @ v, x, None, 2)
        ref = arnoldi.approx_definition(None, None, st)
        assert _rel(y.cpu().numpy(), ref) < 1e-5
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("m", [0, 12])
def test_mixed_apply_vs_exact_small(env, m):
    sg, torch = env
    dims, mu = (3, 3, 3, 4), 0.3
    links = synth.random_links(dims, 32)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    x = synth.gaussian_source(dims, 1001)
    exact = matfunc.sgn_spectral_apply(A, x)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_set_precision(ctx, sg.SGN_PREC_MIXED)
        if m:
            S, T, _, _ = deflation.critical_from_dense(A, m)
            sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        st = sg.sgn_apply(ctx, _dev(torch, x), y, 1e-7, 600)
        info = sg.sgn_last_info(ctx)
        err = _rel(y.cpu().numpy(), exact)
        print("mixed", m, info, err, flush=True)
        assert st == sg.SGN_OK
        assert err < 1e-6
    finally:
        sg.sgn_destroy(ctx)


def test_mixed_8x8_vs_fp64_oracle_arnoldi(env):
    # 8^4, mu = 0.3, m = 30: against the oracle's FP64 Arnoldi at k = 800
    # (self-converged: |y_800 - y_700| / |y_800| <= 1e-8, stored by make_golden.py)
    sg, torch = env
    path = os.path.join(GOLDEN, "c8_mu0.3.npy")
    if not os.path.exists(path):
        pytest.skip("golden file c8_mu0.3 not generated")
    ref = np.load(path, allow_pickle=False)
    dims, mu = (8, 8, 8, 8), 0.3
    links = synth.random_links(dims, synth.GAUGE_SEED)
    x = synth.gaussian_source(dims, 1000)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_set_precision(ctx, sg.SGN_PREC_MIXED)
        sg.sgn_deflate(ctx, 30)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        st = sg.sgn_apply(ctx, _dev(torch, x), y, 1e-7, 800)
        info = sg.sgn_last_info(ctx)
        err = _rel(y.cpu().numpy(), ref)
        print("c3 mixed", info, err, flush=True)
        assert st == sg.SGN_OK
        assert err < 1e-6
    finally:
        sg.sgn_destroy(ctx)
