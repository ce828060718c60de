"""Batched apply (several sources of one field) against single applies and the oracle.

At a fixed Krylov dimension every source of a batch runs exactly the
arithmetic of a single apply (same kernels, same reduction order, each small
matrix sign stopping on its own test), so batched and single results must be
bitwise equal.  With a tolerance the batch shares its checkpoints, so each
source is compared with the exact result instead.
"""
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


@pytest.fixture(scope="module")
def problem():
    dims, mu = (3, 3, 3, 4), 0.3
    links = synth.random_links(dims, 41)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    S, T, _, _ = deflation.critical_from_dense(A.toarray(), 10)
    X = np.stack([synth.gaussian_source(dims, 1000 + r) for r in range(5)])
    return dims, mu, links, A, S, T, X


def _singles(sg, torch, ctx, X, k):
    out = []
    for r in range(X.shape[0]):
        y = torch.empty(X.shape[1], dtype=torch.complex128, device="cuda")
        sg.sgn_apply_fixed(ctx, _dev(torch, X[r]), y, k)
        out.append(y)
    return torch.stack(out)


@pytest.mark.parametrize("prec", [0, 1])  # FP64, mixed
@pytest.mark.parametrize("k", [0, 1, 2, 10, 40])
def test_batched_fixed_is_bitwise_single(env, problem, k, prec):
    sg, torch = env
    dims, mu, links, A, S, T, X = problem
    print("batched fixed", k, prec, flush=True)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_set_precision(ctx, prec)
        sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        Y = torch.empty(X.shape, dtype=torch.complex128, device="cuda")
        infos = sg.sgn_apply_batched_fixed(ctx, _dev(torch, X), Y, k)
        ref = _singles(sg, torch, ctx, X, k)
        assert torch.equal(Y, ref)
        assert [i["k_used"] for i in infos] == [k] * X.shape[0]
        if prec == 0:
            for r in (0, 3):
                st = arnoldi.modified_arnoldi(lambda v: A @ v, X[r], S, k)
                want = arnoldi.approx_definition(S, T, st)
                assert _rel(Y[r].cpu().numpy(), want) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def test_batched_ragged_sources(env, problem):
    """A source inside span(S) stops at k = 0 (exact), the others run on;
    a source repeated in the batch gives the same result twice."""
    sg, torch = env
    dims, mu, links, A, S, T, X = problem
    Xr = np.stack([X[0], S[:, 0] * 2.0 + S[:, 3], X[1], X[0]])
    exact = [matfunc.sgn_spectral_apply(A.toarray(), x) for x in Xr[:3]]
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        Y = torch.empty(Xr.shape, dtype=torch.complex128, device="cuda")
        st, infos = sg.sgn_apply_batched(ctx, _dev(torch, Xr), Y, 1e-11, 600)
        print(infos, flush=True)
        assert st == sg.SGN_OK
        assert infos[1]["k_used"] == 0 and infos[1]["breakdown"] == 1
        for r in range(3):
            assert _rel(Y[r].cpu().numpy(), exact[r]) < 1e-10
        assert torch.equal(Y[0], Y[3])
    finally:
        sg.sgn_destroy(ctx)


def test_batched_more_than_one_launch(env):
    """70 sources run as chunks of 64 and 6; each equals its single apply."""
    sg, torch = env
    dims, mu = (2, 2, 2, 4), 0.2
    links = synth.random_links(dims, 5)
    X = np.stack([synth.gaussian_source(dims, 2000 + r) for r in range(70)])
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        Y = torch.empty(X.shape, dtype=torch.complex128, device="cuda")
        sg.sgn_apply_batched_fixed(ctx, _dev(torch, X), Y, 12)
        ref = _singles(sg, torch, ctx, X[[0, 63, 64, 69]], 12)
        assert torch.equal(Y[[0, 63, 64, 69]], ref)
    finally:
        sg.sgn_destroy(ctx)


def test_batched_6x6_converges_to_exact(env):
    """Four sources at 6^4, mu = 0.2, m = 20 from the library's deflation; the
    first source has a stored exact result, all satisfy sgn(H)^2 x = x."""
    sg, torch = env
    path = os.path.join(GOLDEN, "c6_mu0.2.npy")
    if not os.path.exists(path):
        pytest.skip("stored exact result missing")
    exact = np.load(path, allow_pickle=False)
    dims, mu = (6, 6, 6, 6), 0.2
    links = synth.random_links(dims, synth.GAUGE_SEED)
    X = np.stack([synth.gaussian_source(dims, 1000 + r) for r in range(4)])
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_deflate(ctx, 20)
        Y = torch.empty(X.shape, dtype=torch.complex128, device="cuda")
        st, infos = sg.sgn_apply_batched(ctx, _dev(torch, X), Y, 1e-10, 500)
        print([(i["k_used"], i["err_est"]) for i in infos], flush=True)
        assert st == sg.SGN_OK
        assert _rel(Y[0].cpu().numpy(), exact) < 1e-10
        # sgn(H)^2 = I: applying the batch to its own output gives X back
        Z = torch.empty_like(Y)
        st2, _ = sg.sgn_apply_batched(ctx, Y.clone(), Z, 1e-10, 500)
        assert st2 == sg.SGN_OK
        for r in range(4):
            assert _rel(Z[r].cpu().numpy(), X[r]) < 2e-9
    finally:
        sg.sgn_destroy(ctx)


def test_batched_rejects_bad_input(env, problem):
    sg, torch = env
    dims, mu, links, A, S, T, X = problem
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        Xb = X[:3].copy()
        Xb[1, 7] = np.nan
        Y = torch.empty(Xb.shape, dtype=torch.complex128, device="cuda")
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_apply_batched(ctx, _dev(torch, Xb), Y, 1e-10, 100)
        assert e.value.status == sg.SGN_EINVAL
        with pytest.raises(sg.SgnError):
            sg.sgn_apply_batched(ctx, _dev(torch, X[:3]), Y, -1.0, 100)
        # the context still works afterwards
        Y2 = torch.empty(X[:2].shape, dtype=torch.complex128, device="cuda")
        st, _ = sg.sgn_apply_batched(ctx, _dev(torch, X[:2]), Y2, 1e-9, 600)
        assert st == sg.SGN_OK
    finally:
        sg.sgn_destroy(ctx)


def test_fixed_k_bound_is_the_single_source_bound(env, problem):
    # the composite basis (S V_k) holds at most N columns: k <= N - m for the
    # single and the batched fixed-k entries alike
    sg, torch = env
    dims, mu, links, A, S, T, X = problem
    N, m = X.shape[1], S.shape[1]
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        Xd = _dev(torch, X[:2])
        Y = torch.empty_like(Xd)
        y = torch.empty_like(Xd[0])
        for call in (lambda k: sg.sgn_apply_fixed(ctx, Xd[0], y, k),
                     lambda k: sg.sgn_apply_batched_fixed(ctx, Xd, Y, k)):
            with pytest.raises(sg.SgnError) as e:
                call(N - m + 1)
            assert e.value.status == sg.SGN_EINVAL
    finally:
        sg.sgn_destroy(ctx)
