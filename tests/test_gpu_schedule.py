"""Checkpoint schedule: a first apply (no remembered k) whose tolerance is
reached only near kmax must still be certified.  On this 2x2x2x4 field the
oracle's Arnoldi reaches 1e-12 near k = 320 and the whole complement at
k = N - m = 380; an unbounded jump of the error model from an early
checkpoint straight to kmax left no checkpoint to certify against."""
import numpy as np
import pytest

import synth
from oracle import deflation, matfunc, wilson

pytestmark = pytest.mark.gpu
M_W = -1.6


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


@pytest.fixture(scope="module")
def case():
    dims, mu, m = (2, 2, 2, 4), 0.3, 4
    links = synth.random_links(dims, 5)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    S, T, _, _ = deflation.critical_from_dense(A, m)
    X = np.stack([synth.gaussian_source(dims, 6 + r) for r in range(2)])
    exact = np.stack([matfunc.sgn_spectral_apply(A, x) for x in X])
    return dims, mu, links, S, T, X, exact


def _ctx(sg, torch, case):
    dims, mu, links, S, T = case[:5]
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_deflate_import(ctx, torch.from_numpy(S).cuda(), T)
    return ctx


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_first_apply_certified_near_kmax(env, case):
    sg, torch = env
    X, exact = case[5], case[6]
    kmax = X.shape[1] - case[3].shape[1]
    ctx = _ctx(sg, torch, case)
    try:
        x = torch.from_numpy(X[0]).cuda()
        y = torch.empty_like(x)
        assert sg.sgn_apply(ctx, x, y, 1e-12, kmax) == sg.SGN_OK
        info = sg.sgn_last_info(ctx)
        print(info, flush=True)
        assert info["err_est"] <= 1e-12
        assert _rel(y.cpu().numpy(), exact[0]) < 1e-11
    finally:
        sg.sgn_destroy(ctx)


def test_batched_and_session_certified_near_kmax(env, case):
    sg, torch = env
    X, exact = case[5], case[6]
    kmax = X.shape[1] - case[3].shape[1]
    ctx = _ctx(sg, torch, case)
    try:
        Xd = torch.from_numpy(X).cuda()
        Y = torch.empty_like(Xd)
        st, infos = sg.sgn_apply_batched(ctx, Xd, Y, 1e-12, kmax)
        assert st == sg.SGN_OK and all(i["converged"] for i in infos)
        for r in range(X.shape[0]):
            assert _rel(Y[r].cpu().numpy(), exact[r]) < 1e-11
        ses = sg.Session(ctx, 2, kmax)
        try:
            out = [torch.empty_like(Xd[r]) for r in range(X.shape[0])]
            hs = [ses.submit(Xd[r].contiguous(), out[r], 1e-12, kmax) for r in range(X.shape[0])]
            while ses.active():
                ses.step(16)
            for r, h in enumerate(hs):
                res = ses.poll(h)
                assert res["converged"] == 1, res
                assert _rel(out[r].cpu().numpy(), exact[r]) < 1e-11
        finally:
            ses.destroy()
    finally:
        sg.sgn_destroy(ctx)
