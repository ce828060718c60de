"""Serving sessions (continuous batching on one field).

Each request's checkpoint schedule depends on the request alone and every
kernel computes each slot as it would alone, so a result must be bitwise the
same whether the request runs alone or among others admitted at other
times, and equal to sgn_apply on a fresh context; results are also checked
against the exact sign (oracle).
"""
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
def problem():
    dims, mu = (3, 3, 3, 4), 0.3
    links = synth.random_links(dims, 52)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    S, T, _, _ = deflation.critical_from_dense(A, 10)
    X = np.stack([synth.gaussian_source(dims, 3000 + r) for r in range(6)])
    X[4] = S[:, 1] - 0.5 * S[:, 6]  # inside span(S): exact at k = 0
    return dims, mu, links, A, S, T, X


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _ctx(sg, torch, problem, prec):
    dims, mu, links, A, S, T, X = problem
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_set_precision(ctx, prec)
    sg.sgn_deflate_import(ctx, _dev(torch, S), T)
    return ctx


def _run_alone(sg, torch, problem, prec, tols, kmaxs):
    """Each request alone in a one-slot session."""
    X = problem[6]
    out = []
    ctx = _ctx(sg, torch, problem, prec)
    try:
        for r in range(X.shape[0]):
            ses = sg.Session(ctx, 1, 600)
            x = _dev(torch, X[r])
            y = torch.empty_like(x)
            req = ses.submit(x, y, tols[r], kmaxs[r])
            while ses.poll(req) is None:
                ses.step(7)
            ses.destroy()
            out.append(y)
    finally:
        sg.sgn_destroy(ctx)
    return torch.stack(out)


def _run_mixed(sg, torch, problem, prec, tols, kmaxs, slots=3):
    """All requests through one session with fewer slots than requests,
    admitted as slots free up, at irregular step counts."""
    X = problem[6]
    n = X.shape[0]
    ctx = _ctx(sg, torch, problem, prec)
    xs = [_dev(torch, X[r]) for r in range(n)]
    ys = [torch.empty_like(x) for x in xs]
    infos = [None] * n
    try:
        ses = sg.Session(ctx, slots, 600)
        queue = list(range(n))
        running = {}
        steps = [3, 11, 1, 6, 17, 2]
        t = 0
        while queue or running:
            while queue:
                r = queue[0]
                req = ses.submit(xs[r], ys[r], tols[r], kmaxs[r])
                if req is None:
                    break
                running[req] = r
                queue.pop(0)
                if t % 2 == 0:
                    break  # admit at most one now and then
            ses.step(steps[t % len(steps)])
            t += 1
            for req in list(running):
                info = ses.poll(req)
                if info is not None:
                    infos[running.pop(req)] = info
        ses.destroy()
    finally:
        sg.sgn_destroy(ctx)
    return torch.stack(ys), infos


@pytest.mark.parametrize("prec", [0, 1])
def test_session_alone_equals_mixed(env, problem, prec):
    sg, torch = env
    print("session alone vs mixed", prec, flush=True)
    tols = [1e-10, 1e-8, 1e-11, 1e-9, 1e-10, 1e-10] if prec == 0 else [1e-7] * 6
    kmaxs = [600, 600, 600, 500, 600, 40]  # the last stops at its kmax
    Ya = _run_alone(sg, torch, problem, prec, tols, kmaxs)
    Ym, infos = _run_mixed(sg, torch, problem, prec, tols, kmaxs)
    print([(i["k_used"], i["converged"], i["breakdown"]) for i in infos], flush=True)
    assert torch.equal(Ya, Ym)
    assert infos[4]["k_used"] == 0 and infos[4]["breakdown"] == 1
    assert infos[5]["k_used"] == 40 and infos[5]["converged"] == 0
    A = problem[3]
    bound = 1e-10 if prec == 0 else 1e-6
    for r in (0, 2, 4):
        exact = matfunc.sgn_spectral_apply(A, problem[6][r])
        assert _rel(Ym[r].cpu().numpy(), exact) < bound


def test_session_equals_fresh_apply(env, problem):
    sg, torch = env
    X = problem[6]
    Ys, _ = _run_mixed(sg, torch, problem, 0, [1e-10] * 6, [600] * 6)
    for r in (0, 3):
        ctx = _ctx(sg, torch, problem, 0)
        try:
            y = torch.empty(X.shape[1], dtype=torch.complex128, device="cuda")
            sg.sgn_apply(ctx, _dev(torch, X[r]), y, 1e-10, 600)
            assert torch.equal(y, Ys[r])
        finally:
            sg.sgn_destroy(ctx)


def test_session_admission_and_errors(env, problem):
    sg, torch = env
    X = problem[6]
    ctx = _ctx(sg, torch, problem, 0)
    try:
        ses = sg.Session(ctx, 2, 100)
        xs = [_dev(torch, X[r]) for r in range(3)]
        ys = [torch.empty_like(x) for x in xs]
        a = ses.submit(xs[0], ys[0], 1e-9, 100)
        b = ses.submit(xs[1], ys[1], 1e-9, 100)
        assert a is not None and b is not None and ses.active() == 2
        assert ses.submit(xs[2], ys[2], 1e-9, 100) is None  # no free slot
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_deflate(ctx, 4)  # the Schur pair is held by the session
        assert e.value.status == sg.SGN_ESTATE
        with pytest.raises(sg.SgnError):
            ses.poll(12345)
        while ses.active():
            ses.step(50)
        assert ses.poll(a) is not None and ses.poll(b) is not None
        bad = xs[2].clone()
        bad[5] = float("nan")
        with pytest.raises(sg.SgnError) as e:
            ses.submit(bad, ys[2], 1e-9, 100)
        assert e.value.status == sg.SGN_EINVAL
        with pytest.raises(sg.SgnError):
            ses.submit(xs[2], ys[2], 1e-9, 101)  # above the session's kmax
        assert ses.active() == 0
        ses.destroy()
        sg.sgn_deflate(ctx, 4)  # allowed again once the session is gone
    finally:
        sg.sgn_destroy(ctx)
