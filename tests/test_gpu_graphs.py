"""Captured Arnoldi steps: replaying runs of steps as HIP graphs must give
bitwise the results of direct launches (same kernels, same arguments, step
index read on the device), on every replay, with other GPU work and
synchronisations between the applies; and stay near the exact sign."""
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
def small():
    dims, mu = (4, 4, 4, 4), 0.3
    links = synth.random_links(dims, 71)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    S, T, _, _ = deflation.critical_from_dense(A, 8)
    X = np.stack([synth.gaussian_source(dims, 7000 + r) for r in range(3)])
    return dims, mu, links, A, S, T, X


def _run(sg, torch, small, prec, steps, tol):
    dims, mu, links, A, S, T, X = small
    ctx = sg.sgn_create(links, dims, mu, M_W)
    out, infos = [], []
    try:
        sg.sgn_set_precision(ctx, prec)
        sg.sgn_deflate_import(ctx, torch.from_numpy(S.astype(np.complex128)).cuda(), T)
        sg.sgn_set_step_graphs(ctx, steps)
        for rep in range(2):
            for r in range(X.shape[0]):
                x = torch.from_numpy(X[r]).cuda()
                y = torch.empty_like(x)
                sg.sgn_apply(ctx, x, y, tol, 400)
                infos.append(sg.sgn_last_info(ctx))
                # other GPU work and a synchronisation between applies
                _ = (y * 2.0).abs().sum().item()
                out.append(y)
            y = torch.empty_like(x)
            sg.sgn_apply_fixed(ctx, torch.from_numpy(X[0]).cuda(), y, 90 + 2 * rep)
            out.append(y)
        torch.cuda.synchronize()
    finally:
        sg.sgn_destroy(ctx)
    return torch.stack(out), infos


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_bitwise_equal_direct(env, small, prec):
    sg, torch = env
    tol = 1e-10 if prec == 0 else 1e-7
    print("graphs vs direct, precision", prec, flush=True)
    Yd, infos_d = _run(sg, torch, small, prec, 0, tol)
    for steps in (2, 8, 16):
        print("  steps per graph", steps, flush=True)
        Yg, infos_g = _run(sg, torch, small, prec, steps, tol)
        assert torch.equal(Yg, Yd), steps
        assert [i["k_used"] for i in infos_g] == [i["k_used"] for i in infos_d]
        assert [i["n_matvec"] for i in infos_g] == [i["n_matvec"] for i in infos_d]
    A, X = small[3], small[6]
    bound = 1e-9 if prec == 0 else 1e-6
    exact = matfunc.sgn_spectral_apply(A, X[1])
    got = Yd[1].cpu().numpy()
    assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < bound


def test_graph_setting_errors_and_reuse(env, small):
    sg, torch = env
    dims, mu, links = small[0], small[1], small[2]
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        for bad in (1, -1, 65):
            with pytest.raises(sg.SgnError) as e:
                sg.sgn_set_step_graphs(ctx, bad)
            assert e.value.status == sg.SGN_EINVAL
        x = torch.from_numpy(small[6][0]).cuda()
        y1, y2, y3 = (torch.empty_like(x) for _ in range(3))
        sg.sgn_set_step_graphs(ctx, 8)
        sg.sgn_apply_fixed(ctx, x, y1, 64)
        sg.sgn_set_tuning(ctx, 4, 1)  # drops the graphs; new kernel instances
        sg.sgn_apply_fixed(ctx, x, y2, 64)
        sg.sgn_deflate(ctx, 4)  # new Schur pair: new workspace and graphs
        sg.sgn_apply_fixed(ctx, x, y3, 64)
        sg.sgn_set_step_graphs(ctx, 0)
        y4 = torch.empty_like(x)
        sg.sgn_apply_fixed(ctx, x, y4, 64)
        assert torch.equal(y1, y2)
        assert torch.equal(y3, y4)
        assert not torch.equal(y1, y3)
    finally:
        sg.sgn_destroy(ctx)


def _run_batched(sg, torch, small, prec, steps, tol):
    dims, mu, links, A, S, T, X = small
    ctx = sg.sgn_create(links, dims, mu, M_W)
    out, ks = [], []
    try:
        sg.sgn_set_precision(ctx, prec)
        sg.sgn_deflate_import(ctx, torch.from_numpy(S.astype(np.complex128)).cuda(), T)
        sg.sgn_set_step_graphs(ctx, steps)
        Xd = torch.from_numpy(X).cuda()
        for rep in range(2):
            Y = torch.empty_like(Xd)
            st, infos = sg.sgn_apply_batched(ctx, Xd, Y, tol, 400)
            assert st == sg.SGN_OK
            ks.append([i["k_used"] for i in infos])
            _ = (Y * 2.0).abs().sum().item()  # other GPU work and a synchronisation
            out.append(Y)
            # two of the three sources: another set of running slots
            Y2 = torch.empty_like(Xd[:2])
            sg.sgn_apply_batched_fixed(ctx, Xd[:2].contiguous(), Y2, 70 + 2 * rep)
            out.append(Y2)
        torch.cuda.synchronize()
    finally:
        sg.sgn_destroy(ctx)
    return torch.cat([o.reshape(-1) for o in out]), ks


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_graph_replay_bitwise_equal_direct(env, small, prec):
    sg, torch = env
    tol = 1e-10 if prec == 0 else 1e-7
    print("batched graphs vs direct, precision", prec, flush=True)
    Yd, kd = _run_batched(sg, torch, small, prec, 0, tol)
    for steps in (2, 8, 17):  # 17: runs of 16
        print("  steps per graph", steps, flush=True)
        Yg, kg = _run_batched(sg, torch, small, prec, steps, tol)
        assert torch.equal(Yg, Yd), steps
        assert kg == kd
