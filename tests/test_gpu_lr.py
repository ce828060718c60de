"""LR-deflation through the C ABI (the LR-deflation subsection): fixed-k
parity with the oracle's algorithm, the exact critical components, the k = 0
case, the device setup (left and right eigenvectors) against the oracle's
eigenvalues and relations, mixed precision, the overlap operator, batched
applies and serving sessions on an LR pair, and the import checks."""
import os

import numpy as np
import pytest

import synth
from oracle import deflation, lr, matfunc, overlap, wilson

pytestmark = pytest.mark.gpu

M_W = -1.6
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


@pytest.fixture(scope="module")
def case():
    dims, mu, m = (4, 4, 4, 4), 0.3, 8
    links = synth.random_links(dims, 93)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    R, L, lam = lr.lr_pair_from_dense(A, m)
    Sgn = matfunc.sgn_spectral(A)
    X = np.stack([synth.gaussian_source(dims, 9300 + r) for r in range(2)])
    return dims, mu, links, A, R, L, lam, Sgn, X


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _lr_ctx(sg, torch, case, prec=0):
    dims, mu, links, A, R, L, lam, Sgn, X = case
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_set_precision(ctx, prec)
    sg.sgn_deflate_lr_import(ctx, torch.from_numpy(R).cuda(), torch.from_numpy(L).cuda(), lam)
    assert sg.sgn_deflation_mode(ctx) == sg.SGN_DEFL_LR and sg.sgn_deflation_size(ctx) == R.shape[1]
    return ctx


def test_lr_fixed_k_matches_oracle(env, case):
    sg, torch = env
    A, R, L, lam, X = case[3], case[4], case[5], case[6], case[8]
    ctx = _lr_ctx(sg, torch, case)
    try:
        for k in (10, 60):
            x = torch.from_numpy(X[0]).cuda()
            y = torch.empty_like(x)
            sg.sgn_apply_fixed(ctx, x, y, k)
            ref = lr.sgn_lr_deflated(A, X[0], k, R, L, lam)
            print("k", k, _rel(y.cpu().numpy(), ref), flush=True)
            assert _rel(y.cpu().numpy(), ref) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def test_lr_converged_and_critical_components_exact(env, case):
    sg, torch = env
    R, L, lam, Sgn, X = case[4], case[5], case[6], case[7], case[8]
    ctx = _lr_ctx(sg, torch, case)
    try:
        x = torch.from_numpy(X[1]).cuda()
        y = torch.empty_like(x)
        assert sg.sgn_apply(ctx, x, y, 1e-11, 600) == sg.SGN_OK
        exact = Sgn @ X[1]
        got = y.cpu().numpy()
        assert _rel(got, exact) < 1e-10
        # L^dag y = sgn(Lambda) L^dag x, exactly in the method
        crit = L.conj().T @ got - matfunc.sgn_scalar(lam) * (L.conj().T @ X[1])
        assert np.abs(crit).max() < 1e-11 * np.linalg.norm(X[1])
        # the overlap operator on the LR pair
        yo = torch.empty_like(x)
        assert sg.sgn_overlap_apply(ctx, x, yo, 1e-11, 600) == sg.SGN_OK
        g5 = overlap.gamma5_vector(X.shape[1] // 12)
        assert _rel(yo.cpu().numpy(), X[1] + g5 * exact) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def test_lr_source_in_span_r_exact(env, case):
    sg, torch = env
    R, lam, Sgn = case[4], case[6], case[7]
    ctx = _lr_ctx(sg, torch, case)
    try:
        a = np.arange(1, R.shape[1] + 1) * (0.5 + 1.0j)
        xs = R @ a
        x = torch.from_numpy(xs).cuda()
        y = torch.empty_like(x)
        sg.sgn_apply(ctx, x, y, 1e-10, 100)
        info = sg.sgn_last_info(ctx)
        assert info["k_used"] == 0 and info["breakdown"] == 1
        assert _rel(y.cpu().numpy(), Sgn @ xs) < 1e-12
    finally:
        sg.sgn_destroy(ctx)


def test_lr_mixed_precision(env, case):
    sg, torch = env
    Sgn, X = case[7], case[8]
    ctx = _lr_ctx(sg, torch, case, prec=1)
    try:
        x = torch.from_numpy(X[0]).cuda()
        y = torch.empty_like(x)
        assert sg.sgn_apply(ctx, x, y, 1e-7, 600) == sg.SGN_OK
        assert _rel(y.cpu().numpy(), Sgn @ X[0]) < 1e-6
    finally:
        sg.sgn_destroy(ctx)


def test_lr_device_setup(env, case):
    sg, torch = env
    dims, mu, links, A, R, L, lam = case[:7]
    Sgn, X = case[7], case[8]
    m = R.shape[1]
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_deflate_lr(ctx, m)
        assert sg.sgn_deflation_mode(ctx) == sg.SGN_DEFL_LR
        Rd, Ld, lamd = sg.sgn_deflate_lr_export(ctx)
        Rd, Ld = Rd.cpu().numpy(), Ld.cpu().numpy()
        # the same critical eigenvalues as the dense oracle (as sets)
        for z in lam:
            assert np.min(np.abs(lamd - z)) < 1e-10 * max(1.0, abs(z))
        assert np.abs(Ld.conj().T @ Rd - np.eye(m)).max() < 1e-9
        assert np.linalg.norm(A @ Rd - Rd * lamd) / np.linalg.norm(Rd) < 1e-9
        assert np.linalg.norm(Ld.conj().T @ A - lamd[:, None] * Ld.conj().T) / np.linalg.norm(Ld) < 1e-9
        # the oblique projector does not depend on the eigenvector scaling
        assert np.abs(Rd @ Ld.conj().T - R @ L.conj().T).max() < 1e-9
        x = torch.from_numpy(X[0]).cuda()
        y = torch.empty_like(x)
        assert sg.sgn_apply(ctx, x, y, 1e-11, 600) == sg.SGN_OK
        assert _rel(y.cpu().numpy(), Sgn @ X[0]) < 1e-9
        stats = sg.sgn_deflate_stats(ctx)
        assert stats["residual"] < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def test_lr_batched_and_session(env, case):
    # batched at fixed k: bitwise the single-source result; a session: the
    # same result alone and among other requests, near the exact sign
    sg, torch = env
    X, Sgn = case[8], case[7]
    ctx = _lr_ctx(sg, torch, case)
    try:
        Xd = torch.from_numpy(X).cuda()
        Y = torch.empty_like(Xd)
        sg.sgn_apply_batched_fixed(ctx, Xd, Y, 60)
        for r in range(X.shape[0]):
            y = torch.empty_like(Xd[r])
            sg.sgn_apply_fixed(ctx, Xd[r].contiguous(), y, 60)
            assert torch.equal(y, Y[r])

        def run_session(rows, slots):
            ses = sg.Session(ctx, slots, 500)
            out = {}
            try:
                hs = {}
                for r in rows:
                    out[r] = torch.empty_like(Xd[r])
                    hs[ses.submit(Xd[r].contiguous(), out[r], 1e-11, 500)] = r
                    ses.step(7)  # the next request joins a running one
                while ses.active():
                    ses.step(5)
                for h in hs:
                    assert ses.poll(h)["converged"] == 1
            finally:
                ses.destroy()
            return out

        alone = run_session([1], 1)
        mixed = run_session([0, 1], 2)
        assert torch.equal(alone[1], mixed[1])
        assert _rel(mixed[1].cpu().numpy(), Sgn @ X[1]) < 1e-9
        st, _ = sg.sgn_overlap_apply_batched(ctx, Xd, Y, 1e-11, 500)
        assert st == sg.SGN_OK
    finally:
        sg.sgn_destroy(ctx)


def test_lr_import_checks_then_schur_again(env, case):
    sg, torch = env
    X = case[8]
    ctx = _lr_ctx(sg, torch, case)
    try:
        bad = torch.from_numpy(case[4]).cuda()
        with pytest.raises(sg.SgnError) as e:  # L^dag R != I
            sg.sgn_deflate_lr_import(ctx, bad, bad, case[6])
        assert e.value.status == sg.SGN_EINVAL
        assert sg.sgn_deflation_mode(ctx) == sg.SGN_DEFL_LR  # the failed import left the pair
        sg.sgn_deflate(ctx, 8)  # a Schur pair replaces the LR pair
        assert sg.sgn_deflation_mode(ctx) == sg.SGN_DEFL_SCHUR
        Xd = torch.from_numpy(X).cuda()
        Y = torch.empty_like(Xd)
        st, _ = sg.sgn_apply_batched(ctx, Xd, Y, 1e-10, 600)
        assert st == sg.SGN_OK
        assert _rel(Y[0].cpu().numpy(), case[7] @ X[0]) < 1e-8
        with pytest.raises(sg.SgnError):
            sg.sgn_deflate_lr_export(ctx)
    finally:
        sg.sgn_destroy(ctx)


def test_lr_6x6_field_vs_stored_exact(env):
    sg, torch = env
    path = os.path.join(GOLDEN, "c6_mu0.2.npy")
    if not os.path.exists(path):
        pytest.skip("stored exact result missing")
    dims, mu = (6, 6, 6, 6), 0.2
    exact = np.load(path, allow_pickle=False)
    ctx = sg.sgn_create(synth.random_links(dims, synth.GAUGE_SEED), dims, mu, M_W)
    try:
        sg.sgn_deflate_lr(ctx, 20)
        x = torch.from_numpy(synth.gaussian_source(dims, 1000)).cuda()
        y = torch.empty_like(x)
        assert sg.sgn_apply(ctx, x, y, 1e-11, 500) == sg.SGN_OK
        print("LR 6^4", sg.sgn_last_info(ctx), flush=True)
        assert _rel(y.cpu().numpy(), exact) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def test_lr_adjoint_matches_oracle_and_exact(env, case):
    # sgn(A)^dag x with the same LR pair, L and R exchanged, on A^dag = H_w(-mu)
    sg, torch = env
    A, R, L, lam, Sgn, X = case[3], case[4], case[5], case[6], case[7], case[8]
    ctx = _lr_ctx(sg, torch, case)
    try:
        x = torch.from_numpy(X[0]).cuda()
        y = torch.empty_like(x)
        for k in (10, 60):
            sg.sgn_apply_adjoint_fixed(ctx, x, y, k)
            ref = lr.sgn_lr_adjoint(A, X[0], k, R, L, lam)
            print("adjoint k", k, _rel(y.cpu().numpy(), ref), flush=True)
            assert _rel(y.cpu().numpy(), ref) < 1e-10
        assert sg.sgn_apply_adjoint(ctx, x, y, 1e-11, 600) == sg.SGN_OK
        ya = y.cpu().numpy()
        assert _rel(ya, Sgn.conj().T @ X[0]) < 1e-9
        # <w, sgn(A) x> = <sgn(A)^dag w, x>, both sides through the GPU
        w = torch.from_numpy(X[1]).cuda()
        sw = torch.empty_like(w)
        assert sg.sgn_apply(ctx, w, sw, 1e-11, 600) == sg.SGN_OK
        lhs = np.vdot(X[0], sw.cpu().numpy())
        rhs = np.vdot(ya, X[1])
        assert abs(lhs - rhs) < 1e-9 * np.linalg.norm(X[0]) * np.linalg.norm(X[1])
    finally:
        sg.sgn_destroy(ctx)


def test_lr_adjoint_leaves_the_forward_problem_and_ignores_graphs(env, case):
    sg, torch = env
    X = case[8]
    ctx = _lr_ctx(sg, torch, case)
    try:
        x = torch.from_numpy(X[0]).cuda()
        f0, f1, a0, a1 = (torch.empty_like(x) for _ in range(4))
        sg.sgn_apply_fixed(ctx, x, f0, 40)
        sg.sgn_apply_adjoint_fixed(ctx, x, a0, 40)
        sg.sgn_set_step_graphs(ctx, 8)  # captured steps hold the forward phases
        sg.sgn_apply_fixed(ctx, x, f1, 40)
        sg.sgn_apply_adjoint_fixed(ctx, x, a1, 40)
        assert torch.equal(a0, a1)
        sg.sgn_apply_fixed(ctx, x, a1, 40)
        assert torch.equal(f0, f1) and torch.equal(f0, a1)
        assert not torch.equal(f0, a0)
    finally:
        sg.sgn_destroy(ctx)


def test_adjoint_states(env, case):
    # a Schur pair is refused; no deflation runs the plain method on H_w(-mu)
    sg, torch = env
    dims, mu, links, A, R, L, lam, Sgn, X = case
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        x = torch.from_numpy(X[0]).cuda()
        y = torch.empty_like(x)
        assert sg.sgn_apply_adjoint(ctx, x, y, 1e-11, x.numel()) == sg.SGN_OK
        assert _rel(y.cpu().numpy(), Sgn.conj().T @ X[0]) < 1e-9
        Am = wilson.hw_matrix(links, dims, -mu, M_W).toarray()
        assert np.abs(Am - A.conj().T).max() < 1e-14  # the operator the adjoint runs on
        S, T, _, _ = deflation.critical_from_dense(A, 8)
        sg.sgn_deflate_import(ctx, torch.from_numpy(S).cuda(), T)
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_apply_adjoint(ctx, x, y, 1e-10, 300)
        assert e.value.status == sg.SGN_ESTATE
    finally:
        sg.sgn_destroy(ctx)


def test_lr_adjoint_mixed_precision(env, case):
    sg, torch = env
    Sgn, X = case[7], case[8]
    ctx = _lr_ctx(sg, torch, case, prec=1)
    try:
        x = torch.from_numpy(X[1]).cuda()
        y = torch.empty_like(x)
        assert sg.sgn_apply_adjoint(ctx, x, y, 1e-7, 600) == sg.SGN_OK
        assert _rel(y.cpu().numpy(), Sgn.conj().T @ X[1]) < 1e-6
    finally:
        sg.sgn_destroy(ctx)


def test_overlap_adjoint(env, case):
    # D_ov(mu)^dag x = x + sgn(H_w(mu))^dag gamma5 x against the dense oracle,
    # and <w, D_ov x> = <D_ov^dag w, x> with both sides on the GPU
    sg, torch = env
    A, X = case[3], case[8]
    Dov = overlap.overlap_dense(A)
    ctx = _lr_ctx(sg, torch, case)
    try:
        x = torch.from_numpy(X[0]).cuda()
        w = torch.from_numpy(X[1]).cuda()
        ya, yd = torch.empty_like(x), torch.empty_like(x)
        assert sg.sgn_overlap_apply_adjoint(ctx, w, ya, 1e-11, 600) == sg.SGN_OK
        assert _rel(ya.cpu().numpy(), Dov.conj().T @ X[1]) < 1e-9
        assert sg.sgn_overlap_apply(ctx, x, yd, 1e-11, 600) == sg.SGN_OK
        lhs = np.vdot(X[1], yd.cpu().numpy())
        rhs = np.vdot(ya.cpu().numpy(), X[0])
        assert abs(lhs - rhs) < 1e-9 * np.linalg.norm(X[0]) * np.linalg.norm(X[1])
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_overlap_apply_adjoint(ctx, x, x, 1e-10, 100)  # y aliases x
        assert e.value.status == sg.SGN_EINVAL
    finally:
        sg.sgn_destroy(ctx)


def test_lr_adjoint_batched(env, case):
    # at fixed k each source is bitwise its single-source adjoint; with a
    # tolerance every source is near the exact sgn(A)^dag x
    sg, torch = env
    Sgn, X = case[7], case[8]
    ctx = _lr_ctx(sg, torch, case)
    try:
        Xd = torch.from_numpy(X).cuda()
        Y = torch.empty_like(Xd)
        sg.sgn_apply_adjoint_batched_fixed(ctx, Xd, Y, 40)
        for r in range(X.shape[0]):
            y = torch.empty_like(Xd[r])
            sg.sgn_apply_adjoint_fixed(ctx, Xd[r].contiguous(), y, 40)
            assert torch.equal(y, Y[r])
        st, infos = sg.sgn_apply_adjoint_batched(ctx, Xd, Y, 1e-11, 600)
        assert st == sg.SGN_OK and all(i["converged"] for i in infos)
        for r in range(X.shape[0]):
            assert _rel(Y[r].cpu().numpy(), Sgn.conj().T @ X[r]) < 1e-9
        # the forward batched apply afterwards is unchanged
        Y2 = torch.empty_like(Xd)
        sg.sgn_apply_batched_fixed(ctx, Xd, Y2, 40)
        y = torch.empty_like(Xd[0])
        sg.sgn_apply_fixed(ctx, Xd[0].contiguous(), y, 40)
        assert torch.equal(y, Y2[0])
    finally:
        sg.sgn_destroy(ctx)
