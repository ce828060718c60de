"""Overlap operator D_ov(mu) x = x + gamma5 sgn(H_w(mu)) x (Section 2, Eq.
Dov) through the C ABI: against the dense oracle, against x + gamma5 of the
sign apply (bitwise), the Ginsparg-Wilson relation (Eq. GW:eq) on vectors,
the batched form, the stored exact 6^4 result, and the argument checks."""
import os

import numpy as np
import pytest

import synth
from oracle import deflation, overlap, wilson

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
def field():
    dims, mu = (4, 4, 4, 4), 0.3
    links = synth.random_links(dims, 91)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    S, T, _, _ = deflation.critical_from_dense(A, 8)
    X = np.stack([synth.gaussian_source(dims, 9100 + r) for r in range(4)])
    Dov = overlap.overlap_dense(A)  # one dense sign for every check below
    return dims, mu, links, Dov, S, T, X


def _ctx(sg, torch, field):
    dims, mu, links, _, S, T, X = field
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_deflate_import(ctx, torch.from_numpy(S).cuda(), T)
    return ctx


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_overlap_matches_oracle_and_sign_apply(env, field):
    sg, torch = env
    X = field[6]
    g5 = torch.from_numpy(overlap.gamma5_vector(X.shape[1] // 12)).cuda()
    c1, c2 = _ctx(sg, torch, field), _ctx(sg, torch, field)
    try:
        x = torch.from_numpy(X[0]).cuda()
        yo, ys = torch.empty_like(x), torch.empty_like(x)
        assert sg.sgn_overlap_apply(c1, x, yo, 1e-11, 500) == sg.SGN_OK
        assert sg.sgn_apply(c2, x, ys, 1e-11, 500) == sg.SGN_OK
        assert sg.sgn_last_info(c1)["k_used"] == sg.sgn_last_info(c2)["k_used"]
        # same sign arithmetic, then one IEEE add per entry
        assert torch.equal(yo, x + g5 * ys)
        exact = field[3] @ X[0]
        assert _rel(yo.cpu().numpy(), exact) < 1e-10
    finally:
        sg.sgn_destroy(c1)
        sg.sgn_destroy(c2)


def test_ginsparg_wilson_on_vectors(env, field):
    # {D, g5} x = D g5 D x, with every D applied on the GPU
    sg, torch = env
    X = field[6]
    g5 = torch.from_numpy(overlap.gamma5_vector(X.shape[1] // 12)).cuda()
    ctx = _ctx(sg, torch, field)
    try:
        x = torch.from_numpy(X[1]).cuda()

        def D(v):
            out = torch.empty_like(v)
            assert sg.sgn_overlap_apply(ctx, v.contiguous(), out, 1e-12, 600) == sg.SGN_OK
            return out

        dx = D(x)
        lhs = D(g5 * dx)
        rhs = g5 * dx + D(g5 * x)
        defect = float((lhs - rhs).norm() / x.norm())
        print("GW defect", defect, flush=True)
        assert defect < 1e-9
    finally:
        sg.sgn_destroy(ctx)


def test_overlap_batched(env, field):
    sg, torch = env
    X = field[6]
    ctx = _ctx(sg, torch, field)
    try:
        Xd = torch.from_numpy(X).cuda()
        Y = torch.empty_like(Xd)
        st, infos = sg.sgn_overlap_apply_batched(ctx, Xd, Y, 1e-11, 500)
        assert st == sg.SGN_OK and all(i["converged"] for i in infos)
        for r in range(X.shape[0]):
            exact = field[3] @ X[r]
            assert _rel(Y[r].cpu().numpy(), exact) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def test_overlap_argument_checks(env, field):
    sg, torch = env
    X = field[6]
    ctx = _ctx(sg, torch, field)
    try:
        x = torch.from_numpy(X[0]).cuda()
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_overlap_apply(ctx, x, x, 1e-10, 100)  # y aliases x
        assert e.value.status == sg.SGN_EINVAL
        buf = torch.from_numpy(np.concatenate([X[0], X[1], X[2]])).cuda()
        n = X.shape[1]
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_overlap_apply_batched(ctx, buf[: 2 * n], buf[n:], 1e-10, 100)  # overlapping ranges
        assert e.value.status == sg.SGN_EINVAL
        bad = x.clone()
        bad[3] = float("nan")
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_overlap_apply(ctx, bad, torch.empty_like(x), 1e-10, 100)
        assert e.value.status == sg.SGN_EINVAL
    finally:
        sg.sgn_destroy(ctx)


def test_overlap_6x6_field_vs_stored_exact(env):
    sg, torch = env
    path = os.path.join(GOLDEN, "c6_mu0.2.npy")
    if not os.path.exists(path):
        pytest.skip("stored exact result missing")
    dims, mu = (6, 6, 6, 6), 0.2
    exact_sign = np.load(path, allow_pickle=False)
    x = synth.gaussian_source(dims, 1000)
    exact = x + overlap.gamma5_vector(x.size // 12) * exact_sign
    ctx = sg.sgn_create(synth.random_links(dims, synth.GAUGE_SEED), dims, mu, M_W)
    try:
        sg.sgn_deflate(ctx, 20)
        xd = torch.from_numpy(x).cuda()
        y = torch.empty_like(xd)
        assert sg.sgn_overlap_apply(ctx, xd, y, 1e-11, 500) == sg.SGN_OK
        assert _rel(y.cpu().numpy(), exact) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("mass", [0.2, 2.0])
def test_massive_overlap_solve(env, field, mass):
    # D(m) x = b by GMRES over GPU sign applies, against the oracle's dense
    # solve; m = 2 is 2 times the identity (one outer step)
    sg, torch = env
    dims, mu, links, _, S, T, X = field
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    ref = overlap.massive_overlap_solve(A, X[2], mass)
    ctx = _ctx(sg, torch, field)
    try:
        b = torch.from_numpy(X[2]).cuda()
        x = torch.empty_like(b)
        st, it, res = sg.sgn_overlap_solve(ctx, b, x, mass, 1e-9, max_iter=300, restart=40, inner_tol=1e-12,
                                           inner_kmax=600)
        print("overlap solve", mass, st, it, res, flush=True)
        assert st == sg.SGN_OK and res <= 1e-9
        assert _rel(x.cpu().numpy(), ref) < 1e-7
        if mass == 2.0:
            assert it == 1
        # the residual through the GPU operator: D(m) x = (1 - m/2) D_ov x + m x
        dx = torch.empty_like(x)
        assert sg.sgn_overlap_apply(ctx, x, dx, 1e-12, 600) == sg.SGN_OK
        r = (1 - mass / 2) * dx + mass * x - b
        assert float(r.norm() / b.norm()) < 1e-8
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_overlap_solve(ctx, b, b, mass, 1e-9)  # x aliases b
        assert e.value.status == sg.SGN_EINVAL
    finally:
        sg.sgn_destroy(ctx)


def test_massive_overlap_solve_mixed_precision(env, field):
    sg, torch = env
    dims, mu, links, _, S, T, X = field
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    ref = overlap.massive_overlap_solve(A, X[3], 0.3)
    ctx = _ctx(sg, torch, field)
    try:
        sg.sgn_set_precision(ctx, sg.SGN_PREC_MIXED)
        b = torch.from_numpy(X[3]).cuda()
        x = torch.empty_like(b)
        # inner_tol a decade above the FP32 floor of the inner applies (about
        # 1.4e-7 on this lattice), the outer tolerance a decade above that
        st, it, res = sg.sgn_overlap_solve(ctx, b, x, 0.3, 1e-4, max_iter=300, restart=40, inner_tol=1e-6,
                                           inner_kmax=600)
        print("mixed overlap solve", st, it, res, flush=True)
        assert st == sg.SGN_OK and res <= 1e-4
        assert _rel(x.cpu().numpy(), ref) < 1e-3
    finally:
        sg.sgn_destroy(ctx)
