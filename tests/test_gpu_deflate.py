"""GPU deflation setup (sgn_deflate) against the oracle's critical Schur pair."""
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


def _check_pair(A, S, T, lam_ref, m):
    # invariant subspace: A S = S T, S orthonormal, T upper triangular
    assert np.abs(S.conj().T @ S - np.eye(m)).max() < 1e-12
    assert np.abs(np.tril(T, -1)).max() == 0.0
    res = np.linalg.norm(A @ S - S @ T)
    assert res < 1e-10 * np.abs(lam_ref).max() + 1e-11
    got = np.sort(np.abs(np.diag(T).real))
    assert np.allclose(got, np.sort(np.abs(lam_ref.real)), atol=1e-10)


@pytest.mark.parametrize("degree", [0, 16])  # unfiltered; the default Chebyshev filter
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_deflate_small_matches_dense_oracle(env, mu, degree):
    sg, torch = env
    dims = (3, 3, 3, 4)
    links = synth.random_links(dims, 32)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    Ad = A.toarray()
    m = 12
    S0, T0, lam0, _ = deflation.critical_from_dense(Ad, m)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_set_deflation_filter(ctx, degree)
        sg.sgn_deflate(ctx, m)
        stats = sg.sgn_deflate_stats(ctx)
        print(stats, flush=True)
        assert stats["filter_degree"] == degree  # the filtered run converged (no fallback)
        S, T, ev = sg.sgn_deflate_export(ctx)
        S = S.cpu().numpy()
        _check_pair(A, S, T, lam0, m)
        # same invariant subspace as the oracle
        assert np.abs(S @ S.conj().T - S0 @ S0.conj().T).max() < 1e-9
    finally:
        sg.sgn_destroy(ctx)


def test_deflate_6x6_matches_arpack(env):
    # the default (filtered) setup against the oracle's ARPACK route
    sg, torch = env
    dims, mu, m = (6, 6, 6, 6), 0.2, 20
    links = synth.random_links(dims, synth.GAUGE_SEED)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_deflate(ctx, m)
        stats = sg.sgn_deflate_stats(ctx)
        print(stats, flush=True)
        assert stats["filter_degree"] > 0
        S, T, ev = sg.sgn_deflate_export(ctx)
        S = S.cpu().numpy()
        S0, T0, th0, _ = deflation.critical_from_arpack(A, m)
        _check_pair(A, S, T, np.diag(T0), m)
        assert stats["residual"] < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def test_deflation_krylov_size(env):
    # the eigensolver's basis size changes the iteration, not the result: a
    # narrow basis (about 2 nev), a wide one and the default all find the
    # oracle's critical subspace; a negative size is rejected.  (The smallest
    # basis, nev + 3, adds two vectors per restart and does not reach the
    # 1e-13 residual within its restart limit on this lattice.)
    sg, torch = env
    dims, mu, m = (3, 3, 3, 4), 0.2, 6
    links = synth.random_links(dims, 33)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    S0, T0, lam0, _ = deflation.critical_from_dense(A.toarray(), m)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_set_deflation_krylov(ctx, -1)
        assert e.value.status == sg.SGN_EINVAL
        seen = []
        for ncv in (32, 80, 0):
            sg.sgn_set_deflation_krylov(ctx, ncv)
            sg.sgn_deflate(ctx, m)
            stats = sg.sgn_deflate_stats(ctx)
            print("ncv", ncv, stats, flush=True)
            S, T, _ = sg.sgn_deflate_export(ctx)
            S = S.cpu().numpy()
            _check_pair(A, S, T, lam0, m)
            assert np.abs(S @ S.conj().T - S0 @ S0.conj().T).max() < 1e-9
            seen.append(stats["matvecs"])
        assert len(set(seen)) > 1  # the basis size took effect
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("degree", [8, 16, 24])
def test_filtered_deflation_4x4_mu05_matches_dense_oracle(env, degree):
    # mu = 0.5 (the serving fields' chemical potential): complex spectrum of
    # H_w^2; the filtered setup finds the oracle's critical subspace
    sg, torch = env
    dims, mu, m = (4, 4, 4, 4), 0.5, 20
    links = synth.random_links(dims, synth.GAUGE_SEED)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    S0, T0, lam0, _ = deflation.critical_from_dense(A.toarray(), m)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_set_deflation_filter(ctx, degree)
        sg.sgn_deflate(ctx, m)
        stats = sg.sgn_deflate_stats(ctx)
        print(degree, stats, flush=True)
        assert stats["filter_degree"] == degree and stats["residual"] < 1e-10
        lo, hi = stats["filter_interval"]
        assert 0.0 < lo < hi
        S, T, _ = sg.sgn_deflate_export(ctx)
        S = S.cpu().numpy()
        _check_pair(A, S, T, lam0, m)
        assert np.abs(S @ S.conj().T - S0 @ S0.conj().T).max() < 1e-9
    finally:
        sg.sgn_destroy(ctx)


def test_deflation_filter_arguments(env):
    sg, torch = env
    dims = (2, 2, 2, 4)
    ctx = sg.sgn_create(synth.random_links(dims, 3), dims, 0.3, M_W)
    try:
        for deg, cut in ((-1, 0.0), (201, 0.0), (8, 1.0), (8, -0.5)):
            with pytest.raises(sg.SgnError) as e:
                sg.sgn_set_deflation_filter(ctx, deg, cut)
            assert e.value.status == sg.SGN_EINVAL
        sg.sgn_set_deflation_filter(ctx, 8, 0.1)
        sg.sgn_set_deflation_filter(ctx, 0)
    finally:
        sg.sgn_destroy(ctx)
