"""Pins of the oracle's modified Arnoldi approximation and deflation basis."""
import numpy as np
import pytest

import synth
from oracle import arnoldi, deflation, matfunc, wilson

M_W = -1.6


@pytest.fixture(scope="module")
def tiny():
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 31)
    A = wilson.hw_matrix(U, dims, 0.3, M_W)
    Ad = A.toarray()
    x = synth.gaussian_source(dims, 1000)
    y = matfunc.sgn_spectral_apply(Ad, x)
    return dims, A, Ad, x, y


@pytest.fixture(scope="module")
def small():
    dims = (3, 3, 3, 4)
    U = synth.random_links(dims, 32)
    A = wilson.hw_matrix(U, dims, 0.3, M_W)
    Ad = A.toarray()
    x = synth.gaussian_source(dims, 1001)
    y = matfunc.sgn_spectral_apply(Ad, x)
    S, T, lam, low = deflation.critical_from_dense(Ad, 12)
    return dims, A, Ad, x, y, S, T


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_full_grade_is_exact_without_deflation(tiny):
    # Eq. (interp): at k = grade(x) the Krylov approximation reproduces sgn(A)x
    _, A, Ad, x, y = tiny
    st = arnoldi.modified_arnoldi(lambda v: A @ v, x, None, Ad.shape[0])
    assert _rel(arnoldi.approx_definition(None, None, st), y) < 1e-11


def test_full_grade_is_exact_with_deflation(tiny):
    _, A, Ad, x, y = tiny
    S, T, lam, low = deflation.critical_from_dense(Ad, 8)
    st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, Ad.shape[0] - 8)
    assert _rel(arnoldi.approx_definition(S, T, st), y) < 1e-11
    assert _rel(arnoldi.approx_paper(S, T, st), y) < 1e-9


def test_source_inside_schur_space_is_exact_at_k0(tiny):
    _, A, Ad, x, y = tiny
    S, T, lam, low = deflation.critical_from_dense(Ad, 6)
    xs = S @ np.arange(1, 7)
    st = arnoldi.modified_arnoldi(lambda v: A @ v, xs, S, 10)
    # two Gram-Schmidt passes leave rounding noise of x's size at most
    assert st.beta < 1e-12 * np.linalg.norm(xs)
    ys = arnoldi.approx_definition(S, T, arnoldi.modified_arnoldi(lambda v: A @ v, xs, S, 0))
    assert _rel(ys, matfunc.sgn_spectral_apply(Ad, xs)) < 1e-11


def test_modified_arnoldi_relation_and_orthonormality(small):
    # Eq. (eq:modArnoldi): A V_k = S X + V_{k+1} Hbar, and Q = (S V) orthonormal
    _, A, Ad, x, y, S, T = small
    k = 60
    st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, k)
    lhs = A @ st.V[:, :k]
    rhs = S @ st.X + st.V @ st.Hbar
    assert np.linalg.norm(lhs - rhs) < 1e-13 * np.linalg.norm(lhs)
    Q = np.concatenate([S, st.V], axis=1)
    assert np.abs(Q.conj().T @ Q - np.eye(Q.shape[1])).max() < 1e-13
    # X = S^dag A V_k and H_k = V_k^dag A V_k (Eq. eq:newHQHQ)
    assert np.abs(S.conj().T @ lhs - st.X).max() < 1e-12
    assert np.abs(st.V[:, :k].conj().T @ lhs - st.Hbar[:k]).max() < 1e-12


def test_definition_equals_paper_route(small):
    _, A, Ad, x, y, S, T = small
    for k in (20, 50, 90):
        st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, k)
        assert _rel(arnoldi.approx_paper(S, T, st), arnoldi.approx_definition(S, T, st)) < 1e-10


def test_error_decreases_to_exact(small):
    # Results section: the error falls with k down to rounding level
    _, A, Ad, x, y, S, T = small
    st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, 300)
    errs = []
    for k in (40, 80, 160, 300):
        sub = arnoldi.ArnoldiState(st.V[:, :k + 1], st.Hbar[:k + 1, :k], st.X[:, :k],
                                   st.beta, st.c0, k, False)
        errs.append(_rel(arnoldi.approx_definition(S, T, sub), y))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-10


def test_deflation_helps(small):
    _, A, Ad, x, y, S, T = small
    k = 60
    e0 = _rel(arnoldi.sgn_arnoldi(A, x, k), y)
    e12 = _rel(arnoldi.sgn_arnoldi(A, x, k, S, T), y)
    assert e12 < e0


def test_projection_is_a_lower_bound(small):
    # y_proj = Q Q^dag y is the best approximation in the composite space
    _, A, Ad, x, y, S, T = small
    k = 60
    st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, k)
    Q = np.concatenate([S, st.V[:, :k]], axis=1)
    e_proj = _rel(Q @ (Q.conj().T @ y), y)
    e_arn = _rel(arnoldi.approx_definition(S, T, st), y)
    assert e_proj <= e_arn * (1 + 1e-9)


def test_hermitian_case_is_lanczos():
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 33)
    A = wilson.hw_matrix(U, dims, 0.0, M_W)
    Ad = A.toarray()
    S, T, lam, low = deflation.critical_from_dense(Ad, 6)
    assert np.abs(np.triu(T, 1)).max() < 1e-12  # T diagonal
    assert np.abs(np.diag(T).imag).max() < 1e-12
    x = synth.gaussian_source(dims, 3)
    st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, 40)
    Hk = st.Hbar[:40, :40]
    assert np.abs(np.triu(Hk, 2)).max() < 1e-12  # tridiagonal
    assert np.abs(Hk - Hk.conj().T).max() < 1e-12
    assert np.abs(st.X).max() < 1e-12  # Schur space decouples


def test_dense_deflation_basis(small):
    _, A, Ad, x, y, S, T = small
    lam = np.linalg.eigvals(Ad)
    order = np.sort(np.abs(lam.real))
    assert np.allclose(np.sort(np.abs(np.diag(T).real)), order[:12])
    assert deflation.schur_residual(Ad, S, T) < 1e-12
    assert np.abs(S.conj().T @ S - np.eye(12)).max() < 1e-13
    assert np.abs(np.tril(T, -1)).max() == 0.0


def test_arpack_deflation_matches_dense(small):
    _, A, Ad, x, y, S, T = small
    S2, T2, th, low = deflation.critical_from_arpack(A, 12, extra=8)
    assert np.allclose(np.sort(np.abs(np.diag(T2).real)), np.sort(np.abs(np.diag(T).real)), atol=1e-10)
    assert deflation.schur_residual(A, S2, T2) < 1e-11
    # same invariant subspace: projectors agree
    P1 = S @ S.conj().T
    P2 = S2 @ S2.conj().T
    assert np.abs(P1 - P2).max() < 1e-9
