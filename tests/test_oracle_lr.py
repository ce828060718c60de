"""Pins of the oracle's LR-deflation (the LR-deflation subsection): the
eigenvector relations and biorthonormality (Eqs. Rev, Lev), the exact
extraction of the critical components for every k, the k = 0 result for x in
span R, the full-grade limit, convergence in k, and the relation between the
left eigenvectors and H_w(-mu) = H_w(mu)^dag on which the device setup rests."""
import numpy as np
import pytest

import synth
from oracle import lr, matfunc, wilson

M_W = -1.6
M = 8


@pytest.fixture(scope="module")
def case():
    dims, mu = (2, 2, 2, 4), 0.3
    U = synth.random_links(dims, 41)
    A = wilson.hw_matrix(U, dims, mu, M_W).toarray()
    Am = wilson.hw_matrix(U, dims, -mu, M_W).toarray()
    R, L, lam = lr.lr_pair_from_dense(A, M)
    x = synth.gaussian_source(dims, 4100)
    exact = matfunc.sgn_spectral_apply(A, x)
    return A, Am, R, L, lam, x, exact


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_eigen_relations_and_biorthonormality(case):
    A, _, R, L, lam, _, _ = case
    assert np.abs(L.conj().T @ R - np.eye(M)).max() < 1e-12
    assert np.linalg.norm(A @ R - R * lam) / np.linalg.norm(A) < 1e-12
    assert np.linalg.norm(L.conj().T @ A - lam[:, None] * L.conj().T) / np.linalg.norm(A) < 1e-12
    # the selection is the critical one: smallest |Re lambda| of the whole spectrum
    allre = np.sort(np.abs(np.linalg.eigvals(A).real))
    assert np.isclose(np.max(np.abs(lam.real)), allre[M - 1])


def test_left_vectors_are_right_vectors_of_minus_mu(case):
    # H_w(mu)^dag = H_w(-mu): a left eigenvector of H_w(mu) for lambda is a
    # right eigenvector of H_w(-mu) for conj(lambda)
    A, Am, _, L, lam, _, _ = case
    assert np.allclose(Am, A.conj().T, atol=1e-14)
    assert np.linalg.norm(Am @ L - L * lam.conj()) / np.linalg.norm(L) < 1e-11


@pytest.mark.parametrize("k", [0, 5, 40])
def test_critical_components_exact_for_every_k(case, k):
    # L^dag y = sgn(Lambda) L^dag x = L^dag sgn(A) x, independently of k
    A, _, R, L, lam, x, exact = case
    y = lr.sgn_lr_deflated(A, x, k, R, L, lam)
    assert np.abs(L.conj().T @ y - L.conj().T @ exact).max() < 1e-10 * np.linalg.norm(x)


def test_source_in_span_r_is_exact_at_k0(case):
    A, _, R, L, lam, _, _ = case
    a = np.arange(1, M + 1) * (1.0 - 0.5j)
    x = R @ a
    y = lr.sgn_lr_deflated(A, x, 0, R, L, lam)
    assert _rel(y, matfunc.sgn_spectral_apply(A, x)) < 1e-12


def test_full_grade_is_exact_and_error_decreases(case):
    A, _, R, L, lam, x, exact = case
    errs = [_rel(lr.sgn_lr_deflated(A, x, k, R, L, lam), exact) for k in (10, 40, 120)]
    assert errs[0] > errs[1] > errs[2]
    n = A.shape[0] - M  # K_k(A, x_-) lies in the complementary invariant subspace
    assert _rel(lr.sgn_lr_deflated(A, x, n, R, L, lam), exact) < 1e-10


def test_dropping_the_projection_is_detected(case):
    # a plausible mistake: Arnoldi on x instead of x_- double-counts the
    # critical part; the critical components then differ from the exact ones
    A, _, R, L, lam, x, exact = case
    c = L.conj().T @ x
    from oracle.arnoldi import modified_arnoldi
    st = modified_arnoldi(lambda v: A @ v, x, None, 40)
    y = R @ (matfunc.sgn_scalar(lam) * c) + st.V[:, :40] @ (st.beta * matfunc.sgn_spectral(st.Hbar[:40, :40])[:, 0])
    assert np.abs(L.conj().T @ y - L.conj().T @ exact).max() > 1e-3 * np.linalg.norm(x)


def test_adjoint_full_grade_and_inner_products(case):
    # the adjoint by LR-deflation on A^dag (roles of L and R exchanged): at
    # full grade it is sgn(A)^dag x exactly, and <y, sgn(A) x> = <sgn(A)^dag y, x>
    A, Am, R, L, lam, x, exact = case
    N = A.shape[0]
    y = synth.gaussian_source((2, 2, 2, 4), 4101)
    Sgn = matfunc.sgn_spectral(A)
    ya = lr.sgn_lr_adjoint(A, y, N - M, R, L, lam)
    assert _rel(ya, Sgn.conj().T @ y) < 1e-10
    lhs = np.vdot(y, Sgn @ x)
    rhs = np.vdot(ya, x)
    assert abs(lhs - rhs) < 1e-10 * np.linalg.norm(x) * np.linalg.norm(y)
    # A^dag is H_w(-mu): the adjoint is the sign of the -mu operator
    assert _rel(ya, matfunc.sgn_spectral(Am) @ y) < 1e-10


def test_adjoint_critical_components_exact_for_every_k(case):
    # R^dag sgn(A)^dag y = sgn(conj Lambda) R^dag y exactly, whatever k
    A, _, R, L, lam, _, _ = case
    y = synth.gaussian_source((2, 2, 2, 4), 4102)
    for k in (0, 5, 40):
        ya = lr.sgn_lr_adjoint(A, y, k, R, L, lam)
        crit = R.conj().T @ ya - matfunc.sgn_scalar(np.conj(lam)) * (R.conj().T @ y)
        assert np.abs(crit).max() < 1e-11 * np.linalg.norm(y)
