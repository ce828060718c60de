"""Pins of the oracle's dense sign functions (Section 2, Eq. Roberts) and of
the Appendix A Sylvester recurrence."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import matfunc, sylvester, wilson

M_W = -1.6
RNG = np.random.default_rng(123)


def _rand(n, m=None):
    m = n if m is None else m
    return RNG.standard_normal((n, m)) + 1j * RNG.standard_normal((n, m))


def test_scalar_sign_is_sign_of_real_part():
    z = _rand(200, 1).ravel()
    assert np.allclose(matfunc.sgn_scalar(z), np.sign(z.real))
    assert np.allclose(matfunc.sgn_scalar(z) ** 2, 1)


@pytest.fixture(scope="module")
def hw_small():
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 21)
    return dims, U, wilson.hw_matrix(U, dims, 0.3, M_W).toarray()


def test_spectral_equals_roberts_on_hw(hw_small):
    _, _, H = hw_small
    S1 = matfunc.sgn_spectral(H)
    S2, it = matfunc.sgn_roberts(H)
    assert np.abs(S1 - S2).max() < 1e-12
    assert it < 20  # quadratic convergence


def test_sign_squares_to_identity_and_commutes(hw_small):
    _, _, H = hw_small
    S = matfunc.sgn_spectral(H)
    I = np.eye(H.shape[0])
    assert np.abs(S @ S - I).max() < 1e-12
    assert np.abs(S @ H - H @ S).max() < 1e-12


def test_sign_on_eigenvector(hw_small):
    _, _, H = hw_small
    lam, R = np.linalg.eig(H)
    for i in (0, 5, 77):
        y = matfunc.sgn_spectral_apply(H, R[:, i])
        assert np.allclose(y, np.sign(lam[i].real) * R[:, i], atol=1e-11)


def test_hermitian_routes_and_polar():
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 22)
    H0 = wilson.hw_matrix(U, dims, 0.0, M_W).toarray()
    x = synth.gaussian_source(dims, 1)
    Sh = matfunc.sgn_hermitian(H0)
    assert np.abs(Sh - matfunc.sgn_spectral(H0)).max() < 1e-12
    assert np.abs(Sh - matfunc.polar_factor(H0)).max() < 1e-12
    # sgn of a Hermitian matrix is unitary: |y| = |x|
    assert abs(np.linalg.norm(Sh @ x) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)


def test_polar_differs_at_nonzero_mu(hw_small):
    _, _, H = hw_small
    S = matfunc.sgn_spectral(H)
    P = matfunc.polar_factor(H)
    assert np.abs(S - P).max() > 1e-3
    assert np.abs(P @ P - np.eye(H.shape[0])).max() > 1e-3


def test_roberts_triangular_2x2_closed_form():
    # f(T)_12 for upper triangular T is the divided difference t12 (s1 - s2)/(t11 - t22)
    t11, t22, t12 = 0.7 + 0.2j, -0.4 + 1.1j, 0.3 - 0.5j
    T = np.array([[t11, t12], [0, t22]])
    F, _ = matfunc.sgn_roberts(T)
    s1, s2 = np.sign(t11.real), np.sign(t22.real)
    expect = np.array([[s1, t12 * (s1 - s2) / (t11 - t22)], [0, s2]])
    assert np.allclose(F, expect, atol=1e-14)


def test_roberts_keeps_triangular():
    T = np.triu(_rand(12))
    F, _ = matfunc.sgn_roberts(T)
    assert np.abs(np.tril(F, -1)).max() < 1e-14
    assert np.allclose(np.diag(F), np.sign(np.diag(T).real))


def test_spectral_refuses_imaginary_axis():
    with pytest.raises(ValueError):
        matfunc.sgn_spectral(np.diag([1.0, 2j, -3.0]))


def _hessenberg(n):
    # subdiagonal of the size of the diagonal spread, as in an Arnoldi Hessenberg
    H = np.triu(_rand(n), -1) + 3 * np.eye(n)
    H[np.arange(1, n), np.arange(n - 1)] = 3 + RNG.random(n - 1)
    return H


@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (4, 12), (6, 16)])
def test_sylvester_recurrence_matches_library(m, n):
    T = np.triu(_rand(m)) + 2 * np.eye(m)
    H = _hessenberg(n)
    C = _rand(m, n)
    Y = sylvester.solve_sylvester_hessenberg(T, H, C)
    Y_lib = sla.solve_sylvester(T, -H, C)
    assert np.abs(Y - Y_lib).max() < 1e-10 * max(1, np.abs(Y_lib).max())
    assert np.linalg.norm(T @ Y - Y @ H - C) < 1e-10 * np.linalg.norm(C)


def test_sylvester_recurrence_on_arnoldi_hessenberg():
    # the regime the method uses: H_k from an Arnoldi run on H_w, T from its Schur pair
    from oracle import arnoldi, deflation
    dims = (2, 2, 2, 4)
    A = wilson.hw_matrix(synth.random_links(dims, 41), dims, 0.3, M_W)
    S, T, lam, low = deflation.critical_from_dense(A.toarray(), 5)
    st = arnoldi.modified_arnoldi(lambda v: A @ v, synth.gaussian_source(dims, 4), S, 40)
    Hk = st.Hbar[:40, :40]
    C = matfunc.sgn_spectral(T) @ st.X - st.X @ matfunc.sgn_spectral(Hk)
    Y = sylvester.solve_sylvester_hessenberg(T, Hk, C)
    Y_lib = sla.solve_sylvester(T, -Hk, C)
    assert np.abs(Y - Y_lib).max() < 1e-10 * np.abs(Y_lib).max()


def test_sylvester_single_row_is_a_linear_solve():
    # m = 1: y (t I - H) = c
    H = _hessenberg(9)
    t = 0.3 - 0.8j
    c = _rand(1, 9)
    Y = sylvester.solve_sylvester_hessenberg(np.array([[t]]), H, c)
    y_ref = np.linalg.solve((t * np.eye(9) - H).T, c.ravel())
    assert np.allclose(Y.ravel(), y_ref, atol=1e-12)


def test_sylvester_gives_block_of_composite_sign():
    # Eq. (eq:f_H): the (1,2) block of sgn([[T, X], [0, Hk]]) solves Eq. (SylvEq)
    m, k = 3, 10
    T = np.triu(_rand(m)) + np.diag([1.5, -1.2, 2.0])
    Hk = _hessenberg(k)
    Hk[np.diag_indices(k)] = np.where(np.arange(k) % 2, 3.0, -3.0)
    X = _rand(m, k)
    Hc = np.block([[T, X], [np.zeros((k, m)), Hk]])
    F = matfunc.sgn_spectral(Hc)
    fT = matfunc.sgn_spectral(T)
    fH = matfunc.sgn_spectral(Hk)
    assert np.abs(F[:m, :m] - fT).max() < 1e-10
    assert np.abs(F[m:, m:] - fH).max() < 1e-10
    assert np.abs(F[m:, :m]).max() < 1e-10
    Y = sylvester.solve_sylvester_hessenberg(T, Hk, fT @ X - X @ fH)
    assert np.abs(F[:m, m:] - Y).max() < 1e-9
