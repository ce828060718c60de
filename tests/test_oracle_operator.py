"""Pins of the oracle's operator layer: conventions, Eq. (Dw), free field.

Each test checks the oracle against something other than itself: algebraic
identities, symmetries that Eq. (Dw) implies, and an independent momentum-
space derivation (free field / pure gauge).
"""
import numpy as np
import pytest

import synth
from oracle import conventions, freefield, matfunc, wilson

M_W = -1.6


def test_gamma_algebra():
    g = conventions.gammas()
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * (a == b) * np.eye(4))
    g5 = conventions.gamma5()
    assert np.array_equal(g5, np.diag([1, 1, -1, -1]).astype(complex))
    for a in range(4):
        assert np.allclose(g5 @ g[a] + g[a] @ g5, 0)


def test_kappa():
    assert conventions.kappa(-1.6) == pytest.approx(1 / 4.8)
    assert conventions.kappa(0.0) == pytest.approx(1 / 8)
    with pytest.raises(ValueError):
        conventions.kappa(-4.0)


def test_links_are_su3():
    U = synth.random_links((2, 3, 2, 4), 7).reshape(-1, 3, 3)
    I = np.eye(3)
    assert np.abs(np.einsum("nij,nkj->nik", U, U.conj()) - I).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # deterministic in the seed
    assert np.array_equal(U, synth.random_links((2, 3, 2, 4), 7).reshape(-1, 3, 3))


@pytest.fixture(scope="module")
def small_field():
    dims = (2, 2, 2, 4)
    return dims, synth.random_links(dims, 11)


def test_hermitian_at_zero_mu(small_field):
    dims, U = small_field
    H = wilson.hw_matrix(U, dims, 0.0, M_W).toarray()
    assert np.abs(H - H.conj().T).max() == 0.0


def test_mu_adjoint_relation(small_field):
    # gamma5 D(mu) gamma5 = D(-mu)^dag  <=>  H(mu)^dag = H(-mu)
    dims, U = small_field
    H = wilson.hw_matrix(U, dims, 0.37, M_W).toarray()
    Hm = wilson.hw_matrix(U, dims, -0.37, M_W).toarray()
    assert np.abs(H.conj().T - Hm).max() < 1e-15
    assert np.abs(H - H.conj().T).max() > 0.1  # genuinely non-Hermitian


def test_sparsity_and_diagonal(small_field):
    dims, U = small_field
    V = int(np.prod(dims))
    D = wilson.dirac_wilson(U, dims, 0.3, M_W)
    Dd = D.toarray()
    for n in range(V):
        assert np.allclose(Dd[12 * n:12 * n + 12, 12 * n:12 * n + 12], np.eye(12))
    H = wilson.hw_matrix(U, dims, 0.3, M_W)
    assert H.shape == (12 * V, 12 * V)


def test_gauge_covariance():
    dims = (3, 2, 2, 4)
    U = synth.random_links(dims, 3)
    om = synth.random_su3_field(dims, 4)
    # U'_{n,nu} = Omega_n U_{n,nu} Omega_{n+nu}^dag
    V = int(np.prod(dims))
    Ur = U.reshape(V, 4, 3, 3)
    omr = om.reshape(V, 3, 3)
    Up = np.empty_like(Ur)
    lx, ly, lz, lt = dims
    n = np.arange(V)
    x, y, z, t = n % lx, (n // lx) % ly, (n // (lx * ly)) % lz, n // (lx * ly * lz)
    shifts = [((x + 1) % lx) + lx * (y + ly * (z + lz * t)),
              x + lx * (((y + 1) % ly) + ly * (z + lz * t)),
              x + lx * (y + ly * (((z + 1) % lz) + lz * t)),
              x + lx * (y + ly * (z + lz * ((t + 1) % lt)))]
    for nu in range(4):
        Up[:, nu] = omr @ Ur[:, nu] @ omr[shifts[nu]].conj().transpose(0, 2, 1)
    H = wilson.hw_matrix(U, dims, 0.3, M_W)
    Hp = wilson.hw_matrix(Up.reshape(U.shape), dims, 0.3, M_W)
    psi = synth.gaussian_source(dims, 5)
    lhs = Hp @ synth.gauge_transform_spinor(om, psi)
    rhs = synth.gauge_transform_spinor(om, H @ psi)
    assert np.linalg.norm(lhs - rhs) < 1e-13 * np.linalg.norm(rhs)


def _unit_links(dims):
    U = np.zeros(tuple(reversed(dims)) + (4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


@pytest.mark.parametrize("mu", [0.0, 0.3, -0.45])
def test_free_field_closed_form_matches_dense(mu):
    # independent derivation in momentum space vs the literal Eq. (Dw) + Eq. (fA)
    dims = (2, 2, 2, 4)
    H = wilson.hw_matrix(_unit_links(dims), dims, mu, M_W).toarray()
    x = synth.gaussian_source(dims, 2)
    y_dense = matfunc.sgn_spectral_apply(H, x)
    y_free = freefield.sgn_free_apply(x, dims, mu, M_W)
    assert np.linalg.norm(y_dense - y_free) < 1e-12 * np.linalg.norm(y_dense)


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (3, 2, 4, 2)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_free_field_operator_matches_dense(dims, mu):
    # H(p) by FFT vs the literal Eq. (Dw) matrix (every hop, the boundary sign)
    H = wilson.hw_matrix(_unit_links(dims), dims, mu, M_W)
    x = synth.gaussian_source(dims, 5)
    y = freefield.h_free_apply(x, dims, mu, M_W)
    assert np.linalg.norm(H @ x - y) < 1e-13 * np.linalg.norm(y)


def test_pure_gauge_operator_is_rotated_free_operator():
    # H[U] (Omega x) = Omega H[1] x for U_{n,nu} = Omega_n Omega_{n+nu}^dag
    dims = (2, 3, 2, 4)
    om = synth.random_su3_field(dims, 8)
    U = synth.pure_gauge_links(om)
    x = synth.gaussian_source(dims, 6)
    lhs = wilson.hw_matrix(U, dims, 0.2, M_W) @ synth.gauge_transform_spinor(om, x)
    rhs = synth.gauge_transform_spinor(om, freefield.h_free_apply(x, dims, 0.2, M_W))
    assert np.linalg.norm(lhs - rhs) < 1e-13 * np.linalg.norm(rhs)


def test_free_field_spectrum():
    dims = (2, 2, 2, 4)
    H = wilson.hw_matrix(_unit_links(dims), dims, 0.3, M_W).toarray()
    ev = np.linalg.eigvals(H)
    fe = freefield.free_eigenvalues(dims, 0.3, M_W)
    # every dense eigenvalue has a closed-form partner and vice versa
    d = np.abs(ev[:, None] - fe[None, :])
    assert d.min(axis=1).max() < 1e-8 and d.min(axis=0).max() < 1e-8


def test_free_field_projector_sign_is_pinned():
    # The opposite hop-projector convention ((1 - gamma) forward, (1 + gamma) backward)
    # is D' = gamma5 D gamma5, i.e. H' = gamma5 H gamma5.  The closed form must tell
    # the two apart, so a flipped projector in the oracle would fail the pin above.
    dims = (2, 2, 2, 4)
    U = _unit_links(dims)
    x = synth.gaussian_source(dims, 2)
    H = wilson.hw_matrix(U, dims, 0.3, M_W)
    P = wilson.gamma5_sites(int(np.prod(dims)))
    y_free = freefield.sgn_free_apply(x, dims, 0.3, M_W)
    y_flip = matfunc.sgn_spectral_apply((P @ H @ P).toarray(), x)
    assert np.linalg.norm(y_free - y_flip) > 1e-3 * np.linalg.norm(y_free)
    # and reversing the sign of mu is also told apart
    y_negmu = freefield.sgn_free_apply(x, dims, -0.3, M_W)
    assert np.linalg.norm(y_free - y_negmu) > 1e-3 * np.linalg.norm(y_free)


def test_pure_gauge_covariance_of_sign():
    dims = (2, 2, 2, 4)
    om = synth.random_su3_field(dims, 9)
    Up = synth.pure_gauge_links(om)
    x = synth.gaussian_source(dims, 3)
    H = wilson.hw_matrix(Up, dims, 0.3, M_W).toarray()
    y = matfunc.sgn_spectral_apply(H, synth.gauge_transform_spinor(om, x))
    y_ref = synth.gauge_transform_spinor(om, freefield.sgn_free_apply(x, dims, 0.3, M_W))
    assert np.linalg.norm(y - y_ref) < 1e-12 * np.linalg.norm(y)
