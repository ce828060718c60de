"""Pins of the oracle's overlap operator D_ov(mu) = 1 + gamma5 sgn(H_w(mu))
(Section 2, Eq. Dov): the Ginsparg-Wilson relation (Eq. GW:eq), its
violation by the polar factor at mu != 0, the circle spectrum at mu = 0, the
free-field closed form, and the gamma5 layout."""
import numpy as np
import pytest

import synth
from oracle import conventions, matfunc, overlap, wilson

M_W = -1.6


@pytest.fixture(scope="module")
def fields():
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 31)
    return dims, U, {mu: wilson.hw_matrix(U, dims, mu, M_W).toarray() for mu in (0.0, 0.3)}


def test_gamma5_vector_matches_site_kronecker():
    V = 3
    g5 = overlap.gamma5_vector(V)
    dense = wilson.gamma5_sites(V).toarray()
    assert np.array_equal(np.diag(dense).real, g5)
    assert np.array_equal(g5[:12], [1] * 6 + [-1] * 6)
    assert np.allclose(np.diag(conventions.gamma5()), [1, 1, -1, -1])


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_ginsparg_wilson_relation_holds(fields, mu):
    H = fields[2][mu]
    D = overlap.overlap_dense(H)
    assert overlap.gw_defect(D) < 1e-12


def test_polar_factor_breaks_ginsparg_wilson_at_nonzero_mu(fields):
    # Section 2: with pol(H) in place of sgn(H) the relation fails for mu != 0
    # (pol^2 != I), and holds at mu = 0 where pol = sgn
    H3, H0 = fields[2][0.3], fields[2][0.0]
    assert overlap.gw_defect(overlap.overlap_dense(H3, sign=matfunc.polar_factor)) > 1e-4
    assert overlap.gw_defect(overlap.overlap_dense(H0, sign=matfunc.polar_factor)) < 1e-12


def test_gw_detects_a_dropped_gamma5(fields):
    # D = 1 + sgn(H) (gamma5 forgotten) does not satisfy the relation
    H = fields[2][0.3]
    D = np.eye(H.shape[0]) + matfunc.sgn_spectral(H)
    assert overlap.gw_defect(D) > 1e-2


def test_spectrum_on_circle_at_zero_mu(fields):
    H0 = fields[2][0.0]
    lam = np.linalg.eigvals(overlap.overlap_dense(H0))
    assert np.abs(np.abs(lam - 1.0) - 1.0).max() < 1e-12
    lam3 = np.linalg.eigvals(overlap.overlap_dense(fields[2][0.3]))
    assert np.abs(np.abs(lam3 - 1.0) - 1.0).max() > 1e-3  # off the circle at mu != 0


@pytest.mark.parametrize("mu", [0.0, 0.4])
def test_free_field_closed_form(mu):
    dims = (2, 2, 4, 4)
    lx, ly, lz, lt = dims
    U = np.broadcast_to(np.eye(3, dtype=complex), (lt, lz, ly, lx, 4, 3, 3)).copy()
    H = wilson.hw_matrix(U, dims, mu, M_W).toarray()
    x = synth.gaussian_source(dims, 3100)
    ref = overlap.overlap_apply(H, x)
    got = overlap.overlap_free_apply(x, dims, mu, M_W)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


def test_apply_matches_dense(fields):
    H = fields[2][0.3]
    x = synth.gaussian_source(fields[0], 3200)
    assert np.allclose(overlap.overlap_apply(H, x), overlap.overlap_dense(H) @ x, atol=1e-12)


def test_massive_overlap_reading_and_solve():
    # D(m) = (1 - m/2) D_ov + m: D(0) = D_ov, D(2) = 2 (so x = b/2), the
    # expanded form (1 + m/2) + (1 - m/2) gamma5 sgn, at mu = 0 a spectrum on
    # |lambda - (1 + m/2)| = 1 - m/2, and the solve's residual
    dims = (2, 2, 2, 2)
    U = synth.random_links(dims, 61)
    b = synth.gaussian_source(dims, 6100)
    n = b.size
    for mu in (0.0, 0.3):
        A = wilson.hw_matrix(U, dims, mu, M_W).toarray()
        D = overlap.overlap_dense(A)
        assert np.abs(overlap.massive_overlap_dense(A, 0.0) - D).max() < 1e-14
        assert np.abs(overlap.massive_overlap_dense(A, 2.0) - 2.0 * np.eye(n)).max() < 1e-14
        assert np.abs(overlap.massive_overlap_solve(A, b, 2.0) - 0.5 * b).max() < 1e-14
        m = 0.2
        g5 = overlap.gamma5_vector(n // 12)
        expanded = (1 + m / 2) * np.eye(n) + (1 - m / 2) * g5[:, None] * matfunc.sgn_spectral(A)
        Dm = overlap.massive_overlap_dense(A, m)
        assert np.abs(Dm - expanded).max() < 1e-13
        x = overlap.massive_overlap_solve(A, b, m)
        assert np.linalg.norm(Dm @ x - b) < 1e-12 * np.linalg.norm(b)
        if mu == 0.0:
            ev = np.linalg.eigvals(Dm)
            assert np.abs(np.abs(ev - (1 + m / 2)) - (1 - m / 2)).max() < 1e-12
