"""Closed form of sgn(H_w(mu)) x for the free field U = 1 (any lattice size).

Not in the paper; derived here from Eq. (Dw).  For U = 1, a plane wave
psi_n = e^{i p.n} u is mapped by D_w(mu) to e^{i p.n} D(p) u with
    D(p) = 1 - kappa sum_nu [ (1 + gamma_nu) e^{+mu d_nu4} e^{+i p_nu}
                             + (1 - gamma_nu) e^{-mu d_nu4} e^{-i p_nu} ],
where p_i = 2 pi n_i / L_i (periodic) and p_4 = (2 n_4 + 1) pi / L_t
(antiperiodic; the -1 on the boundary hop is exactly e^{i p_4 L_t}).
With p~_nu = p_nu - i mu d_nu4 this is D(p) = a - i sum_nu b_nu gamma_nu,
a = 1 - 2 kappa sum cos p~_nu, b_nu = 2 kappa sin p~_nu, and because the
gamma_nu anticommute, H(p)^2 = (gamma5 D(p))^2 = c(p) I with
c = a^2 + sum b_nu^2.  The eigenvalues of H(p) are +-sqrt(c), so Eq. (sgnz)
gives sgn(H(p)) = H(p)/sqrt(c(p)) with the principal square root.

Pure gauge fields U_{n,nu} = Omega_n Omega_{n+nu}^dag are a gauge rotation of
U = 1, so sgn(H[U]) (Omega x) = Omega sgn(H[1]) x holds exactly at any size.
"""
from __future__ import annotations

import numpy as np

from .conventions import gamma5, gammas, kappa


def momentum_matrices(dims, mu: float, m_w: float):
    """H(p) = gamma5 D(p) (4x4) and c(p), on the FFT momentum grid (t,z,y,x)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    g = gammas()
    g5 = gamma5()
    k = kappa(m_w)
    px = 2 * np.pi * np.fft.fftfreq(lx) * 1.0
    py = 2 * np.pi * np.fft.fftfreq(ly)
    pz = 2 * np.pi * np.fft.fftfreq(lz)
    pt = 2 * np.pi * np.fft.fftfreq(lt) + np.pi / lt
    PT, PZ, PY, PX = np.meshgrid(pt, pz, py, px, indexing="ij")
    P = [PX, PY, PZ, PT]
    D = np.zeros(PX.shape + (4, 4), dtype=np.complex128)
    D += np.eye(4)
    for nu in range(4):
        ef = np.exp(mu) if nu == 3 else 1.0
        eb = np.exp(-mu) if nu == 3 else 1.0
        fwd = (ef * np.exp(1j * P[nu]))[..., None, None] * (np.eye(4) + g[nu])
        bwd = (eb * np.exp(-1j * P[nu]))[..., None, None] * (np.eye(4) - g[nu])
        D -= k * (fwd + bwd)
    H = np.einsum("ab,...bc->...ac", g5, D)
    pmu = [PX, PY, PZ, PT - 1j * mu]
    a = 1 - 2 * k * sum(np.cos(q) for q in pmu)
    c = a * a + sum((2 * k * np.sin(q)) ** 2 for q in pmu)
    return H, c


def _momentum_apply(x: np.ndarray, dims, M: np.ndarray) -> np.ndarray:
    """Apply the per-momentum 4x4 spin matrices M(p) to x (colour untouched).

    The antiperiodic time direction enters as the phase e^{-i pi t / L_t}
    before the FFT (momenta p_4 = (2 n_4 + 1) pi / L_t) and its inverse after.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    psi = x.reshape(lt, lz, ly, lx, 4, 3)
    tph = np.exp(-1j * np.pi * np.arange(lt) / lt)[:, None, None, None, None, None]
    f = np.fft.fftn(psi * tph, axes=(0, 1, 2, 3))
    f = np.einsum("...ab,...bc->...ac", M, f)
    out = np.fft.ifftn(f, axes=(0, 1, 2, 3)) / tph
    return out.reshape(-1)


def h_free_apply(x: np.ndarray, dims, mu: float, m_w: float) -> np.ndarray:
    """H_w(mu) x for U = 1 (Eq. Dw times gamma5), by FFT: H(p) per momentum."""
    H, _ = momentum_matrices(dims, mu, m_w)
    return _momentum_apply(x, dims, H)


def sgn_free_apply(x: np.ndarray, dims, mu: float, m_w: float) -> np.ndarray:
    """sgn(H_w(mu)) x for U = 1, by FFT and the closed form H(p)/sqrt(c(p))."""
    lx, ly, lz, lt = (int(d) for d in dims)
    H, c = momentum_matrices(dims, mu, m_w)
    if np.min(np.abs(np.sqrt(c).real)) < 1e-8:
        raise ValueError("free-field spectrum touches the imaginary axis")
    # sanity of the closed form: H(p)^2 = c(p) I
    H2 = np.einsum("...ab,...bc->...ac", H, H)
    assert np.allclose(H2, c[..., None, None] * np.eye(4), atol=1e-12)
    M = H / np.sqrt(c)[..., None, None]
    return _momentum_apply(x, dims, M)


def free_eigenvalues(dims, mu: float, m_w: float) -> np.ndarray:
    """All eigenvalues of the free H_w(mu): +-sqrt(c(p)), each 6-fold (2 spin x 3 colour)."""
    _, c = momentum_matrices(dims, mu, m_w)
    r = np.sqrt(c).ravel()
    return np.concatenate([np.repeat(r, 6), np.repeat(-r, 6)])
