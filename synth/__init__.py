"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module produces *inputs only*: SU(3) gauge links, source vectors and
random gauge transformations.  It contains none of the sign-function method's
arithmetic (no Dirac operator, no Krylov step, no matrix function), so that
the oracle and the HIP path can consume identical inputs without sharing any
implementation.

Layouts (the C-ABI layout):
  * site index   n = x + Lx*(y + Ly*(z + Lz*t)),  dims = (Lx, Ly, Lz, Lt)
  * gauge links  U[t][z][y][x][nu][row][col], complex128, nu = 0..3 <-> x,y,z,t
                 (U[n][nu] is the link from site n to n + e_nu)
  * spinors      psi[n][spin][colour], complex128, 12 entries per site

The paper's own gauge configurations (quenched Wilson plaquette action at
beta = 5.1, Results section) are not available; the random-link ensemble
below stands in for them with the same lattice shapes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "su3_from_algebra",
    "random_links",
    "random_su3_field",
    "pure_gauge_links",
    "gauge_transform_spinor",
    "gaussian_source",
    "ones_source",
    "volume",
    "GAUGE_SEED",
]

#: Gauge seed of the benchmark ensemble (the paper's date, 26 April 2007).
GAUGE_SEED = 20070426


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, normalised Tr(l_a l_b) = 2 delta_ab."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def su3_from_algebra(g: np.ndarray, scale: float = 0.5) -> np.ndarray:
    """U = exp(i * scale * sum_a g_a l_a / 2) for a stack of 8-vectors g[..., 8].

    The exponential is taken through the eigendecomposition of the Hermitian,
    traceless generator, so U is unitary with det U = 1 to rounding.
    """
    lam = gell_mann()
    m = scale * np.einsum("...a,aij->...ij", g, lam) / 2.0
    w, v = np.linalg.eigh(m)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def random_links(dims, seed: int, scale: float = 0.5) -> np.ndarray:
    """Random-link gauge field U[t][z][y][x][nu][3][3].

    g_a ~ N(0, 1) per link and generator, U = exp(i*scale*sum_a g_a l_a/2).
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((lt, lz, ly, lx, 4, 8))
    return np.ascontiguousarray(su3_from_algebra(g, scale))


def random_su3_field(dims, seed: int, scale: float = 2.0) -> np.ndarray:
    """One random SU(3) matrix per site, Omega[t][z][y][x][3][3]."""
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((lt, lz, ly, lx, 8))
    return np.ascontiguousarray(su3_from_algebra(g, scale))


def pure_gauge_links(omega: np.ndarray) -> np.ndarray:
    """Pure-gauge field U_{n,nu} = Omega_n Omega_{n+nu}^dagger (periodic wrap).

    omega has shape (Lt, Lz, Ly, Lx, 3, 3).  The result has the link layout.
    """
    lt, lz, ly, lx = omega.shape[:4]
    out = np.empty((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    # axis of each direction nu in the (t, z, y, x) array
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    for nu in range(4):
        fwd = np.roll(omega, -1, axis=axis[nu])  # Omega_{n + e_nu}
        out[..., nu, :, :] = np.einsum("...ij,...kj->...ik", omega, fwd.conj())
    return out


def gauge_transform_spinor(omega: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(Omega psi)_n = Omega_n psi_n acting on colour; psi is flat (12 V,)."""
    v = omega.shape[0] * omega.shape[1] * omega.shape[2] * omega.shape[3]
    om = omega.reshape(v, 3, 3)
    p = psi.reshape(v, 4, 3)
    return np.einsum("nij,nsj->nsi", om, p).reshape(-1)


def gaussian_source(dims, seed: int) -> np.ndarray:
    """x = (a + i b)/sqrt(2) with (a, b) ~ N(0, 1), length N = 12 V."""
    n = 12 * volume(dims)
    rng = np.random.default_rng(seed)
    ab = rng.standard_normal((n, 2))
    return (ab[:, 0] + 1j * ab[:, 1]) / np.sqrt(2.0)


def ones_source(dims) -> np.ndarray:
    """x = (1, 1, ..., 1), the source used for the paper's accuracy figures."""
    return np.ones(12 * volume(dims), dtype=np.complex128)
