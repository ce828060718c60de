"""Conventions the paper leaves open, fixed once for the oracle.

Section 2 of the paper defines gamma5 = gamma1 gamma2 gamma3 gamma4 with
Euclidean Dirac matrices but does not print a representation.  We use the
Euclidean chiral basis
    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]   (k = 1, 2, 3)
    gamma_4 = [[0, 1], [1, 0]]
for which gamma1 gamma2 gamma3 gamma4 = diag(1, 1, -1, -1).  Any unitarily
equivalent representation gives a unitarily equivalent sgn(H_w); both the
oracle and the GPU path use exactly these matrices.

Indexing (site-major, spin-major-over-colour):
    n = x + Lx*(y + Ly*(z + Lz*t)),  component = 12 n + 3 spin + colour.
Direction nu = 0, 1, 2, 3 is the paper's 1, 2, 3, 4 (4 = time).
Boundary conditions (not stated in the paper): periodic in x, y, z and
antiperiodic in t.
"""
from __future__ import annotations

import numpy as np

SIGMA = np.array(
    [
        [[0, 1], [1, 0]],
        [[0, -1j], [1j, 0]],
        [[1, 0], [0, -1]],
    ],
    dtype=np.complex128,
)


def gammas() -> np.ndarray:
    """gamma_1..gamma_4 (index 0..3) in the Euclidean chiral basis."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    z = np.zeros((2, 2))
    for k in range(3):
        g[k] = np.block([[z, -1j * SIGMA[k]], [1j * SIGMA[k], z]])
    g[3] = np.block([[z, np.eye(2)], [np.eye(2), z]])
    return g


def gamma5() -> np.ndarray:
    """gamma5 = gamma1 gamma2 gamma3 gamma4 (Section 2)."""
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def kappa(m_w: float) -> float:
    """Hopping parameter kappa = 1/(8 + 2 m_w) of Eq. (Dw)."""
    d = 8.0 + 2.0 * m_w
    if d <= 0:
        raise ValueError("8 + 2 m_w must be positive")
    return 1.0 / d


def site_index(x, y, z, t, dims):
    lx, ly, lz, _ = dims
    return x + lx * (y + ly * (z + lz * t))


def coords(dims):
    """Arrays (x, y, z, t) of every site, in site-index order."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(
        np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij"
    )
    return x.ravel(), y.ravel(), z.ravel(), t.ravel()
