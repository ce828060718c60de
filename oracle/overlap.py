"""The overlap Dirac operator at nonzero chemical potential (Section 2).

    D_ov(mu) = 1 + gamma5 sgn(H_w(mu)),            Eq. (Dov)

with the sign function of Eqs. (fA)/(signA) and gamma5 = diag(1, 1, -1, -1)
in spin (chiral basis), acting on every site.  Test infrastructure only, like
the rest of this package.

Because sgn(A)^2 = I for any A, D_ov satisfies the Ginsparg-Wilson relation
{D_ov, gamma5} = D_ov gamma5 D_ov (Eq. GW:eq); replacing the sign by the
polar factor breaks it at mu != 0 (Section 2).  At mu = 0, H_w is Hermitian,
gamma5 sgn(H_w) is unitary and the spectrum of D_ov lies on the circle
|lambda - 1| = 1.
"""
from __future__ import annotations

import numpy as np

from . import freefield, matfunc
from .conventions import gamma5


def gamma5_vector(V: int) -> np.ndarray:
    """Diagonal of gamma5 on V sites in the component order 12 n + 3 spin + colour."""
    return np.tile(np.repeat(np.diag(gamma5()).real, 3), V)


def overlap_dense(A_hw: np.ndarray, sign=matfunc.sgn_spectral) -> np.ndarray:
    """Eq. (Dov) as a dense matrix from the dense H_w(mu); `sign` is the
    matrix function used for sgn (the polar factor gives the operator the
    paper rejects at mu != 0)."""
    n = A_hw.shape[0]
    g5 = gamma5_vector(n // 12)
    return np.eye(n, dtype=complex) + g5[:, None] * sign(A_hw)


def overlap_apply(A_hw: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D_ov(mu) x = x + gamma5 sgn(H_w(mu)) x, with the spectral sign."""
    g5 = gamma5_vector(x.size // 12)
    return x + g5 * matfunc.sgn_spectral_apply(A_hw, x)


def overlap_free_apply(x: np.ndarray, dims, mu: float, m_w: float) -> np.ndarray:
    """D_ov(mu) x for the free field U = 1, from the closed form of sgn(H(p))."""
    g5 = gamma5_vector(x.size // 12)
    return x + g5 * freefield.sgn_free_apply(x, dims, mu, m_w)


def gw_defect(D: np.ndarray) -> float:
    """|| {D, gamma5} - D gamma5 D ||_F / ||D||_F (zero for Eq. GW:eq)."""
    g5 = gamma5_vector(D.shape[0] // 12)
    lhs = D * g5[None, :] + g5[:, None] * D
    rhs = (D * g5[None, :]) @ D
    return float(np.linalg.norm(lhs - rhs) / np.linalg.norm(D))


def massive_overlap_dense(A_hw: np.ndarray, mass: float) -> np.ndarray:
    """The massive overlap operator, a reading (the paper leaves the inversion
    of D_ov to future work and names no mass term): the usual
    D(m) = (1 - m/2) D_ov(mu) + m = (1 + m/2) + (1 - m/2) gamma5 sgn(H_w(mu)),
    which is D_ov at m = 0 and 2 at m = 2."""
    n = A_hw.shape[0]
    return (1.0 - 0.5 * mass) * overlap_dense(A_hw) + mass * np.eye(n, dtype=complex)


def massive_overlap_solve(A_hw: np.ndarray, b: np.ndarray, mass: float) -> np.ndarray:
    """x with D(m) x = b, by a dense LU solve."""
    return np.linalg.solve(massive_overlap_dense(A_hw, mass), np.asarray(b, dtype=np.complex128))
