"""Step (i) of the Schur-deflation algorithm: the partial Schur pair (S_m, T_m).

Section 5.2: from m critical eigenvectors one builds orthonormal Schur
vectors S_m and the upper triangular T_m = S_m^dag A S_m with A S_m = S_m T_m
(Eq. pSd); the diagonal of T_m holds the critical eigenvalues.

"Critical" are the eigenvalues nearest the imaginary axis, i.e. smallest
|Re lambda| (Section 5.1).  Ties are broken by smaller |lambda|, then larger
Im lambda.  Two sources of eigenvectors:
  * ``critical_from_dense``  -- the full eigendecomposition (small lattices);
  * ``critical_from_arpack`` -- the Results-section recipe: ARPACK's
    smallest-magnitude mode on H_w^2 (so the wanted eigenvalues sit on the
    boundary of the convex hull), followed by a Rayleigh-Ritz step with H_w on
    the span of the returned vectors and the same selection.
The Schur vectors are the Q factor of the selected eigenvector block
(R_sel = S G with G upper triangular, hence T_m = G Lambda G^{-1}).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def select_critical(lam: np.ndarray, m: int) -> np.ndarray:
    """Indices of the m eigenvalues with smallest |Re lambda| (ties: |lambda|, -Im)."""
    order = np.lexsort((np.arange(lam.size), -lam.imag, np.abs(lam), np.abs(lam.real)))
    return order[:m]


def schur_pair_from_vectors(A, R: np.ndarray):
    """Orthonormalise R (QR) and form T = S^dag A S; returns (S, T, |tril(T,-1)|)."""
    S, _ = np.linalg.qr(R)
    AS = A @ S
    T = S.conj().T @ AS
    low = float(np.linalg.norm(np.tril(T, -1)))
    T = np.triu(T)
    return S, T, low


def critical_from_dense(A_dense: np.ndarray, m: int):
    """Critical Schur pair from a full eigendecomposition (Eq. pSd)."""
    lam, U = np.linalg.eig(A_dense)
    idx = select_critical(lam, m)
    S, T, low = schur_pair_from_vectors(A_dense, U[:, idx])
    return S, T, lam[idx], low


def critical_from_arpack(A_sparse, m: int, extra: int = 10, tol: float = 1e-13,
                         maxiter: int = 100000, ncv=None, v0=None):
    """Critical Schur pair via ARPACK 'SM' on A^2, then Rayleigh-Ritz with A."""
    N = A_sparse.shape[0]
    A2 = spla.LinearOperator((N, N), matvec=lambda v: A_sparse @ (A_sparse @ v),
                             dtype=np.complex128)
    nev = m + extra
    _, vecs = spla.eigs(A2, k=nev, which="SM", tol=tol, maxiter=maxiter, ncv=ncv, v0=v0)
    Z, _ = np.linalg.qr(vecs)
    B = Z.conj().T @ (A_sparse @ Z)
    theta, W = np.linalg.eig(B)
    idx = select_critical(theta, m)
    S, T, low = schur_pair_from_vectors(A_sparse, Z @ W[:, idx])
    return S, T, theta[idx], low


def schur_residual(A, S: np.ndarray, T: np.ndarray) -> float:
    """||A S - S T||_F, the accuracy measure of the deflation basis."""
    return float(np.linalg.norm(A @ S - S @ T))
