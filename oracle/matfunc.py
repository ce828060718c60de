"""Dense matrix sign function: the definitions the paper builds on.

* ``sgn_scalar``     -- Eq. (sgnz): sgn(z) = z / sqrt(z^2) = sgn(Re z), with the
                        square-root cut on the negative real axis.
* ``sgn_spectral``   -- Eqs. (fA), (signA): sgn(A) = U sgn(Lambda) U^{-1} for a
                        diagonalisable A with no eigenvalue on the imaginary axis.
* ``sgn_roberts``    -- Eq. (Roberts): S^{n+1} = (S^n + (S^n)^{-1})/2, S^0 = A,
                        unscaled as printed.
* ``sgn_hermitian``  -- the Hermitian case (Section 2): sgn(A) = W sgn(w) W^dag
                        from an eigh decomposition; equals the polar factor.
* ``polar_factor``   -- pol(A) = A (A^dag A)^{-1/2} (Section 2), which differs
                        from sgn(A) when A is not Hermitian.
"""
from __future__ import annotations

import numpy as np


def sgn_scalar(z):
    """Eq. (sgnz): z/sqrt(z^2) with numpy's principal square root."""
    z = np.asarray(z, dtype=np.complex128)
    return z / np.sqrt(z * z)


def eig_checked(A: np.ndarray, rel_gap: float = 1e-10):
    """Eigen-decomposition A = U diag(lam) U^{-1}; refuses |Re lam| ~ 0."""
    lam, U = np.linalg.eig(A)
    scale = np.max(np.abs(lam)) if lam.size else 1.0
    if lam.size and np.min(np.abs(lam.real)) <= rel_gap * scale:
        raise ValueError("eigenvalue on the imaginary axis: sgn undefined")
    return lam, U


def sgn_spectral(A: np.ndarray) -> np.ndarray:
    """Eqs. (fA), (signA): U sgn(Re Lambda) U^{-1}."""
    lam, U = eig_checked(A)
    s = np.sign(lam.real)
    return (U * s[None, :]) @ np.linalg.inv(U)


def sgn_spectral_apply(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sgn(A) x = U sgn(Re Lambda) U^{-1} x via one solve (no explicit inverse)."""
    lam, U = eig_checked(A)
    z = np.linalg.solve(U, x)
    return U @ (np.sign(lam.real) * z)


def sgn_roberts(A: np.ndarray, tol: float = 1e-14, maxit: int = 100):
    """Eq. (Roberts), unscaled.  Returns (sgn(A), iterations).

    Stops once d_n = ||S_{n+1} - S_n||_F / ||S_{n+1}||_F <= tol, or once d_n has
    reached rounding level (d_n < 1e-8 and no longer shrinking, d_n > d_{n-1}/2,
    where a quadratically convergent iteration would have squared it), and then
    takes one more step to settle the last digits.
    """
    S = np.array(A, dtype=np.complex128)
    prev = np.inf
    for it in range(1, maxit + 1):
        S_new = 0.5 * (S + np.linalg.inv(S))
        d = np.linalg.norm(S_new - S) / np.linalg.norm(S_new)
        S = S_new
        if d <= tol or (d < 1e-8 and d > 0.5 * prev):
            S = 0.5 * (S + np.linalg.inv(S))
            return S, it + 1
        prev = d
    raise RuntimeError("Roberts iteration did not converge")


def sgn_hermitian(A: np.ndarray) -> np.ndarray:
    """Hermitian A: W sgn(w) W^dag from numpy.linalg.eigh."""
    w, W = np.linalg.eigh(A)
    return (W * np.sign(w)[None, :]) @ W.conj().T


def polar_factor(A: np.ndarray) -> np.ndarray:
    """pol(A) = A (A^dag A)^{-1/2}, through the SVD A = P s R^dag -> P R^dag."""
    P, _, Rh = np.linalg.svd(A)
    return P @ Rh
