"""LR-deflation (the subsection on LR-deflation, Eqs. Rev, Lev, xdec, fAxLR,
fARLx, LRArnoldi, fAxLRArn).  Test infrastructure only, like the rest of this
package.

With m critical right eigenvectors R (A R = R Lambda, Eq. Rev) and left
eigenvectors L (L^dag A = Lambda L^dag, Eq. Lev) normalised to L^dag R = I,
R L^dag is an oblique projector on their span, and

    f(A) x = R f(Lambda) L^dag x + f(A) x_-,   x_- = (1 - R L^dag) x,

where the second term is approximated by the plain Arnoldi method on
K_k(A, x_-):  f(A) x ~ R f(Lambda) L^dag x + beta V_k f(H_k) e_1.
The algorithm's steps, as the paper lists them: (i) left and right
eigenvectors of the critical eigenvalues, (ii) f(lambda_i), (iii) x_-,
(iv) the Arnoldi basis V_k and H_k = V_k^dag A V_k, (v) f(H_k), (vi) the sum.

The same pair serves the adjoint f(A)^dag x = f(A^dag) x (the remark closing
the subsection): A^dag L = L conj(Lambda) and R^dag A^dag = conj(Lambda) R^dag,
so L and R exchange roles, with R^dag L = I.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .arnoldi import modified_arnoldi
from .deflation import select_critical
from .matfunc import sgn_scalar, sgn_spectral


def lr_pair_from_dense(A_dense: np.ndarray, m: int):
    """Step (i): right and left eigenvectors of the m critical eigenvalues
    (smallest |Re lambda|, the same selection as the Schur deflation), from a
    full eigendecomposition, with L rescaled so that L^dag R = I."""
    lam, Lv, Rv = sla.eig(A_dense, left=True, right=True)
    idx = select_critical(lam, m)
    R, L = Rv[:, idx], Lv[:, idx]
    M = L.conj().T @ R  # diagonal up to rounding for distinct eigenvalues
    L = L @ np.linalg.inv(M).conj().T
    return R, L, lam[idx]


def sgn_lr_deflated(A, x: np.ndarray, k: int, R: np.ndarray, L: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Steps (ii)-(vi) for f = sgn: R sgn(Lambda) L^dag x + beta V_k sgn(H_k) e_1."""
    x = np.asarray(x, dtype=np.complex128)
    c = L.conj().T @ x                                         # L^dag x
    x_minus = x - R @ c                                        # Eq. (xdec)
    st = modified_arnoldi(lambda v: A @ v, x_minus, None, k)   # Eq. (LRArnoldi)
    y = R @ (sgn_scalar(lam) * c)                              # Eq. (fARLx)
    if st.k:
        fH = sgn_spectral(st.Hbar[: st.k, : st.k])
        y = y + st.V[:, : st.k] @ (st.beta * fH[:, 0])         # Eq. (fAxLRArn)
    return y


def sgn_lr_adjoint(A, x: np.ndarray, k: int, R: np.ndarray, L: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """sgn(A)^dag x by the LR-deflated method on A^dag: the left eigenvectors
    L are A^dag's right eigenvectors and R its left ones, for the eigenvalues
    conj(Lambda); the Krylov space is K_k(A^dag, (1 - L R^dag) x)."""
    Ah = A.conj().T
    return sgn_lr_deflated(Ah, x, k, L, R, np.conj(lam))
