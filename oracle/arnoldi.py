"""The modified (Schur-deflated) Arnoldi approximation of sgn(A) x.

Section 5.2 (Schur deflation), steps (iii)-(vi):
  (iii) x_perp = (1 - S_m S_m^dag) x,  beta = |x_perp|,  v_1 = x_perp / beta;
  (iv)  every new vector A v_j is orthogonalised against the Schur vectors
        and against all previous Arnoldi vectors (Eq. eq:modArnoldi), which
        builds V_k, the Hessenberg H_k and X = S_m^dag A V_k;
  (v)   sgn of the composite H = [[T_m, X], [0, H_k]] (Eq. eq:newH), whose
        upper-right block Y solves T_m Y - Y H_k = sgn(T_m) X - X sgn(H_k)
        (Eq. SylvEq);
  (vi)  y = S_m sgn(T_m) S_m^dag x + (S_m V_k) [Y; sgn(H_k)] beta e_1
        (Eq. eq:formula).
With m = 0 this is the plain Arnoldi approximation beta V_k sgn(H_k) e_1 of
Section 4 (Eq. yproj3).

The orthogonalisation is modified Gram-Schmidt, Schur vectors first and then
V_j, repeated once in full (the paper notes that reorthogonalisation may be
needed in floating point); the coefficients of both passes are summed into
X and H.  Two evaluations of step (v)-(vi) are provided:
  * ``approx_definition``: Q sgn(H) Q^dag x with the composite sign taken from
    its spectral definition (Eqs. yproj4, fA) -- the plainest statement;
  * ``approx_paper``: the paper's route -- Roberts' iteration on T_m and H_k,
    Appendix A for Y, then Eq. (eq:formula).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .matfunc import sgn_roberts, sgn_spectral
from .sylvester import solve_sylvester_hessenberg


@dataclass
class ArnoldiState:
    V: np.ndarray  # N x (k+1), orthonormal, V[:, k] = v_{k+1}
    Hbar: np.ndarray  # (k+1) x k upper Hessenberg
    X: np.ndarray  # m x k, S^dag A V_k
    beta: float  # |x_perp|
    c0: np.ndarray  # S^dag x
    k: int  # Krylov dimension actually built (smaller on breakdown)
    breakdown: bool


def _mgs(w, B, coef):
    """One modified Gram-Schmidt sweep of w against the columns of B."""
    for i in range(B.shape[1]):
        h = np.vdot(B[:, i], w)
        w = w - h * B[:, i]
        coef[i] += h
    return w


def modified_arnoldi(matvec, x: np.ndarray, S: np.ndarray, k: int, passes: int = 2,
                     breakdown_tol: float = 1e-14) -> ArnoldiState:
    """Steps (iii)-(iv): build V_k, H_k and X for the source x."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    S = np.zeros((N, 0), dtype=np.complex128) if S is None else np.asarray(S, np.complex128)
    m = S.shape[1]
    c0 = np.zeros(m, dtype=np.complex128)
    w = x.copy()
    for _ in range(passes):
        w = _mgs(w, S, c0)
    beta = float(np.linalg.norm(w))
    V = np.zeros((N, k + 1), dtype=np.complex128)
    Hbar = np.zeros((k + 1, k), dtype=np.complex128)
    X = np.zeros((m, k), dtype=np.complex128)
    if beta == 0.0 or k == 0:
        return ArnoldiState(V[:, :1], Hbar[:1, :0], X[:, :0], beta, c0, 0, beta == 0.0)
    V[:, 0] = w / beta
    for j in range(k):
        w = matvec(V[:, j])
        for _ in range(passes):
            w = _mgs(w, S, X[:, j])
            w = _mgs(w, V[:, : j + 1], Hbar[: j + 1, j])
        h = float(np.linalg.norm(w))
        Hbar[j + 1, j] = h
        if h <= breakdown_tol * max(1.0, np.linalg.norm(Hbar[: j + 2, : j + 1])):
            kk = j + 1
            return ArnoldiState(V[:, : kk + 1], Hbar[: kk + 1, :kk], X[:, :kk], beta, c0, kk, True)
        V[:, j + 1] = w / h
    return ArnoldiState(V, Hbar, X, beta, c0, k, False)


def composite_h(T: np.ndarray, st: ArnoldiState) -> np.ndarray:
    """H = [[T_m, X], [0, H_k]] of Eq. (eq:newH)."""
    m = T.shape[0]
    k = st.k
    H = np.zeros((m + k, m + k), dtype=np.complex128)
    H[:m, :m] = T
    H[:m, m:] = st.X
    H[m:, m:] = st.Hbar[:k, :k]
    return H


def approx_definition(S, T, st: ArnoldiState) -> np.ndarray:
    """y = Q sgn(H) Q^dag x (Eq. yproj4) with sgn(H) from Eq. (fA)."""
    N = st.V.shape[0]
    S = np.zeros((N, 0), dtype=np.complex128) if S is None else S
    T = np.zeros((0, 0), dtype=np.complex128) if T is None else T
    m = S.shape[1]
    k = st.k
    Q = np.concatenate([S, st.V[:, :k]], axis=1)
    g = np.zeros(m + k, dtype=np.complex128)
    g[:m] = st.c0  # S^dag x
    if k:
        g[m] = st.beta  # V_k^dag x = beta e_1
    if m + k == 0:
        return np.zeros(N, dtype=np.complex128)
    F = sgn_spectral(composite_h(T, st))
    return Q @ (F @ g)


def approx_paper(S, T, st: ArnoldiState, sgnT=None) -> np.ndarray:
    """Steps (v)-(vi) as printed: Roberts on T_m and H_k, Appendix A, Eq. (eq:formula)."""
    N = st.V.shape[0]
    m = 0 if S is None else S.shape[1]
    k = st.k
    y = np.zeros(N, dtype=np.complex128)
    Vk = st.V[:, :k]
    Hk = st.Hbar[:k, :k]
    fH = sgn_roberts(Hk)[0] if k else np.zeros((0, 0))
    if m:
        fT = sgn_roberts(T)[0] if sgnT is None else sgnT
        y += S @ (fT @ st.c0)
        if k:
            C = fT @ st.X - st.X @ fH
            Y = solve_sylvester_hessenberg(T, Hk, C)
            y += S @ (st.beta * Y[:, 0])
    if k:
        y += Vk @ (st.beta * fH[:, 0])
    return y


def sgn_arnoldi(A, x, k: int, S=None, T=None, how: str = "definition") -> np.ndarray:
    """Convenience: the deflated Arnoldi approximation for a (sparse) matrix A."""
    st = modified_arnoldi(lambda v: A @ v, x, S, k)
    if how == "definition":
        return approx_definition(S, T, st)
    return approx_paper(S, T, st)

