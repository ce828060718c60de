"""The gamma5-Wilson-Dirac matrix H_w(mu) = gamma5 D_w(mu) as a sparse matrix.

Follows Eq. (Dw) of Section 2 term by term:
    [D_w(mu)]_{nm} = delta_{nm}
        - kappa sum_{j=1..3} (1 + gamma_j) U_{n,j} delta_{n+j,m}
        - kappa sum_{j=1..3} (1 - gamma_j) U^dag_{n-j,j} delta_{n-j,m}
        - kappa (1 + gamma_4) e^{+mu} U_{n,4} delta_{n+4,m}
        - kappa (1 - gamma_4) e^{-mu} U^dag_{n-4,4} delta_{n-4,m}
with kappa = 1/(8 + 2 m_w), and H_w(mu) = gamma5 D_w(mu) (Section 2).
Every 12x12 block is kron(spin matrix, colour matrix), matching the
component order 3*spin + colour.  A hop that crosses the time boundary
(t = Lt-1 <-> 0) carries an extra factor -1 (antiperiodic in time); the
spatial directions are periodic.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .conventions import coords, gamma5, gammas, kappa, site_index


def _neighbour(dims, nu, step):
    """Site index of n + step*e_nu for every n, and the boundary sign."""
    lx, ly, lz, lt = dims
    x, y, z, t = coords(dims)
    c = [x, y, z, t]
    L = [lx, ly, lz, lt]
    moved = (c[nu] + step) % L[nu]
    crossed = (c[nu] + step < 0) | (c[nu] + step >= L[nu])
    c2 = list(c)
    c2[nu] = moved
    m = site_index(c2[0], c2[1], c2[2], c2[3], dims)
    sign = np.ones(len(x))
    if nu == 3:
        sign[crossed] = -1.0
    return m, sign


def dirac_wilson(links: np.ndarray, dims, mu: float, m_w: float) -> sp.csr_matrix:
    """Sparse D_w(mu) of Eq. (Dw), N x N with N = 12 V."""
    dims = tuple(int(d) for d in dims)
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    U = np.asarray(links, dtype=np.complex128).reshape(V, 4, 3, 3)
    g = gammas()
    eye4 = np.eye(4)
    k = kappa(m_w)
    rows, cols, vals = [], [], []
    n = np.arange(V)

    def add_blocks(src, dst, blocks):
        # blocks: (V, 12, 12) placed at block (src, dst)
        r = 12 * src[:, None, None] + np.arange(12)[None, :, None]
        c = 12 * dst[:, None, None] + np.arange(12)[None, None, :]
        rows.append(np.broadcast_to(r, blocks.shape).ravel())
        cols.append(np.broadcast_to(c, blocks.shape).ravel())
        vals.append(blocks.ravel())

    # diagonal term delta_{nm}
    add_blocks(n, n, np.broadcast_to(np.eye(12, dtype=np.complex128), (V, 12, 12)).copy())
    for nu in range(4):
        phase_f = np.exp(mu) if nu == 3 else 1.0
        phase_b = np.exp(-mu) if nu == 3 else 1.0
        # forward hop: -kappa (1 + gamma_nu) e^{+mu delta_{nu4}} U_{n,nu} psi_{n+nu}
        m_f, s_f = _neighbour(dims, nu, +1)
        blk = np.einsum("ab,nij->naibj", eye4 + g[nu], U[:, nu]).reshape(V, 12, 12)
        add_blocks(n, m_f, (-k * phase_f * s_f)[:, None, None] * blk)
        # backward hop: -kappa (1 - gamma_nu) e^{-mu delta_{nu4}} U^dag_{n-nu,nu} psi_{n-nu}
        m_b, s_b = _neighbour(dims, nu, -1)
        udag = np.conj(np.transpose(U[m_b, nu], (0, 2, 1)))
        blk = np.einsum("ab,nij->naibj", eye4 - g[nu], udag).reshape(V, 12, 12)
        add_blocks(n, m_b, (-k * phase_b * s_b)[:, None, None] * blk)
    N = 12 * V
    D = sp.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)
    ).tocsr()
    D.sum_duplicates()
    return D


def gamma5_sites(V: int) -> sp.csr_matrix:
    """gamma5 acting on every site: kron(I_V, gamma5, I_3)."""
    return sp.kron(sp.identity(V, format="csr"), sp.kron(gamma5(), np.eye(3)), format="csr")


def hw_matrix(links: np.ndarray, dims, mu: float, m_w: float) -> sp.csr_matrix:
    """H_w(mu) = gamma5 D_w(mu) (Section 2), sparse CSR, complex128."""
    V = int(np.prod(dims))
    return (gamma5_sites(V) @ dirac_wilson(links, dims, mu, m_w)).tocsr()
