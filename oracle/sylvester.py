"""Appendix A: the row recurrence for T Y - Y H = C.

T is m x m upper triangular, H is n x n upper Hessenberg, C and Y are m x n.
Element (i, j) of the equation reads
    sum_{k>=i} T_ik y_kj - sum_{k<=min(j+1,n)} y_ik H_kj = c_ij .
(The printed upper summation limit max(j+1, n) is a typo: H is upper
Hessenberg, so column j of H has nonzeros only in rows 1..j+1, and the limit
must be min(j+1, n).)

Rows are solved bottom to top.  Inside row i every entry is written as
y_ij = a_j y_i1 + b_j with a_1 = 1, b_1 = 0 and the two-term recurrences of
Eq. (abij); the last column's equation then fixes y_i1.  The recurrence is
numerically delicate for long rows (|a_j| grows like 1/prod H_{l+1,l}), which
the tests measure against a library solver and against the (1,2) block of the
composite sign.
"""
from __future__ import annotations

import numpy as np


def solve_sylvester_hessenberg(T: np.ndarray, H: np.ndarray, C: np.ndarray) -> np.ndarray:
    T = np.asarray(T, dtype=np.complex128)
    H = np.asarray(H, dtype=np.complex128)
    C = np.asarray(C, dtype=np.complex128)
    m, n = C.shape
    Y = np.zeros((m, n), dtype=np.complex128)
    for i in range(m - 1, -1, -1):
        # c~_ij = c_ij - sum_{k>i} T_ik y_kj
        ct = C[i] - T[i, i + 1 :] @ Y[i + 1 :]
        tii = T[i, i]
        a = np.zeros(n, dtype=np.complex128)
        b = np.zeros(n, dtype=np.complex128)
        a[0], b[0] = 1.0, 0.0
        for j in range(n - 1):
            # Eq. (abij), columns 1..j of H (0-based 0..j)
            sa = a[: j + 1] @ H[: j + 1, j]
            sb = b[: j + 1] @ H[: j + 1, j]
            a[j + 1] = -(-tii * a[j] + sa) / H[j + 1, j]
            b[j + 1] = -(ct[j] - tii * b[j] + sb) / H[j + 1, j]
        # last column fixes y_i1
        num = ct[n - 1] - tii * b[n - 1] + b @ H[:, n - 1]
        den = tii * a[n - 1] - a @ H[:, n - 1]
        y1 = num / den
        Y[i] = a * y1 + b
    return Y
