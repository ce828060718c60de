// Small dense complex linear algebra on the host (deflation setup only).
#pragma once

#include <complex>
#include <vector>

namespace hostla {

using cplx = std::complex<double>;

// In-place Householder reduction of the column-major n x n matrix H to upper
// Hessenberg form; Q receives the unitary factor (A = Q H Q^H).
void hessenberg(int n, cplx* H, cplx* Q);

// Implicit single-shift QR iteration on a Hessenberg H (in place) to the
// complex Schur form; Z is right-multiplied by the rotations.  false if the
// iteration did not converge.
bool schur_from_hessenberg(int n, cplx* H, cplx* Z);

// Eigenvalues w and unit-norm right eigenvectors V (columns) of a general
// complex n x n matrix A (column-major).  false if the QR iteration failed.
bool eig(int n, const cplx* A, cplx* w, cplx* V);

// Orthonormalise the columns of the rows x cols matrix A in place (modified
// Gram-Schmidt, two passes).  Columns that fall below rank_tol times their
// original norm are zeroed.  Returns the numerical rank.
int thin_qr(int rows, int cols, cplx* A, double rank_tol);

}  // namespace hostla
