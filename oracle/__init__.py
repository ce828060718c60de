"""Oracle: a plain, slow, FP64 CPU implementation of sgn(H_w(mu)) x.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call anything in this package; the
product path (the HIP library and its Python binding) never does, and this
package imports nothing from the product.  The two share no code: the only
common dependency is the seeded input generator module ``synth``.

Contents, each following the paper (Bloch, Frommer, Lang, Wettig 2007):
  * conventions -- gamma matrices (chiral basis), site ordering, kappa
  * wilson      -- sparse H_w(mu) = gamma5 D_w(mu) from Eq. (Dw)
  * matfunc     -- spectral sign (Eqs. fA, sgnz, signA), Roberts' iteration
                   (Eq. Roberts), Hermitian eigh route, polar factor
  * freefield   -- momentum-space closed form of sgn(H_w) for U = 1
  * sylvester   -- Appendix A row recurrence for T Y - Y H = C
  * arnoldi     -- the modified Arnoldi method with Schur deflation
                   (Eqs. eq:modArnoldi, eq:newH, yproj4, eq:f_H, SylvEq,
                   eq:formula) and the undeflated Arnoldi (Eq. yproj3)
  * deflation   -- partial Schur pair (S_m, T_m) from critical eigenvectors
                   (Eq. pSd), from a dense eigendecomposition or from ARPACK
                   on H_w^2 as in the Results section
  * overlap     -- the overlap operator D_ov(mu) = 1 + gamma5 sgn(H_w(mu))
                   (Eq. Dov), its Ginsparg-Wilson defect (Eq. GW:eq), and
                   the massive operator (1 - m/2) D_ov + m with its dense
                   solve (a reading: the paper leaves the inversion open)
  * lr          -- LR-deflation: left/right critical eigenvectors and the
                   approximation R f(Lambda) L^dag x + beta V_k f(H_k) e_1
                   (Eqs. Rev, Lev, xdec, fARLx, LRArnoldi, fAxLRArn), and
                   the adjoint sgn(A)^dag x from the same pair

Parity status: every function listed above is pinned by the CPU tests in
tests/test_oracle_*.py against facts the paper and the mathematics fix
(sgn(A)^2 = I, Hermiticity at mu = 0, the spectral/Newton agreement, the
free-field closed form, exactness of the Krylov approximation at full grade,
library Sylvester solves, brute-force small cases).  The paper's printed
numbers (Tables EVratio and CPUtime) need gauge ensembles that are not
available; they are not matched ("parity unpinned" for those tables only).
"""
