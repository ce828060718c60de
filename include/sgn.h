/*
 * sgn.h -- C ABI of the MI355X (gfx950) implementation of y = sgn(H_w(mu)) x
 *
 * Method: Bloch, Frommer, Lang, Wettig, "An iterative method to compute the
 * sign function of a non-Hermitian matrix and its application to the overlap
 * Dirac operator at nonzero chemical potential" (2007).
 *   H_w(mu) = gamma5 D_w(mu), D_w(mu) the Wilson-Dirac operator of Eq. (Dw)
 *   (Section 2) with kappa = 1/(8 + 2 m_w), e^{+mu} on forward and e^{-mu}
 *   on backward time hops.  sgn(A) is the spectral sign of Eqs. (fA), (sgnz).
 *   y is approximated by the Schur-deflated modified Arnoldi method of
 *   Section 5.2, steps (i)-(vi).
 *
 * Conventions fixed by this library (the paper does not print them):
 *   - chiral gamma basis: gamma_k = [[0,-i s_k],[i s_k,0]] (k=1,2,3),
 *     gamma_4 = [[0,1],[1,0]], gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1,1,-1,-1);
 *   - periodic boundary conditions in x, y, z; antiperiodic in t.
 *
 * Layouts at the ABI (all complex numbers are interleaved complex128, i.e.
 * two doubles re, im):
 *   - dims = {Lx, Ly, Lz, Lt}, every L >= 2;  V = Lx Ly Lz Lt,  N = 12 V;
 *   - site index n = x + Lx (y + Ly (z + Lz t));
 *   - spinor:  psi[n][spin][colour]   (component 12 n + 3 spin + colour);
 *   - gauge:   U[n][nu][row][col], nu = 0,1,2,3 <-> x,y,z,t, the SU(3) link
 *              from n to n + e_nu (host memory, 4 V 9 complex numbers);
 *   - S (deflation basis): column-major N x m, column j contiguous (device);
 *   - T: column-major m x m upper triangular (host).
 *
 * Ownership: the gauge array is copied during sgn_create.  Vectors x, y are
 * caller-owned device buffers that must stay valid for the duration of the
 * call; y may alias x.  The context owns every internal buffer (links, Schur
 * basis, Krylov workspace) and frees them in sgn_destroy.  A context is not
 * thread-safe; use one context per host thread.
 *
 * Errors: functions return SGN_OK (0) or a negative status; no C++ exception
 * crosses the ABI.  sgn_last_error() gives a message for the last failure on
 * a context, sgn_create_error() for the last failed sgn_create on the calling
 * thread.  All calls are synchronous with respect to the host: when they
 * return, device results are written.
 */
#ifndef SGN_H
#define SGN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgn_ctx sgn_ctx;

enum {
  SGN_OK = 0,
  SGN_EINVAL = -1,     /* bad argument: dims, m_w, tol, kmax, NaN/Inf in x, ... */
  SGN_ENOMEM = -2,     /* device allocation failed or budget exceeded */
  SGN_EHIP = -3,       /* HIP runtime error */
  SGN_ENOCONV = -4,    /* soft: kmax reached before tol; y holds the kmax estimate */
  SGN_ESINGULAR = -5,  /* singular Newton iterate / eigenvalue on the imaginary axis */
  SGN_ESTATE = -6,     /* call not valid in the current state (NULL context, ...) */
  SGN_EDEFL = -7       /* deflation basis not accurate enough (||AS - ST|| too large) */
};

enum { SGN_PREC_FP64 = 0, SGN_PREC_MIXED = 1 };

/* Orthogonalisation of step (iv).  Both orthogonalise every new vector
 * against the Schur vectors and all previous Arnoldi vectors twice (classical
 * Gram-Schmidt with one re-orthogonalisation); they differ in scheduling:
 *   SGN_ORTH_CGS2:    two passes per step (four sweeps over the basis);
 *   SGN_ORTH_DELAYED: the re-orthogonalisation of v_j is merged with the
 *                     first pass of v_{j+1} (one reduction, two sweeps over
 *                     the basis per step; the default). */
enum { SGN_ORTH_CGS2 = 0, SGN_ORTH_DELAYED = 1 };

/* Per-apply statistics (sgn_last_info). */
typedef struct sgn_info {
  int k_used;         /* Krylov dimension of the returned approximation */
  int converged;      /* 1 if the stopping rule (sgn_apply) certified tol */
  int newton_iters;   /* small-matrix sign iterations summed over all checkpoints */
  int n_matvec;       /* applications of H_w(mu) */
  int n_checkpoints;  /* evaluations of the small-matrix sign */
  int breakdown;      /* 1 if the Krylov space became invariant (exact result): the
                       * orthogonalised candidate fell below 1e-12 (FP64) or 1e-6
                       * (mixed: FP32 basis) of its size before orthogonalisation */
  double err_est;     /* ||c_k - c_k'|| / ||c_k|| at the last checkpoint */
  double beta;        /* |x_perp| = |(1 - S S^dag) x| */
  double ms_arnoldi;  /* wall time of the Arnoldi steps (device-synchronous) */
  double ms_sign;     /* wall time of the small-matrix sign evaluations */
  double ms_total;
} sgn_info;

/* ---- context ---------------------------------------------------------- */

/* Create a context for one gauge field (Eq. Dw).  gauge: host complex128
 * U[V][4][3][3] of SU(3) matrices (unitary with determinant 1 to 1e-10: the
 * stencil keeps two rows of each link and rebuilds the third, so other
 * matrices are refused); dims: {Lx,Ly,Lz,Lt}, each >= 2; requires
 * 8 + 2 m_w > 0.  The context uses the null stream until sgn_set_stream is
 * called.  Returns NULL on failure (see sgn_create_error). */
sgn_ctx* sgn_create(const double* gauge, const int dims[4], double mu, double m_w);

/* Message of the last failed sgn_create on this thread ("" if none). */
const char* sgn_create_error(void);

/* Free every device buffer of the context.  NULL is accepted. */
void sgn_destroy(sgn_ctx* ctx);

/* Launch all work of this context on the given hipStream_t (NULL = null
 * stream).  The stream must use the default priority. */
int sgn_set_stream(sgn_ctx* ctx, void* hip_stream);

/* Lattice extents and vector length N = 12 V of a context. */
int sgn_get_dims(const sgn_ctx* ctx, int dims[4], long long* n);

/* ---- deflation (Section 5.2, steps (i)-(ii)) ------------------------- */

/* Compute and install the partial Schur pair of the m critical eigenvalues
 * (smallest |Re lambda|) of H_w(mu) on the device (Section 5.2, steps (i)-(ii);
 * Results section): Arnoldi on H_w^2 for its smallest-magnitude eigenvalues
 * with thick restarts, a Rayleigh-Ritz step with H_w on the converged span,
 * selection by |Re lambda|, S_m = orthonormalised eigenvectors, T_m =
 * S_m^dag A S_m, then sgn(T_m) on the device (the small-matrix sign of
 * sgn_set_sign_method: Newton-Schulz by default).  m = 0 removes
 * deflation.  SGN_EDEFL if ||A S - S T||_F / ||A|| > 1e-10 or the eigensolver
 * does not converge.  Requires 0 <= m <= N/4. */
int sgn_deflate(sgn_ctx* ctx, int m);

/* Statistics of the last sgn_deflate: restarts, applications of H_w(mu),
 * and the relative Schur residual ||A S - S T||_F / ||A||. */
int sgn_deflate_stats(const sgn_ctx* ctx, int* restarts, int* matvecs, double* residual);

/* Install a partial Schur pair A S = S T (Eq. pSd) computed elsewhere.
 * S: device complex128, column-major N x m, orthonormal columns;
 * T: host complex128, column-major m x m, upper triangular (the strictly
 * lower part is ignored).  Computes sgn(T) on the device with the
 * small-matrix sign of sgn_set_sign_method.  m = 0 removes deflation.  Returns SGN_EINVAL if
 * m < 0 or m > N/4, SGN_ESINGULAR if T has a diagonal entry with Re = 0. */
int sgn_deflate_import(sgn_ctx* ctx, int m, const double* S, const double* T);

/* Copy the installed pair out: S to device (N x m), T to host (m x m),
 * evals to host (m complex = diag T).  Any pointer may be NULL. */
int sgn_deflate_export(const sgn_ctx* ctx, double* S, double* T, double* evals);

/* Krylov subspace size of the deflation eigensolver (sgn_deflate,
 * sgn_deflate_lr: thick-restart Arnoldi on H_w^2): ncv basis vectors per
 * cycle, of which about (ncv + nev) / 2 are kept at a restart; nev =
 * m + max(10, m / 2).  0 restores the default max(3 nev, nev + 40); values
 * below nev + 3 are raised to it, above N - 1 lowered to it.  SGN_EINVAL for
 * ncv < 0.  A fixed ncv is not enlarged when the solver stalls: a basis of
 * only a few vectors more than nev gains little per restart and can end in
 * SGN_EDEFL (no convergence within 3000 restarts); about 2 nev or more is
 * safe.  Device memory grows by 2 ncv N complex128 during the setup. */
int sgn_set_deflation_krylov(sgn_ctx* ctx, int ncv);

/* Chebyshev filter of the deflation eigensolver (sgn_deflate, sgn_deflate_lr;
 * the faster setup the Results section's ARPACK run on H_w^2 asks for): the
 * thick-restart Arnoldi method runs on p(H_w^2) = T_d((H_w^2 - c) / e), the
 * degree-d Chebyshev polynomial of the interval [alpha, beta] = [c - e,
 * c + e] = [cut rho, rho] of H_w^2's spectrum (rho its spectral radius,
 * estimated by a 40-step Arnoldi run, with 10 % margin).  p stays within
 * [-1, 1] on that interval and grows fast below it, so the smallest-
 * magnitude eigenvalues of H_w^2 become the largest of p(H_w^2), found in few
 * restarts; the eigenvectors are the same, and the Rayleigh-Ritz step with
 * H_w, the selection and the Schur-residual test follow as without the
 * filter.  Each Arnoldi step costs 2 d stencil applications instead of 2, so
 * the filter pays where orthogonalisation and restarts dominate (large
 * lattices, clustered spectra).  If the filtered run has not converged within
 * 300 restarts (for instance when fewer than m + max(10, m/2) eigenvalues lie
 * below alpha), the unfiltered solver runs.  degree 0 disables the filter;
 * cut 0 selects the default 1/16.  Default degree 16.  SGN_EINVAL for degree
 * outside [0, 200] or cut outside (0, 1). */
int sgn_set_deflation_filter(sgn_ctx* ctx, int degree, double cut);
/* Of the last sgn_deflate / sgn_deflate_lr: the filter degree of the run that
 * converged (0: unfiltered) and its interval [alpha, beta]. */
int sgn_deflate_filter_stats(const sgn_ctx* ctx, int* degree, double* alpha, double* beta);

/* Number of installed deflation vectors, Schur or LR (0 if none, <0 on error). */
int sgn_deflation_size(const sgn_ctx* ctx);

/* LR-deflation (the LR-deflation subsection; Eqs. Rev, Lev, xdec, fARLx,
 * LRArnoldi, fAxLRArn): with right eigenvectors R (A R = R Lambda) and left
 * eigenvectors L (L^dag A = Lambda L^dag) of the m critical eigenvalues,
 * L^dag R = I, an apply computes R sgn(Lambda) L^dag x + beta V_k sgn(H_k) e1
 * with the plain Arnoldi method on x_- = (1 - R L^dag) x (no projection
 * inside the Krylov steps).  An LR pair replaces any Schur pair and vice
 * versa; every apply (single, batched, overlap, serving sessions) uses the
 * installed one.
 * sgn_deflate_lr computes it on the device: the critical Schur pairs of
 * H_w(mu) and of H_w(-mu) = H_w(mu)^dag (same method as sgn_deflate; its
 * left eigenvectors are the right ones of H_w(-mu) for conj(lambda)), their
 * eigenvectors, paired by eigenvalue and rescaled to L^dag R = I
 * (SGN_EDEFL if the eigenvalues do not pair up or L^dag R deviates from I by
 * more than 1e-8); 1 <= m <= N/4.  sgn_deflate_lr_import takes R and L
 * (device, interface layout, N x m column-major) and the eigenvalues (host,
 * m complex); SGN_EINVAL unless L^dag R = I to 1e-8.  sgn_deflate_lr_export
 * copies them out (any pointer may be NULL; SGN_ESTATE without an LR pair).
 * sgn_deflation_mode: SGN_DEFL_NONE, SGN_DEFL_SCHUR or SGN_DEFL_LR. */
enum { SGN_DEFL_NONE = 0, SGN_DEFL_SCHUR = 1, SGN_DEFL_LR = 2 };
int sgn_deflate_lr(sgn_ctx* ctx, int m);
int sgn_deflate_lr_import(sgn_ctx* ctx, int m, const double* R, const double* L, const double* lam);
int sgn_deflate_lr_export(const sgn_ctx* ctx, double* R, double* L, double* lam);
int sgn_deflation_mode(const sgn_ctx* ctx);

/* ---- the hot path (Section 5.2, steps (iii)-(vi)) ---------------------- */

/* y = sgn(H_w(mu)) x by the deflated modified Arnoldi method.  The small
 * sign is evaluated at even-k checkpoints (Section 4); the relative change e
 * of y between two checkpoints k' < k is exact (Q has orthonormal columns).
 * Stopping rule (not in the paper, which measures only against the exact y):
 * the changes fit a geometric error model err(k) ~ exp(r k), under which
 * e / (1 - exp(r (k - k'))) estimates the error of y_k'; the apply stops
 * once that estimate is <= tol and returns y_k (a factor exp(r (k - k')),
 * at most 1/2 for a confirming checkpoint, more accurate), or at k = kmax
 * (then SGN_ENOCONV with y holding the kmax approximation).  x, y: device
 * complex128, N entries.  Requires tol > 0, 2 <= kmax <= N.  Returns
 * SGN_EINVAL for NaN/Inf in x. */
int sgn_apply(sgn_ctx* ctx, const double* x, double* y, double tol, int kmax);

/* Fixed Krylov dimension: exactly k modified Arnoldi steps (fewer only on an
 * exact breakdown), then steps (v)-(vi) once.  0 <= k <= N - d, d the
 * installed deflation size (Schur m or the LR pair's m), else SGN_EINVAL:
 * the composite basis holds at most N orthonormal columns. */
int sgn_apply_fixed(sgn_ctx* ctx, const double* x, double* y, int k);

/* Several sources of one field: Y_r = sgn(H_w(mu)) X_r for r < nrhs.
 * X, Y: device complex128, nrhs x N (source r at X + 2 N r doubles); Y may
 * alias X.  The sources advance together (one stencil, dot and update launch
 * per Arnoldi step for all unfinished sources, at most 64 per launch; larger
 * nrhs run in chunks of 64); each stops at the first shared even-k
 * checkpoint where its own change is <= tol.  info: host array of nrhs
 * entries (nullable).  Always the one-reduction schedule.  Per source the
 * arithmetic is that of sgn_apply, so sgn_apply_batched_fixed returns
 * bitwise the sgn_apply_fixed results; with a tolerance the shared
 * checkpoints can stop a source at a later k than sgn_apply would.
 * Returns SGN_ENOCONV if any source reached kmax unconverged (its Y_r holds
 * the kmax approximation, info[r].converged = 0).  The workspace holds
 * sgn_footprint_bytes(ctx, kmax, min(nrhs, 64)) bytes and is kept for reuse. */
int sgn_apply_batched(sgn_ctx* ctx, int nrhs, const double* X, double* Y, double tol, int kmax, sgn_info* info);

/* Batched counterpart of sgn_apply_fixed: exactly k steps per source, with
 * the same bound 0 <= k <= N - d. */
int sgn_apply_batched_fixed(sgn_ctx* ctx, int nrhs, const double* X, double* Y, int k, sgn_info* info);

/* The overlap Dirac operator at nonzero chemical potential (Section 2, Eq.
 * Dov): y = D_ov(mu) x = x + gamma5 sgn(H_w(mu)) x, gamma5 = diag(1, 1, -1,
 * -1) in spin.  The sign is applied exactly as by sgn_apply (same tol, kmax,
 * status, sgn_last_info); the batched form as by sgn_apply_batched, with
 * the same info array.  x, y (X, Y: nrhs x N): device complex128 in the
 * interface layout; they must not overlap (SGN_EINVAL), since x is read
 * again after the sign is formed.  Complete on return. */
int sgn_overlap_apply(sgn_ctx* ctx, const double* x, double* y, double tol, int kmax);
int sgn_overlap_apply_batched(sgn_ctx* ctx, int nrhs, const double* X, double* Y, double tol, int kmax,
                              sgn_info* info);

/* The adjoint y = sgn(H_w(mu))^dag x = sgn(H_w(-mu)) x (the LR-deflation
 * subsection's closing remark: the left and right eigenvectors exchange
 * roles).  Runs the method on A^dag = H_w(-mu) with the installed LR pair
 * (sgn_deflate_lr or sgn_deflate_lr_import), L as A^dag's right and R as its
 * left eigenvectors for conj(Lambda), or with no deflation; tol, kmax,
 * status and sgn_last_info as for sgn_apply, and the fixed form as
 * sgn_apply_fixed.  SGN_ESTATE with a Schur pair installed (a Schur basis of
 * A is none of A^dag) or while a serving session is open on the context.
 * Captured step graphs (sgn_set_step_graphs) are not used by these calls. */
int sgn_apply_adjoint(sgn_ctx* ctx, const double* x, double* y, double tol, int kmax);
int sgn_apply_adjoint_fixed(sgn_ctx* ctx, const double* x, double* y, int k);
/* Several sources, as sgn_apply_batched / sgn_apply_batched_fixed: Y_r =
 * sgn(H_w(mu))^dag X_r, per source bitwise the single-source adjoint at
 * fixed k; the same requirements as sgn_apply_adjoint. */
int sgn_apply_adjoint_batched(sgn_ctx* ctx, int nrhs, const double* X, double* Y, double tol, int kmax,
                              sgn_info* info);
int sgn_apply_adjoint_batched_fixed(sgn_ctx* ctx, int nrhs, const double* X, double* Y, int k, sgn_info* info);

/* The adjoint of the overlap operator (Eq. Dov): y = D_ov(mu)^dag x =
 * x + sgn(H_w(mu))^dag gamma5 x, the sign applied as by sgn_apply_adjoint
 * (same requirements and status) to gamma5 x.  At mu != 0 this is not
 * gamma5 D_ov gamma5.  x, y: device complex128 in the interface layout; they
 * must not overlap (SGN_EINVAL).  Complete on return. */
int sgn_overlap_apply_adjoint(sgn_ctx* ctx, const double* x, double* y, double tol, int kmax);

/* Solve D(m) x = b for the massive overlap operator
 *   D(m) = (1 - m/2) D_ov(mu) + m = (1 + m/2) + (1 - m/2) gamma5 sgn(H_w(mu)),
 * a reading: the paper leaves the inversion of D_ov to future work (each
 * outer step needs one sign apply, which is where deflation's one-off cost
 * pays) and names no mass term; this is the usual one, D_ov at m = 0.
 * Restarted GMRES (restart outer vectors, 1..500) with the sign applied as
 * by sgn_apply(inner_tol, inner_kmax) on the installed deflation; the outer
 * basis is orthogonalised twice with classical Gram-Schmidt on the device.
 * Stops when the true relative residual |b - D x| / |b| <= tol (checked at
 * every restart) or after max_iter outer steps (then SGN_ENOCONV, x the
 * last iterate).  The operator is only as accurate as inner_tol, so choose
 * inner_tol well below tol; in mixed precision (sgn_set_precision) the
 * inner applies run on the FP32 basis, which bounds inner_tol at about
 * 1e-7.  b, x: device complex128, N entries, not
 * overlapping.  iters, rel_res (host, nullable): outer steps taken and the
 * final true relative residual.  SGN_ENOCONV also when an inner apply
 * misses inner_tol.  Allocates (restart + 2) N complex128 per call. */
int sgn_overlap_solve(sgn_ctx* ctx, const double* b, double* x, double mass, double tol, int max_iter, int restart,
                      double inner_tol, int inner_kmax, int* iters, double* rel_res);

/* ---- serving: continuous batching on one resident field ---------------- */

/* A session keeps up to max_slots (1..64) requests of one context in flight,
 * each with its own Krylov workspace of kmax vectors (device bytes:
 * sgn_footprint_bytes(ctx, kmax, max_slots)).  sgn_session_submit admits a
 * request into a free slot (source projection, step (iii)); each
 * sgn_session_step runs one Arnoldi step (step (iv)) for every occupied slot,
 * all in one stencil, dot and update launch, each request at its own Krylov
 * dimension; a request reaching one of its checkpoints evaluates the small
 * sign (step (v)) and, once its change is <= tol (or its space is invariant,
 * or it reached its kmax), writes y (step (vi)) and frees its slot.  The
 * checkpoint schedule depends on the request alone, so y is bitwise the same
 * whatever else is in flight (and equal to sgn_apply on a fresh context).
 * x, y: device complex128, N entries, caller-owned; x is read during submit
 * only, y must stay valid until poll reports the request done.  The context
 * keeps its Schur pair and precision while sessions are open (sgn_deflate,
 * sgn_deflate_import, sgn_set_precision return SGN_ESTATE); a session uses
 * the context's stream and is not thread-safe; destroy sessions before their
 * context. */
typedef struct sgn_session sgn_session;
/* NULL on failure (sgn_last_error(ctx) says why). */
sgn_session* sgn_session_create(sgn_ctx* ctx, int max_slots, int kmax);
/* Admit a request; *req receives its handle.  SGN_ENOMEM if every slot is
 * busy (the request is not admitted), SGN_EINVAL for NaN/Inf in x, tol <= 0
 * or kmax outside [2, session kmax]. */
int sgn_session_submit(sgn_session* s, const double* x, double* y, double tol, int kmax, int* req);
/* Advance every occupied slot by up to nsteps Arnoldi steps (stops early when
 * no slot is occupied); returns the number of requests finished (>= 0). */
int sgn_session_step(sgn_session* s, int nsteps);
/* 1: request done, y written, info filled (nullable; the handle is then
 * forgotten; info.converged = 0 if it stopped at its kmax); 0: running;
 * < 0: the request failed (SGN_EINVAL: non-finite values) or the handle is
 * unknown. */
int sgn_session_poll(sgn_session* s, int req, sgn_info* info);
/* Occupied slots. */
int sgn_session_active(const sgn_session* s);
void sgn_session_destroy(sgn_session* s);

/* Arithmetic of the Krylov loop.  SGN_PREC_FP64 (default): everything FP64.
 * SGN_PREC_MIXED: the links, the stencil and the stored Krylov vectors v_j are
 * FP32; the Schur vectors S_m, the candidate vector being orthogonalised,
 * every dot product, the re-orthogonalisation, the composite matrix H, its
 * sign (sgn_set_sign_method) and the assembly of y stay FP64 (always the
 * delayed schedule).  x and y stay complex128 at the ABI. */
int sgn_set_precision(sgn_ctx* ctx, int prec);
/* The context's precision (SGN_PREC_*), or SGN_ESTATE for a NULL context. */
int sgn_get_precision(const sgn_ctx* ctx);

/* Evaluation of sgn of the small composite matrix (step (v)):
 *   SGN_SIGN_SCHULZ (default): inverse-free Newton-Schulz iteration
 *     X <- X (3I - X^2)/2 from X_0 = H/|H|_1 (two complex GEMMs per step);
 *     falls back to Roberts' iteration if it does not converge;
 *   SGN_SIGN_ROBERTS: Roberts' iteration S <- (S + S^{-1})/2 (Eq. Roberts)
 *     with determinantal scaling and Gauss-Jordan inverses. */
enum { SGN_SIGN_SCHULZ = 0, SGN_SIGN_ROBERTS = 1 };
int sgn_set_sign_method(sgn_ctx* ctx, int method);

/* Select the orthogonalisation schedule (SGN_ORTH_*); default DELAYED. */
int sgn_set_orthogonalization(sgn_ctx* ctx, int mode);

/* Block (s-step) form of step (iv) (Eq. eq:modArnoldi) for the FP64 applies
 * of this context (sgn_apply, sgn_apply_fixed, the batched applies, the
 * adjoint and overlap applies and the overlap solve's inner applies; mixed
 * precision and serving sessions keep one vector per step).  Each block of
 * `s` steps takes s Krylov directions from the Chebyshev recurrence on
 * [-e, e], e = sqrt(1.1) x the spectral radius estimate of A (40 Arnoldi
 * steps on A^2, once per context, on the first block apply), orthogonalises
 * them against the composite basis by block classical Gram-Schmidt with one
 * full second pass and a Cholesky factor, and recovers the block's Hessenberg
 * columns from the change of basis.  In exact arithmetic basis, Hessenberg
 * matrix and result are those of the one-vector process; in floating point
 * they agree to rounding amplified by the block's condition (measured up to
 * 60 at s = 8 and 250 at s = 16 on the 4^4 to 6^4 fields).  Checkpoints fall
 * on whole blocks (k a multiple of s, or kmax).  The basis is read four
 * times per block instead of twice per step.  A block that is not
 * numerically of full rank (a Cholesky pivot below 1e-12 of the block's
 * size or 1e-7 of its largest pivot) makes the apply (or batch) start again
 * with one-vector steps (an invariant subspace, a tiny lattice).  s: 0 (off,
 * the default) or 1..16; SGN_EINVAL otherwise.  e_out (nullable): the
 * interval half-width in use (0 before the first block apply). */
int sgn_set_block_steps(sgn_ctx* ctx, int s);
int sgn_get_block_steps(const sgn_ctx* ctx, int* s, double* e_out);

/* Launch shape of the Arnoldi step's two sweeps over the basis (Eq.
 * eq:modArnoldi; the Gram-Schmidt dot and update passes of step (iv)):
 * update_batch (4, 8 or 16) basis columns whose loads each lane of the
 * update pass issues before their arithmetic, dot_cols (1, 2 or 4) basis
 * columns per wavefront of the dot pass, and update_waves (8 or 16)
 * wavefronts per 64-row workgroup of the update pass.  update_batch and
 * dot_cols form every sum in the same order, so results are bitwise the
 * same for all their values; update_waves changes which columns each
 * wavefront sums, so results differ between its values at the rounding
 * level.  Defaults 8, 4, 8.  Applies to later applies, batched applies and
 * session steps on this context (which all use the same shape, so they stay
 * bitwise consistent with each other).  SGN_EINVAL for other values. */
int sgn_set_tuning(sgn_ctx* ctx, int update_batch, int dot_cols, int update_waves);
int sgn_get_tuning(const sgn_ctx* ctx, int* update_batch, int* dot_cols, int* update_waves);

/* Captured Arnoldi steps of sgn_apply / sgn_apply_fixed and of the batched
 * applies (step (iv)): runs of `steps` consecutive steps between two
 * checkpoints are replayed as one HIP graph, whose kernels read the step
 * index from device memory; shorter runs, profiled applies, the adjoint
 * applies and the two-pass schedule launch each kernel directly.  A batch
 * replays runs of an even number of steps (steps rounded down) that start
 * at an even step, one graph per set of running sources.  The graphs (one
 * per 32 columns of basis size, captured on first use on a stream the
 * context owns) hold the workspace's addresses and are dropped when it, the
 * Schur pair, the precision, the launch shape or `steps` changes.  The
 * kernels and their arguments are the same in both modes, so results are
 * bitwise the same.  steps: 0 (off) or 2..64; default 0 (off: on MI355X the
 * step's kernels already run back to back, and replay measured no faster).
 * SGN_EINVAL for other values. */
int sgn_set_step_graphs(sgn_ctx* ctx, int steps);

/* Order in which the stencil's workgroups walk the lattice (Eq. Dw; results
 * are bitwise the same for every order): 4D blocks of Lx x By x Bz x Bt
 * sites, walked block by block so that neighbour spinors and links are
 * reused from cache.  By, Bz, Bt must divide Ly, Lz, Lt with Lx*By a
 * multiple of 32; (0, 0, 0) restores the default (on lattices of 65536
 * sites or more the first of By = 4, 8, 2, 16, 1, Bz = 16, 8, 4, 2, 1,
 * Bt = 4, 8, 2, 1 that fits; natural order below); By < 0 selects the
 * natural order.  SGN_EINVAL otherwise. */
int sgn_set_stencil_blocks(sgn_ctx* ctx, int By, int Bz, int Bt);

/* Checkpoint placement of sgn_apply.  The small-matrix sign is evaluated at
 * even checkpoints; the first successful sgn_apply on a field records the k
 * at which convergence to tol was certified, and later applies with the same
 * tol start checkpointing there (results then no longer depend on what ran
 * before).  sgn_set_schedule sets that k explicitly (0: record it again on
 * the next apply).  The stopping test is the same in every case. */
int sgn_set_schedule(sgn_ctx* ctx, int k_first, double tol);

/* Statistics of the last sgn_apply / sgn_apply_fixed (after a batched
 * apply: k_used and err_est are the largest over the sources, converged is 1
 * only if all converged). */
int sgn_last_info(const sgn_ctx* ctx, sgn_info* info);

/* Device bytes an apply with this kmax needs beyond the resident field
 * (nrhs = 1: sgn_apply; nrhs > 1: sgn_apply_batched with min(nrhs, 64)
 * sources per chunk). */
size_t sgn_footprint_bytes(const sgn_ctx* ctx, int kmax, int nrhs);

/* ---- building blocks exposed for testing and measurement -------------- */

/* y = H_w(mu) x = gamma5 D_w(mu) x (Eq. Dw), FP64.  x, y: device, N entries;
 * y must not alias x. */
int sgn_matvec(sgn_ctx* ctx, const double* x, double* y);

/* sgn_matvec for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same y = H_w(mu) x, bitwise, with the two staging vectors (packed x and its
 * image) in a static per-device buffer of 64 MiB instead of per-call
 * allocations.  The call allocates nothing.  Limit: 2 * 16 * ceil(12 V / 64)
 * * 64 bytes <= 64 MiB, i.e. at most 174762 lattice sites (20^4 fits, 24^4
 * does not); larger lattices give SGN_EINVAL.  The context's device must be
 * current (SGN_ESTATE otherwise).  Every call on one GPU shares that GPU's
 * buffer: calls that overlap in time on one GPU (several host threads, or
 * contexts on different streams) race, so serialise them.  Synchronous like
 * every call of this library.  x, y: device, N entries, distinct. */
int sgn_matvec_noalloc(sgn_ctx* ctx, const double* x, double* y);

/* F = sgn(A) for a dense n x n complex128 column-major device matrix, by the
 * context's sign method (sgn_set_sign_method): the inverse-free
 * Newton-Schulz iteration on the matrix cores from A / |A|_1, falling back to
 * Roberts' iteration (Eq. Roberts) with a Gauss-Jordan inverse, or Roberts'
 * iteration alone.  Uses the context's stream and workspace.  iters
 * (nullable) receives the iteration count.  SGN_ESINGULAR on a singular
 * iterate. */
int sgn_dense_sign(sgn_ctx* ctx, int n, const double* A, double* F, int* iters);

/* C = A B for complex128 column-major device matrices (A: M x K, ld lda;
 * B: K x N, ld ldb; C: M x N, ld ldc), on the matrix cores with the kernel
 * of the small-matrix sign's Newton-Schulz products (FP64 MFMA).  Uses the
 * context's stream.  SGN_EINVAL for negative sizes or short leading
 * dimensions. */
int sgn_zgemm(sgn_ctx* ctx, int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C,
              int ldc);

/* Kernel-level timing with HIP events on the context's stream.  When on,
 * every launch of the instrumented kernels is bracketed by events and its
 * duration and algorithmic bytes are accumulated per kernel class. */
int sgn_set_profiling(sgn_ctx* ctx, int on);

typedef struct sgn_kstat {
  char name[32];      /* kernel class */
  long long launches;
  double ms;          /* summed event-measured launch durations */
  double bytes;       /* summed algorithmic bytes */
  double flops;       /* summed algorithmic flops */
} sgn_kstat;

/* Copy up to max entries of the accumulated statistics; returns the count. */
int sgn_profile_read(const sgn_ctx* ctx, sgn_kstat* out, int max);
int sgn_profile_reset(sgn_ctx* ctx);

/* Host-only helper (no GPU needed): eigenvalues w (n complex) and unit-norm
 * right eigenvectors V (n x n column-major) of a dense complex n x n matrix
 * A (column-major), by Householder-Hessenberg reduction and shifted QR.  This
 * is the small eigensolver of the deflation setup.  SGN_ESINGULAR if the QR
 * iteration does not converge. */
int sgn_host_eig(int n, const double* A, double* w, double* V);

/* Copy the leading n x n block of the device composite matrix H of Eq.
 * (eq:newH) from the last apply (before the final re-orthogonalisation of
 * its last column in the delayed schedule) to host H (column-major), c0 =
 * S^dag x (m entries) and beta = |x_perp|.  Any pointer may be NULL. */
int sgn_debug_hessenberg(const sgn_ctx* ctx, int n, double* H, double* c0, double* beta);

/* ---- errors ------------------------------------------------------------ */
const char* sgn_strerror(int status);
const char* sgn_last_error(const sgn_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SGN_H */
