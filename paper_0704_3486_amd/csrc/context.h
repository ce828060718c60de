// The sgn_ctx structure shared by the translation units that drive kernels.
#pragma once

#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "krylov.h"

// Workspace of the batched apply (batch.hip): per slot r the Krylov columns,
// candidates, stencil results, composite Hessenberg matrix and coefficients,
// each at a fixed slot stride.  VT = FP64 (double2) or, in mixed precision,
// FP32 (float2) for the Krylov columns and stencil operands.
struct BatchWork {
  int nslots = 0, kcap = 0, ncap = 0, prec = -1, m = -1, lrm = -1;
  size_t ldq = 0;
  void* V = nullptr;         // [slot] ldq x (kcap + 1), VT
  size_t vstride = 0;
  double2* u = nullptr;      // [2][slot] ldq, FP64 candidates (ping-pong halves)
  void* ulo = nullptr;       // [2][slot] ldq, VT copies of the candidates (mixed)
  void* z = nullptr;         // [slot] ldq, VT stencil results
  double2* xin = nullptr;    // [slot] ldq, packed sources
  double2* y = nullptr;      // [slot] ldq, packed results
  double2* H = nullptr;      // [slot] ncap x ncap
  double2* F = nullptr;      // [launch slot] (m + kcap)^2, signs of one checkpoint
  double2* c0 = nullptr;     // [slot] max(m, 1)
  double2* lrc = nullptr;    // [slot] max(lr_m, 1): L^dag x of the LR-deflation
  double2* cv = nullptr;     // [2][slot] ncap, coefficients (ping-pong halves)
  double* beta = nullptr;    // [slot]
  double* err = nullptr;     // [slot]
  double* ref = nullptr;     // [slot] |x| (reference size of the first breakdown test)
  double* inv = nullptr;     // [slot] scratch of the source normalisation
  int* flag = nullptr;       // [slot] breakdown record
  int* fin = nullptr;        // [slot] non-finite input flag
  double* hpin = nullptr;    // pinned host mirror: err [slot], beta [slot], flag, fin [slot]
  GsWork gs;
  KrylovWork kw;
  DenseWork dense;
  BlockWork blk;  // block (s-step) process, per slot
  // checkpoint placement learned by earlier batched applies (as k_hint, rate_hint)
  int k_hint = 0;
  double tol_hint = 0.0;
  double rate_hint = 0.0;
  // captured runs of Arnoldi steps (sgn_set_step_graphs): the step index comes
  // from jdev; one graph per set of running slots and 32-column bucket of the
  // step index; they hold the workspace's addresses
  int* jdev = nullptr;
  std::map<std::pair<std::vector<int>, int>, hipGraphExec_t> graphs;

  void drop_graphs() {
    for (auto& g : graphs)
      if (g.second) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
  }

  size_t vt() const { return prec == SGN_PREC_MIXED ? sizeof(float2) : sizeof(double2); }
  void release() {
    drop_graphs();
    for (void** p : {&V, (void**)&u, &ulo, &z, (void**)&xin, (void**)&y, (void**)&H, (void**)&F, (void**)&c0,
                     (void**)&lrc, (void**)&cv, (void**)&beta, (void**)&err, (void**)&ref, (void**)&inv,
                     (void**)&flag, (void**)&fin, (void**)&jdev})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
    if (hpin) (void)hipHostFree(hpin);
    hpin = nullptr;
    gs_free(gs);
    krylov_free(kw);
    dense_destroy(dense);
    block_free(blk);
    nslots = kcap = ncap = 0;
    prec = m = lrm = -1;
  }
  // bytes ensure() allocates (kcap Krylov vectors for nslots right-hand sides)
  static size_t bytes(size_t ldq, int m, int kcap, int nslots, size_t vt) {
    const size_t ncap = (size_t)m + kcap + 1, n = (size_t)m + kcap, S = (size_t)nslots;
    size_t b = S * ldq * (kcap + 1) * vt;                    // V
    b += S * ldq * (2 * sizeof(double2) + 3 * vt + 2 * sizeof(double2));  // u, ulo, z, xin, y
    b += S * sizeof(double2) * (ncap * ncap + n * n + (size_t)std::max(m, 1) + 2 * ncap);  // H, F, c0, cv
    b += S * sizeof(double2) * 2 * (ncap + (ldq + 511) / 512 * ncap);  // dot partials, a, b
    b += 3 * sizeof(double2) * n * n * S;                    // sign work matrices
    return b;
  }
};

// default filter of the deflation eigensolver (sgn_set_deflation_filter)
constexpr int kDefaultFilterDegree = 16;
constexpr double kDefaultFilterCut = 1.0 / 16.0;

struct sgn_ctx {
  int device = -1;  // HIP device current at sgn_create
  Lattice lat{};
  int N = 0;
  size_t ldq = 0;
  double mu = 0, m_w = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  sgn_info info{};
  Profiler prof;

  double2* links = nullptr;  // [4][9][V]

  // deflation
  int m = 0;
  int defl_restarts = 0, defl_matvecs = 0;
  int defl_ncv = 0;  // Krylov subspace size of the deflation eigensolver (0: default rule)
  // Chebyshev filter of the deflation eigensolver: degree (0: A^2 itself) and
  // the damped interval's lower end as a fraction of A^2's spectral radius
  int defl_degree = kDefaultFilterDegree;
  double defl_cut = kDefaultFilterCut;
  int defl_used_degree = 0;  // last sgn_deflate: degree of the run that converged (0: unfiltered)
  double defl_alpha = 0.0, defl_beta = 0.0;
  double defl_residual = 0.0;
  double2* S = nullptr;       // internal layout, ldq x m
  std::vector<double2> T;     // host m x m (column-major, upper triangular)
  double2* Tdev = nullptr;    // m x m
  double2* sgnT = nullptr;    // m x m
  // LR-deflation pair, installed in place of a Schur pair (then m = 0 and
  // the Krylov part is the plain Arnoldi method): right and left critical
  // eigenvectors in the internal layout (ldq x lr_m, L^dag R = I), sgn of
  // their eigenvalues, and the per-apply coefficients L^dag x
  int lr_m = 0;
  double2* lrR = nullptr;
  double2* lrL = nullptr;
  double2* lrSgn = nullptr;       // lr_m entries (sgn Re lambda_i, 0)
  double2* lrC = nullptr;         // lr_m entries
  std::vector<double2> lrLam;     // host eigenvalues

  // Krylov workspace
  int kcap = 0;               // capacity in Krylov vectors
  int ncap = 0;               // m + kcap + 1 (columns of Q, rows of H)
  double2* Q = nullptr;       // ldq x ncap
  double2* Hc = nullptr;      // ncap x ncap, column-major (ld = ncap)
  double2* F = nullptr;       // sign output (m + kcap)^2, ld = n
  double2* wA = nullptr;
  double2* wB = nullptr;
  double2* xin = nullptr;
  double2* hbuf1 = nullptr;
  double2* hbuf2 = nullptr;
  double2* c0 = nullptr;
  double2* cvec = nullptr;
  double2* cprev = nullptr;
  double* scal = nullptr;     // [0] beta0 [1] inv_beta [2] err [3] scratch
  int* flag = nullptr;        // [0] breakdown/finite flag
  double* hpin = nullptr;     // pinned host mirror
  double2* wC = nullptr;
  // mixed precision: FP32 links, Krylov columns and stencil operands
  int prec = SGN_PREC_FP64;
  float2* links32 = nullptr;
  float2* V32 = nullptr;   // ldq x (kcap + 1)
  float2* u32a = nullptr;  // FP32 copies of the candidate (ping-pong)
  float2* u32b = nullptr;
  float2* z32 = nullptr;
  GsWork gs;
  KrylovWork kw;
  DenseWork dense;
  BatchWork bw;
  // convergence history of previous applies on this field (checkpoint placement only)
  int k_hint = 0;
  double tol_hint = 0.0;
  double rate_hint = 0.0;
  KrylovTune tune;  // launch shape of the Krylov dot/update passes (results do not depend on it)
  // captured Arnoldi steps: graph_steps consecutive steps of sgn_apply per
  // replay (0: direct launches), one graph per 32-column bucket of the basis
  // size, captured on cap_stream when first needed; they hold the workspace's
  // addresses and are dropped with it
  int graph_steps = 0;
  hipStream_t cap_stream = nullptr;
  int* jdev = nullptr;  // device step index read by the captured steps
  std::vector<hipGraphExec_t> graphs;
  int orth = 1;  // 0: two classical Gram-Schmidt passes per step; 1: one reduction, delayed re-orthogonalisation
  // block (s-step) Arnoldi process for FP64 applies: block size (0: off) and
  // the half-width of its Chebyshev interval (estimated on first use)
  int block_s = 0;
  double cheb_e = 0.0;
  BlockWork blk;
  int sessions = 0;  // open serving sessions (they hold the Schur pair and the precision fixed)

  ~sgn_ctx() { release(); }

  void release_workspace() {
    for (double2** p : {&Q, &Hc, &F, &wA, &wB, &wC, &xin, &hbuf1, &hbuf2, &c0, &cvec, &cprev})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
    for (float2** p : {&V32, &u32a, &u32b, &z32})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
    gs_free(gs);
    krylov_free(kw);
    block_free(blk);
    drop_graphs();
    if (jdev) (void)hipFree(jdev);
    jdev = nullptr;
    kcap = 0;
    ncap = 0;
  }

  void drop_lr() {
    for (double2** p : {&lrR, &lrL, &lrSgn, &lrC})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
    lrLam.clear();
    lr_m = 0;
  }

  void drop_graphs() {
    for (hipGraphExec_t& g : graphs)
      if (g) (void)hipGraphExecDestroy(g);
    graphs.clear();
    bw.drop_graphs();
  }

  void release() {
    if (stream || true) (void)hipDeviceSynchronize();
    release_workspace();
    dense_destroy(dense);
    bw.release();
    drop_lr();
    for (double2** p : {&links, &S, &Tdev, &sgnT})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
    if (links32) (void)hipFree(links32);
    links32 = nullptr;
    if (scal) (void)hipFree(scal);
    if (flag) (void)hipFree(flag);
    if (hpin) (void)hipHostFree(hpin);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    scal = nullptr;
    flag = nullptr;
    hpin = nullptr;
  }

  // make sure the Krylov workspace holds m + kmax + 1 columns
  void ensure_workspace(int kmax) {
    if (kmax <= kcap && Q) return;
    release_workspace();
    kcap = kmax;
    ncap = m + kcap + 1;
    // FP64 mode keeps S and the Krylov columns in one matrix; mixed mode keeps
    // only S in FP64 and the Krylov columns in V32
    const size_t qcols = (prec == SGN_PREC_MIXED) ? (size_t)std::max(m, 1) : (size_t)ncap;
    SGN_HIP(hipMalloc(&Q, sizeof(double2) * ldq * qcols));
    if (prec == SGN_PREC_MIXED) {
      SGN_HIP(hipMalloc(&V32, sizeof(float2) * ldq * (size_t)(kcap + 1)));
      SGN_HIP(hipMalloc(&u32a, sizeof(float2) * ldq));
      SGN_HIP(hipMalloc(&u32b, sizeof(float2) * ldq));
      SGN_HIP(hipMalloc(&z32, sizeof(float2) * ldq));
    }
    SGN_HIP(hipMalloc(&Hc, sizeof(double2) * (size_t)ncap * ncap));
    SGN_HIP(hipMalloc(&F, sizeof(double2) * (size_t)(m + kcap) * (m + kcap)));
    SGN_HIP(hipMalloc(&wA, sizeof(double2) * ldq));
    SGN_HIP(hipMalloc(&wB, sizeof(double2) * ldq));
    SGN_HIP(hipMalloc(&wC, sizeof(double2) * ldq));
    SGN_HIP(hipMalloc(&xin, sizeof(double2) * ldq));
    SGN_HIP(hipMalloc(&hbuf1, sizeof(double2) * (size_t)ncap));
    SGN_HIP(hipMalloc(&hbuf2, sizeof(double2) * (size_t)ncap));
    SGN_HIP(hipMalloc(&c0, sizeof(double2) * (size_t)(m > 0 ? m : 1)));
    SGN_HIP(hipMalloc(&cvec, sizeof(double2) * (size_t)ncap));
    SGN_HIP(hipMalloc(&cprev, sizeof(double2) * (size_t)ncap));
    SGN_HIP(hipMalloc(&jdev, sizeof(int)));
    gs_alloc(gs, N, ldq, std::max(ncap, lr_m));
    krylov_alloc(kw, N, ldq, ncap, 1);
    dense_reserve(dense, m + kcap, 1);
    // the Schur block of Q and of H never changes between applies
    if (m > 0) {
      SGN_HIP(hipMemcpy2D(Q, ldq * sizeof(double2), S, ldq * sizeof(double2), ldq * sizeof(double2), m,
                          hipMemcpyDeviceToDevice));
    }
    SGN_HIP(hipMemset(Hc, 0, sizeof(double2) * (size_t)ncap * ncap));
    if (m > 0) dev_copy_mat(Tdev, m, Hc, ncap, m, m, nullptr);
    SGN_HIP(hipDeviceSynchronize());
  }
};


// The adjoint problem on this context, for the duration of one call:
// A^dag = H_w(mu)^dag = H_w(-mu) (the time hops' e^{+mu} and e^{-mu}
// exchanged), with the LR pair's roles exchanged (L holds A^dag's right
// eigenvectors and R its left ones, for conj(Lambda), whose signs are those of
// Lambda).  Captured step graphs hold the forward phases among their kernel
// arguments, so none are replayed meanwhile.
struct AdjointScope {
  sgn_ctx* c;
  int graph_steps;
  explicit AdjointScope(sgn_ctx* cc) : c(cc), graph_steps(cc->graph_steps) {
    std::swap(c->lat.emu, c->lat.emmu);
    std::swap(c->lrR, c->lrL);
    c->graph_steps = 0;
  }
  ~AdjointScope() {
    std::swap(c->lat.emu, c->lat.emmu);
    std::swap(c->lrR, c->lrL);
    c->graph_steps = graph_steps;
  }
};

inline void check_adjoint(const sgn_ctx* c) {
  SGN_REQUIRE(c->m == 0, SGN_ESTATE,
              "the adjoint needs an LR pair (sgn_deflate_lr) or no deflation: a Schur basis of A is none of A^dag");
  SGN_REQUIRE(c->sessions == 0, SGN_ESTATE, "a serving session runs on this field");
}


// A block of the block Arnoldi process was not of full rank: the apply is
// repeated with one-vector steps.
struct BlockFallback {};

// 1.1 x the spectral radius of A^2 from an Arnoldi run of `steps` steps on A^2
// (deflate.hip)
double sq_radius_estimate(sgn_ctx* c, int steps, unsigned long long seed);

inline int fail(sgn_ctx* c, const SgnError& e) {
  if (c) c->last_error = e.msg;
  return e.status;
}

template <class F>
inline int guarded(sgn_ctx* c, F&& f) {
  if (!c) return SGN_ESTATE;
  try {
    return f();
  } catch (const SgnError& e) {
    return fail(c, e);
  } catch (const std::bad_alloc&) {
    return fail(c, SgnError{SGN_ENOMEM, "host allocation failed"});
  } catch (...) {
    return fail(c, SgnError{SGN_EHIP, "unexpected error"});
  }
}


// Install a partial Schur pair (S in the internal layout, device, ldq x m;
// T host column-major m x m, upper triangular) and compute sgn(T) on the device.
void install_schur_pair(sgn_ctx* c, int m, const double2* S_internal, const std::vector<double2>& T);
// Install an LR-deflation pair (R, L internal layout ldq x m, L^dag R = I;
// eigenvalues on the host) in place of any Schur pair.
void install_lr_pair(sgn_ctx* c, int m, const double2* R_internal, const double2* L_internal,
                     const std::vector<double2>& lam);
