// Internal declarations shared by the HIP translation units of libsgn.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sgn.h"

// ----------------------------------------------------------------------------
// complex helpers (double2 = re, im)
// ----------------------------------------------------------------------------
__host__ __device__ inline double2 cmake(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// acc + a * b
__host__ __device__ inline double2 cfma(double2 a, double2 b, double2 acc) {
  return make_double2(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}
// acc + conj(a) * b
__host__ __device__ inline double2 cfmac(double2 a, double2 b, double2 acc) {
  return make_double2(acc.x + a.x * b.x + a.y * b.y, acc.y + a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// i * a
__host__ __device__ inline double2 cmuli(double2 a) { return make_double2(-a.y, a.x); }
__host__ __device__ inline double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }

// ----------------------------------------------------------------------------
// status helpers
// ----------------------------------------------------------------------------
struct SgnError {
  int status;
  std::string msg;
};

#define SGN_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw SgnError{SGN_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)};     \
  } while (0)

#define SGN_REQUIRE(cond, st, msg)                 \
  do {                                             \
    if (!(cond)) throw SgnError{(st), (msg)};      \
  } while (0)

// ----------------------------------------------------------------------------
// kernel profiling (HIP events on the context stream)
// ----------------------------------------------------------------------------
// one class per kernel on the apply path, so that a class's average duration
// is that kernel's (the Gauss-Jordan class brackets all panels of one inverse)
enum KClass {
  K_WILSON = 0,      // wilson_hw_*_kernel
  K_KDOT,            // kdot_kernel
  K_KRED,            // kred_kernel
  K_KUPDATE,         // kupdate_kernel
  K_KCOMBINE,        // kcombine_kernel
  K_NS_GEMM,         // zgemm_kernel (Newton-Schulz)
  K_GJ_PANEL,        // gj_panel_kernel x panels (Newton inverse)
  K_NEWTON_COMBINE,  // newton_combine_kernel
  K_CGS_DOT,         // gs_dot_kernel (deflation setup)
  K_CGS_UPDATE,      // gs_update_kernel (deflation setup)
  K_BDOT,            // bdot_kernel (block steps: Q^dag W)
  K_BRED,            // bred_kernel (block steps: sum of the dot partials)
  K_BUPDATE,         // bupdate_kernel (block steps: W - Q C)
  K_BSMALL,          // bsmall_kernel (block steps: Cholesky factor and H times the coefficients)
  K_MISC,
  K_NCLASS
};

struct Profiler {
  bool on = false;
  hipStream_t stream = nullptr;
  long long launches[K_NCLASS] = {};
  double ms[K_NCLASS] = {};
  double bytes[K_NCLASS] = {};
  double flops[K_NCLASS] = {};
  struct Pending {
    hipEvent_t a, b;
    int cls;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t get_event();
  // bracket a launch: returns index of pending record or -1
  int begin(int cls);

  // count: launches the interval counts as (0: accounted by the caller)
  void end(int idx, double nbytes, double nflops, int count = 1);
  void flush();  // synchronise and accumulate the pending durations
  void reset();
  ~Profiler();
};

// Launch kernel<<<grid, block, shm, s>>>(args...); with profiling on, bracket
// it with events on s (recorded in stream order, so the interval never covers
// earlier work; it includes the launch gap, about 2 us on the 6^4 workload).
template <typename F, typename... Args>
inline void prof_launch(Profiler* prof, int cls, double nbytes, double nflops, F kernel, dim3 grid, dim3 block,
                        uint32_t shm, hipStream_t s, Args... args) {
  const int idx = prof ? prof->begin(cls) : -1;
  hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
  SGN_HIP(hipGetLastError());
  if (prof) prof->end(idx, nbytes, nflops);
}

// ----------------------------------------------------------------------------
// device workspace for Gram-Schmidt passes
// ----------------------------------------------------------------------------
struct GsWork {
  int nrt_dot = 0;      // row tiles of the dot kernel
  int nblk_upd = 0;     // 64-row blocks of the update kernel
  int ncol_cap = 0;     // max columns
  double2* P = nullptr;        // dot partials [nrt_dot][ncol_cap]
  double* normpart = nullptr;  // |w|^2 per update block [nblk_upd]
};

// GS kernels (gs.hip)
void gs_alloc(GsWork& g, int N, size_t ldq, int ncol_cap);
void gs_free(GsWork& g);
// h[c] = sum_i conj(Q[c][i]) w[i], c < ncol
void gs_dot(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* w, double2* h,
            hipStream_t s, Profiler* prof);
// w -= Q h ; if fin: also hout[c] = h1[c] + h[c] (h1 may be null), beta = |w|, inv_beta = 1/beta,
// breakdown flag when beta <= tiny * |hout|
struct GsFinal {
  const double2* h1;  // first-pass coefficients (nullable)
  double2* hout;      // ncol+1 outputs: sums, then beta as complex at hout[ncol] (nullable)
  double* beta;       // device scalar (nullable)
  double* inv_beta;   // device scalar (nullable)
  int* flag;          // device int: set to 1 on breakdown / non-finite (nullable)
};
// kval: Krylov dimension completed by this pass; a breakdown records flag = kval + 1
void gs_update(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* h, double2* w,
               const GsFinal* fin, int kval, hipStream_t s, Profiler* prof);
// beta = |w|, inv_beta = 1/beta (single vector, no projection)
void gs_norm(const GsWork& g, int N, const double2* w, double* beta, double* inv_beta, int* flag,
             hipStream_t s, Profiler* prof);

// Wilson kernels (wilson.hip)
struct Lattice {
  int L[4];
  int V;
  double kappa;
  double emu, emmu;  // e^{+mu}, e^{-mu}
  // stencil walk blocks (By, Bz, Bt): {0,0,0} the default rule, {-1,...} the
  // natural site order; otherwise these extents (results do not depend on it)
  int blk[3] = {0, 0, 0};
};
// links in the internal layout (rows 0, 1 of each SU(3) link; wilson_link_entries(V)
// complex entries); *bad = 1 (device) for a link that is not SU(3) to 1e-10
void wilson_pack_links(const Lattice& lat, const double2* gauge_abi, double2* links, int* bad, hipStream_t s);
size_t wilson_link_entries(int V);
void wilson_pack(const Lattice& lat, const double2* x_abi, double2* v, hipStream_t s);
void wilson_unpack(const Lattice& lat, const double2* v, double2* y_abi, hipStream_t s);
// walk blocks acceptable for this lattice (0,0,0: default; negative By: natural order)
bool wilson_blocks_valid(const Lattice& lat, int By, int Bz, int Bt);
// y = x + gamma5 y over n entries in the interface layout (n a multiple of 12)
void overlap_finish(const double2* x, double2* y, size_t n, hipStream_t s);
// D_ov^dag x = x + sgn^dag (gamma5 x): y = gamma5 x, then (after the sign) y = x + y
void overlap_adjoint_start(const double2* x, double2* y, size_t n, hipStream_t s);
void overlap_adjoint_finish(const double2* x, double2* y, size_t n, hipStream_t s);
// y = a x + b g y with g = gamma5 (g5) or 1, interface layout, n entries; x may be y
void axpby_abi(const double2* x, double2* y, double a, double b, bool g5, size_t n, hipStream_t s);
// out = H_w(mu) (in * scale), optional copy_out = in * scale; scale = *inv_beta (or 1 if null)
void wilson_apply(const Lattice& lat, const double2* links, const double2* in, double2* out,
                  const double* inv_beta, double2* copy_out, hipStream_t s, Profiler* prof);


// most right-hand sides one launch carries; launch index z (blockIdx) works
// on slot[z], aux[z] is a per-slot integer the caller defines
constexpr int kMaxBatch = 64;
struct SlotMap {
  int n = 0;
  int slot[kMaxBatch] = {};
  int aux[kMaxBatch] = {};
};

// Out_slot = H_w(mu) In_slot for the slots of map (one hop per thread, the
// same arithmetic per slot as wilson_apply), In/Out at fixed slot strides
template <typename C>
void wilson_apply_slots(const Lattice& lat, const C* links, const C* in, size_t istride, C* out, size_t ostride,
                        const SlotMap& map, hipStream_t s, Profiler* prof);

// Out_r = H_w(mu) In_r for nrhs vectors at fixed strides, one launch.  split: one
// hop per thread for every right-hand side (each result bitwise independent of
// nrhs); otherwise, for nrhs >= 2, one site per thread with the link shared.
void wilson_apply_multi(const Lattice& lat, const double2* links, const double2* in, size_t istride, double2* out,
                        size_t ostride, int nrhs, bool split, hipStream_t s, Profiler* prof);
// FP32 links and spinors (mixed precision)
void wilson_apply_multi32(const Lattice& lat, const float2* links, const float2* in, size_t istride, float2* out,
                          size_t ostride, int nrhs, bool split, hipStream_t s, Profiler* prof);
void wilson_links_f32(const double2* links, float2* links32, int V, hipStream_t s);

// workspace of the block (s-step) Arnoldi process (block.hip), per slot at
// the given strides (nslots right-hand sides)
constexpr int kBlockMax = 16;  // largest block
struct BlockWork {
  int ncap = 0;               // basis columns the buffers serve
  int nslots = 0;
  double2* W = nullptr;       // ldq x kBlockMax block vectors
  double2* part = nullptr;    // dot partials [chunk][column][kBlockMax]
  double2* C1 = nullptr;      // [ncap][kBlockMax] first-pass coefficients
  double2* C2 = nullptr;      // [ncap][kBlockMax] second-pass coefficients
  double2* Ct = nullptr;      // [ncap][kBlockMax] their sum
  double2* P = nullptr;       // [kBlockMax][ncap] H times Ct
  double2* G = nullptr;       // [kBlockMax][kBlockMax] Gram matrix of the projected block
  double2* R = nullptr;       // [3][kBlockMax][kBlockMax]: Cholesky factor R, R^-1, Rb^-1
  int* flag = nullptr;        // set when a block is not of full rank
  size_t wstride = 0, pstride = 0, cstride = 0, gstride = 0, rstride = 0;
};
void block_alloc(BlockWork& b, int N, size_t ldq, int ncap, int nslots);
void block_free(BlockWork& b);
// The composite bases of one launch of the block process: Schur columns S
// (m, shared), Krylov columns V_r = V + r vstride (basis column c >= m is
// V_r[c - m]), Hessenberg matrices H + r hstride (ld ldh); nb slots act[z];
// p + s <= ncap for every block.
struct BlockSpan {
  const double2* S = nullptr;
  double2* V = nullptr;
  size_t vstride = 0, ldq = 0;
  int m = 0, N = 0, ncap = 0;
  double2* H = nullptr;
  size_t hstride = 0;
  int ldh = 0;
  int nb = 0;
  int act[kMaxBatch] = {};
};
// v_1 of every slot: V_r[0] = u_r * inv_r (u at ustride, inv at istride)
void block_first(const BlockSpan& sp, const double2* u, size_t ustride, const double* inv, int istride,
                 hipStream_t s);
// One block of sb <= kBlockMax Arnoldi steps from k finished steps for every
// slot: basis columns m + k + 1 .. m + k + sb and Hessenberg columns
// m + k .. m + k + sb - 1; e: half-width of the Chebyshev interval.  A block
// that is not of full rank raises its slot's b.flag.
void block_step(const BlockSpan& sp, BlockWork& b, const Lattice& lat, const double2* links, int k, int sb, double e,
                hipStream_t s, Profiler* prof);

// Out_r = ca H_w(mu) In_r + cb Prev_r (Prev nullable) for the slots of map,
// at fixed slot strides: one step of a three-term polynomial recurrence in
// the stencil
void wilson_apply_cheb_slots(const Lattice& lat, const double2* links, const double2* in, size_t istride,
                             double2* out, size_t ostride, const double2* prev, size_t pstride, double ca, double cb,
                             const SlotMap& map, hipStream_t s, Profiler* prof);

// dense kernels (dense.hip)
struct DenseWork {
  int method = 0;         // 0: Newton-Schulz with Roberts/Gauss-Jordan fallback; 1: Roberts only
  double* spart = nullptr;  // Newton-Schulz residual partials
  size_t nspart = 0;
  int* ns_state = nullptr;  // Newton-Schulz per-matrix state [nb] and iterations [nb]
  int* host_state = nullptr;  // pinned mirror
  int nstate = 0;
  int last_iters = 0;       // iterations the previous call needed (when the host first looks)
  int ncap = 0;
  int nbcap = 0;          // matrices per batch
  int* host_flag = nullptr;
  double2* S = nullptr;   // n x n iterate
  double2* Ma = nullptr;  // Gauss-Jordan ping-pong
  double2* Mb = nullptr;
  int* rowpiv = nullptr;  // pivot row of each column
  double* logpiv = nullptr;
  double* scal = nullptr;  // [0] change, [1] |S|, [2] prev change, [3] mu
  double* host_scal = nullptr;  // pinned mirror
  int* flag = nullptr;          // singular flag
  unsigned* counters = nullptr;
  double* part = nullptr;  // reduction partials
  int npart = 0;
};
void dense_alloc(DenseWork& d, int n);
void dense_alloc(DenseWork& d, int n, int nb);
// free the buffers
void dense_free(DenseWork& d);
void dense_destroy(DenseWork& d);
// allocate everything dense_sign_batched needs up to order n and batch nb,
// so that later calls of at most that size allocate nothing
void dense_reserve(DenseWork& d, int n, int nb);
// F = sgn(A) (n x n, ld = lda); returns iterations; throws SGN_ESINGULAR.
// radius: an estimate of the spectral radius of A's eigenvalues of largest
// modulus (0: none); see dense_sign_batched
int dense_sign(DenseWork& d, int n, const double2* A, int lda, double2* F, int ldf, hipStream_t s,
               Profiler* prof, double radius = 0.0);
// F_b = sgn(A_b) for nb <= kMaxBatch matrices at strides astride / fstride;
// each matrix stops on its own test, so F_b is bitwise the single-matrix result.
// The Newton-Schulz start X_0 = A / |A|_1, or A / max(radius, |A|_1 / 1.5)
// when 0 < radius < |A|_1: the composite Arnoldi matrices' largest Ritz
// values sit near the operator's spectral radius, well below the 1-norm
// (1.6-1.9x at 4^4-6^4), and the smaller divisor saves steps that grow the
// small eigenvalues; the bound keeps every |z| <= 1.5, inside the
// iteration's basin on the real axis
int dense_sign_batched(DenseWork& d, int n, int nb, const double2* A, int lda, size_t astride, double2* F, int ldf,
                       size_t fstride, hipStream_t s, Profiler* prof, double radius = 0.0);
// c[i] = sum_{q<m} F[i][q] c0[q] + beta * F[i][m]  (i < n); err = |c - cprev_pad| / |c| if cprev
void dense_coeffs(int n, int m, const double2* F, int ldf, const double2* c0, const double* beta, double2* c,
                  const double2* cprev, int nprev, double* err, hipStream_t s);
// dense_coeffs for map.n matrices: F_z (stride fstride) belongs to slot
// r = map.slot[z]; c0, beta, c, cprev, err are indexed by r; map.aux[z] is
// that slot's nprev (< 0: no previous coefficients)
void dense_coeffs_batched(int n, int m, const double2* F, int ldf, size_t fstride, const double2* c0, int c0stride,
                          const double* beta, double2* c, const double2* cprev, int cstride, const SlotMap& map,
                          double* err, hipStream_t s);
// zero a device vector
void dev_zero(double2* p, size_t n, hipStream_t s);
void dev_copy_mat(const double2* A, int lda, double2* B, int ldb, int rows, int cols, hipStream_t s);
// w += sum_c Q[c] h[c]
void gs_add(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* h, double2* w,
            hipStream_t s, Profiler* prof);
// y = sum_c Q[c] coef[c]  (fresh output)
void gs_combine(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* coef,
                double2* y, double2* scratch_neg, hipStream_t s, Profiler* prof);
// out = -in
void dev_negate(const double2* in, double2* out, int n, hipStream_t s);
// C = A B (column-major, complex; matrix-core kernel of zgemm.hip, deterministic)
void dev_zgemm_nn(DenseWork& d, int M, int N, int K, const double2* A, int lda, const double2* B, int ldb,
                  double2* C, int ldc, hipStream_t s);
// x[i] = a[i] x[i] (complex, n entries)
void dev_cmul(const double2* a, double2* x, int n, hipStream_t s);
// precision conversion
void dev_to_f32(const double2* in, float2* out, size_t n, hipStream_t s);
// any non-finite entry -> flag = 1
void dev_check_finite(const double2* v, size_t n, int* flag, hipStream_t s);

// complex FP64 products on the matrix cores (zgemm.hip)
// C_b = alpha A_b B_b (M x K times K x N, column-major) for nb matrices at strides
void zgemm(int M, int N, int K, double alpha, const double2* A, int lda, size_t astride, const double2* B, int ldb,
           size_t bstride, double2* C, int ldc, size_t cstride, int nb, hipStream_t s);
// Newton-Schulz step of nb n x n matrices at stride `stride`: Y = 3I - X X with
// per-wavefront partials of |X X - I|^2 (zgemm_ns_parts(n, nb) per matrix),
// skipped for matrices whose state is not 0
void zgemm_ns_square(int n, const double2* X, double2* Y, size_t stride, int nb, const int* state, double* part,
                     hipStream_t s);
// Xn = X Y / 2, also into F_b (ld ldf, stride fstride) where state == 1;
// skipped where state > 1
void zgemm_ns_update(int n, const double2* X, const double2* Y, double2* Xn, size_t stride, int nb, const int* state,
                     double2* F, int ldf, size_t fstride, hipStream_t s);
int zgemm_ns_parts(int n, int nb);
// per matrix: residual from the partials and the state transition of iteration it
void ns_check(const double* part, int nparts, int n, int* state, int* iters, int it, int maxit, int nb,
              hipStream_t s);
