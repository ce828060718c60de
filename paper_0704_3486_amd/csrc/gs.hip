// Classical Gram-Schmidt passes against the composite basis Q = (S_m V_j)
// (Section 5.2, step (iv): every new vector is orthogonalised against the
// Schur vectors and all previous Arnoldi vectors).
//
// Q is column-major with leading dimension ldq; a pass is
//     h = Q^dag w            (gs_dot:    tall-skinny GEMV^H, HBM-bound)
//     w = w - Q h            (gs_update: tall-skinny GEMV,   HBM-bound)
// For a single right-hand side these are matrix-vector products (0.5 flop
// per byte), so they are written as streaming kernels, not MFMA tiles.
//
// Reductions are deterministic: partial sums are written per row tile and
// combined in a fixed order by a separate small kernel, so a result is
// bitwise reproducible for a given problem shape.  No kernel synchronises
// with another workgroup.
#include <algorithm>

#include "internal.h"

namespace {

constexpr int kDotRpl = 8;                     // dot: rows per lane
constexpr int kDotRows = 64 * kDotRpl;         // dot: rows per tile (512)
constexpr int kDotCpw = 4;                     // dot: columns per wavefront
constexpr int kDotCols = 4 * kDotCpw;          // dot: columns per workgroup (4 wavefronts)
constexpr int kUpdWaves = 8;                   // update: wavefronts per 64-row workgroup
constexpr int kUpdThreads = 64 * kUpdWaves;
constexpr int kUpdBatch = 8;                   // update: column loads issued together per lane

__device__ inline double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

__device__ inline double wave_sum1(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// partial sums P[rt][c] = sum over the rows of tile rt of conj(Q[c][i]) w[i];
// workgroup id = rt + nrt cg, column group cg = 16 columns (4 per wavefront).
// Rows past N carry zero weight and load row N-1 (unconditional loads).
__global__ void __launch_bounds__(256)
gs_dot_part_kernel(const double2* __restrict__ Q, size_t ldq, int N, int ncol, const double2* __restrict__ w,
                   double2* __restrict__ P, int ldp, int nrt) {
  const int rt = blockIdx.x % nrt, cg = blockIdx.x / nrt;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row0 = rt * kDotRows;
  double2 wv[kDotRpl];
#pragma unroll
  for (int t = 0; t < kDotRpl; ++t) {
    const int i = row0 + t * 64 + lane;
    wv[t] = (i < N) ? w[i] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int cc = 0; cc < kDotCpw; ++cc) {
    const int c = (cg * 4 + wave) * kDotCpw + cc;
    if (c < ncol) {
      const double2* __restrict__ q = Q + (size_t)c * ldq;
      double2 qv[kDotRpl];
#pragma unroll
      for (int t = 0; t < kDotRpl; ++t) qv[t] = q[min(row0 + t * 64 + lane, N - 1)];
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < kDotRpl; ++t) acc = cfmac(qv[t], wv[t], acc);
      acc = wave_sum(acc);
      if (lane == 0) P[(size_t)rt * ldp + c] = acc;
    }
  }
}

// h[c] = sum over row tiles of P[rt][c] in a fixed order: 32 columns per
// workgroup, 8 threads per column (each sums every 8th tile), then in order
__global__ void __launch_bounds__(256)
gs_dot_red_kernel(const double2* __restrict__ P, int ldp, int nrt, int ncol, double2* __restrict__ h) {
  const int cl = threadIdx.x & 31, part = threadIdx.x >> 5;
  const int c = blockIdx.x * 32 + cl;
  const double2 zero = make_double2(0.0, 0.0);
  double2 acc = zero;
  // tiles t = part, part + 8, ... in that order, eight loads in flight
  if (c < ncol)
    for (int t0 = part; t0 < nrt; t0 += 64) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (t0 + 8 * u < nrt) ? P[(size_t)(t0 + 8 * u) * ldp + c] : zero;
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
    }
  __shared__ double2 red[8][33];
  red[part][cl] = acc;
  __syncthreads();
  if (part == 0 && c < ncol) {
    double2 sum = red[0][cl];
    for (int q = 1; q < 8; ++q) sum = cadd(sum, red[q][cl]);
    h[c] = sum;
  }
}

struct FinDev {
  const double2* h1;
  double2* hout;
  double* beta;
  double* inv_beta;
  int* flag;
  int kval;  // Krylov dimension this pass completes (for the breakdown record)
  int active;
};

// w += sgn Q h: each workgroup owns 64 rows and all columns; its wavefronts
// take the columns c = wave, wave + 8, ... (batches of kUpdBatch loads in
// flight; past ncol, column ncol-1 is reloaded with weight zero) and are
// combined in LDS in a fixed order.  With want_norm, normpart[blk] = |w|^2
// over the block's rows.
__global__ void __launch_bounds__(kUpdThreads)
gs_update_kernel(const double2* __restrict__ Q, size_t ldq, int N, int ncol, const double2* __restrict__ h,
                 double sgn, double2* __restrict__ w, double* __restrict__ normpart, int want_norm) {
  const int blk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = blk * 64 + lane;
  const bool ok = i < N;
  const int il = ok ? i : N - 1;
  const double2 zero = make_double2(0.0, 0.0);
  double2 acc = zero;
  for (int c = wave; c < ncol; c += kUpdBatch * kUpdWaves) {
    double2 qv[kUpdBatch], hv[kUpdBatch];
#pragma unroll
    for (int t = 0; t < kUpdBatch; ++t) {
      const int cc = c + t * kUpdWaves, cl = min(cc, ncol - 1);
      qv[t] = Q[(size_t)cl * ldq + il];
      hv[t] = (cc < ncol) ? h[cl] : zero;
    }
#pragma unroll
    for (int t = 0; t < kUpdBatch; ++t) acc = cfma(qv[t], hv[t], acc);
  }
  __shared__ double2 ps[kUpdWaves][64];
  ps[wave][lane] = acc;
  __syncthreads();
  if (wave != 0) return;
  double2 sum = ps[0][lane];
#pragma unroll
  for (int q = 1; q < kUpdWaves; ++q) sum = cadd(sum, ps[q][lane]);
  double nrm = 0.0;
  if (ok) {
    const double2 wi = make_double2(w[i].x + sgn * sum.x, w[i].y + sgn * sum.y);
    w[i] = wi;
    nrm = cabs2(wi);
  }
  if (want_norm) {
    nrm = wave_sum1(nrm);
    if (lane == 0) normpart[blk] = nrm;
  }
}

// beta = |w| from the block partials (fixed order), then the coefficient
// column hout = h1 + h with beta appended, 1/beta and the breakdown record
__global__ void __launch_bounds__(256)
gs_final_kernel(const double* __restrict__ normpart, int nblk, int ncol, const double2* __restrict__ h, FinDev fin) {
  const int tid = threadIdx.x;
  __shared__ double tred[256];
  double s = 0.0;
  for (int r = tid; r < nblk; r += 256) s += normpart[r];
  tred[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) tred[tid] += tred[tid + off];
    __syncthreads();
  }
  const double beta = sqrt(tred[0]);
  __shared__ double hn2[256];
  double hsum = 0.0;
  if (fin.hout) {
    for (int c = tid; c < ncol; c += 256) {
      double2 v = h[c];
      if (fin.h1) v = cadd(v, fin.h1[c]);
      fin.hout[c] = v;
      hsum += cabs2(v);
    }
  }
  hn2[tid] = hsum;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) hn2[tid] += hn2[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    const double hnorm = sqrt(hn2[0]);
    const bool finite = isfinite(beta) && isfinite(hnorm);
    // invariant Krylov space: the new vector is at the rounding level of the
    // coefficients removed from it
    const bool brk = !(beta > 1e-12 * fmax(hnorm, 1e-300)) || beta == 0.0;
    if (fin.hout) fin.hout[ncol] = make_double2(finite ? beta : 0.0, 0.0);
    if (fin.beta) *fin.beta = beta;
    if (fin.inv_beta) *fin.inv_beta = (finite && !brk) ? 1.0 / beta : 0.0;
    if (fin.flag) {
      if (!finite)
        *fin.flag = -1;
      else if (brk && *fin.flag == 0)
        *fin.flag = fin.kval + 1;
    }
  }
}

}  // namespace

void gs_alloc(GsWork& g, int N, size_t ldq, int ncol_cap) {
  gs_free(g);
  (void)ldq;
  g.nrt_dot = (N + kDotRows - 1) / kDotRows;
  g.nblk_upd = (N + 63) / 64;
  g.ncol_cap = ncol_cap;
  SGN_HIP(hipMalloc(&g.P, sizeof(double2) * (size_t)g.nrt_dot * std::max(ncol_cap, 1)));
  SGN_HIP(hipMalloc(&g.normpart, sizeof(double) * (size_t)g.nblk_upd));
}

void gs_free(GsWork& g) {
  if (g.P) (void)hipFree(g.P);
  if (g.normpart) (void)hipFree(g.normpart);
  g = GsWork{};
}

void gs_dot(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* w, double2* h,
            hipStream_t s, Profiler* prof) {
  if (ncol <= 0) return;
  SGN_REQUIRE(ncol <= g.ncol_cap, SGN_EINVAL, "gs_dot: ncol exceeds workspace");
  const size_t nwg = (size_t)g.nrt_dot * ((ncol + kDotCols - 1) / kDotCols);
  SGN_REQUIRE(nwg * 256 < (size_t(1) << 32), SGN_EINVAL, "gs_dot: grid too large");
  const int idx = prof ? prof->begin(K_CGS_DOT) : -1;
  hipLaunchKernelGGL(gs_dot_part_kernel, dim3((unsigned)nwg), dim3(256), 0, s, Q, ldq, N, ncol, w, g.P,
                     g.ncol_cap, g.nrt_dot);
  SGN_HIP(hipGetLastError());
  hipLaunchKernelGGL(gs_dot_red_kernel, dim3((unsigned)((ncol + 31) / 32)), dim3(256), 0, s, g.P, g.ncol_cap,
                     g.nrt_dot, ncol, h);
  SGN_HIP(hipGetLastError());
  if (prof) prof->end(idx, 16.0 * ((double)N * ncol + N + ncol), 8.0 * (double)N * ncol);
}

static void update_launch(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* h,
                          double sgn, double2* w, const GsFinal* fin, int kval, hipStream_t s, Profiler* prof) {
  SGN_REQUIRE(ncol >= 0 && ncol <= g.ncol_cap, SGN_EINVAL, "gs_update: ncol exceeds workspace");
  SGN_REQUIRE((size_t)g.nblk_upd * kUpdThreads < (size_t(1) << 32), SGN_EINVAL, "gs_update: grid too large");
  const int idx = prof ? prof->begin(K_CGS_UPDATE) : -1;
  hipLaunchKernelGGL(gs_update_kernel, dim3(g.nblk_upd), dim3(kUpdThreads), 0, s, Q, ldq, N, ncol, h, sgn, w,
                     g.normpart, fin ? 1 : 0);
  SGN_HIP(hipGetLastError());
  if (fin) {
    FinDev fd{};
    fd.h1 = fin->h1;
    fd.hout = fin->hout;
    fd.beta = fin->beta;
    fd.inv_beta = fin->inv_beta;
    fd.flag = fin->flag;
    fd.kval = kval;
    fd.active = 1;
    hipLaunchKernelGGL(gs_final_kernel, dim3(1), dim3(256), 0, s, g.normpart, g.nblk_upd, ncol, h, fd);
    SGN_HIP(hipGetLastError());
  }
  if (prof) prof->end(idx, 16.0 * ((double)N * ncol + 2.0 * N + ncol), 8.0 * (double)N * ncol);
}

void gs_update(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* h, double2* w,
               const GsFinal* fin, int kval, hipStream_t s, Profiler* prof) {
  update_launch(g, Q, ldq, N, ncol, h, -1.0, w, fin, kval, s, prof);
}

void gs_add(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* h, double2* w,
            hipStream_t s, Profiler* prof) {
  update_launch(g, Q, ldq, N, ncol, h, +1.0, w, nullptr, 0, s, prof);
}

void gs_norm(const GsWork& g, int N, const double2* w, double* beta, double* inv_beta, int* flag,
             hipStream_t s, Profiler* prof) {
  GsFinal fin{nullptr, nullptr, beta, inv_beta, flag};
  update_launch(g, nullptr, 0, N, 0, nullptr, -1.0, const_cast<double2*>(w), &fin, 0, s, prof);
}

void gs_combine(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* coef, double2* y,
                double2* /*scratch*/, hipStream_t s, Profiler* prof) {
  dev_zero(y, (size_t)N, s);
  update_launch(g, Q, ldq, N, ncol, coef, +1.0, y, nullptr, 0, s, prof);
}
