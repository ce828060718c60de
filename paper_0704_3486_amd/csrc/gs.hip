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
// Reductions are deterministic: partial sums are combined in a fixed order by
// the last workgroup to finish (atomic ticket + device-scope fences), so a
// result is bitwise reproducible for a given problem shape.
#include "internal.h"

namespace {

constexpr int kDotRpl = 16;                 // rows per lane
constexpr int kDotCpw = 4;                  // columns per wavefront
constexpr int kDotWaves = 4;                // wavefronts per workgroup
constexpr int kDotRows = 64 * kDotRpl;      // rows per tile (1024)
constexpr int kDotCols = kDotCpw * kDotWaves;  // columns per workgroup (16)

constexpr int kUpdRpt = 4;                  // rows per thread
constexpr int kUpdRows = 256 * kUpdRpt;     // rows per tile (1024)
constexpr int kUpdCols = 32;                // columns per workgroup

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

// Atomic ticket: returns true in every thread of the workgroup that finished last.
__device__ inline bool last_block(unsigned* counter, unsigned total) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == total - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = is_last != 0;
  if (last) __threadfence();
  return last;
}

__device__ inline void reset_counter(unsigned* counter) {
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256)
gs_dot_kernel(const double2* __restrict__ Q, size_t ldq, int N, int ncol, const double2* __restrict__ w,
              double2* __restrict__ P, int ldp, double2* __restrict__ h, unsigned* __restrict__ counters,
              int nrt) {
  const int rt = blockIdx.x, cg = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = rt * kDotRows;
  double2 wv[kDotRpl];
#pragma unroll
  for (int r = 0; r < kDotRpl; ++r) {
    const int i = row0 + r * 64 + lane;
    wv[r] = (i < N) ? w[i] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int cc = 0; cc < kDotCpw; ++cc) {
    const int c = cg * kDotCols + wave * kDotCpw + cc;
    if (c < ncol) {
      const double2* __restrict__ q = Q + (size_t)c * ldq;
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < kDotRpl; ++r) {
        const int i = row0 + r * 64 + lane;
        if (i < N) acc = cfmac(q[i], wv[r], acc);
      }
      acc = wave_sum(acc);
      if (lane == 0) P[(size_t)rt * ldp + c] = acc;
    }
  }
  if (!last_block(&counters[cg], (unsigned)nrt)) return;
  // fixed-order reduction over row tiles: 16 columns x 16 interleaved subsets
  __shared__ double2 red[16][kDotCols + 1];
  const int cc = threadIdx.x & 15, sub = threadIdx.x >> 4;
  const int c = cg * kDotCols + cc;
  double2 acc = make_double2(0.0, 0.0);
  if (c < ncol)
    for (int r = sub; r < nrt; r += 16) acc = cadd(acc, P[(size_t)r * ldp + c]);
  red[sub][cc] = acc;
  __syncthreads();
  if (threadIdx.x < 16 && c < ncol) {
    double2 s = red[0][cc];
    for (int k = 1; k < 16; ++k) s = cadd(s, red[k][cc]);
    h[c] = s;
  }
  reset_counter(&counters[cg]);
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

__global__ void __launch_bounds__(256)
gs_update_kernel(const double2* __restrict__ Q, size_t ldq, int N, int ncol, const double2* __restrict__ h,
                 double sgn, double2* __restrict__ w, double2* __restrict__ Upart, int ngroups,
                 unsigned* __restrict__ cnt_rows, unsigned* __restrict__ cnt_norm, int nrt,
                 double* __restrict__ normpart, FinDev fin) {
  const int rt = blockIdx.x, g = blockIdx.y;
  const int tid = threadIdx.x;
  const int row0 = rt * kUpdRows;
  __shared__ double2 hs[kUpdCols];
  const int c0 = g * kUpdCols;
  const int nc = min(kUpdCols, ncol - c0);
  if (tid < nc) hs[tid] = h[c0 + tid];
  __syncthreads();
  double2 u[kUpdRpt];
#pragma unroll
  for (int r = 0; r < kUpdRpt; ++r) u[r] = make_double2(0.0, 0.0);
  for (int c = 0; c < nc; ++c) {
    const double2* __restrict__ q = Q + (size_t)(c0 + c) * ldq;
    const double2 hc = hs[c];
#pragma unroll
    for (int r = 0; r < kUpdRpt; ++r) {
      const int i = row0 + r * 256 + tid;
      if (i < N) u[r] = cfma(q[i], hc, u[r]);
    }
  }
  if (ngroups > 1) {
#pragma unroll
    for (int r = 0; r < kUpdRpt; ++r) {
      const int i = row0 + r * 256 + tid;
      if (i < N) Upart[(size_t)g * ldq + i] = u[r];
    }
    if (!last_block(&cnt_rows[rt], (unsigned)ngroups)) return;
#pragma unroll
    for (int r = 0; r < kUpdRpt; ++r) {
      const int i = row0 + r * 256 + tid;
      double2 s = make_double2(0.0, 0.0);
      if (i < N)
        for (int gg = 0; gg < ngroups; ++gg) s = cadd(s, Upart[(size_t)gg * ldq + i]);
      u[r] = s;
    }
    reset_counter(&cnt_rows[rt]);
  }
  double nrm = 0.0;
#pragma unroll
  for (int r = 0; r < kUpdRpt; ++r) {
    const int i = row0 + r * 256 + tid;
    if (i < N) {
      const double2 wi = make_double2(w[i].x + sgn * u[r].x, w[i].y + sgn * u[r].y);
      w[i] = wi;
      nrm += cabs2(wi);
    }
  }
  if (!fin.active) return;
  // workgroup sum of |w|^2 over this row tile, fixed order
  __shared__ double wred[4];
  nrm = wave_sum1(nrm);
  if ((tid & 63) == 0) wred[tid >> 6] = nrm;
  __syncthreads();
  if (tid == 0) normpart[rt] = ((wred[0] + wred[1]) + wred[2]) + wred[3];
  if (!last_block(cnt_norm, (unsigned)nrt)) return;
  __shared__ double tred[256];
  double s = 0.0;
  for (int r = tid; r < nrt; r += 256) s += normpart[r];
  tred[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) tred[tid] += tred[tid + off];
    __syncthreads();
  }
  const double beta = sqrt(tred[0]);
  // coefficient column: hout = h1 + h, then beta (as a complex entry)
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
  reset_counter(cnt_norm);
}

}  // namespace

void gs_alloc(GsWork& g, int N, size_t ldq, int ncol_cap) {
  gs_free(g);
  g.nrt_dot = (N + kDotRows - 1) / kDotRows;
  g.nrt_upd = (N + kUpdRows - 1) / kUpdRows;
  g.ncol_cap = ncol_cap;
  g.ngroups_cap = (ncol_cap + kUpdCols - 1) / kUpdCols;
  const int ndotgroups = (ncol_cap + kDotCols - 1) / kDotCols;
  g.ncounters = ndotgroups + g.nrt_upd + 1;
  SGN_HIP(hipMalloc(&g.P, sizeof(double2) * (size_t)g.nrt_dot * ncol_cap));
  SGN_HIP(hipMalloc(&g.Upart, sizeof(double2) * ldq * (size_t)(g.ngroups_cap > 1 ? g.ngroups_cap : 1)));
  SGN_HIP(hipMalloc(&g.normpart, sizeof(double) * (size_t)g.nrt_upd));
  SGN_HIP(hipMalloc(&g.counters, sizeof(unsigned) * (size_t)g.ncounters));
  SGN_HIP(hipMemset(g.counters, 0, sizeof(unsigned) * (size_t)g.ncounters));
  SGN_HIP(hipDeviceSynchronize());
}

void gs_free(GsWork& g) {
  if (g.P) (void)hipFree(g.P);
  if (g.Upart) (void)hipFree(g.Upart);
  if (g.normpart) (void)hipFree(g.normpart);
  if (g.counters) (void)hipFree(g.counters);
  g = GsWork{};
}

void gs_dot(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* w, double2* h,
            hipStream_t s, Profiler* prof) {
  if (ncol <= 0) return;
  SGN_REQUIRE(ncol <= g.ncol_cap, SGN_EINVAL, "gs_dot: ncol exceeds workspace");
  const int ngroups = (ncol + kDotCols - 1) / kDotCols;
  const int idx = prof ? prof->begin(K_CGS_DOT) : -1;
  hipLaunchKernelGGL(gs_dot_kernel, dim3(g.nrt_dot, ngroups), dim3(256), 0, s, Q, ldq, N, ncol, w, g.P,
                     g.ncol_cap, h, g.counters, g.nrt_dot);
  SGN_HIP(hipGetLastError());
  if (prof) prof->end(idx, 16.0 * ((double)N * ncol + N + ncol), 8.0 * (double)N * ncol);
}

static void update_launch(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* h,
                          double sgn, double2* w, const GsFinal* fin, int kval, hipStream_t s, Profiler* prof) {
  SGN_REQUIRE(ncol >= 0 && ncol <= g.ncol_cap, SGN_EINVAL, "gs_update: ncol exceeds workspace");
  const int ngroups = ncol > 0 ? (ncol + kUpdCols - 1) / kUpdCols : 1;
  FinDev fd{};
  if (fin) {
    fd.h1 = fin->h1;
    fd.hout = fin->hout;
    fd.beta = fin->beta;
    fd.inv_beta = fin->inv_beta;
    fd.flag = fin->flag;
    fd.kval = kval;
    fd.active = 1;
  }
  const int ndotgroups = (g.ncol_cap + kDotCols - 1) / kDotCols;
  unsigned* cnt_rows = g.counters + ndotgroups;
  unsigned* cnt_norm = cnt_rows + g.nrt_upd;
  const int idx = prof ? prof->begin(K_CGS_UPDATE) : -1;
  hipLaunchKernelGGL(gs_update_kernel, dim3(g.nrt_upd, ngroups), dim3(256), 0, s, Q, ldq, N, ncol, h, sgn, w,
                     g.Upart, ngroups, cnt_rows, cnt_norm, g.nrt_upd, g.normpart, fd);
  SGN_HIP(hipGetLastError());
  if (prof) prof->end(idx, 16.0 * ((double)N * ncol + 2.0 * N + ncol), 8.0 * (double)N * ncol);
}

void gs_update(const GsWork& g, const double2* Q, size_t ldq, int N, int ncol, const double2* h, double2* w,
                 const GsFinal* fin, int kval, hipStream_t s, Profiler* prof) {
  update_launch(g, Q, ldq, N, ncol, h, -1.0, w, fin, kval, s, prof);
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

