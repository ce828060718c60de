// Sign of the small dense composite matrix H (Eq. eq:newH) on the device:
// Roberts' iteration S <- (S + S^{-1})/2, S_0 = H (Eq. Roberts), in FP64,
// with determinantal scaling S <- (mu S + (mu S)^{-1})/2, mu = |det S|^{-1/n},
// while the iterates still move by more than 1e-2 (relative Frobenius norm).
//
// The inverse is a blocked in-place Gauss-Jordan elimination with partial
// pivoting by rows.  Pivoting is implicit: no rows are swapped; column p is
// eliminated with pivot row r_p, rows already used are excluded from later
// pivot searches, and the inverse is read back as
//     A^{-1}[p][q] = M[r_p][r^{-1}(q)].
// One launch handles a panel of BP columns.  Every workgroup loads the panel
// into LDS and factorises it redundantly (identical data and code, so every
// workgroup picks the same pivots), then applies the accumulated elimination
//     M[:, j] <- (I - P_R) M[:, j] + G M[R, j]        (R = panel pivot rows)
// to its own tile of columns, where G (n x BP) is the factorised panel.  The
// matrix is ping-ponged between two buffers so no workgroup reads data that
// another one writes in the same launch.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace {

constexpr int kGjThreads = 256;
constexpr int kGjTile = 4;  // columns per workgroup in the trailing update

// panel rows are padded to bp + 1 entries so that a column of the panel
// (one entry per row) spreads over the LDS banks
inline size_t gj_lds_bytes(int n, int bp) {
  return sizeof(double2) * (size_t)n * (bp + 1) + sizeof(int) * (size_t)(2 * n + (n & 1)) + sizeof(double2) * (size_t)n;
}

__device__ inline void argmax_merge(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// LDS layout: panel[n][BP] (double2), used[n] (int), inR[n] (int), fcol[n] (double2)
template <int BP>
__global__ void __launch_bounds__(kGjThreads)
gj_panel_kernel(const double2* __restrict__ Min, double2* __restrict__ Mout, int n, int p0,
                int* __restrict__ rowpiv, double* __restrict__ logpiv, int* __restrict__ flag, size_t mstride) {
  // blockIdx.y selects the matrix of a batch
  Min += (size_t)blockIdx.y * mstride;
  Mout += (size_t)blockIdx.y * mstride;
  rowpiv += (size_t)blockIdx.y * n;
  logpiv += (size_t)blockIdx.y * n;
  flag += blockIdx.y;
  constexpr int PS = BP + 1;  // padded row stride
  extern __shared__ double2 smem[];
  double2* panel = smem;                                   // n * PS
  int* used = reinterpret_cast<int*>(panel + (size_t)n * PS);  // n
  int* inR = used + n;                                     // n
  double2* fcol = reinterpret_cast<double2*>(inR + n + (n & 1));  // n (16-byte aligned)
  __shared__ int rp[BP];
  __shared__ double redv[kGjThreads / 64];
  __shared__ int redi[kGjThreads / 64];
  __shared__ double2 pivinv;
  const int tid = threadIdx.x;
  const int b = min(BP, n - p0);

  for (int idx = tid; idx < n * BP; idx += kGjThreads) {
    const int col = idx / n, row = idx - col * n;  // coalesced over rows of the global column
    panel[row * PS + col] = (col < b) ? Min[(size_t)(p0 + col) * n + row] : make_double2(0.0, 0.0);
  }
  for (int i = tid; i < n; i += kGjThreads) {
    used[i] = 0;
    inR[i] = 0;
  }
  __syncthreads();
  for (int p = tid; p < p0; p += kGjThreads) used[rowpiv[p]] = 1;
  __syncthreads();

  for (int t = 0; t < b; ++t) {
    // pivot search over unused rows (ties -> smallest row index)
    double bv = -1.0;
    int bi = n;
    for (int i = tid; i < n; i += kGjThreads)
      if (!used[i]) argmax_merge(bv, bi, cabs2(panel[i * PS + t]), i);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double v2 = __shfl_xor(bv, off, 64);
      const int i2 = __shfl_xor(bi, off, 64);
      argmax_merge(bv, bi, v2, i2);
    }
    if ((tid & 63) == 0) {
      redv[tid >> 6] = bv;
      redi[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double v = redv[0];
      int i = redi[0];
      for (int w = 1; w < kGjThreads / 64; ++w) argmax_merge(v, i, redv[w], redi[w]);
      if (i >= n) i = 0;  // cannot happen for a valid permutation; keeps indices in range
      rp[t] = i;
      used[i] = 1;
      inR[i] = 1;
      double2 piv = panel[i * PS + t];
      double a2 = cabs2(piv);
      if (!(a2 > 0.0) || !isfinite(a2)) {
        if (blockIdx.x == 0) *flag = 1;
        piv = make_double2(1.0, 0.0);
        a2 = 1.0;
      }
      pivinv = make_double2(piv.x / a2, -piv.y / a2);
      if (blockIdx.x == 0) {
        rowpiv[p0 + t] = i;
        logpiv[p0 + t] = 0.5 * log(a2);
      }
    }
    __syncthreads();
    const int r = rp[t];
    const double2 inv = pivinv;
    // scale the pivot row; the eliminated entry becomes 1/piv
    if (tid < BP) {
      const double2 v = panel[r * PS + tid];
      panel[r * PS + tid] = (tid == t) ? inv : cmul(v, inv);
    }
    __syncthreads();
    // eliminate column t from every other row (multipliers staged first)
    for (int i = tid; i < n; i += kGjThreads) fcol[i] = panel[i * PS + t];
    __syncthreads();
    for (int idx = tid; idx < n * BP; idx += kGjThreads) {
      const int i = idx / BP, s = idx - i * BP;
      if (i == r) continue;
      const double2 base = (s == t) ? make_double2(0.0, 0.0) : panel[i * PS + s];
      panel[i * PS + s] = csub(base, cmul(fcol[i], panel[r * PS + s]));
    }
    __syncthreads();
  }

  // workgroup 0 stores the factorised panel (G) into the output
  if (blockIdx.x == 0) {
    for (int idx = tid; idx < n * b; idx += kGjThreads) {
      const int col = idx / n, row = idx - col * n;
      Mout[(size_t)(p0 + col) * n + row] = panel[row * PS + col];
    }
  }
  // trailing update of this workgroup's column tile
  __shared__ double2 mr[kGjTile][BP];
  const int j0 = blockIdx.x * kGjTile;
  for (int jj = 0; jj < kGjTile; ++jj) {
    const int j = j0 + jj;
    if (tid < BP) {
      mr[jj][tid] = (j < n && tid < b && !(j >= p0 && j < p0 + b)) ? Min[(size_t)j * n + rp[tid]]
                                                                   : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  for (int jj = 0; jj < kGjTile; ++jj) {
    const int j = j0 + jj;
    if (j >= n || (j >= p0 && j < p0 + b)) continue;
    for (int i = tid; i < n; i += kGjThreads) {
      double2 acc = inR[i] ? make_double2(0.0, 0.0) : Min[(size_t)j * n + i];
#pragma unroll
      for (int s = 0; s < BP; ++s)
        if (s < b) acc = cfma(panel[i * PS + s], mr[jj][s], acc);
      Mout[(size_t)j * n + i] = acc;
    }
  }
}

// S <- (mu S + Ainv / mu) / 2 with Ainv[p][q] = M[r_p][rinv[q]]; accumulates
// |S_new - S|^2 and |S_new|^2; the last workgroup writes the relative change
// to scal[0], keeps it in scal[2] for the next scaling decision and scal[3] = mu.
__global__ void __launch_bounds__(256)
newton_combine_kernel(double2* __restrict__ S, const double2* __restrict__ M, int n,
                      const int* __restrict__ rowpiv, const double* __restrict__ logpiv,
                      double* __restrict__ scal, double* __restrict__ part, unsigned* __restrict__ counter,
                      int nblk, size_t mstride) {
  // blockIdx.y selects the matrix of a batch
  S += (size_t)blockIdx.y * mstride;
  M += (size_t)blockIdx.y * mstride;
  rowpiv += (size_t)blockIdx.y * n;
  logpiv += (size_t)blockIdx.y * n;
  scal += (size_t)blockIdx.y * 8;
  part += (size_t)blockIdx.y * 2 * nblk;
  counter += blockIdx.y;
  extern __shared__ int rinv[];  // n
  __shared__ double red[2][256];
  __shared__ double mu_s;
  __shared__ int is_last;
  const int tid = threadIdx.x;
  // rowpiv is a permutation unless a singular/non-finite pivot was flagged; the
  // zero fill keeps every gathered index in range even then.
  for (int q = tid; q < n; q += 256) rinv[q] = 0;
  __syncthreads();
  for (int p = tid; p < n; p += 256) {
    const int r = rowpiv[p];
    if (r >= 0 && r < n) rinv[r] = p;
  }
  if (tid == 0) {
    double mu = 1.0;
    if (scal[2] > 1e-2) {
      double ld = 0.0;
      for (int p = 0; p < n; ++p) ld += logpiv[p];
      mu = exp(-ld / n);
      if (!(mu > 0.0) || !isfinite(mu)) mu = 1.0;
    }
    mu_s = mu;
  }
  __syncthreads();
  const double mu = mu_s, imu = 1.0 / mu;
  double dsum = 0.0, ssum = 0.0;
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * 256 + tid; e < total; e += (size_t)gridDim.x * 256) {
    const int q = (int)(e / n), p = (int)(e - (size_t)q * n);
    const double2 s_old = S[e];
    const int rp = min(max(rowpiv[p], 0), n - 1);
    const double2 ai = M[(size_t)rinv[q] * n + rp];
    const double2 s_new = make_double2(0.5 * (mu * s_old.x + imu * ai.x), 0.5 * (mu * s_old.y + imu * ai.y));
    S[e] = s_new;
    dsum += cabs2(csub(s_new, s_old));
    ssum += cabs2(s_new);
  }
  red[0][tid] = dsum;
  red[1][tid] = ssum;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      red[0][tid] += red[0][tid + off];
      red[1][tid] += red[1][tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == (unsigned)nblk - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (tid == 0) {
    double d = 0.0, s = 0.0;
    for (int b = 0; b < nblk; ++b) {
      d += part[2 * b];
      s += part[2 * b + 1];
    }
    const double ch = sqrt(d / fmax(s, 1e-300));
    scal[0] = ch;
    scal[1] = sqrt(s);
    scal[2] = ch;
    scal[3] = mu;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void copy_mat_kernel(const double2* __restrict__ A, int lda, double2* __restrict__ B, int ldb, int rows,
                                int cols) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rows * cols) return;
  const int c = (int)(e / rows), r = (int)(e - (size_t)c * rows);
  B[(size_t)c * ldb + r] = A[(size_t)c * lda + r];
}

__global__ void zero_kernel(double2* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

__global__ void set_scal_kernel(double* scal, int* flag, int nb) {
  for (int b = 0; b < nb; ++b) {
    scal[8 * b + 0] = 1e30;
    scal[8 * b + 1] = 0.0;
    scal[8 * b + 2] = 1e30;
    scal[8 * b + 3] = 1.0;
    flag[b] = 0;
  }
}

// batched strided copy: B_b = A_b (rows x cols), blockIdx.y = b
__global__ void copy_mat_batched_kernel(const double2* __restrict__ A, int lda, size_t astride,
                                        double2* __restrict__ B, int ldb, size_t bstride, int rows, int cols) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)rows * cols) return;
  const int c = (int)(e / rows), r = (int)(e - (size_t)c * rows);
  B[(size_t)blockIdx.y * bstride + (size_t)c * ldb + r] = A[(size_t)blockIdx.y * astride + (size_t)c * lda + r];
}

// c[i] = sum_{q<m} F[i][q] c0[q] + beta F[i][m];  err = |c - [cprev; 0]| / |c|
__global__ void __launch_bounds__(256)
coeffs_kernel(int n, int m, const double2* __restrict__ F, int ldf, size_t fstride, const double2* __restrict__ c0,
              int c0stride, const double* __restrict__ beta, double2* __restrict__ c,
              const double2* __restrict__ cprev, int cstride, SlotMap map, double* __restrict__ err) {
  const int z = blockIdx.x, r = map.slot[z], nprev = map.aux[z];
  F += (size_t)z * fstride;
  c0 += (size_t)r * c0stride;
  beta += r;
  c += (size_t)r * cstride;
  if (nprev < 0) cprev = nullptr;
  if (cprev) cprev += (size_t)r * cstride;
  if (err) err += r;
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  const double b = *beta;
  double dsum = 0.0, csum = 0.0;
  for (int i = tid; i < n; i += 256) {
    double2 acc = make_double2(0.0, 0.0);
    for (int q = 0; q < m; ++q) acc = cfma(F[(size_t)q * ldf + i], c0[q], acc);
    if (m < n) acc = cadd(acc, cscale(F[(size_t)m * ldf + i], b));
    c[i] = acc;
    const double2 prev = (cprev && i < nprev) ? cprev[i] : make_double2(0.0, 0.0);
    dsum += cabs2(csub(acc, prev));
    csum += cabs2(acc);
  }
  red[0][tid] = dsum;
  red[1][tid] = csum;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      red[0][tid] += red[0][tid + off];
      red[1][tid] += red[1][tid + off];
    }
    __syncthreads();
  }
  if (tid == 0 && err) *err = cprev ? sqrt(red[0][0] / fmax(red[1][0], 1e-300)) : 1e30;
}

__global__ void negate_kernel(const double2* __restrict__ in, double2* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cneg(in[i]);
}

__global__ void cmul_kernel(const double2* __restrict__ a, double2* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = cmul(a[i], x[i]);
}

__global__ void to_f32_kernel(const double2* __restrict__ in, float2* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

__global__ void finite_kernel(const double2* __restrict__ v, size_t n, int* __restrict__ flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 a = v[i];
    if (!isfinite(a.x) || !isfinite(a.y)) *flag = 1;
  }
}

size_t lds_budget();

template <int BP>
void launch_panel(const double2* Min, double2* Mout, int n, int p0, int nb, DenseWork& d, hipStream_t s) {
  const size_t lds = gj_lds_bytes(n, BP);
  // allow the kernel the whole budget once (thread-safe: contexts may run on
  // several host threads)
  static const bool configured = [] {
    SGN_HIP(hipFuncSetAttribute((const void*)gj_panel_kernel<BP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_budget()));
    return true;
  }();
  (void)configured;
  const int nblk = (n + kGjTile - 1) / kGjTile;
  hipLaunchKernelGGL(gj_panel_kernel<BP>, dim3(nblk, nb), dim3(kGjThreads), lds, s, Min, Mout, n, p0, d.rowpiv,
                     d.logpiv, d.flag, (size_t)n * n);
}

}  // namespace

namespace {
size_t lds_budget() {
  static const size_t cached = [] {
    int dev = 0, v = 0;
    SGN_HIP(hipGetDevice(&dev));
    SGN_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // leave room for the kernel's static LDS arrays
    return (size_t)std::max(v, 16384) - 2048;
  }();
  return cached;
}
}  // namespace

static int panel_width(int n) {
  const size_t budget = lds_budget();
  for (int bp : {16, 8, 4, 2}) {
    if (gj_lds_bytes(n, bp) <= budget) return bp;
  }
  return 0;
}

void dense_alloc(DenseWork& d, int n, int nb) {
  if (n <= d.ncap && nb <= d.nbcap) return;
  const int ncap = std::max(n, d.ncap), nbcap = std::max(nb, d.nbcap);
  dense_free(d);
  d.ncap = ncap;
  d.nbcap = nbcap;
  const size_t nn = (size_t)ncap * ncap * nbcap;
  SGN_HIP(hipMalloc(&d.S, sizeof(double2) * nn));
  SGN_HIP(hipMalloc(&d.Ma, sizeof(double2) * nn));
  SGN_HIP(hipMalloc(&d.Mb, sizeof(double2) * nn));
  SGN_HIP(hipMalloc(&d.rowpiv, sizeof(int) * (size_t)ncap * nbcap));
  SGN_HIP(hipMalloc(&d.logpiv, sizeof(double) * (size_t)ncap * nbcap));
  SGN_HIP(hipMalloc(&d.scal, sizeof(double) * 8 * (size_t)nbcap));
  SGN_HIP(hipHostMalloc(&d.host_scal, sizeof(double) * 8 * (size_t)nbcap, hipHostMallocDefault));
  SGN_HIP(hipHostMalloc(&d.host_flag, sizeof(int) * (size_t)nbcap, hipHostMallocDefault));
  SGN_HIP(hipMalloc(&d.flag, sizeof(int) * (size_t)nbcap));
  SGN_HIP(hipMalloc(&d.counters, sizeof(unsigned) * (size_t)nbcap));
  SGN_HIP(hipMemset(d.counters, 0, sizeof(unsigned) * (size_t)nbcap));
  d.npart = 1024;
  SGN_HIP(hipMalloc(&d.part, sizeof(double) * 2 * (size_t)d.npart * nbcap));
  SGN_HIP(hipDeviceSynchronize());
}

void dense_alloc(DenseWork& d, int n) { dense_alloc(d, n, 1); }



void dense_free(DenseWork& d) {
  if (d.S) (void)hipFree(d.S);
  if (d.Ma) (void)hipFree(d.Ma);
  if (d.Mb) (void)hipFree(d.Mb);
  if (d.rowpiv) (void)hipFree(d.rowpiv);
  if (d.logpiv) (void)hipFree(d.logpiv);
  if (d.scal) (void)hipFree(d.scal);
  if (d.host_scal) (void)hipHostFree(d.host_scal);
  if (d.host_flag) (void)hipHostFree(d.host_flag);
  if (d.flag) (void)hipFree(d.flag);
  if (d.counters) (void)hipFree(d.counters);
  if (d.part) (void)hipFree(d.part);
  if (d.spart) (void)hipFree(d.spart);
  if (d.ns_state) (void)hipFree(d.ns_state);
  if (d.host_state) (void)hipHostFree(d.host_state);
  const int method = d.method;
  const int last_iters = d.last_iters;
  d = DenseWork{};
  d.method = method;
  d.last_iters = last_iters;
}

void dense_destroy(DenseWork& d) { dense_free(d); }

void dev_zero(double2* p, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  SGN_HIP(hipGetLastError());
}

void dev_copy_mat(const double2* A, int lda, double2* B, int ldb, int rows, int cols, hipStream_t s) {
  const size_t tot = (size_t)rows * cols;
  if (tot == 0) return;
  hipLaunchKernelGGL(copy_mat_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, A, lda, B, ldb, rows,
                     cols);
  SGN_HIP(hipGetLastError());
}

void dev_negate(const double2* in, double2* out, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(negate_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n);
  SGN_HIP(hipGetLastError());
}

void dev_cmul(const double2* a, double2* x, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cmul_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, x, n);
  SGN_HIP(hipGetLastError());
}

void dev_to_f32(const double2* in, float2* out, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  SGN_HIP(hipGetLastError());
}

void dev_check_finite(const double2* v, size_t n, int* flag, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(finite_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n, flag);
  SGN_HIP(hipGetLastError());
}

void dense_coeffs(int n, int m, const double2* F, int ldf, const double2* c0, const double* beta, double2* c,
                  const double2* cprev, int nprev, double* err, hipStream_t s) {
  SlotMap one;
  one.n = 1;
  one.aux[0] = cprev ? nprev : -1;
  dense_coeffs_batched(n, m, F, ldf, 0, c0, 0, beta, c, cprev, 0, one, err, s);
}

void dense_coeffs_batched(int n, int m, const double2* F, int ldf, size_t fstride, const double2* c0, int c0stride,
                          const double* beta, double2* c, const double2* cprev, int cstride, const SlotMap& map,
                          double* err, hipStream_t s) {
  if (map.n <= 0) return;
  hipLaunchKernelGGL(coeffs_kernel, dim3(map.n), dim3(256), 0, s, n, m, F, ldf, fstride, c0, c0stride, beta, c, cprev,
                     cstride, map, err);
  SGN_HIP(hipGetLastError());
}

static int dense_sign_newton_batched(DenseWork& d, int n, int nb, const double2* A, int lda, size_t astride,
                                     double2* F, int ldf, size_t fstride, hipStream_t s, Profiler* prof) {
  SGN_REQUIRE(n >= 1 && nb >= 1, SGN_EINVAL, "dense_sign: n and the batch must be positive");
  const int bp = panel_width(n);
  SGN_REQUIRE(bp > 0, SGN_EINVAL, "dense_sign: matrix too large for the LDS panel");
  dense_alloc(d, n, nb);
  const size_t nn = (size_t)n * n;
  {
    const size_t tot = nn;
    hipLaunchKernelGGL(copy_mat_batched_kernel, dim3((unsigned)((tot + 255) / 256), nb), dim3(256), 0, s, A, lda,
                       astride, d.S, n, nn, n, n);
    SGN_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(set_scal_kernel, dim3(1), dim3(1), 0, s, d.scal, d.flag, nb);
  SGN_HIP(hipGetLastError());
  const int npanel = (n + bp - 1) / bp;
  const int nblk_comb = (int)std::min<size_t>((size_t)d.npart, (nn + 255) / 256);
  const int maxit = 100;
  std::vector<double> prev(nb, 1e30);
  std::vector<char> done(nb, 0);
  bool extra = false;
  for (int it = 1; it <= maxit; ++it) {
    const int idx = prof ? prof->begin(K_GJ_PANEL) : -1;
    const double2* Min = d.S;
    double2* bufs[2] = {d.Ma, d.Mb};
    for (int pi = 0; pi < npanel; ++pi) {
      double2* Mout = bufs[pi & 1];
      switch (bp) {
        case 16: launch_panel<16>(Min, Mout, n, pi * bp, nb, d, s); break;
        case 8: launch_panel<8>(Min, Mout, n, pi * bp, nb, d, s); break;
        case 4: launch_panel<4>(Min, Mout, n, pi * bp, nb, d, s); break;
        default: launch_panel<2>(Min, Mout, n, pi * bp, nb, d, s); break;
      }
      SGN_HIP(hipGetLastError());
      Min = Mout;
    }
    if (prof) prof->end(idx, nb * 2.0 * 16.0 * (double)nn * npanel, nb * 8.0 * (double)nn * n);
    const int idx2 = prof ? prof->begin(K_NEWTON_COMBINE) : -1;
    hipLaunchKernelGGL(newton_combine_kernel, dim3(nblk_comb, nb), dim3(256), sizeof(int) * (size_t)n, s, d.S, Min,
                       n, d.rowpiv, d.logpiv, d.scal, d.part, d.counters, nblk_comb, nn);
    SGN_HIP(hipGetLastError());
    if (prof) prof->end(idx2, nb * 3.0 * 16.0 * (double)nn, nb * 10.0 * (double)nn);
    SGN_HIP(hipMemcpyAsync(d.host_scal, d.scal, sizeof(double) * 8 * nb, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipMemcpyAsync(d.host_flag, d.flag, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b) {
      if (d.host_flag[b]) throw SgnError{SGN_ESINGULAR, "Roberts iteration met a singular iterate"};
      if (!std::isfinite(d.host_scal[8 * b]))
        throw SgnError{SGN_ESINGULAR, "Roberts iteration diverged (non-finite iterate)"};
    }
    if (extra) {
      hipLaunchKernelGGL(copy_mat_batched_kernel, dim3((unsigned)((nn + 255) / 256), nb), dim3(256), 0, s, d.S, n,
                         nn, F, ldf, fstride, n, n);
      SGN_HIP(hipGetLastError());
      return it;
    }
    // converged (or stagnated at rounding level): one more step settles the last digits
    bool all = true;
    for (int b = 0; b < nb; ++b) {
      const double ch = d.host_scal[8 * b];
      if (ch <= 1e-13 || (it > 4 && ch < 1e-9 && ch > 0.5 * prev[b])) done[b] = 1;
      prev[b] = ch;
      all = all && done[b];
    }
    if (all) extra = true;
  }
  throw SgnError{SGN_ESINGULAR, "Roberts iteration did not converge in 100 steps"};
}

// ---------------------------------------------------------------------------
// Inverse-free evaluation: Newton-Schulz iteration X <- X (3I - X^2) / 2 from
// X_0 = A / |A|_1.  It converges to sgn(A) when every eigenvalue z of X_0
// satisfies |1 - z^2| < 1, which holds for the composite Arnoldi matrices of
// this method (their Ritz values have |Im| well below |Re| once the critical
// eigenvalues are deflated); growth of the small eigenvalues is 3/2 per step,
// then quadratic.  Each step is two complex products on the matrix cores
// (zgemm.hip), one launch each for the whole batch, and a per-matrix check
// of |X^2 - I|_F / sqrt(n) on the device; a matrix stops once it is below
// 1e-7 (the next iterate is then at rounding level), or when it diverges or
// has not settled within 60 steps (then the caller falls back to Roberts'
// iteration with Gauss-Jordan inverses, which converges for any matrix
// without eigenvalues on the imaginary axis).  The host reads the per-matrix
// states only every other step from the step where the previous call
// settled, so launches run back to back in between; a finished matrix's
// later launches return at once.
// ---------------------------------------------------------------------------
namespace {

// X_b = A_b / |A_b|_1 (max column sum of |a_ij|); one workgroup per matrix
// column sums of |A_ij| (one wavefront per column, lanes over rows)
__global__ void __launch_bounds__(256) colsum_kernel(const double2* __restrict__ A, int lda, size_t astride,
                                                     double* __restrict__ cs, int n) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const double2* col = A + (size_t)blockIdx.y * astride + (size_t)j * lda;
  double sum = 0.0;
  for (int i = lane; i < n; i += 64) sum += sqrt(cabs2(col[i]));
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
  if (lane == 0) cs[(size_t)blockIdx.y * n + j] = sum;
}

// X = A / |A|_1 (the 1-norm as the largest column sum; every workgroup takes
// the maximum itself), or A / max(radius, |A|_1 / 1.5) for a smaller radius
__global__ void __launch_bounds__(256) scale_by_norm1_kernel(const double2* __restrict__ A, int lda, size_t astride,
                                                             const double* __restrict__ cs, double2* __restrict__ X,
                                                             int n, size_t nn, double radius) {
  const int b = blockIdx.y;
  __shared__ double red[256];
  double mx = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) mx = fmax(mx, cs[(size_t)b * n + j]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  // the divisor: |A|_1, or the radius estimate when it is smaller but not
  // below 2/3 of the 1-norm: every eigenvalue then has |z| <= 1.5 < sqrt(3),
  // and a real z in (0, sqrt(3)) stays positive under z (3 - z^2) / 2, so a
  // radius estimate that is too small cannot turn a real eigenvalue's sign
  const double n1 = red[0];
  const double div = (radius > 0.0 && radius < n1) ? fmax(radius, n1 / 1.5) : n1;
  const double inv = div > 0.0 ? 1.0 / div : 1.0;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nn) return;
  const int j = (int)(e / n), i = (int)(e - (size_t)j * n);
  X[(size_t)b * nn + e] = cscale(A[(size_t)b * astride + (size_t)j * lda + i], inv);
}

__global__ void ns_init_kernel(int* state, int* iters, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) {
    state[b] = 0;
    iters[b] = 0;
  }
}

}  // namespace

// C = A B (column-major, complex) on the matrix cores
void dev_zgemm_nn(DenseWork& d, int M, int N, int K, const double2* A, int lda, const double2* B, int ldb,
                  double2* C, int ldc, hipStream_t s) {
  (void)d;
  zgemm(M, N, K, 1.0, A, lda, 0, B, ldb, 0, C, ldc, 0, 1, s);
}

static void ns_reserve(DenseWork& d, int n, int nb) {
  // residual partials of the squaring launches; also the column sums (n per matrix)
  const size_t nparts = (size_t)std::max(zgemm_ns_parts(n, nb), n) * nb;
  if (d.nspart < nparts) {
    if (d.spart) (void)hipFree(d.spart);
    SGN_HIP(hipMalloc(&d.spart, sizeof(double) * nparts));
    d.nspart = nparts;
  }
  if (d.nstate < nb) {
    if (d.ns_state) (void)hipFree(d.ns_state);
    if (d.host_state) (void)hipHostFree(d.host_state);
    SGN_HIP(hipMalloc(&d.ns_state, sizeof(int) * 2 * (size_t)nb));
    SGN_HIP(hipHostMalloc(&d.host_state, sizeof(int) * 2 * (size_t)nb, hipHostMallocDefault));
    d.nstate = nb;
  }
}

// Newton-Schulz for nb matrices; returns the iterations run.  done marks the
// matrices whose iteration met the stopping test (their F_b is written); the
// others diverged or did not settle within the iteration limit.
static int dense_sign_ns_batched(DenseWork& d, int n, int nb, const double2* A, int lda, size_t astride, double2* F,
                                 int ldf, size_t fstride, hipStream_t s, Profiler* prof, unsigned long long& done,
                                 double radius) {
  SGN_REQUIRE(nb <= kMaxBatch, SGN_EINVAL, "dense_sign: batch too large");
  dense_alloc(d, n, nb);
  const size_t nn = (size_t)n * n;
  ns_reserve(d, n, nb);
  int* state = d.ns_state;
  int* iters = d.ns_state + nb;
  // the column sums use the partial-sum buffer (sized above for both uses)
  hipLaunchKernelGGL(colsum_kernel, dim3((n + 3) / 4, nb), dim3(256), 0, s, A, lda, astride, d.spart, n);
  SGN_HIP(hipGetLastError());
  hipLaunchKernelGGL(scale_by_norm1_kernel, dim3((unsigned)((nn + 255) / 256), nb), dim3(256), 0, s, A, lda, astride,
                     d.spart, d.S, n, nn, radius);
  SGN_HIP(hipGetLastError());
  hipLaunchKernelGGL(ns_init_kernel, dim3((nb + 63) / 64), dim3(64), 0, s, state, iters, nb);
  SGN_HIP(hipGetLastError());
  double2* X = d.S;
  double2* Y = d.Ma;
  double2* Xn = d.Mb;
  const int nparts = zgemm_ns_parts(n, nb);
  const int maxit = 60;
  const int first_look = std::max(6, std::min(d.last_iters, maxit));
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    int idx = prof ? prof->begin(K_NS_GEMM) : -1;
    zgemm_ns_square(n, X, Y, nn, nb, state, d.spart, s);
    if (prof) prof->end(idx, 0.0, 0.0, 0);
    ns_check(d.spart, nparts, n, state, iters, it, maxit, nb, s);
    idx = prof ? prof->begin(K_NS_GEMM) : -1;
    zgemm_ns_update(n, X, Y, Xn, nn, nb, state, F, ldf, fstride, s);
    if (prof) prof->end(idx, 0.0, 0.0, 0);
    std::swap(X, Xn);
    if (it >= first_look && ((it - first_look) % 2 == 0 || it == maxit)) {
      SGN_HIP(hipMemcpyAsync(d.host_state, state, sizeof(int) * 2 * (size_t)nb, hipMemcpyDeviceToHost, s));
      SGN_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (int b = 0; b < nb; ++b) all = all && d.host_state[b] != 0;
      if (all) break;
    }
  }
  it = std::min(it, maxit);
  // a final read (the loop may have ended at maxit without one)
  SGN_HIP(hipMemcpyAsync(d.host_state, state, sizeof(int) * 2 * (size_t)nb, hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  done = 0;
  int most = 0;
  double gemm_matrices = 0.0;  // matrix products that did work
  for (int b = 0; b < nb; ++b) {
    const int st = d.host_state[b];
    if (st == 1 || st == 2) {
      done |= 1ull << b;
      most = std::max(most, d.host_state[nb + b]);
      gemm_matrices += 2.0 * d.host_state[nb + b];
    } else {
      gemm_matrices += 2.0 * it;
    }
  }
  if (most > 0) d.last_iters = most;
  if (prof) {
    // per product: read two n x n operands, write one; 8 n^3 real flops
    prof->bytes[K_NS_GEMM] += gemm_matrices * 3.0 * 16.0 * (double)nn;
    prof->flops[K_NS_GEMM] += gemm_matrices * 8.0 * (double)nn * n;
    prof->launches[K_NS_GEMM] += 2 * (long long)std::max(most, done == 0 ? it : most);
  }
  return done ? most : it;
}

void dense_reserve(DenseWork& d, int n, int nb) {
  dense_alloc(d, n, nb);
  ns_reserve(d, n, nb);
}

int dense_sign_batched(DenseWork& d, int n, int nb, const double2* A, int lda, size_t astride, double2* F, int ldf,
                       size_t fstride, hipStream_t s, Profiler* prof, double radius) {
  SGN_REQUIRE(n >= 1 && nb >= 1, SGN_EINVAL, "dense_sign: n and the batch must be positive");
  if (d.method == 1) return dense_sign_newton_batched(d, n, nb, A, lda, astride, F, ldf, fstride, s, prof);
  unsigned long long done = 0;
  int it = dense_sign_ns_batched(d, n, nb, A, lda, astride, F, ldf, fstride, s, prof, done, radius);
  // Roberts' iteration for each matrix Newton-Schulz did not settle, one at a
  // time (as it would run for that matrix alone)
  for (int b = 0; b < nb; ++b)
    if (!((done >> b) & 1ull))
      it = std::max(it, dense_sign_newton_batched(d, n, 1, A + (size_t)b * astride, lda, astride,
                                                  F + (size_t)b * fstride, ldf, fstride, s, prof));
  return it;
}

int dense_sign(DenseWork& d, int n, const double2* A, int lda, double2* F, int ldf, hipStream_t s,
               Profiler* prof, double radius) {
  return dense_sign_batched(d, n, 1, A, lda, 0, F, ldf, 0, s, prof, radius);
}
