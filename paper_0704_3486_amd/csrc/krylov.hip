// One-reduction modified Arnoldi step with delayed re-orthogonalisation
// (Section 5.2, step (iv), Eq. eq:modArnoldi), for FP64 or FP32 Krylov-vector
// storage and for a batch of right-hand sides advancing in lock step.
//
// State before step j (J = m + j finished columns of Q = (S_m v_1 .. v_j)):
// u, the candidate for column J, orthogonalised once against Q_J but neither
// re-orthogonalised nor normalised.  With z = A u (the stencil, outside):
//   dot:    a = Q_J^dag u, b = Q_J^dag z, c = u^dag u, d = u^dag z   (1 sweep)
//           rho = sqrt(c - |a|^2),  gam = (d - a^dag b) / rho
//   update: v_J = (u - Q_J a) / rho                                    (1 sweep)
//           u'  = (z - (gam/rho) u - Q_J (b - (gam/rho) a)) / rho
//               = (1 - Q_{J+1} Q_{J+1}^dag) A v_J
//           column J-1 of H += a, H[J][J-1] = rho  (re-orthogonalisation)
//           column J of H = ([b; gam] - Hbar_J a) / rho
// Hbar_J is the (J+1) x J leading block of the composite H with the corrected
// column J-1, so that A Q_J = Q_{J+1} Hbar_J.  At j = 0 the correction goes to
// c0 = S^dag x and rho is beta = |x_perp|.  This is classical Gram-Schmidt
// with one full re-orthogonalisation, rescheduled so that each step needs a
// single global reduction and two sweeps over the basis.
//
// Precision: S, u, H, all dot products and all coefficients are FP64; the
// Krylov columns v_j and the stencil operand/result (z) are stored as VT
// (double2, or float2 in mixed precision).
//
// Batching: each workgroup serves one right-hand side; per-RHS buffers are
// laid out at fixed strides.  The dot and update passes number their
// workgroups with the right-hand side varying fastest, so the workgroups of
// all right-hand sides that read the same rows of the shared Schur block S run
// together and S comes from cache after the first of them.  Every reduction
// has a fixed order, so results are bitwise independent of the batch.
#include "internal.h"
#include "krylov.h"

namespace {

constexpr int kRpl = 8;                 // dot: rows per lane
constexpr int kDRows = 64 * kRpl;       // dot: rows per tile (4 wavefronts of CPW columns each)
constexpr int kUWaves = 8;              // combine (and the default update): wavefronts per 64-row workgroup
constexpr int kUThreads = 64 * kUWaves;
constexpr int kCBatch = 8;              // combine: column loads issued together per lane

__device__ inline double2 ld2(const double2* p, size_t i) { return p[i]; }
__device__ inline double2 ld2(const float2* p, size_t i) {
  const float2 v = p[i];
  return make_double2((double)v.x, (double)v.y);
}
__device__ inline void st2(double2* p, size_t i, double2 v) { p[i] = v; }
__device__ inline void st2(float2* p, size_t i, double2 v) { p[i] = make_float2((float)v.x, (float)v.y); }

// two adjacent rows il, il + 1 of one column (il even): FP32 columns in one
// 16-byte load per lane, FP64 columns in two
__device__ inline void ld_pair(const double2* __restrict__ p, int il, double2& q0, double2& q1) {
  q0 = p[il];
  q1 = p[il + 1];
}
__device__ inline void ld_pair(const float2* __restrict__ p, int il, double2& q0, double2& q1) {
  const float4 v = *reinterpret_cast<const float4*>(p + il);
  q0 = make_double2((double)v.x, (double)v.y);
  q1 = make_double2((double)v.z, (double)v.w);
}

// Rows per lane group of the dot and update passes: 1 with FP64 Krylov
// columns, 2 with FP32 columns, whose lanes then take adjacent row pairs so
// that a column load is 16 bytes per lane
template <typename VT>
constexpr int rows_per_lane() { return sizeof(VT) == 8 ? 2 : 1; }

__device__ inline double2 wsum2(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}
__device__ inline double wsum1(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// wavefront index as a scalar (uniform) value
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// column c of Q for right-hand side slot r
template <typename VT>
__device__ inline double2 qload(const KrylovArgs& A, int r, int c, int i) {
  if (c < A.m) return A.S[(size_t)c * A.ldq + i];
  const VT* V = static_cast<const VT*>(A.V) + (size_t)r * A.vstride + (size_t)(c - A.m) * A.ldq;
  return ld2(V, i);
}

// launch position z (an index into the batch) -> buffer slot and step
__device__ inline int slot_of(const KrylovArgs& A, int z) { return A.act[z]; }
__device__ inline int step_of(const KrylovArgs& A, int z) { return A.jdev ? *A.jdev + A.joff : A.jv[z]; }

// ---------------------------------------------------------------------------
// dot pass: per (row tile, column group) partial sums of Q^dag u and Q^dag z,
// plus |u|^2, u^dag z, |z|^2 per row tile.  No cross-workgroup communication:
// the partials are reduced by kred_kernel in a fixed order.
// the rows past N carry zero weights (uv = zv = 0 there) and load a valid
// row instead: unconditional loads, all in flight together
// Row of a lane's slot t in a tile: R = 1, row0 + 64 t + lane; R = 2 (FP32
// columns), the pair row0 + 128 (t / 2) + 2 lane + {0, 1}
template <int R>
__device__ inline int dot_row(int row0, int t, int lane) {
  return R == 1 ? row0 + t * 64 + lane : row0 + (t >> 1) * 128 + 2 * lane + (t & 1);
}

template <typename QT, int R>
__device__ inline void dot_cols(const QT* __restrict__ q, const double2 uv[kRpl], const double2 zv[kRpl], int row0,
                                int lane, int N, double2& aa, double2& bb) {
  double2 qv[kRpl];
  if constexpr (R == 1) {
#pragma unroll
    for (int t = 0; t < kRpl; ++t) qv[t] = ld2(q, min(dot_row<1>(row0, t, lane), N - 1));
  } else {
    // N is even, so a pair lies wholly below N or wholly at or above it
#pragma unroll
    for (int t = 0; t < kRpl; t += 2) ld_pair(q, min(dot_row<2>(row0, t, lane), N - 2), qv[t], qv[t + 1]);
  }
#pragma unroll
  for (int t = 0; t < kRpl; ++t) {
    aa = cfmac(qv[t], uv[t], aa);
    bb = cfmac(qv[t], zv[t], bb);
  }
}

// workgroup id = z + nb (rt + nrt cg): batch position fastest, then row
// tile; column group cg holds columns [4 CPW cg, 4 CPW (cg + 1)), CPW per wavefront
template <typename VT, int CPW>
__global__ void __launch_bounds__(256) kdot_kernel(KrylovArgs A, int with_z) {
  constexpr int R = rows_per_lane<VT>();
  const int zb = blockIdx.x % A.nb, rest = blockIdx.x / A.nb;
  const int rt = rest % A.nrt_dot, cg = rest / A.nrt_dot;
  const int r = slot_of(A, zb);
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int N = A.N, J = A.m + step_of(A, zb);
  const int row0 = rt * kDRows;
  const double2* __restrict__ u = A.u + (size_t)r * A.ustride;
  const VT* __restrict__ z = static_cast<const VT*>(A.z) + (size_t)r * A.zstride;
  double2* Pa = A.Pa + (size_t)r * A.pstride;
  double2* Pb = A.Pb + (size_t)r * A.pstride;
  double* Pcd = A.Pcd + (size_t)r * A.cdstride;

  double2 uv[kRpl], zv[kRpl];
#pragma unroll
  for (int t = 0; t < kRpl; ++t) {
    const int i = dot_row<R>(row0, t, lane);
    uv[t] = (i < N) ? u[i] : make_double2(0.0, 0.0);
    zv[t] = (with_z && i < N) ? ld2(z, i) : make_double2(0.0, 0.0);
  }
  const int cw = (cg * 4 + wave) * CPW;  // first column of this wavefront
#pragma unroll
  for (int cc = 0; cc < CPW; ++cc) {
    const int c = cw + cc;
    if (c < J) {
      double2 aa = make_double2(0.0, 0.0), bb = make_double2(0.0, 0.0);
      if (c < A.m) {
        dot_cols<double2, R>(A.S + (size_t)c * A.ldq, uv, zv, row0, lane, N, aa, bb);
      } else {
        const VT* q = static_cast<const VT*>(A.V) + (size_t)r * A.vstride + (size_t)(c - A.m) * A.ldq;
        dot_cols<VT, R>(q, uv, zv, row0, lane, N, aa, bb);
      }
      aa = wsum2(aa);
      bb = wsum2(bb);
      if (lane == 0) {
        Pa[(size_t)rt * A.ldp + c] = aa;
        Pb[(size_t)rt * A.ldp + c] = bb;
      }
    }
  }
  if (cg == 0 && wave == 0) {
    // |u|^2, u^dag z, |z|^2 of this row tile (the four wavefronts hold the
    // same rows, so one of them accounts for the tile)
    double cs = 0.0, zs = 0.0;
    double2 ds = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < kRpl; ++t) {
      cs += cabs2(uv[t]);
      zs += cabs2(zv[t]);
      ds = cfmac(uv[t], zv[t], ds);
    }
    cs = wsum1(cs);
    zs = wsum1(zs);
    ds = wsum2(ds);
    if (lane == 0) {
      Pcd[4 * rt + 0] = cs;
      Pcd[4 * rt + 1] = ds.x;
      Pcd[4 * rt + 2] = ds.y;
      Pcd[4 * rt + 3] = zs;
    }
  }
}

// reduce the dot partials over row tiles in a fixed order: 32 columns per
// workgroup, 8 threads per column (each sums every 8th row tile), then a
// fixed-order combine; workgroup 0 also sums the scalars c, d, |z|^2
__global__ void __launch_bounds__(256) kred_kernel(KrylovArgs A) {
  const int r = slot_of(A, blockIdx.z);
  const int J = A.m + step_of(A, blockIdx.z), nrt = A.nrt_dot;
  const double2* Pa = A.Pa + (size_t)r * A.pstride;
  const double2* Pb = A.Pb + (size_t)r * A.pstride;
  const double* Pcd = A.Pcd + (size_t)r * A.cdstride;
  const int cl = threadIdx.x & 31, part = threadIdx.x >> 5;
  const int c = blockIdx.x * 32 + cl;
  const double2 zero = make_double2(0.0, 0.0);
  double2 sa = zero, sb = zero;
  // tiles t = part, part + 8, ... in that order, eight loads in flight
  if (c < J)
    for (int t0 = part; t0 < nrt; t0 += 64) {
      double2 va[8], vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + 8 * u;
        va[u] = t < nrt ? Pa[(size_t)t * A.ldp + c] : zero;
        vb[u] = t < nrt ? Pb[(size_t)t * A.ldp + c] : zero;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        sa = cadd(sa, va[u]);
        sb = cadd(sb, vb[u]);
      }
    }
  __shared__ double2 ra[8][33], rb[8][33];
  ra[part][cl] = sa;
  rb[part][cl] = sb;
  __syncthreads();
  if (part == 0 && c < J) {
    double2 ta = ra[0][cl], tb = rb[0][cl];
    for (int q = 1; q < 8; ++q) {
      ta = cadd(ta, ra[q][cl]);
      tb = cadd(tb, rb[q][cl]);
    }
    A.a[(size_t)r * A.abstride + c] = ta;
    A.b[(size_t)r * A.abstride + c] = tb;
  }
  if (blockIdx.x == 0) {
    // wavefront q sums scalar q over the row tiles: lane partials (tiles
    // lane, lane + 64, ...) then a fixed butterfly
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc = 0.0;
    for (int t0 = lane; t0 < nrt; t0 += 64 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (t0 + 64 * u < nrt) ? Pcd[4 * (t0 + 64 * u) + q] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    acc = wsum1(acc);
    if (lane == 0) A.sc[(size_t)r * kScStride + kScRawC + q] = acc;
  }
}

// Step scalars from a, b and the raw sums.  Each thread brings its partial
// sums over the columns c = tid, tid + NT, ... (|a_c|^2 and conj(a_c) b_c);
// they are combined by wavefront butterflies and then over the wavefronts in
// a fixed order, so every workgroup computes them identically.
struct StepScalars {
  double rho, inv;
  double2 gam, gr;
  bool brk, finite;
  double scale;
};

// this thread's columns of a and b: the first two are loaded by the caller
// (early, so their latency overlaps other work), the rest here
template <int NT>
__device__ inline void scalar_partials(const double2* av, const double2* bv, int J, double2 a0, double2 b0,
                                       double2 a1, double2 b1, double& s0, double2& s12) {
  const int tid = threadIdx.x;
  s0 = cabs2(a0) + cabs2(a1);
  s12 = cadd(cmulc(a0, b0), cmulc(a1, b1));
  for (int c = tid + 2 * NT; c < J; c += NT) {
    const double2 x1 = av[c], x2 = bv[c];
    s0 += cabs2(x1);
    s12 = cadd(s12, cmulc(x1, x2));
  }
}

template <int NW>
__device__ StepScalars step_scalars(const KrylovArgs& A, int r, int j, double s0, double2 s12,
                                    double* red /* LDS [3][NW] */) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  s0 = wsum1(s0);
  s12 = wsum2(s12);
  if (lane == 0) {
    red[wave] = s0;
    red[NW + wave] = s12.x;
    red[2 * NW + wave] = s12.y;
  }
  __syncthreads();
  double aa = red[0];
  double2 ab = make_double2(red[NW], red[2 * NW]);
  for (int w = 1; w < NW; ++w) {
    aa += red[w];
    ab.x += red[NW + w];
    ab.y += red[2 * NW + w];
  }
  const double* sc = A.sc + (size_t)r * kScStride;
  StepScalars st;
  const double c = sc[kScRawC];
  const double2 d = make_double2(sc[kScRawC + 1], sc[kScRawC + 2]);
  const double zz = sc[kScRawC + 3];
  const double rho2 = c - aa;
  const double rho = rho2 > 0.0 ? sqrt(rho2) : 0.0;
  st.finite = isfinite(c) && isfinite(d.x) && isfinite(d.y) && isfinite(zz);
  st.brk = !(rho > A.brk_tol * sc[kScRef + (j & 1)]) || !st.finite;
  st.inv = st.brk ? 0.0 : 1.0 / rho;
  st.rho = st.brk ? 0.0 : rho;
  st.gam = cscale(csub(d, ab), st.inv);
  st.gr = cscale(st.gam, st.inv);
  st.scale = sqrt(zz) * st.inv;
  return st;
}

// Hessenberg column J and the re-orthogonalisation of column J-1, one row per
// wavefront (the lanes split the sum over columns); at j = 0 the correction
// goes to c0 instead.
__device__ void hcol_row_wave(const KrylovArgs& A, int r, int j, int row, int lane, const StepScalars& st) {
  const int J = A.m + j;
  const double2* a = A.a + (size_t)r * A.abstride;
  const double2* b = A.b + (size_t)r * A.abstride;
  double2* H = A.H + (size_t)r * A.hstride;
  const int ldh = A.ldh;
  const int lim = (j > 0) ? J - 1 : J;
  double2 ha = make_double2(0.0, 0.0);
  if (row < J)  // row J of columns < J-1 is below the subdiagonal (zero)
    // columns l = lane, lane + 64, ... in order, 4 loads of each operand in
    // flight per lane (deeper batches raise the kernel's register count, and
    // with it lower the occupancy of the sweep workgroups)
    for (int l0 = 0; l0 < lim; l0 += 4 * 64) {
      double2 hv[4], xv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int l = l0 + t * 64 + lane;
        if (l < lim) {
          hv[t] = H[(size_t)l * ldh + row];
          xv[t] = a[l];
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (l0 + t * 64 + lane < lim) ha = cfma(hv[t], xv[t], ha);
    }
  ha = wsum2(ha);
  if (lane != 0) return;
  const double rho = st.rho, inv = st.inv;
  const double2 g = (row < J) ? b[row] : st.gam;
  if (j > 0) {
    const double2 hl = (row < J) ? cadd(H[(size_t)(J - 1) * ldh + row], a[row]) : make_double2(rho, 0.0);
    ha = cfma(hl, a[J - 1], ha);
    H[(size_t)(J - 1) * ldh + row] = hl;
  } else if (row < A.m) {
    double2* c0 = A.c0 + (size_t)r * A.c0stride;
    c0[row] = cadd(c0[row], a[row]);
  }
  H[(size_t)J * ldh + row] = cscale(csub(g, ha), inv);
}

// sa += sum_c q_c[i] a_c, sb += sum_c q_c[i] b_c over the columns c = c0,
// c0 + NW, ... < cend, in that order; column c sits at base + (c - cofs)
// ldq.  Each batch of KB column loads (and their coefficients) is issued
// before its arithmetic, the last, partial batch too, so a sweep costs
// ceil(ncols / KB) memory round trips: a slot past cend reloads column
// cend - 1 (a cache hit) and adds it with coefficient zero, which leaves the
// sums unchanged since basis vectors are finite.
// (rows past N load row N-1 and are never written: unconditional loads; c
// is wavefront-uniform, so the coefficients come through scalar loads)
template <typename QT, bool HasB, int KB, int NW>
__device__ inline void sweep_cols(const QT* __restrict__ base, int cofs, size_t ldq, int c, int cend, int i,
                                  const double2* __restrict__ av, const double2* __restrict__ bv, double2& sa,
                                  double2& sb) {
  const double2 zero = make_double2(0.0, 0.0);
  for (; c < cend; c += KB * NW) {
    double2 qv[KB], ca[KB], cb[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) {
      const int cc = c + t * NW, cl = min(cc, cend - 1);
      qv[t] = ld2(base + (size_t)(cl - cofs) * ldq, i);
      ca[t] = av[cl];
      if constexpr (HasB) cb[t] = bv[cl];
      if (cc >= cend) {
        ca[t] = zero;
        if constexpr (HasB) cb[t] = zero;
      }
    }
#pragma unroll
    for (int t = 0; t < KB; ++t) {
      sa = cfma(qv[t], ca[t], sa);
      if constexpr (HasB) sb = cfma(qv[t], cb[t], sb);
    }
  }
}


// sweep_cols for two adjacent rows per lane: each row's sums take the same
// columns in the same order as sweep_cols, so the results are bitwise those
// of one row per lane
template <typename QT, int KB, int NW>
__device__ inline void sweep_cols_pair(const QT* __restrict__ base, int cofs, size_t ldq, int c, int cend, int il,
                                       const double2* __restrict__ av, const double2* __restrict__ bv,
                                       double2 (&sa)[2], double2 (&sb)[2]) {
  const double2 zero = make_double2(0.0, 0.0);
  for (; c < cend; c += KB * NW) {
    double2 q0[KB], q1[KB], ca[KB], cb[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) {
      const int cc = c + t * NW, cl = min(cc, cend - 1);
      ld_pair(base + (size_t)(cl - cofs) * ldq, il, q0[t], q1[t]);
      ca[t] = av[cl];
      cb[t] = bv[cl];
      if (cc >= cend) {
        ca[t] = zero;
        cb[t] = zero;
      }
    }
#pragma unroll
    for (int t = 0; t < KB; ++t) {
      sa[0] = cfma(q0[t], ca[t], sa[0]);
      sb[0] = cfma(q0[t], cb[t], sb[0]);
      sa[1] = cfma(q1[t], ca[t], sa[1]);
      sb[1] = cfma(q1[t], cb[t], sb[1]);
    }
  }
}

// first column >= m that wavefront w of NW takes (c = w mod NW)
template <int NW>
__device__ inline int first_col(int m, int w) { return m + ((w - m % NW) + NW) % NW; }

// update pass.  Per slot, the first nh workgroups compute the Hessenberg
// column J (one row per wavefront), the next nblk each own 64 R rows and all
// J columns: their NW wavefronts take interleaved columns, combined in LDS in
// a fixed order.  R = 1 for FP64 columns; R = 2 for FP32 columns, whose lanes
// then take two adjacent rows each, so that a column load is 16 bytes per
// lane (every row's sums are the same as with R = 1).  Workgroup id = z + nb b
// (batch position fastest).  Both kinds compute the step scalars; the
// Hessenberg rows, a strided gather, so run beside the sweeps instead of
// after them.
template <typename VT, int KB, int NW>
__global__ void __launch_bounds__(64 * NW) kupdate_kernel(KrylovArgs A, int nh) {
  constexpr int NT = 64 * NW;
  constexpr int R = rows_per_lane<VT>();
  const int zb = blockIdx.x % A.nb, bb = blockIdx.x / A.nb;
  const int r = slot_of(A, zb);
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int N = A.N, j = step_of(A, zb), J = A.m + j;
  const double2* av = A.a + (size_t)r * A.abstride;
  const double2* bv = A.b + (size_t)r * A.abstride;
  const double2 zero = make_double2(0.0, 0.0);
  // this thread's first two coefficients for the step scalars (loaded after
  // the sweep in the sweep workgroups, whose registers the sweep needs)
  double2 a0 = zero, b0 = zero, a1 = zero, b1 = zero;
  auto load_coef = [&]() {
    if (tid < J) {
      a0 = av[tid];
      b0 = bv[tid];
    }
    if (tid + NT < J) {
      a1 = av[tid + NT];
      b1 = bv[tid + NT];
    }
  };
  __shared__ double red[3 * NW];
  double s0;
  double2 s12;
  if (bb < nh) {
    load_coef();
    scalar_partials<NT>(av, bv, J, a0, b0, a1, b1, s0, s12);
    const StepScalars st = step_scalars<NW>(A, r, j, s0, s12, red);
    const int row = bb * NW + wave;
    if (row <= J) hcol_row_wave(A, r, j, row, lane, st);
    return;
  }
  const int blk = bb - nh;
  const int i = blk * 64 * R + R * lane;  // this lane's first row
  const bool ok = i < N;                  // N is even: with R = 2, row i + 1 < N too
  // sweep: sa = Q a, sb = Q b (the step scalars enter only afterwards:
  // Q (b - gr a) = sb - gr sa)
  __shared__ double2 ps[2][NW][64 * R];
  const int il = ok ? i : N - R;
  if constexpr (R == 1) {
    double2 sa = zero, sb = zero;
    sweep_cols<double2, true, KB, NW>(A.S, 0, A.ldq, wave, min(J, A.m), il, av, bv, sa, sb);
    sweep_cols<VT, true, KB, NW>(static_cast<const VT*>(A.V) + (size_t)r * A.vstride, A.m, A.ldq,
                                 first_col<NW>(A.m, wave), J, il, av, bv, sa, sb);
    ps[0][wave][lane] = sa;
    ps[1][wave][lane] = sb;
  } else {
    // FP64 Schur columns take two loads per lane: half the batch keeps the
    // bytes in flight (the batch size does not change any sum)
    double2 sa[2] = {zero, zero}, sb[2] = {zero, zero};
    sweep_cols_pair<double2, (KB > 4 ? KB / 2 : 2), NW>(A.S, 0, A.ldq, wave, min(J, A.m), il, av, bv, sa, sb);
    sweep_cols_pair<VT, KB, NW>(static_cast<const VT*>(A.V) + (size_t)r * A.vstride, A.m, A.ldq,
                                first_col<NW>(A.m, wave), J, il, av, bv, sa, sb);
    ps[0][wave][2 * lane] = sa[0];
    ps[0][wave][2 * lane + 1] = sa[1];
    ps[1][wave][2 * lane] = sb[0];
    ps[1][wave][2 * lane + 1] = sb[1];
  }
  load_coef();
  scalar_partials<NT>(av, bv, J, a0, b0, a1, b1, s0, s12);
  const StepScalars st = step_scalars<NW>(A, r, j, s0, s12, red);  // contains __syncthreads
  if (blk == 0 && tid == 0) {
    double* sc = A.sc + (size_t)r * kScStride;
    sc[kScRho] = st.rho;
    sc[kScInv] = st.inv;
    sc[kScGamRe] = st.gam.x;
    sc[kScGamIm] = st.gam.y;
    sc[kScGrRe] = st.gr.x;
    sc[kScGrIm] = st.gr.y;
    sc[kScScale] = st.scale;
    // reference size for the next step's breakdown test (the other parity
    // slot: this step's slot is still being read by other workgroups)
    sc[kScRef + ((j + 1) & 1)] = st.scale;
    if (j == 0 && A.beta) A.beta[r] = st.rho;
    if (A.flag) {
      int* f = A.flag + r;
      if (!st.finite)
        *f = -1;
      else if (st.brk && *f == 0)
        *f = j + 1;
    }
  }
  // combine the wavefronts (fixed order) and write v_J and u'
  if (wave == 0 && ok) {
    // u may be updated in place (unext == u): each lane reads its u[i]
    // before writing u'[i], and no other thread of the step touches row i of u
    const double2* u = A.u + (size_t)r * A.ustride;
    const VT* __restrict__ z = static_cast<const VT*>(A.z) + (size_t)r * A.zstride;
    VT* vout = static_cast<VT*>(A.V) + (size_t)r * A.vstride + (size_t)(J - A.m) * A.ldq;
    double2 vo[R], nx[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int row = R * lane + q;
      double2 ta = ps[0][0][row], tb = ps[1][0][row];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        ta = cadd(ta, ps[0][w][row]);
        tb = cadd(tb, ps[1][w][row]);
      }
      const double2 te = csub(tb, cmul(st.gr, ta));
      const double2 ui = u[i + q];
      vo[q] = cscale(csub(ui, ta), st.inv);
      nx[q] = cscale(csub(csub(ld2(z, i + q), cmul(st.gr, ui)), te), st.inv);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      st2(vout, i + q, vo[q]);
      A.unext[(size_t)r * A.ustride + i + q] = nx[q];
      if (A.ulonext) st2(static_cast<VT*>(A.ulonext) + (size_t)r * A.zstride, i + q, nx[q]);
    }
  }
}

// y = S c_S + V c_V for slot r (coefficients c[0..ncol)): 64 rows per
// workgroup, wavefront w sums the columns c = w mod kUWaves, fixed-order combine
template <typename VT>
__global__ void __launch_bounds__(kUThreads) kcombine_kernel(KrylovArgs A, const double2* __restrict__ coef,
                                                             int cstride, double2* __restrict__ y, size_t ystride,
                                                             int ncol) {
  const int r = slot_of(A, blockIdx.z);
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int i = blockIdx.x * 64 + lane;
  const bool ok = i < A.N;
  const double2* cf = coef + (size_t)r * cstride;
  double2 acc = make_double2(0.0, 0.0), unused = make_double2(0.0, 0.0);
  const int il = ok ? i : A.N - 1;
  sweep_cols<double2, false, kCBatch, kUWaves>(A.S, 0, A.ldq, wave, min(ncol, A.m), il, cf, nullptr, acc, unused);
  sweep_cols<VT, false, kCBatch, kUWaves>(static_cast<const VT*>(A.V) + (size_t)r * A.vstride, A.m, A.ldq,
                                          first_col<kUWaves>(A.m, wave), ncol, il, cf, nullptr, acc, unused);
  __shared__ double2 ps[kUWaves][64];
  ps[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && ok) {
    double2 t = ps[0][lane];
#pragma unroll
    for (int w = 1; w < kUWaves; ++w) t = cadd(t, ps[w][lane]);
    y[(size_t)r * ystride + i] = t;
  }
}

__global__ void set_index_kernel(int* p, int v, int add) {
  if (threadIdx.x == 0) *p = add ? *p + v : v;
}

// dst = H[:n,:n] with column n-1 += a (slot r), dst dense n x n per slot
__global__ void kpatch_kernel(KrylovArgs A, int n, double2* __restrict__ dst, size_t dstride, int with_a) {
  const int r = slot_of(A, blockIdx.z);
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int c = (int)(e / n), row = (int)(e - (size_t)c * n);
  const double2* H = A.H + (size_t)r * A.hstride;
  double2 v = H[(size_t)c * A.ldh + row];
  if (with_a && c == n - 1) v = cadd(v, A.a[(size_t)r * A.abstride + row]);
  dst[(size_t)blockIdx.z * dstride + e] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void krylov_alloc(KrylovWork& w, int N, size_t ldq, int ncol_cap, int nslots) {
  krylov_free(w);
  (void)ldq;
  w.nrt_dot = (N + kDRows - 1) / kDRows;
  w.ncol_cap = ncol_cap;
  w.nslots = nslots;
  w.ldp = ncol_cap;
  w.pstride = (size_t)w.nrt_dot * ncol_cap;
  w.cdstride = (size_t)4 * w.nrt_dot;
  w.abstride = (size_t)ncol_cap;
  const size_t S = (size_t)nslots;
  SGN_HIP(hipMalloc(&w.Pa, sizeof(double2) * w.pstride * S));
  SGN_HIP(hipMalloc(&w.Pb, sizeof(double2) * w.pstride * S));
  SGN_HIP(hipMalloc(&w.Pcd, sizeof(double) * w.cdstride * S));
  SGN_HIP(hipMalloc(&w.a, sizeof(double2) * w.abstride * S));
  SGN_HIP(hipMalloc(&w.b, sizeof(double2) * w.abstride * S));
  SGN_HIP(hipMalloc(&w.sc, sizeof(double) * kScStride * S));
  SGN_HIP(hipMemset(w.sc, 0, sizeof(double) * kScStride * S));
  SGN_HIP(hipDeviceSynchronize());
}

void krylov_free(KrylovWork& w) {
  for (void* p : {(void*)w.Pa, (void*)w.Pb, (void*)w.Pcd, (void*)w.a, (void*)w.b, (void*)w.sc})
    if (p) (void)hipFree(p);
  w = KrylovWork{};
}

void krylov_bind(const KrylovWork& w, KrylovArgs& A) {
  A.Pa = w.Pa;
  A.Pb = w.Pb;
  A.Pcd = w.Pcd;
  A.ldp = w.ldp;
  A.pstride = w.pstride;
  A.cdstride = w.cdstride;
  A.a = w.a;
  A.b = w.b;
  A.abstride = w.abstride;
  A.sc = w.sc;
  A.nrt_dot = w.nrt_dot;
}

static void check_args(const KrylovWork& w, const KrylovArgs& A) {
  SGN_REQUIRE(A.nb >= 1 && A.nb <= w.nslots && A.nb <= kMaxBatch, SGN_EINVAL, "krylov: batch exceeds workspace");
  // a device step index is shared by every launch slot (all at the same step)
  SGN_REQUIRE(!A.jdev || A.joff >= 0, SGN_EINVAL, "krylov: negative step offset");
  for (int z = 0; z < A.nb; ++z) {
    SGN_REQUIRE(A.act[z] >= 0 && A.act[z] < w.nslots, SGN_EINVAL, "krylov: slot out of range");
    SGN_REQUIRE(A.jv[z] >= 0 && A.m + A.jv[z] <= w.ncol_cap, SGN_EINVAL, "krylov: J exceeds workspace");
  }
}

// columns a launch reads, for the algorithmic byte counts: the FP64 Schur
// part, shared by the slots (once), and the sum of the slots' Krylov parts
static void col_sums(const KrylovArgs& A, double& sum_m, double& sum_k) {
  sum_m = A.m;
  sum_k = 0.0;
  for (int z = 0; z < A.nb; ++z) sum_k += A.jv[z];
}

bool krylov_tune_valid(const KrylovTune& t) {
  return (t.ub == 4 || t.ub == 8 || t.ub == 16) && (t.cpw == 1 || t.cpw == 2 || t.cpw == 4) &&
         (t.uw == 8 || t.uw == 16);
}

template <typename VT>
static auto dot_kernel_for(int cpw) {
  switch (cpw) {
    case 1: return kdot_kernel<VT, 1>;
    case 2: return kdot_kernel<VT, 2>;
    default: return kdot_kernel<VT, 4>;
  }
}

template <typename VT, int NW>
static auto update_kernel_nw(int ub) {
  switch (ub) {
    case 4: return kupdate_kernel<VT, 4, NW>;
    case 16: return kupdate_kernel<VT, 16, NW>;
    default: return kupdate_kernel<VT, 8, NW>;
  }
}

template <typename VT>
static auto update_kernel_for(const KrylovTune& t) {
  return t.uw == 16 ? update_kernel_nw<VT, 16>(t.ub) : update_kernel_nw<VT, 8>(t.ub);
}

// 16-byte loads of row pairs of the FP32 columns (dot and update passes)
template <typename VT>
static void check_pairs(const KrylovArgs& A) {
  static_assert(kRpl % 2 == 0, "dot tiles hold whole row pairs");
  if (rows_per_lane<VT>() == 2) {
    SGN_REQUIRE(A.N % 2 == 0 && A.ldq % 2 == 0 && A.vstride % 2 == 0 && (reinterpret_cast<uintptr_t>(A.V) & 15) == 0,
                SGN_EINVAL, "krylov: FP32 basis needs an even row count and strides and a 16-byte aligned base");
  }
}

template <typename VT>
void krylov_dot(const KrylovWork& w, const KrylovArgs& Ain, bool with_z, hipStream_t s, Profiler* prof) {
  KrylovArgs A = Ain;
  krylov_bind(w, A);
  check_args(w, A);
  check_pairs<VT>(A);
  SGN_REQUIRE(krylov_tune_valid(A.tune), SGN_EINVAL, "krylov: invalid launch shape");
  const int Jmax = A.m + A.jmax();
  const int gcols = 4 * A.tune.cpw;
  const int ngroups = Jmax > 0 ? (Jmax + gcols - 1) / gcols : 1;
  const double vb = (double)sizeof(VT);
  double sm, sk;
  col_sums(A, sm, sk);
  const double qbytes = (double)A.N * (16.0 * sm + vb * sk);
  // algorithmic bytes: Q, u, z read once; a, b written
  const size_t nwg = (size_t)w.nrt_dot * ngroups * A.nb;
  SGN_REQUIRE(nwg * 256 < (size_t(1) << 32), SGN_EINVAL, "krylov: dot grid too large");
  // per-slot work counts S for every slot
  const double cols = A.nb * (double)A.m + sk;
  prof_launch(prof, K_KDOT, qbytes + A.nb * A.N * (16.0 + (with_z ? vb : 0.0)) + 32.0 * cols,
              16.0 * (double)A.N * cols, dot_kernel_for<VT>(A.tune.cpw), dim3((unsigned)nwg), dim3(256), 0, s,
              A, with_z ? 1 : 0);
  // partial sums of every row tile read, a, b written
  prof_launch(prof, K_KRED, 32.0 * cols * (w.nrt_dot + 1.0) + 32.0 * A.nb * w.nrt_dot,
              4.0 * cols * w.nrt_dot, kred_kernel, dim3(std::max(1, (Jmax + 31) / 32), 1, A.nb), dim3(256), 0, s,
              A);
}

template <typename VT>
void krylov_update(const KrylovWork& w, const KrylovArgs& Ain, hipStream_t s, Profiler* prof) {
  KrylovArgs A = Ain;
  krylov_bind(w, A);
  check_args(w, A);
  SGN_REQUIRE(A.m + A.jmax() + 1 <= A.ldh, SGN_EINVAL, "krylov: H too small");
  SGN_REQUIRE(krylov_tune_valid(A.tune), SGN_EINVAL, "krylov: invalid launch shape");
  // per slot: Hessenberg-row workgroups for rows 0..m+jmax, then the blocks
  // of 64 R rows
  const int nh = (A.m + A.jmax() + 1 + A.tune.uw - 1) / A.tune.uw;
  const int rows = 64 * rows_per_lane<VT>();
  check_pairs<VT>(A);
  const size_t nwg = ((size_t)((A.N + rows - 1) / rows) + nh) * A.nb;
  const int nthr = 64 * A.tune.uw;
  SGN_REQUIRE(nwg * nthr < (size_t(1) << 32), SGN_EINVAL, "krylov: update grid too large");
  const double vb = (double)sizeof(VT);
  double sm, sk;
  col_sums(A, sm, sk);
  const double qbytes = (double)A.N * (16.0 * sm + vb * sk);
  // read Q, u, z; write v_J, u' (+ its low-precision copy)
  const double vec = A.N * (16.0 + vb + vb + 16.0 + (A.ulonext ? vb : 0.0));
  const double cols = A.nb * (double)A.m + sk;  // per-slot work counts S for every slot
  prof_launch(prof, K_KUPDATE, qbytes + A.nb * vec + 32.0 * cols, 16.0 * (double)A.N * cols,
              update_kernel_for<VT>(A.tune), dim3((unsigned)nwg), dim3(nthr), 0, s, A, nh);
}

template <typename VT>
void krylov_combine(const KrylovWork& w, const KrylovArgs& Ain, const double2* coef, int cstride, double2* y,
                    size_t ystride, int ncol, hipStream_t s, Profiler* prof) {
  KrylovArgs A = Ain;
  krylov_bind(w, A);
  check_args(w, A);
  SGN_REQUIRE(ncol >= 0 && ncol <= w.ncol_cap, SGN_EINVAL, "krylov: ncol exceeds workspace");
  const double vb = (double)sizeof(VT);
  const int nm = std::min(ncol, A.m);
  prof_launch(prof, K_KCOMBINE, (double)A.N * (16.0 * nm + A.nb * (vb * (ncol - nm) + 16.0)),
              A.nb * 8.0 * (double)A.N * ncol, kcombine_kernel<VT>, dim3((A.N + 63) / 64, 1, A.nb), dim3(kUThreads),
              0, s, A, coef, cstride, y, ystride, ncol);
}

void krylov_set_index(int* p, int v, bool add, hipStream_t s) {
  hipLaunchKernelGGL(set_index_kernel, dim3(1), dim3(64), 0, s, p, v, add ? 1 : 0);
  SGN_HIP(hipGetLastError());
}

void krylov_patch(const KrylovWork& w, const KrylovArgs& Ain, int n, double2* dst, size_t dstride, bool with_a,
                  hipStream_t s) {
  KrylovArgs A = Ain;
  krylov_bind(w, A);
  check_args(w, A);
  const size_t tot = (size_t)n * n;
  if (tot == 0) return;
  hipLaunchKernelGGL(kpatch_kernel, dim3((unsigned)((tot + 255) / 256), 1, A.nb), dim3(256), 0, s, A, n, dst,
                     dstride, with_a ? 1 : 0);
  SGN_HIP(hipGetLastError());
}

template void krylov_dot<double2>(const KrylovWork&, const KrylovArgs&, bool, hipStream_t, Profiler*);
template void krylov_dot<float2>(const KrylovWork&, const KrylovArgs&, bool, hipStream_t, Profiler*);
template void krylov_update<double2>(const KrylovWork&, const KrylovArgs&, hipStream_t, Profiler*);
template void krylov_update<float2>(const KrylovWork&, const KrylovArgs&, hipStream_t, Profiler*);
template void krylov_combine<double2>(const KrylovWork&, const KrylovArgs&, const double2*, int, double2*, size_t,
                                      int, hipStream_t, Profiler*);
template void krylov_combine<float2>(const KrylovWork&, const KrylovArgs&, const double2*, int, double2*, size_t, int,
                                     hipStream_t, Profiler*);
