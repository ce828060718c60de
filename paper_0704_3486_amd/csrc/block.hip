// Block (s-step) form of the modified Arnoldi process of Section 5.2, step
// (iv), for FP64 Krylov columns.
//
// One block takes the composite basis Q = (S_m v_1 .. v_k) from p = m + k + 1
// to p + s columns.  q_{p-1} = v_{k+1} is the newest column, not yet
// multiplied by A:
//   * Krylov directions from the Chebyshev recurrence on [-e, e] (e a bound
//     of A's spectral radius, so the directions stay well conditioned):
//       W_0 = q_{p-1},  W_1 = A W_0 / e,  W_{i+1} = 2 A W_i / e - W_{i-1},
//     that is A W_{0..s-1} = W_{0..s} Th with Th the (s+1) x s tridiagonal
//     matrix of the recurrence (Th[1][0] = e, Th[j-1][j] = Th[j+1][j] = e/2);
//   * block classical Gram-Schmidt against Q with one full second pass:
//       C1 = Q^dag W, W -= Q C1;  C2 = Q^dag W, G = W^dag W, W -= Q C2;
//     R = chol(G - C2^dag C2) (upper), new columns q_p .. q_{p+s-1} = W R^-1;
//   * the Hessenberg columns p-1 .. p+s-2 from the change of basis: with
//       Rc = [e_{p-1} | (C1 + C2; R)]   ((p + s) x (s + 1), W_{0..s} = Q Rc)
//     A Q Rc' = Q Rc Th (Rc' its first s columns), and A's action on the
//     first p - 1 columns is the known H_{p x (p-1)}, so
//       H(:, p-1 .. p+s-2) = (Rc Th - [H_{p x (p-1)} Rc'_top; 0]) Rb^-1,
//     Rb = rows p-1 .. p+s-2 of Rc' (upper triangular, diagonal 1, R_ii).
// In exact arithmetic this is the Krylov space, basis and Hessenberg matrix
// of the one-vector process (A Q_k = Q_{k+1} Hbar_k, Eq. eq:modArnoldi): the
// Schur columns enter through A S = S T, which the T block of H records.  It
// reads Q four times per block of s steps instead of twice per step.
//
// The two block products are tall and skinny (Q^dag W: p x N times N x s;
// Q C: N x p times p x s), so they run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64) with the real and imaginary parts of the s <= 8
// block vectors side by side in the 16-wide dimension: two real products per
// 16 x 4 fragment of Q give the complex result without cross-lane sums.
// Every sum has a fixed order, so results do not depend on the launch.
#include "internal.h"
#include "context.h"

typedef double v4d __attribute__((ext_vector_type(4)));

// A complex zero in device memory for lanes outside the block (their loads
// read it, so every load is issued unconditionally; see zgemm.hip)
__device__ double2 sgn_block_zero_entry;

namespace {

__device__ inline v4d mfma(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

__device__ inline double2 wsum2(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// ---------------------------------------------------------------------------
// dot pass: partial sums of conj(col_c) . W_v over row chunks.  Columns c < p
// are Q's; with ncol = p + s, columns p + u are W_u (the Gram matrix).
// Wavefront: 16 columns x rpw rows; lane (li, lk) = (lane % 16, lane / 16)
// holds, per k-step of four rows, row lk of column li (B fragment) and of
// block vector li % 8, real part for li < 8, imaginary for li >= 8 (A
// fragment).  D1 = A Re(Q), D2 = A Im(Q) give
//   Re C[j][v] = D1[v][j] + D2[v+8][j],  Im C[j][v] = D1[v+8][j] - D2[v][j].
// Workgroup: four wavefronts on consecutive row ranges, summed in order.
struct BDot {
  const double2* Q;
  size_t ldq;
  int p;
  const double2* W;
  size_t ldw;
  int s;
  int ncol;
  int N;
  int rpw;        // rows per wavefront, a multiple of 4
  double2* part;  // [chunk][ncol][kBlockMax]
};

__global__ void __launch_bounds__(256) bdot_kernel(BDot a) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int c = blockIdx.x * 16 + li;
  const int v = li & 7;
  const bool imag = li >= 8;
  const int r0 = (blockIdx.y * 4 + wave) * a.rpw;
  const int r1 = min(r0 + a.rpw, a.N);
  const int nit = r1 > r0 ? (r1 - r0) >> 2 : 0;
  // a column past ncol reads column ncol - 1 (its sums are not written)
  const int cc = min(c, a.ncol - 1);
  const double2* qp = (cc < a.p ? a.Q + (size_t)cc * a.ldq : a.W + (size_t)(cc - a.p) * a.ldw) + r0 + lk;
  // the A fragment: the lane's real or imaginary part, loaded as one double
  const bool vok = v < a.s;
  const double* wp = vok ? reinterpret_cast<const double*>(a.W + (size_t)v * a.ldw + r0 + lk) + (imag ? 1 : 0)
                         : reinterpret_cast<const double*>(&sgn_block_zero_entry);
  const int dw = vok ? 8 : 0;  // four rows, in doubles
  v4d d1 = {0.0, 0.0, 0.0, 0.0}, d2 = {0.0, 0.0, 0.0, 0.0};
  int it = 0;
  for (; it + 4 <= nit; it += 4) {
    double2 qv[4];
    double wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      qv[u] = qp[4 * u];
      wv[u] = wp[dw * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      d1 = mfma(wv[u], qv[u].x, d1);
      d2 = mfma(wv[u], qv[u].y, d2);
    }
    qp += 16;
    wp += 4 * dw;
  }
  for (; it < nit; ++it) {
    const double2 qv = *qp;
    const double wv = *wp;
    d1 = mfma(wv, qv.x, d1);
    d2 = mfma(wv, qv.y, d2);
    qp += 4;
    wp += dw;
  }
  // lane (j = li, lk): items t hold rows lk + 4 t of D: vectors lk, lk + 4
  double2 c0 = make_double2(d1[0] + d2[2], d1[2] - d2[0]);
  double2 c1 = make_double2(d1[1] + d2[3], d1[3] - d2[1]);
  __shared__ double2 red[4][64][2];
  red[wave][lane][0] = c0;
  red[wave][lane][1] = c1;
  __syncthreads();
  if (wave == 0 && c < a.ncol) {
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      c0 = cadd(c0, red[w][lane][0]);
      c1 = cadd(c1, red[w][lane][1]);
    }
    // vectors past s have zero fragments, so their sums are zero
    double2* o = a.part + ((size_t)blockIdx.y * a.ncol + c) * kBlockMax;
    o[lk] = c0;
    o[lk + 4] = c1;
  }
}

// sum of the dot partials over chunks in a fixed order: 32 entries per
// workgroup, 8 threads per entry (every 8th chunk), then the 8 in order.
// Entry e = c * kBlockMax + v; c < p goes to C[c][v] (and C1[c][v] + C[c][v]
// to Ct[c][v] if Ct), c >= p to G[c - p][v].
__global__ void __launch_bounds__(256) bred_kernel(const double2* __restrict__ part, int nchunk, int nent, int p,
                                                   double2* __restrict__ C, double2* __restrict__ G,
                                                   const double2* __restrict__ C1, double2* __restrict__ Ct) {
  const int el = threadIdx.x & 31, q = threadIdx.x >> 5;
  const int e = blockIdx.x * 32 + el;
  const double2 zero = make_double2(0.0, 0.0);
  double2 acc = zero;
  if (e < nent)
    for (int t0 = q; t0 < nchunk; t0 += 64) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + 8 * u;
        const double2 x = part[(size_t)min(t, nchunk - 1) * nent + e];
        v[u] = make_double2(t < nchunk ? x.x : 0.0, t < nchunk ? x.y : 0.0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
    }
  __shared__ double2 r[8][33];
  r[q][el] = acc;
  __syncthreads();
  if (q == 0 && e < nent) {
    double2 t = r[0][el];
    for (int w = 1; w < 8; ++w) t = cadd(t, r[w][el]);
    const int c = e / kBlockMax;
    if (c < p) {
      C[e] = t;
      if (Ct) Ct[e] = cadd(C1[e], t);
    } else {
      G[e - p * kBlockMax] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Q C on the matrix cores: 16 rows of Q (column-major, ld ldq) times the
// coefficients C[c][v] of columns c < ncol, for the k-steps (four columns)
// k0, k0 + dk, ... .  Lane (li, lk) holds row li of column 4 ks + lk (A
// fragment) and that column's coefficient for block vector li % 8 (B
// fragment), so that
//   D += Re(Q) [Re C | Im C] + Im(Q) [-Im C | Re C]
// is [Re | Im] of (Q C) for the 16 rows and 8 vectors (rows lk + 4 t in item
// t, vector li % 8, real part for li < 8).  A partial last k-step reads the
// zero entry for columns past ncol.
__device__ inline v4d qc_steps(const double2* __restrict__ Q, size_t ldq, int row, int ncol,
                               const double2* __restrict__ C, int v, bool imag, bool vok, int lk, int k0, int dk,
                               v4d d) {
  const double2* zero = &sgn_block_zero_entry;
  const int nfull = ncol >> 2, nk = (ncol + 3) >> 2;
  const double2* qp = Q + (size_t)(4 * k0 + lk) * ldq + row;
  const double2* cp = vok ? C + (size_t)(4 * k0 + lk) * kBlockMax + v : zero;
  const size_t dq = (size_t)4 * dk * ldq;
  const int dc = vok ? 4 * dk * kBlockMax : 0;
  int ks = k0;
  for (; ks + 3 * dk < nfull; ks += 4 * dk) {
    double2 qv[4], cv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      qv[u] = qp[u * dq];
      cv[u] = cp[u * dc];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double b1 = imag ? cv[u].y : cv[u].x;
      const double b2 = imag ? cv[u].x : -cv[u].y;
      d = mfma(qv[u].x, b1, d);
      d = mfma(qv[u].y, b2, d);
    }
    qp += 4 * dq;
    cp += 4 * dc;
  }
  for (; ks < nfull; ks += dk) {
    const double2 qv = *qp, cv = *cp;
    const double b1 = imag ? cv.y : cv.x;
    const double b2 = imag ? cv.x : -cv.y;
    d = mfma(qv.x, b1, d);
    d = mfma(qv.y, b2, d);
    qp += dq;
    cp += dc;
  }
  if (ks < nk) {
    const bool ok = 4 * ks + lk < ncol;
    const double2 qv = *(ok ? qp : zero), cv = *(ok ? cp : zero);
    const double b1 = imag ? cv.y : cv.x;
    const double b2 = imag ? cv.x : -cv.y;
    d = mfma(qv.x, b1, d);
    d = mfma(qv.y, b2, d);
  }
  return d;
}

// complex entries (Re in lane li < 8, Im from lane li + 8) of a Q C tile
__device__ inline void qc_pairs(const v4d& d, double2 (&res)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) res[t] = make_double2(d[t], __shfl_xor(d[t], 8, 64));
}

// The block's Hessenberg columns p-1 .. p+s-2, one thread per (row r, column
// j): M[i] = (Rc Th)[r][i] - P[r][i-1] for i <= j (P = H_{p x (p-1)} Ct, zero
// for rows r >= p), H[r][p-1+j] = sum_{i <= j} M[i] Rbi[i][j]; zero below the
// subdiagonal.  Rc(r, 0) = [r == p-1]; Rc(r, i) = Ct[r][i-1] (r < p) or
// R[r-p][i-1] (r >= p, upper triangular).
struct BHess {
  int p, s;
  double e;
  const double2* Ct;   // [p][kBlockMax]
  const double2* P;    // [v][r], ld ldp: H_{p x (p-1)} Ct
  int ldp;
  const double2* R;    // [kBlockMax][kBlockMax]
  const double2* Rbi;  // [kBlockMax][kBlockMax]
  double2* H;
  int ldh;
};

__device__ inline double2 rc_entry(const BHess& h, int r, int i) {
  if (i == 0) return make_double2(r == h.p - 1 ? 1.0 : 0.0, 0.0);
  if (r < h.p) return h.Ct[(size_t)r * kBlockMax + i - 1];
  const int rr = r - h.p;
  return rr <= i - 1 ? h.R[rr * kBlockMax + i - 1] : make_double2(0.0, 0.0);
}

__device__ void hess_entry(const BHess& h, int idx) {
  const int r = idx / kBlockMax, j = idx % kBlockMax;
  if (r >= h.p + h.s || j >= h.s) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int i = 0; i <= j; ++i) {
    double2 mi;
    if (i == 0) {
      mi = cscale(rc_entry(h, r, 1), h.e);
    } else {
      mi = cscale(cadd(rc_entry(h, r, i - 1), rc_entry(h, r, i + 1)), 0.5 * h.e);
      if (r < h.p) mi = csub(mi, h.P[(size_t)(i - 1) * h.ldp + r]);
    }
    acc = cfma(mi, h.Rbi[i * kBlockMax + j], acc);
  }
  // column p-1+j has its subdiagonal in row p+j; below it H is zero
  h.H[(size_t)(h.p - 1 + j) * h.ldh + r] = (r <= h.p + j) ? acc : make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------------------
// update pass: Wout = (Win - Q C) [Rinv].  Wavefront: 16 rows x all p
// columns.  With Rinv (the second pass) the workgroups past the rows also
// write the block's Hessenberg columns (hess).
struct BUpd {
  const double2* Q;
  size_t ldq;
  int p;
  const double2* C;  // [p][kBlockMax]
  const double2* Win;
  double2* Wout;
  size_t ldw;
  int s;
  const double2* Rinv;  // [kBlockMax][kBlockMax] upper triangular, or null
  int N;
  int nrowblk;          // workgroups on rows
  BHess hess;
};

__global__ void __launch_bounds__(256) bupdate_kernel(BUpd a) {
  if ((int)blockIdx.x >= a.nrowblk) {
    hess_entry(a.hess, ((int)blockIdx.x - a.nrowblk) * 256 + threadIdx.x);
    return;
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = (blockIdx.x * 4 + wave) * 16;
  const bool active = r0 < a.N;  // wavefront-uniform
  const int row = min(r0 + li, a.N - 1);
  const int v = li & 7;
  const bool vok = v < a.s;
  v4d d = {0.0, 0.0, 0.0, 0.0};
  if (active) d = qc_steps(a.Q, a.ldq, row, a.p, a.C, v, li >= 8, vok, lk, 0, 1, d);
  double2 res[4];
  qc_pairs(d, res);
  if (!a.Rinv) {
    if (active && li < 8 && vok)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int rr = r0 + lk + 4 * t;
        if (rr < a.N) {
          const size_t o = (size_t)v * a.ldw + rr;
          a.Wout[o] = csub(a.Win[o], res[t]);
        }
      }
    return;
  }
  // second pass: W'' = Win - Q C, then W'' Rinv per row (through LDS)
  __shared__ double2 tile[4][16][kBlockMax];
  if (li < 8)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rr = r0 + lk + 4 * t;
      double2 val = make_double2(0.0, 0.0);
      if (active && vok && rr < a.N) val = csub(a.Win[(size_t)v * a.ldw + rr], res[t]);
      tile[wave][lk + 4 * t][v] = val;
    }
  __syncthreads();
  if (!active) return;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int idx = lane + 64 * h;
    const int rl = idx >> 3, vv = idx & 7;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < kBlockMax; ++u) acc = cfma(tile[wave][rl][u], a.Rinv[u * kBlockMax + vv], acc);
    const int rr = r0 + rl;
    if (vv < a.s && rr < a.N) a.Wout[(size_t)vv * a.ldw + rr] = acc;
  }
}

// ---------------------------------------------------------------------------
// Between the two passes' reductions and the second update: workgroup 0
// factors the block, G'' = G - C2^dag C2 = R^dag R (R upper), and forms R^-1
// and Rb^-1 (Rb = [1, Ct[p-1][0 .. s-2]; 0, R[0 .. s-2][0 .. s-2]]); it
// raises flag when the block is not numerically of full rank (a pivot below
// 1e-12 of the block's size, or below 1e-7 of the largest pivot) or not
// finite.  Workgroups 1.. form P = H_{p x (p-1)} Ct for 16 rows each (the
// four wavefronts take every fourth k-step, summed in order), from the
// first column where a row of the tile can be nonzero (H is upper
// Hessenberg below the T block, T upper triangular).
struct BSmall {
  int p, s, m;
  const double2* C2;  // [p][kBlockMax]
  const double2* Ct;  // [p][kBlockMax] C1 + C2
  const double2* G;   // [s][kBlockMax]
  const double2* H;
  int ldh;
  double2* P;  // [v][r], ld ldp
  int ldp;
  double2* R;     // [kBlockMax][kBlockMax]
  double2* Rinv;  // [kBlockMax][kBlockMax]
  double2* Rbi;   // [kBlockMax][kBlockMax]
  int* flag;
};

__device__ void block_factor(const BSmall& a) {
  const int tid = threadIdx.x;
  const int s = a.s, p = a.p;
  __shared__ double2 red[4][64];
  __shared__ double redn[4][64];
  __shared__ double2 g[kBlockMax][kBlockMax], R[kBlockMax][kBlockMax], Ri[kBlockMax][kBlockMax],
      Rb[kBlockMax][kBlockMax], Rbi[kBlockMax][kBlockMax];
  __shared__ double piv[kBlockMax], ref_s;
  __shared__ int bad;
  const int ent = tid & 63, q = tid >> 6, u = ent >> 3, v = ent & 7;
  {
    // G'' entries (u, v) by four threads (columns c = q, q + 4, ...), and
    // |Ct[:, v]|^2 (the block vectors' size before projection)
    double2 acc = make_double2(0.0, 0.0);
    double nn = 0.0;
    if (u < s && v < s)
      for (int cb = q; cb < p; cb += 32) {
        // eight columns' loads in flight (clamped), then their sums in order
        double2 x[8], y[8], z[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const size_t c = (size_t)min(cb + 4 * t, p - 1) * kBlockMax;
          x[t] = a.C2[c + u];
          y[t] = a.C2[c + v];
          z[t] = a.Ct[c + v];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (cb + 4 * t < p) {
            acc = cfmac(x[t], y[t], acc);
            nn += cabs2(z[t]);
          }
      }
    red[q][ent] = acc;
    redn[q][ent] = nn;
  }
  if (tid < kBlockMax * kBlockMax) {
    R[u][v] = make_double2(0.0, 0.0);
    Ri[u][v] = make_double2(0.0, 0.0);
    Rb[u][v] = make_double2(0.0, 0.0);
    Rbi[u][v] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (tid < kBlockMax * kBlockMax) {
    const double2 sub = cadd(cadd(red[0][tid], red[1][tid]), cadd(red[2][tid], red[3][tid]));
    g[u][v] = (u < s && v < s) ? csub(a.G[u * kBlockMax + v], sub) : make_double2(0.0, 0.0);
  }
  if (tid == 0) {
    bad = 0;
    double r = 0.0;
    for (int w = 0; w < s; ++w) {
      const int e = w * kBlockMax + w;
      r = fmax(r, a.G[e].x + redn[0][e] + redn[1][e] + redn[2][e] + redn[3][e]);
    }
    ref_s = r;
  }
  __syncthreads();
  // right-looking Cholesky: step j forms row j of R and updates the trailing block
  for (int j = 0; j < s; ++j) {
    if (tid == 0) {
      double dj = g[j][j].x;
      if (!(dj > 0.0) || !isfinite(dj)) {
        bad = 1;
        dj = 1.0;
      }
      piv[j] = sqrt(dj);
    }
    __syncthreads();
    if (tid < kBlockMax && tid >= j && tid < s)
      R[j][tid] = tid == j ? make_double2(piv[j], 0.0) : cscale(g[j][tid], 1.0 / piv[j]);
    __syncthreads();
    if (tid < kBlockMax * kBlockMax && u > j && v > j && u < s && v < s) g[u][v] = csub(g[u][v], cmulc(R[j][u], R[j][v]));
    __syncthreads();
  }
  // Rb from R and the last basis column's coefficients
  if (tid < kBlockMax * kBlockMax && u < s && v < s) {
    if (u == 0)
      Rb[0][v] = v == 0 ? make_double2(1.0, 0.0) : a.Ct[(size_t)(p - 1) * kBlockMax + v - 1];
    else if (v >= u)
      Rb[u][v] = R[u - 1][v - 1];
  }
  __syncthreads();
  // inverses of the two upper triangular factors, one column per thread
  if (tid < 2 * kBlockMax) {
    const int col = tid & 7;
    const bool second = tid >= kBlockMax;
    auto& M = second ? Rb : R;
    auto& X = second ? Rbi : Ri;
    if (col < s) {
      X[col][col] = make_double2(1.0 / M[col][col].x, 0.0);
      for (int i = col - 1; i >= 0; --i) {
        double2 t = make_double2(0.0, 0.0);
        for (int l = i + 1; l <= col; ++l) t = cfma(M[i][l], X[l][col], t);
        X[i][col] = cscale(cneg(t), 1.0 / M[i][i].x);
      }
    }
  }
  __syncthreads();
  if (tid < kBlockMax * kBlockMax) {
    a.R[tid] = R[u][v];
    a.Rinv[tid] = Ri[u][v];
    a.Rbi[tid] = Rbi[u][v];
  }
  if (tid == 0) {
    double dmin = HUGE_VAL, dmax = 0.0;
    for (int j = 0; j < s; ++j) {
      dmin = fmin(dmin, piv[j]);
      dmax = fmax(dmax, piv[j]);
    }
    const double r = ref_s;
    if (bad || !(r > 0.0) || !isfinite(r) || dmin * dmin < 1e-24 * r || dmin < 1e-7 * dmax) a.flag[0] = 1;
  }
}

__global__ void __launch_bounds__(256) bsmall_kernel(BSmall a) {
  if (blockIdx.x == 0) {
    block_factor(a);
    return;
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = (blockIdx.x - 1) * 16;
  const int row = min(r0 + li, a.p - 1);
  const int v = li & 7;
  const int c0 = r0 < a.m ? r0 : max(a.m, r0 - 1);  // columns below c0 are zero in these rows
  v4d d = {0.0, 0.0, 0.0, 0.0};
  d = qc_steps(a.H, a.ldh, row, a.p - 1, a.Ct, v, li >= 8, v < a.s, lk, (c0 >> 2) + wave, 4, d);
  __shared__ v4d red[4][64];
  red[wave][lane] = d;
  __syncthreads();
  if (wave != 0) return;
  d = red[0][lane];
#pragma unroll
  for (int w = 1; w < 4; ++w) d += red[w][lane];
  double2 res[4];
  qc_pairs(d, res);
  if (li < 8 && v < a.s)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rr = r0 + lk + 4 * t;
      if (rr < a.p) a.P[(size_t)v * a.ldp + rr] = res[t];
    }
}

int nchunks_for(int N, int& rpw) {
  // rows per wavefront: 64 or more, so that at most 128 chunks of four
  // wavefronts cover N
  const int want = (N + 4 * 128 - 1) / (4 * 128);
  rpw = std::max(64, (want + 3) & ~3);
  return (N + 4 * rpw - 1) / (4 * rpw);
}

}  // namespace

void block_alloc(BlockWork& b, int N, size_t ldq, int ncap) {
  block_free(b);
  int rpw = 0;
  const int nch = nchunks_for(N, rpw);
  SGN_HIP(hipMalloc(&b.W, sizeof(double2) * ldq * kBlockMax));
  SGN_HIP(hipMalloc(&b.part, sizeof(double2) * (size_t)nch * (ncap + kBlockMax) * kBlockMax));
  SGN_HIP(hipMalloc(&b.C1, sizeof(double2) * (size_t)ncap * kBlockMax));
  SGN_HIP(hipMalloc(&b.C2, sizeof(double2) * (size_t)ncap * kBlockMax));
  SGN_HIP(hipMalloc(&b.Ct, sizeof(double2) * (size_t)ncap * kBlockMax));
  SGN_HIP(hipMalloc(&b.P, sizeof(double2) * (size_t)ncap * kBlockMax));
  SGN_HIP(hipMalloc(&b.G, sizeof(double2) * kBlockMax * kBlockMax));
  SGN_HIP(hipMalloc(&b.R, sizeof(double2) * kBlockMax * kBlockMax * 3));
  b.Rinv = b.R + kBlockMax * kBlockMax;
  b.Rbi = b.R + 2 * kBlockMax * kBlockMax;
  SGN_HIP(hipMalloc(&b.flag, sizeof(int)));
  b.ncap = ncap;
}

void block_free(BlockWork& b) {
  for (double2** p : {&b.W, &b.part, &b.C1, &b.C2, &b.Ct, &b.P, &b.G, &b.R})
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  b.Rinv = b.Rbi = nullptr;
  if (b.flag) (void)hipFree(b.flag);
  b.flag = nullptr;
  b.ncap = 0;
}

void block_step(sgn_ctx* c, int k, int sb, double e, hipStream_t s, Profiler* prof) {
  BlockWork& b = c->blk;
  const int m = c->m, N = c->N, p = m + 1 + k;
  const size_t ldq = c->ldq;
  SGN_REQUIRE(sb >= 1 && sb <= kBlockMax && p + sb <= c->ncap && b.ncap >= c->ncap, SGN_EINVAL,
              "block step exceeds the workspace");
  double2* Q = c->Q;
  double2* W = b.W;
  const double2* w0 = Q + (size_t)(p - 1) * ldq;
  // Krylov directions: W_1 = A W_0 / e, W_{i+1} = 2 A W_i / e - W_{i-1}
  if (k == 0)  // W_0 = v_1 = x_perp / beta, written to Q on the way
    wilson_apply_cheb(c->lat, c->links, c->wA, W, &c->scal[1], Q + (size_t)m * ldq, nullptr, 1.0 / e, 0.0, s, prof);
  else
    wilson_apply_cheb(c->lat, c->links, w0, W, nullptr, nullptr, nullptr, 1.0 / e, 0.0, s, prof);
  for (int i = 1; i < sb; ++i)
    wilson_apply_cheb(c->lat, c->links, W + (size_t)(i - 1) * ldq, W + (size_t)i * ldq, nullptr, nullptr,
                      i == 1 ? w0 : W + (size_t)(i - 2) * ldq, 2.0 / e, -1.0, s, prof);
  int rpw = 0;
  const int nch = nchunks_for(N, rpw);
  auto dot = [&](double2* C, int ncol, const double2* C1, double2* Ct) {
    BDot d{Q, ldq, p, W, ldq, sb, ncol, N, rpw, b.part};
    // Q (and W as columns) read once, W once per column group, partials written
    const double bytes = 16.0 * N * ((double)ncol + sb) + 16.0 * nch * ncol * kBlockMax;
    prof_launch(prof, K_BDOT, bytes, 8.0 * N * ncol * sb, bdot_kernel, dim3((ncol + 15) / 16, nch), dim3(256), 0,
                s, d);
    const int nent = ncol * kBlockMax;
    prof_launch(prof, K_BRED, 16.0 * (double)nch * nent + 16.0 * nent, 2.0 * nch * nent, bred_kernel,
                dim3((nent + 31) / 32), dim3(256), 0, s, (const double2*)b.part, nch, nent, p, C, b.G, C1, Ct);
  };
  const int nrowblk = (N + 63) / 64;
  // pass 1
  dot(b.C1, p, nullptr, nullptr);
  {
    BUpd u{Q, ldq, p, b.C1, W, W, ldq, sb, nullptr, N, nrowblk, BHess{}};
    prof_launch(prof, K_BUPDATE, 16.0 * N * ((double)p + 2.0 * sb) + 16.0 * p * sb, 8.0 * N * p * sb, bupdate_kernel,
                dim3(nrowblk), dim3(256), 0, s, u);
  }
  // pass 2 with the Gram matrix of the projected block
  dot(b.C2, p + sb, b.C1, b.Ct);
  {
    BSmall sm{p, sb, m, b.C2, b.Ct, b.G, c->Hc, c->ncap, b.P, c->ncap, b.R, b.Rinv, b.Rbi, b.flag};
    const double hb = 16.0 * ((double)p * p / 2 + 3.0 * p * sb);
    prof_launch(prof, K_BSMALL, hb, 8.0 * p * p * sb / 2, bsmall_kernel, dim3(1 + (p + 15) / 16), dim3(256), 0, s,
                sm);
  }
  {
    BHess h{p, sb, e, b.Ct, b.P, c->ncap, b.R, b.Rbi, c->Hc, c->ncap};
    BUpd u{Q, ldq, p, b.C2, W, Q + (size_t)p * ldq, ldq, sb, b.Rinv, N, nrowblk, h};
    const int nh = ((p + sb) * kBlockMax + 255) / 256;
    prof_launch(prof, K_BUPDATE, 16.0 * N * ((double)p + 2.0 * sb) + 16.0 * p * sb, 8.0 * N * p * sb, bupdate_kernel,
                dim3(nrowblk + nh), dim3(256), 0, s, u);
  }
}
