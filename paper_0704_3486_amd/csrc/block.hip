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
// (v_mfma_f64_16x16x4f64) with the real and imaginary parts of 8 block
// vectors side by side in the 16-wide dimension (s <= 16: two halves): two
// real products per 16 x 4 fragment of Q and half give the complex result
// without cross-lane sums.
// Every sum has a fixed order, so results do not depend on the launch.
//
// A launch carries one or several right-hand sides of one field at the same
// basis size (the batched applies advance in lockstep): the Schur columns S
// are shared, each source has its own Krylov columns V_r, block vectors,
// coefficients, factors and Hessenberg matrix at fixed strides, and the
// launch position z (fastest in the workgroup numbering, so that the
// workgroups reading the same rows of S run together) selects slot act[z].
// Per slot the arithmetic does not depend on the other slots.
#include "internal.h"
#include "context.h"

typedef double v4d __attribute__((ext_vector_type(4)));

// A complex zero in device memory for lanes outside the block (their loads
// read it, so every load is issued unconditionally; see zgemm.hip)
__device__ double2 sgn_block_zero_entry;

namespace {

__device__ inline v4d mfma(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Loads through pointers known to address device (global) memory: global
// rather than flat instructions, which would also wait on the LDS counter.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef const d2v __attribute__((address_space(1)))* gptr;
__device__ inline gptr to_global(const double2* p) { return (gptr)p; }
__device__ inline double2 gload(gptr p) {
  const d2v v = *p;
  return make_double2(v.x, v.y);
}

// k-steps whose loads a lane issues together in the block products
constexpr int kUnroll = 8;
// fewest rows per wavefront of the dot pass, and its tiles of 16 columns
// per wavefront (sharing the block-vector loads)
constexpr int kMinRowsPerWave = 128;
constexpr int kDotTiles = 2;
// tiles per wavefront of the three-multiplication dot pass in a launch of
// kWideFrom or more slots (the block-vector loads shared by four tiles);
// launches of fewer slots keep two, for twice the workgroups
constexpr int kDot3Tiles = 4;
constexpr int kDot3TilesSingle = 2;
// slots from which a launch takes the wide tiles (dot) and row blocks (update)
constexpr int kWideFrom = 4;

// the composite basis of one launch: column c < m is S[c], column c >= m of
// slot r is V_r[c - m] (V_r = V + r vstride), all with leading dimension ldq
struct BlockGeo {
  const double2* S;
  const double2* V;
  size_t vstride;
  size_t ldq;
  int m, p, s, N;
  int nb;
  int act[kMaxBatch];
};

// Workgroup i runs on XCD i % 8 (round-robin dispatch).  Map i to (tile b,
// index z within the tile, z < per) so that the workgroups of one tile run on
// one XCD, whose L2 then serves what they share (the rows of the Schur
// columns for every slot, the slot's block vectors for every column group):
// i = 8 (z + per q) + x -> b = 8 q + x.  A grid of 8 per ceil(ntiles / 8)
// workgroups covers every (b, z) once; false for the padding (b >= ntiles).
__device__ inline bool xcd_tile(int i, int per, int ntiles, int& b, int& z) {
  const int x = i & 7, l = i >> 3;
  z = l % per;
  b = (l / per) * 8 + x;
  return b < ntiles;
}
inline unsigned xcd_grid(int per, int ntiles) { return 8u * (unsigned)per * (unsigned)((ntiles + 7) / 8); }

__device__ inline const double2* qcol(const double2* S, const double2* Vr, int m, size_t ldq, int c) {
  return c < m ? S + (size_t)c * ldq : Vr + (size_t)(c - m) * ldq;
}

__device__ inline double2 wsum2(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// v_1 = u * inv per slot: the first Krylov column
__global__ void bstart_kernel(BlockGeo g, const double2* __restrict__ u, size_t ustride,
                              const double* __restrict__ inv, int istride) {
  const int z = blockIdx.y, r = g.act[z];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  double2* v = const_cast<double2*>(g.V) + (size_t)r * g.vstride;
  v[i] = cscale(u[(size_t)r * ustride + i], inv[(size_t)r * istride]);
}

// ---------------------------------------------------------------------------
// The s <= 16 block vectors fill the matrix instruction's 16-wide dimension
// in halves of 8: half h holds vectors 8 h .. 8 h + 7, real parts in rows
// (or columns) 0..7 and imaginary parts in 8..15.  kHalves halves cover
// kBlockMax vectors; a launch uses nh = ceil(s / 8) of them.
constexpr int kHalves = kBlockMax / 8;

// dot pass: partial sums of conj(col_c) . W_v over row chunks.  Columns c < p
// are the basis; with ncol = p + s, columns p + u are W_u (the Gram matrix).
// Wavefront: 32 columns (two tiles of 16 sharing the A fragments) x rpw
// rows; lane (li, lk) = (lane % 16, lane / 16) holds, per k-step of four
// rows, row lk of column li of each tile (B fragment) and, per half, of
// block vector 8 h + li % 8, real part for li < 8, imaginary for li >= 8 (A
// fragment).  D1 = A Re(Q), D2 = A Im(Q) give
//   Re C[j][v] = D1[v][j] + D2[v+8][j],  Im C[j][v] = D1[v+8][j] - D2[v][j].
// Workgroup: four wavefronts on consecutive row ranges, summed in order.
struct BDot {
  const double2* W;  // slot block vectors, ld ldq
  size_t wstride;
  int ncol;
  int rpw;  // rows per wavefront, a multiple of 4
  int ncg;  // column groups
  int nch;  // row chunks
  double2* part;  // per slot [chunk][ncol][kBlockMax]
  size_t pstride;
};

__global__ void __launch_bounds__(256) bdot_kernel(BlockGeo g, BDot a) {
  // tile = row chunk: all slots and column groups of a chunk on one XCD
  int chunk, inner;
  if (!xcd_tile(blockIdx.x, g.nb * a.ncg, a.nch, chunk, inner)) return;
  const int z = inner % g.nb, cg = inner / g.nb;
  const int r = g.act[z];
  const double2* Vr = g.V + (size_t)r * g.vstride;
  const double2* Wr = a.W + (size_t)r * a.wstride;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int v = li & 7;
  const bool imag = li >= 8;
  const int nh = (g.s + 7) >> 3;  // halves in use (uniform)
  const int r0 = (chunk * 4 + wave) * a.rpw;
  const int r1 = min(r0 + a.rpw, g.N);
  const int nit = r1 > r0 ? (r1 - r0) >> 2 : 0;
  // a column past ncol reads column ncol - 1 (its sums are not written)
  const double2* qp[kDotTiles];
#pragma unroll
  for (int t = 0; t < kDotTiles; ++t) {
    const int cc = min((cg * kDotTiles + t) * 16 + li, a.ncol - 1);
    qp[t] = (cc < g.p ? qcol(g.S, Vr, g.m, g.ldq, cc) : Wr + (size_t)(cc - g.p) * g.ldq) + r0 + lk;
  }
  // the A fragments: the lane's real or imaginary part, loaded as one double
  const double* wp[kHalves];
  int dw[kHalves];
#pragma unroll
  for (int h = 0; h < kHalves; ++h) {
    const bool vok = 8 * h + v < g.s;
    wp[h] = vok ? reinterpret_cast<const double*>(Wr + (size_t)(8 * h + v) * g.ldq + r0 + lk) + (imag ? 1 : 0)
                : reinterpret_cast<const double*>(&sgn_block_zero_entry);
    dw[h] = vok ? 8 : 0;  // four rows, in doubles
  }
  v4d d1[kHalves][kDotTiles], d2[kHalves][kDotTiles];
#pragma unroll
  for (int h = 0; h < kHalves; ++h)
#pragma unroll
    for (int t = 0; t < kDotTiles; ++t) {
      d1[h][t] = v4d{0.0, 0.0, 0.0, 0.0};
      d2[h][t] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  constexpr int U = kUnroll / 2;
  int it = 0;
  for (; it + U <= nit; it += U) {
    double2 qv[U][kDotTiles];
    double wv[U][kHalves];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int t = 0; t < kDotTiles; ++t) qv[u][t] = qp[t][4 * u];
#pragma unroll
      for (int h = 0; h < kHalves; ++h) wv[u][h] = wp[h][dw[h] * u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int h = 0; h < kHalves; ++h)
        if (h < nh)
#pragma unroll
          for (int t = 0; t < kDotTiles; ++t) {
            d1[h][t] = mfma(wv[u][h], qv[u][t].x, d1[h][t]);
            d2[h][t] = mfma(wv[u][h], qv[u][t].y, d2[h][t]);
          }
#pragma unroll
    for (int t = 0; t < kDotTiles; ++t) qp[t] += 4 * U;
#pragma unroll
    for (int h = 0; h < kHalves; ++h) wp[h] += U * dw[h];
  }
  for (; it < nit; ++it) {
    double wv[kHalves];
#pragma unroll
    for (int h = 0; h < kHalves; ++h) wv[h] = *wp[h];
#pragma unroll
    for (int t = 0; t < kDotTiles; ++t) {
      const double2 qv = *qp[t];
#pragma unroll
      for (int h = 0; h < kHalves; ++h)
        if (h < nh) {
          d1[h][t] = mfma(wv[h], qv.x, d1[h][t]);
          d2[h][t] = mfma(wv[h], qv.y, d2[h][t]);
        }
      qp[t] += 4;
    }
#pragma unroll
    for (int h = 0; h < kHalves; ++h) wp[h] += dw[h];
  }
  // lane (j = li, lk): items of half h's D hold rows lk + 4 t: vectors
  // 8 h + lk and 8 h + lk + 4
  __shared__ double2 red[4][64][2 * kDotTiles * kHalves];
  double2 cs[kDotTiles][kHalves][2];
#pragma unroll
  for (int t = 0; t < kDotTiles; ++t)
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      cs[t][h][0] = make_double2(d1[h][t][0] + d2[h][t][2], d1[h][t][2] - d2[h][t][0]);
      cs[t][h][1] = make_double2(d1[h][t][1] + d2[h][t][3], d1[h][t][3] - d2[h][t][1]);
      red[wave][lane][(t * kHalves + h) * 2] = cs[t][h][0];
      red[wave][lane][(t * kHalves + h) * 2 + 1] = cs[t][h][1];
    }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int t = 0; t < kDotTiles; ++t) {
    const int c = (cg * kDotTiles + t) * 16 + li;
    if (c >= a.ncol) continue;
    double2* o = a.part + (size_t)r * a.pstride + ((size_t)chunk * a.ncol + c) * kBlockMax;
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      double2 c0 = cs[t][h][0], c1 = cs[t][h][1];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        c0 = cadd(c0, red[w][lane][(t * kHalves + h) * 2]);
        c1 = cadd(c1, red[w][lane][(t * kHalves + h) * 2 + 1]);
      }
      // vectors past s have zero fragments, so their sums are zero
      o[8 * h + lk] = c0;
      o[8 * h + lk + 4] = c1;
    }
  }
}

// The dot pass for s > 8 with three real products per fragment (the
// Gauss form of the complex product): lane (li, lk) holds row lk of block
// vector li (A fragment, both parts) and of column li of each tile (B
// fragment);
//   T1 = Wr^T Re(Q),  T2 = Wi^T Im(Q),  T3 = (Wr + Wi)^T (Re(Q) - Im(Q)),
//   Re C = T1 + T2,  Im C = T3 - T1 + T2,
// a quarter fewer matrix-core instructions than two halves of 8.
template <int T>
__global__ void __launch_bounds__(256) bdot3_kernel(BlockGeo g, BDot a) {
  int chunk, inner;
  if (!xcd_tile(blockIdx.x, g.nb * a.ncg, a.nch, chunk, inner)) return;
  const int z = inner % g.nb, cg = inner / g.nb;
  const int r = g.act[z];
  const double2* Vr = g.V + (size_t)r * g.vstride;
  const double2* Wr = a.W + (size_t)r * a.wstride;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = (chunk * 4 + wave) * a.rpw;
  const int r1 = min(r0 + a.rpw, g.N);
  const int nit = r1 > r0 ? (r1 - r0) >> 2 : 0;
  gptr qp[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int cc = min((cg * T + t) * 16 + li, a.ncol - 1);
    qp[t] = to_global((cc < g.p ? qcol(g.S, Vr, g.m, g.ldq, cc) : Wr + (size_t)(cc - g.p) * g.ldq) + r0 + lk);
  }
  const bool vok = li < g.s;
  gptr wp = to_global(vok ? Wr + (size_t)li * g.ldq + r0 + lk : &sgn_block_zero_entry);
  const int dw = vok ? 4 : 0;
  v4d t1[T], t2[T], t3[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    t1[t] = v4d{0.0, 0.0, 0.0, 0.0};
    t2[t] = v4d{0.0, 0.0, 0.0, 0.0};
    t3[t] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // groups of U k-steps, the loads of the next group issued before the
  // products of the current one (two register sets)
  constexpr int U = kUnroll / 4;
  auto load = [&](double2 (&qv)[U][T], double2 (&wv)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int t = 0; t < T; ++t) qv[u][t] = gload(qp[t] + 4 * u);
      wv[u] = gload(wp + dw * u);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) qp[t] += 4 * U;
    wp += U * dw;
  };
  auto mul = [&](const double2 (&qv)[U][T], const double2 (&wv)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double ws = wv[u].x + wv[u].y;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        t1[t] = mfma(wv[u].x, qv[u][t].x, t1[t]);
        t2[t] = mfma(wv[u].y, qv[u][t].y, t2[t]);
        t3[t] = mfma(ws, qv[u][t].x - qv[u][t].y, t3[t]);
      }
    }
  };
  int it = 0;
  {
    double2 qa[U][T], wa[U], qb[U][T], wb[U];
    if (nit >= U) load(qa, wa);
    for (; it + 2 * U <= nit; it += 2 * U) {
      load(qb, wb);
      mul(qa, wa);
      if (it + 3 * U <= nit) load(qa, wa);
      mul(qb, wb);
    }
    if (it + U <= nit) {
      mul(qa, wa);
      it += U;
    }
  }
  for (; it < nit; ++it) {
    const double2 wv = gload(wp);
    const double ws = wv.x + wv.y;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const double2 qv = gload(qp[t]);
      t1[t] = mfma(wv.x, qv.x, t1[t]);
      t2[t] = mfma(wv.y, qv.y, t2[t]);
      t3[t] = mfma(ws, qv.x - qv.y, t3[t]);
      qp[t] += 4;
    }
    wp += dw;
  }
  // lane (j = li, lk): item q holds vector lk + 4 q of column j
  __shared__ double2 red[4][64][4 * T];
  double2 cs[T][4];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cs[t][q] = make_double2(t1[t][q] + t2[t][q], t3[t][q] - t1[t][q] + t2[t][q]);
      red[wave][lane][4 * t + q] = cs[t][q];
    }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int c = (cg * T + t) * 16 + li;
    if (c >= a.ncol) continue;
    double2* o = a.part + (size_t)r * a.pstride + ((size_t)chunk * a.ncol + c) * kBlockMax;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double2 acc = cs[t][q];
#pragma unroll
      for (int w = 1; w < 4; ++w) acc = cadd(acc, red[w][lane][4 * t + q]);
      o[lk + 4 * q] = acc;  // zero for vectors past s
    }
  }
}

// sum of the dot partials over chunks in a fixed order: 32 entries per
// workgroup, 8 threads per entry (every 8th chunk), then the 8 in order.
// Entry e = c * kBlockMax + v; c < p goes to C[c][v] (and C1[c][v] + C[c][v]
// to Ct[c][v] if Ct), c >= p to G[c - p][v].
struct BRed {
  const double2* part;
  size_t pstride;
  int nchunk, nent, nblk;
  double2* C;
  const double2* C1;
  double2* Ct;
  size_t cstride;
  double2* G;
  size_t gstride;
};

__global__ void __launch_bounds__(256) bred_kernel(BlockGeo g, BRed a) {
  const int z = blockIdx.x % g.nb, blk = blockIdx.x / g.nb;
  const int r = g.act[z];
  const double2* __restrict__ part = a.part + (size_t)r * a.pstride;
  const int el = threadIdx.x & 31, q = threadIdx.x >> 5;
  const int e = blk * 32 + el;
  const int nchunk = a.nchunk, nent = a.nent;
  double2 acc = make_double2(0.0, 0.0);
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
  __shared__ double2 rs[8][33];
  rs[q][el] = acc;
  __syncthreads();
  if (q == 0 && e < nent) {
    double2 t = rs[0][el];
    for (int w = 1; w < 8; ++w) t = cadd(t, rs[w][el]);
    const int c = e / kBlockMax;
    const size_t co = (size_t)r * a.cstride;
    if (c < g.p) {
      a.C[co + e] = t;
      if (a.Ct) a.Ct[co + e] = cadd(a.C1[co + e], t);
    } else {
      a.G[(size_t)r * a.gstride + e - g.p * kBlockMax] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Q C on the matrix cores: 16 rows of the composite basis (S, Vr; ld ldq)
// times the coefficients C[c][v] of columns c < ncol, for the k-steps (four
// columns) k0, k0 + dk, ... .  Lane (li, lk) holds row li of column
// 4 ks + lk (A fragment) and that column's coefficient for block vector
// 8 h + li % 8 of each half h (B fragments), so that
//   D[h] += Re(Q) [Re C | Im C] + Im(Q) [-Im C | Re C]
// is [Re | Im] of (Q C) for the 16 rows and half h's 8 vectors (rows lk + 4 t
// in item t, vector 8 h + li % 8, real part for li < 8).  Columns past ncol
// read the zero entry; halves h >= nh are skipped.
__device__ inline void qc_steps(const double2* __restrict__ S, const double2* __restrict__ Vr, int m, size_t ldq,
                                int row, int ncol, const double2* __restrict__ C, int v, bool imag, int s, int lk,
                                int k0, int dk, v4d (&d)[kHalves]) {
  const double2* zero = &sgn_block_zero_entry;
  const int nk = (ncol + 3) >> 2;
  const int nh = (s + 7) >> 3;
  bool vok[kHalves];
#pragma unroll
  for (int h = 0; h < kHalves; ++h) vok[h] = 8 * h + v < s;
  int ks = k0;
  constexpr int U = kUnroll / kHalves;
  for (; ks + (U - 1) * dk < nk; ks += U * dk) {
    double2 qv[U], cv[U][kHalves];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int col = 4 * (ks + u * dk) + lk;
      const bool ok = col < ncol;
      qv[u] = *(ok ? qcol(S, Vr, m, ldq, col) + row : zero);
#pragma unroll
      for (int h = 0; h < kHalves; ++h)
        cv[u][h] = *((ok & vok[h]) ? C + (size_t)col * kBlockMax + 8 * h + v : zero);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int h = 0; h < kHalves; ++h)
        if (h < nh) {
          const double b1 = imag ? cv[u][h].y : cv[u][h].x;
          const double b2 = imag ? cv[u][h].x : -cv[u][h].y;
          d[h] = mfma(qv[u].x, b1, d[h]);
          d[h] = mfma(qv[u].y, b2, d[h]);
        }
  }
  for (; ks < nk; ks += dk) {
    const int col = 4 * ks + lk;
    const bool ok = col < ncol;
    const double2 qv = *(ok ? qcol(S, Vr, m, ldq, col) + row : zero);
#pragma unroll
    for (int h = 0; h < kHalves; ++h)
      if (h < nh) {
        const double2 cv = *((ok & vok[h]) ? C + (size_t)col * kBlockMax + 8 * h + v : zero);
        const double b1 = imag ? cv.y : cv.x;
        const double b2 = imag ? cv.x : -cv.y;
        d[h] = mfma(qv.x, b1, d[h]);
        d[h] = mfma(qv.y, b2, d[h]);
      }
  }
}

// Q C for s > 8 with three real products per fragment (the Gauss form):
// lane (li, lk) holds row li of column 4 ks + lk (A fragment) and that
// column's coefficient for block vector li (B fragment);
//   T1 = Re(Q) Re(C),  T2 = Im(Q) Im(C),  T3 = (Re Q + Im Q)(Re C + Im C),
//   Re(Q C) = T1 - T2,  Im(Q C) = T3 - T1 - T2
// for the 16 rows (rows lk + 4 t in item t) and vector li.  RB blocks of 16
// rows (rows[b]: this lane's row of block b) share each coefficient load.
template <int RB>
__device__ inline void qc_steps3(const double2* __restrict__ S, const double2* __restrict__ Vr, int m, size_t ldq,
                                 const int (&rows)[RB], int ncol, const double2* __restrict__ C, int s, int li,
                                 int lk, int k0, int dk, v4d (&t1)[RB], v4d (&t2)[RB], v4d (&t3)[RB]) {
  const gptr zero = to_global(&sgn_block_zero_entry);
  const int nk = (ncol + 3) >> 2;
  const bool vok = li < s;
  int ks = k0;
  constexpr int U = kUnroll / (2 * RB);
  for (; ks + (U - 1) * dk < nk; ks += U * dk) {
    double2 qv[U][RB], cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int col = 4 * (ks + u * dk) + lk;
      const bool ok = col < ncol;
      const double2* qc = qcol(S, Vr, m, ldq, col);
#pragma unroll
      for (int b = 0; b < RB; ++b) qv[u][b] = gload(ok ? to_global(qc + rows[b]) : zero);
      cv[u] = gload((ok & vok) ? to_global(C + (size_t)col * kBlockMax + li) : zero);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double cs = cv[u].x + cv[u].y;
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        t1[b] = mfma(qv[u][b].x, cv[u].x, t1[b]);
        t2[b] = mfma(qv[u][b].y, cv[u].y, t2[b]);
        t3[b] = mfma(qv[u][b].x + qv[u][b].y, cs, t3[b]);
      }
    }
  }
  for (; ks < nk; ks += dk) {
    const int col = 4 * ks + lk;
    const bool ok = col < ncol;
    const double2* qc = qcol(S, Vr, m, ldq, col);
    const double2 cv = gload((ok & vok) ? to_global(C + (size_t)col * kBlockMax + li) : zero);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const double2 qv = gload(ok ? to_global(qc + rows[b]) : zero);
      t1[b] = mfma(qv.x, cv.x, t1[b]);
      t2[b] = mfma(qv.y, cv.y, t2[b]);
      t3[b] = mfma(qv.x + qv.y, cv.x + cv.y, t3[b]);
    }
  }
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
// R[r-p][i-1] (r >= p, upper triangular).  Per slot: Ct, P at cstride (P
// laid out [v][r] with ld ldp), R and Rbi at rstride, H at hstride.
struct BHess {
  double e;
  const double2* Ct;
  const double2* P;
  size_t cstride;
  int ldp;
  const double2* R;
  const double2* Rbi;
  size_t rstride;
  double2* H;
  size_t hstride;
  int ldh;
};

__device__ void hess_entry(const BlockGeo& g, const BHess& h, int r_slot, int idx) {
  const int r = idx / kBlockMax, j = idx % kBlockMax;
  const int p = g.p;
  if (r >= p + g.s || j >= g.s) return;
  const double2* Ct = h.Ct + (size_t)r_slot * h.cstride;
  const double2* P = h.P + (size_t)r_slot * h.cstride;
  const double2* R = h.R + (size_t)r_slot * h.rstride;
  const double2* Rbi = h.Rbi + (size_t)r_slot * h.rstride;
  auto rc = [&](int i) -> double2 {
    if (i == 0) return make_double2(r == p - 1 ? 1.0 : 0.0, 0.0);
    if (r < p) return Ct[(size_t)r * kBlockMax + i - 1];
    const int rr = r - p;
    return rr <= i - 1 ? R[rr * kBlockMax + i - 1] : make_double2(0.0, 0.0);
  };
  double2 acc = make_double2(0.0, 0.0);
  for (int i = 0; i <= j; ++i) {
    double2 mi;
    if (i == 0) {
      mi = cscale(rc(1), h.e);
    } else {
      mi = cscale(cadd(rc(i - 1), rc(i + 1)), 0.5 * h.e);
      if (r < p) mi = csub(mi, P[(size_t)(i - 1) * h.ldp + r]);
    }
    acc = cfma(mi, Rbi[i * kBlockMax + j], acc);
  }
  // column p-1+j has its subdiagonal in row p+j; below it H is zero
  h.H[(size_t)r_slot * h.hstride + (size_t)(p - 1 + j) * h.ldh + r] = (r <= p + j) ? acc : make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------------------
// update pass: Wout = (Win - Q C) [Rinv].  Wavefront: 16 rows x all p
// columns.  With Rinv (the second pass) the workgroups past the rows also
// write the block's Hessenberg columns (hess).  Tile = row block; the slots
// of a row block run on one XCD.
struct BUpd {
  const double2* C;
  size_t cstride;
  const double2* Win;
  size_t winstride;
  double2* Wout;
  size_t woutstride;
  const double2* Rinv;  // per slot [kBlockMax][kBlockMax] upper triangular at rstride, or null
  size_t rstride;
  int nrowblk;  // workgroups on rows
  int nhess;    // workgroups on the Hessenberg columns (with Rinv)
  BHess hess;
};

template <bool G, int RB>
__global__ void __launch_bounds__(256) bupdate_kernel(BlockGeo g, BUpd a) {
  // RB blocks of 16 rows per wavefront, sharing each coefficient load (the
  // three-multiplication form only; the packed form takes one)
  static_assert(G || RB == 1, "row blocks need the three-multiplication form");
  int z, bid;
  if (!xcd_tile(blockIdx.x, g.nb, a.nrowblk + a.nhess, bid, z)) return;
  const int rs = g.act[z];
  if (bid >= a.nrowblk) {
    hess_entry(g, a.hess, rs, (bid - a.nrowblk) * 256 + threadIdx.x);
    return;
  }
  const double2* Vr = g.V + (size_t)rs * g.vstride;
  const double2* Cr = a.C + (size_t)rs * a.cstride;
  const double2* Win = a.Win + (size_t)rs * a.winstride;
  double2* Wout = a.Wout + (size_t)rs * a.woutstride;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = (bid * 4 + wave) * 16 * RB;
  const bool active = r0 < g.N;  // wavefront-uniform
  const int v = li & 7;
  // res[b][h][t]: (Q C)[row r0 + 16 b + lk + 4 t][vector vec(h)] in the lanes
  // that own one
  double2 res[RB][kHalves][4];
  bool own[kHalves];
  int vec[kHalves];
  if constexpr (G) {
    v4d t1[RB], t2[RB], t3[RB];
    int rows[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      t1[b] = v4d{0.0, 0.0, 0.0, 0.0};
      t2[b] = t1[b];
      t3[b] = t1[b];
      rows[b] = min(r0 + 16 * b + li, g.N - 1);
    }
    if (active) qc_steps3<RB>(g.S, Vr, g.m, g.ldq, rows, g.p, Cr, g.s, li, lk, 0, 1, t1, t2, t3);
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        res[b][0][t] = make_double2(t1[b][t] - t2[b][t], t3[b][t] - t1[b][t] - t2[b][t]);
    own[0] = li < g.s;
    vec[0] = li;
#pragma unroll
    for (int h = 1; h < kHalves; ++h) own[h] = false;
  } else {
    const int row = min(r0 + li, g.N - 1);
    v4d d[kHalves];
#pragma unroll
    for (int h = 0; h < kHalves; ++h) d[h] = v4d{0.0, 0.0, 0.0, 0.0};
    if (active) qc_steps(g.S, Vr, g.m, g.ldq, row, g.p, Cr, v, li >= 8, g.s, lk, 0, 1, d);
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      qc_pairs(d[h], res[0][h]);
      vec[h] = 8 * h + v;
      own[h] = li < 8 && vec[h] < g.s;
    }
  }
  if (!a.Rinv) {
    if (active)
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int h = 0; h < kHalves; ++h) {
          if (!own[h]) continue;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int rr = r0 + 16 * b + lk + 4 * t;
            if (rr < g.N) {
              const size_t o = (size_t)vec[h] * g.ldq + rr;
              Wout[o] = csub(Win[o], res[b][h][t]);
            }
          }
        }
    return;
  }
  // second pass: W'' = Win - Q C, then W'' Rinv per row (through LDS; the
  // workgroup's slot is the same for all four wavefronts)
  __shared__ double2 tile[4][16 * RB][kBlockMax];
  __shared__ double2 ri[kBlockMax * kBlockMax];
  {
    const double2* Ri = a.Rinv + (size_t)rs * a.rstride;
    for (int e = threadIdx.x; e < kBlockMax * kBlockMax; e += 256) ri[e] = Ri[e];
  }
  // every (row, vector) of the tile: vectors past s and rows past N as zero
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      const bool writer = G ? h == 0 : li < 8;
      if (!writer) continue;
      const int vv = G ? li : 8 * h + v;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int rl = 16 * b + lk + 4 * t, rr = r0 + rl;
        double2 val = make_double2(0.0, 0.0);
        if (active && own[h] && rr < g.N) val = csub(Win[(size_t)vv * g.ldq + rr], res[b][h][t]);
        tile[wave][rl][vv] = val;
      }
    }
  __syncthreads();
  if (!active) return;
  constexpr int kOut = 16 * RB * kBlockMax / 64;  // outputs per lane
  // (not unrolled: this epilogue would otherwise set the kernel's register
  // count, and with it the occupancy of the sweep above)
#pragma unroll 1
  for (int q = 0; q < kOut; ++q) {
    const int idx = lane + 64 * q;
    const int rl = idx / kBlockMax, vv = idx % kBlockMax;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
    for (int u = 0; u < kBlockMax; ++u) acc = cfma(tile[wave][rl][u], ri[u * kBlockMax + vv], acc);
    const int rr = r0 + rl;
    if (vv < g.s && rr < g.N) Wout[(size_t)vv * g.ldq + rr] = acc;
  }
}

// ---------------------------------------------------------------------------
// Between the two passes' reductions and the second update: per slot, one
// workgroup factors the block, G'' = G - C2^dag C2 = R^dag R (R upper), and
// forms R^-1 and Rb^-1 (Rb = [1, Ct[p-1][0 .. s-2]; 0, R[0 .. s-2][0 .. s-2]]);
// it raises the slot's flag when the block is not numerically of full rank
// (a pivot below 1e-12 of the block's size, or below 1e-7 of the largest
// pivot) or not finite.  C2^dag C2 and the diagonal of Ct^dag Ct (the block
// vectors' size before projection) run on the matrix cores, the four
// wavefronts taking every fourth k-step.  The other workgroups form
// P = H_{p x (p-1)} Ct for 16 rows each (the four wavefronts take every
// fourth k-step, summed in order), from the first column where a row of the
// tile can be nonzero (H is upper Hessenberg below the T block, T upper
// triangular).  Workgroup id = z + nb t: t = 0 factors, t >= 1 is row tile
// t - 1.
struct BSmall {
  const double2* C2;
  const double2* Ct;
  size_t cstride;
  const double2* G;
  size_t gstride;
  const double2* H;
  size_t hstride;
  int ldh;
  double2* P;  // [v][r], ld ldp
  int ldp;
  double2* R;  // per slot: R, R^-1, Rb^-1 (kBlockMax^2 each) at rstride
  size_t rstride;
  int* flag;
};

__device__ void block_factor(const BlockGeo& gg, const BSmall& a, int rs) {
  constexpr int B = kBlockMax;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int s = gg.s, p = gg.p;
  const double2* C2 = a.C2 + (size_t)rs * a.cstride;
  const double2* Ct = a.Ct + (size_t)rs * a.cstride;
  const double2* G = a.G + (size_t)rs * a.gstride;
  double2* Rout = a.R + (size_t)rs * a.rstride;
  __shared__ v4d red[4][4][64];
  __shared__ double redn[4][64];
  __shared__ double2 g[B][B], R[B][B], Ri[B][B], Rb[B][B], Rbi[B][B];
  __shared__ double piv[B], ref_s;
  __shared__ int bad;
  // C2^dag C2 (16 x 16 complex) on the matrix cores: A = C2^dag (row u, k = c),
  // B = C2 (k = c, column v); lane (li, lk) loads C2[c][li] for c = 4 ks + lk.
  // Re += Re A Re B + Im A Im B... with A = conj(C2)^T:
  //   Re(conj(a) b) = ar br + ai bi,  Im(conj(a) b) = ar bi - ai br
  {
    const int li = lane & 15, lk = lane >> 4;
    v4d dre = {0.0, 0.0, 0.0, 0.0}, dim = {0.0, 0.0, 0.0, 0.0};
    double nn = 0.0;
    const double2* zero = &sgn_block_zero_entry;
    const int nk = (p + 3) >> 2;
    // the loads of kUnroll k-steps first (one wait per group, not per step)
    int ks = wave;
    for (; ks + 4 * (kUnroll - 1) < nk; ks += 4 * kUnroll) {
      double2 x[kUnroll], y[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int c = 4 * (ks + 4 * u) + lk;
        const bool ok = c < p && li < s;
        x[u] = *(ok ? C2 + (size_t)c * B + li : zero);
        y[u] = *(ok ? Ct + (size_t)c * B + li : zero);
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        dre = mfma(x[u].x, x[u].x, dre);
        dre = mfma(x[u].y, x[u].y, dre);
        dim = mfma(x[u].x, x[u].y, dim);
        dim = mfma(-x[u].y, x[u].x, dim);
        nn += cabs2(y[u]);
      }
    }
    for (; ks < nk; ks += 4) {
      const int c = 4 * ks + lk;
      const bool ok = c < p && li < s;
      const double2 x = *(ok ? C2 + (size_t)c * B + li : zero);
      const double2 y = *(ok ? Ct + (size_t)c * B + li : zero);
      dre = mfma(x.x, x.x, dre);
      dre = mfma(x.y, x.y, dre);
      dim = mfma(x.x, x.y, dim);
      dim = mfma(-x.y, x.x, dim);
      nn += cabs2(y);
    }
    red[wave][0][lane] = dre;
    red[wave][1][lane] = dim;
    redn[wave][lane] = nn;
  }
  if (tid < B * B) {
    const int u = tid / B, v = tid % B;
    R[u][v] = make_double2(0.0, 0.0);
    Ri[u][v] = make_double2(0.0, 0.0);
    Rb[u][v] = make_double2(0.0, 0.0);
    Rbi[u][v] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (tid < 64) {
    // D[u][v] sits in lane v + 16 (u % 4), item u / 4
    const int v = tid & 15, u0 = tid >> 4;
    v4d sre = red[0][0][tid], sim = red[0][1][tid];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      sre += red[w][0][tid];
      sim += red[w][1][tid];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int u = u0 + 4 * t;
      g[u][v] = (u < s && v < s) ? csub(G[u * B + v], make_double2(sre[t], sim[t])) : make_double2(0.0, 0.0);
    }
  }
  if (tid == 0) {
    bad = 0;
    // |Ct[:, v]|^2 summed over the lanes holding v (li = v) and the wavefronts
    double rf = 0.0;
    for (int v = 0; v < s; ++v) {
      double t = 0.0;
      for (int w = 0; w < 4; ++w)
        for (int q = 0; q < 4; ++q) t += redn[w][v + 16 * q];
      rf = fmax(rf, G[v * B + v].x + t);
    }
    ref_s = rf;
  }
  __syncthreads();
  // right-looking Cholesky: step j forms row j of R and updates the trailing
  // block.  Every thread takes the pivot from g[j][j] itself and row j of R
  // from row j of g (which step j leaves alone), so a step needs one barrier.
  for (int j = 0; j < s; ++j) {
    double dj = g[j][j].x;
    const bool okp = dj > 0.0 && isfinite(dj);
    if (!okp) dj = 1.0;
    const double pj = sqrt(dj), ip = 1.0 / pj;
    if (tid == 0) {
      piv[j] = pj;
      if (!okp) bad = 1;
    }
    if (tid < B && tid >= j && tid < s) R[j][tid] = tid == j ? make_double2(pj, 0.0) : cscale(g[j][tid], ip);
    if (tid < B * B) {
      const int u = tid / B, v = tid % B;
      if (u > j && v > j && u < s && v < s) g[u][v] = csub(g[u][v], cmulc(cscale(g[j][u], ip), cscale(g[j][v], ip)));
    }
    __syncthreads();
  }
  // Rb from R and the last basis column's coefficients
  if (tid < B * B) {
    const int u = tid / B, v = tid % B;
    if (u < s && v < s) {
      if (u == 0)
        Rb[0][v] = v == 0 ? make_double2(1.0, 0.0) : Ct[(size_t)(p - 1) * B + v - 1];
      else if (v >= u)
        Rb[u][v] = R[u - 1][v - 1];
    }
  }
  __syncthreads();
  // inverses of the two upper triangular factors, one column per thread
  if (tid < 2 * B) {
    const int col = tid % B;
    const bool second = tid >= B;
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
  if (tid < B * B) {
    const int u = tid / B, v = tid % B;
    Rout[tid] = R[u][v];
    Rout[B * B + tid] = Ri[u][v];
    Rout[2 * B * B + tid] = Rbi[u][v];
  }
  if (tid == 0) {
    double dmin = HUGE_VAL, dmax = 0.0;
    for (int j = 0; j < s; ++j) {
      dmin = fmin(dmin, piv[j]);
      dmax = fmax(dmax, piv[j]);
    }
    const double rf = ref_s;
    if (bad || !(rf > 0.0) || !isfinite(rf) || dmin * dmin < 1e-24 * rf || dmin < 1e-7 * dmax) a.flag[rs] = 1;
  }
}

template <bool G>
__global__ void __launch_bounds__(256) bsmall_kernel(BlockGeo g, BSmall a) {
  const int z = blockIdx.x % g.nb, t = blockIdx.x / g.nb;
  const int rs = g.act[z];
  if (t == 0) {
    block_factor(g, a, rs);
    return;
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int p = g.p;
  const int r0 = (t - 1) * 16;
  const int row = min(r0 + li, p - 1);
  const int v = li & 7;
  const int c0 = r0 < g.m ? r0 : max(g.m, r0 - 1);  // columns below c0 are zero in these rows
  const double2* H = a.H + (size_t)rs * a.hstride;
  const double2* Ct = a.Ct + (size_t)rs * a.cstride;
  double2* P = a.P + (size_t)rs * a.cstride;
  // only the columns 0 .. s-2 of Ct enter P
  if constexpr (G) {
    v4d t1[1] = {v4d{0.0, 0.0, 0.0, 0.0}}, t2[1] = {t1[0]}, t3[1] = {t1[0]};
    const int rows[1] = {row};
    qc_steps3<1>(H, H, 0, (size_t)a.ldh, rows, p - 1, Ct, g.s - 1, li, lk, (c0 >> 2) + wave, 4, t1, t2, t3);
    __shared__ v4d red3[4][3][64];
    red3[wave][0][lane] = t1[0];
    red3[wave][1][lane] = t2[0];
    red3[wave][2][lane] = t3[0];
    __syncthreads();
    if (wave != 0) return;
    v4d u1 = t1[0], u2 = t2[0], u3 = t3[0];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      u1 += red3[w][0][lane];
      u2 += red3[w][1][lane];
      u3 += red3[w][2][lane];
    }
    if (li < g.s - 1)
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const int rr = r0 + lk + 4 * tt;
        if (rr < p) P[(size_t)li * a.ldp + rr] = make_double2(u1[tt] - u2[tt], u3[tt] - u1[tt] - u2[tt]);
      }
  } else {
    v4d d[kHalves];
#pragma unroll
    for (int h = 0; h < kHalves; ++h) d[h] = v4d{0.0, 0.0, 0.0, 0.0};
    qc_steps(H, H, 0, (size_t)a.ldh, row, p - 1, Ct, v, li >= 8, g.s - 1, lk, (c0 >> 2) + wave, 4, d);
    __shared__ v4d red[4][kHalves][64];
#pragma unroll
    for (int h = 0; h < kHalves; ++h) red[wave][h][lane] = d[h];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int h = 0; h < kHalves; ++h) {
      v4d dh = red[0][h][lane];
#pragma unroll
      for (int w = 1; w < 4; ++w) dh += red[w][h][lane];
      double2 res[4];
      qc_pairs(dh, res);
      if (li < 8 && 8 * h + v < g.s - 1)
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const int rr = r0 + lk + 4 * tt;
          if (rr < p) P[(size_t)(8 * h + v) * a.ldp + rr] = res[tt];
        }
    }
  }
}

int nchunks_for(int N, int& rpw) {
  // rows per wavefront: kMinRowsPerWave or more, so that at most 128 chunks
  // of four wavefronts cover N
  const int want = (N + 4 * 128 - 1) / (4 * 128);
  rpw = std::max(kMinRowsPerWave, (want + 3) & ~3);
  return (N + 4 * rpw - 1) / (4 * rpw);
}

BlockGeo make_geo(const BlockSpan& sp) {
  BlockGeo g;
  g.S = sp.S;
  g.V = sp.V;
  g.vstride = sp.vstride;
  g.ldq = sp.ldq;
  g.m = sp.m;
  g.p = 0;
  g.s = 0;
  g.N = sp.N;
  g.nb = sp.nb;
  for (int z = 0; z < sp.nb; ++z) g.act[z] = sp.act[z];
  return g;
}

}  // namespace

void block_alloc(BlockWork& b, int N, size_t ldq, int ncap, int nslots) {
  block_free(b);
  int rpw = 0;
  const int nch = nchunks_for(N, rpw);
  const size_t S = (size_t)nslots;
  b.nslots = nslots;
  b.wstride = ldq * kBlockMax;
  b.pstride = (size_t)nch * (ncap + kBlockMax) * kBlockMax;
  b.cstride = (size_t)ncap * kBlockMax;
  b.gstride = kBlockMax * kBlockMax;
  b.rstride = 3 * kBlockMax * kBlockMax;
  SGN_HIP(hipMalloc(&b.W, sizeof(double2) * b.wstride * S));
  SGN_HIP(hipMalloc(&b.part, sizeof(double2) * b.pstride * S));
  SGN_HIP(hipMalloc(&b.C1, sizeof(double2) * b.cstride * S));
  SGN_HIP(hipMalloc(&b.C2, sizeof(double2) * b.cstride * S));
  SGN_HIP(hipMalloc(&b.Ct, sizeof(double2) * b.cstride * S));
  SGN_HIP(hipMalloc(&b.P, sizeof(double2) * b.cstride * S));
  SGN_HIP(hipMalloc(&b.G, sizeof(double2) * b.gstride * S));
  SGN_HIP(hipMalloc(&b.R, sizeof(double2) * b.rstride * S));
  SGN_HIP(hipMalloc(&b.flag, sizeof(int) * S));
  b.ncap = ncap;
}

void block_free(BlockWork& b) {
  for (double2** p : {&b.W, &b.part, &b.C1, &b.C2, &b.Ct, &b.P, &b.G, &b.R})
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  if (b.flag) (void)hipFree(b.flag);
  b.flag = nullptr;
  b.ncap = 0;
  b.nslots = 0;
}

void block_first(const BlockSpan& sp, const double2* u, size_t ustride, const double* inv, int istride,
                 hipStream_t s) {
  BlockGeo g = make_geo(sp);
  hipLaunchKernelGGL(bstart_kernel, dim3((sp.N + 255) / 256, sp.nb), dim3(256), 0, s, g, u, ustride, inv, istride);
  SGN_HIP(hipGetLastError());
}

void block_step(const BlockSpan& sp, BlockWork& b, const Lattice& lat, const double2* links, int k, int sb, double e,
                hipStream_t s, Profiler* prof) {
  const int m = sp.m, N = sp.N, p = m + 1 + k, nb = sp.nb;
  const size_t ldq = sp.ldq;
  SGN_REQUIRE(sb >= 1 && sb <= kBlockMax && p + sb <= sp.ncap && b.ncap >= sp.ncap && nb >= 1 && nb <= kMaxBatch &&
                  nb <= b.nslots,
              SGN_EINVAL, "block step exceeds the workspace");
  BlockGeo g = make_geo(sp);
  g.p = p;
  g.s = sb;
  // the newest basis column q_{p-1} = V_r[p-1-m]
  const double2* w0 = sp.V + (size_t)(p - 1 - m) * ldq;
  // Krylov directions: W_1 = A W_0 / e, W_{i+1} = 2 A W_i / e - W_{i-1}
  SlotMap map;
  map.n = nb;
  for (int z = 0; z < nb; ++z) map.slot[z] = sp.act[z];
  wilson_apply_cheb_slots(lat, links, w0, sp.vstride, b.W, b.wstride, nullptr, 0, 1.0 / e, 0.0, map, s, prof);
  for (int i = 1; i < sb; ++i)
    wilson_apply_cheb_slots(lat, links, b.W + (size_t)(i - 1) * ldq, b.wstride, b.W + (size_t)i * ldq, b.wstride,
                            i == 1 ? w0 : b.W + (size_t)(i - 2) * ldq, i == 1 ? sp.vstride : b.wstride, 2.0 / e,
                            -1.0, map, s, prof);
  int rpw = 0;
  const int nch = nchunks_for(N, rpw);
  // more than 8 block vectors: the products in their three-multiplication form
  const bool gauss = sb > 8;
  // launches of several slots: four column tiles per dot wavefront and two
  // blocks of 16 rows per update wavefront (three-multiplication form); the
  // arithmetic of every entry is the same either way
  const bool wide = gauss && nb >= kWideFrom;
  const int tiles = !gauss ? kDotTiles : wide ? kDot3Tiles : kDot3TilesSingle;
  void (*dot_kernel)(BlockGeo, BDot) =
      !gauss ? bdot_kernel : wide ? bdot3_kernel<kDot3Tiles> : bdot3_kernel<kDot3TilesSingle>;
  const int rb = wide ? 2 : 1;
  void (*upd_kernel)(BlockGeo, BUpd) =
      !gauss ? bupdate_kernel<false, 1> : wide ? bupdate_kernel<true, 2> : bupdate_kernel<true, 1>;
  auto dot = [&](double2* C, int ncol, const double2* C1, double2* Ct) {
    const int ncg = (ncol + 16 * tiles - 1) / (16 * tiles);
    BDot d{b.W, b.wstride, ncol, rpw, ncg, nch, b.part, b.pstride};
    // the basis read once (S once for the launch, the slots' own columns and
    // W as columns per slot), W once per slot, partials written
    const double bytes =
        16.0 * N * ((double)m + (double)nb * (ncol - m + sb)) + 16.0 * nch * ncol * kBlockMax * (double)nb;
    prof_launch(prof, K_BDOT, bytes, 8.0 * N * ncol * sb * nb, dot_kernel, dim3(xcd_grid(nb * ncg, nch)), dim3(256),
                0, s, g, d);
    const int nent = ncol * kBlockMax, nblk = (nent + 31) / 32;
    BRed rd{b.part, b.pstride, nch, nent, nblk, C, C1, Ct, b.cstride, b.G, b.gstride};
    prof_launch(prof, K_BRED, (16.0 * (double)nch * nent + 16.0 * nent) * nb, 2.0 * nch * nent * nb, bred_kernel,
                dim3(nblk * nb), dim3(256), 0, s, g, rd);
  };
  const int nrowblk = (N + 64 * rb - 1) / (64 * rb);
  // the basis (S once for the launch), W read and written, the coefficients
  const double upd_bytes = 16.0 * N * ((double)m + (double)nb * (p - m + 2.0 * sb)) + 16.0 * p * sb * (double)nb;
  // pass 1
  dot(b.C1, p, nullptr, nullptr);
  {
    BUpd u{b.C1, b.cstride, b.W, b.wstride, b.W, b.wstride, nullptr, 0, nrowblk, 0, BHess{}};
    prof_launch(prof, K_BUPDATE, upd_bytes, 8.0 * N * p * sb * nb, upd_kernel, dim3(xcd_grid(nb, nrowblk)), dim3(256),
                0, s, g, u);
  }
  // pass 2 with the Gram matrix of the projected block
  dot(b.C2, p + sb, b.C1, b.Ct);
  {
    BSmall sm{b.C2, b.Ct, b.cstride, b.G, b.gstride, sp.H, sp.hstride, sp.ldh, b.P, sp.ncap, b.R, b.rstride, b.flag};
    const double hb = 16.0 * ((double)p * p / 2 + 3.0 * p * sb) * nb;
    prof_launch(prof, K_BSMALL, hb, 8.0 * p * p * sb / 2 * nb, sb - 1 > 8 ? bsmall_kernel<true> : bsmall_kernel<false>,
                dim3((1 + (p + 15) / 16) * nb), dim3(256), 0, s, g, sm);
  }
  {
    BHess h{e, b.Ct, b.P, b.cstride, sp.ncap, b.R, b.R + 2 * kBlockMax * kBlockMax, b.rstride, sp.H, sp.hstride,
            sp.ldh};
    const int nh = ((p + sb) * kBlockMax + 255) / 256;
    BUpd u{b.C2, b.cstride, b.W, b.wstride, const_cast<double2*>(sp.V) + (size_t)(p - m) * ldq, sp.vstride,
           b.R + kBlockMax * kBlockMax, b.rstride, nrowblk, nh, h};
    prof_launch(prof, K_BUPDATE, upd_bytes, 8.0 * N * p * sb * nb, upd_kernel, dim3(xcd_grid(nb, nrowblk + nh)),
                dim3(256), 0, s, g, u);
  }
}
