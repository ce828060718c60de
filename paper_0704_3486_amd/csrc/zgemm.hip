// Complex FP64 matrix products on the matrix cores of gfx950.
//
// C = alpha A B for column-major complex matrices, built from the real
// instruction v_mfma_f64_16x16x4f64 (one 16 x 16 real block += 16 x 4 times
// 4 x 16 per wavefront): a complex 16 x 16 block takes four of them per
// k-step of four,
//     Re C += Re A Re B - Im A Im B,     Im C += Re A Im B + Im A Re B,
// or, in the Newton-Schulz products, three (the three-multiplication form:
// Re A Re B, Im A Im B and (Re A + Im A)(Re B + Im B)).
// Operand fragments come straight from global memory (the small sign's
// matrices live in L2; a lane loads one complex entry per fragment, rows of
// A and columns of B 16 entries apart), two k-steps ahead of the products,
// clamped at the matrix edges and zeroed outside.  Three launch shapes by
// the number of 16 x 16 output blocks: up to a couple of thousand blocks the
// four wavefronts of a workgroup split the k-steps of one block (or of 2 x 2
// blocks in launches of several large enough matrices), summed in a fixed
// order through LDS; otherwise 2 x 2 wavefronts each own 1 x 1 or 2 x 2
// blocks.  blockIdx.z selects the matrix of a batch.  The shape
// depends on a matrix's size only, so every matrix's arithmetic is the same
// alone and in any batch (no cross-matrix sums).
//
// Two epilogues serve the inverse-free Newton-Schulz iteration of the
// small-matrix sign (step (v)), X <- X (3I - X^2) / 2:
//   * NS_SQUARE: P = X X, writes Y = 3I - P and, per wavefront, the partial
//     sum of |P - I|^2 (summed in a fixed order by ns_check_kernel);
//   * NS_UPDATE: X' = X Y / 2, also into the caller's output F for a matrix
//     whose iteration has just met its stopping test.
// A per-matrix state word (0 running, 1 final, 2 done, 3 stopped unconverged)
// lets finished matrices skip later launches, so the host looks at the
// states only every few iterations.
#include "internal.h"

typedef double v4d __attribute__((ext_vector_type(4)));

// A complex zero in device memory (external linkage, so the compiler cannot
// fold loads from it): lanes outside the matrix load from here, so every
// load is issued unconditionally.  A per-lane select of the value instead of
// the address is turned into a branch around the load, which serialises the
// loads of a k-step.
__device__ double2 sgn_zgemm_zero_entry;

namespace {

enum { ZG_PLAIN = 0, ZG_NS_SQUARE = 1, ZG_NS_UPDATE = 2 };

struct ZgArgs {
  int M, N, K;
  double alpha;
  const double2* A;
  int lda;
  size_t astride;
  const double2* B;
  int ldb;
  size_t bstride;
  double2* C;
  int ldc;
  size_t cstride;
  const int* state;  // NS modes: per matrix
  double* part;      // NS_SQUARE: per matrix, nparts partial sums of |P - I|^2
  int nparts;
  double2* F;        // NS_UPDATE: output of a final matrix
  int ldf;
  size_t fstride;
};

__device__ inline v4d mfma(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// operand fragments of one k-step (four k) for TM row blocks of A and TN
// column blocks of B: lane (li, lk) takes row li / column li at k = k0 + lk
template <int TM, int TN>
struct Frag {
  double2 a[TM], b[TN];
};

// Walks the k-steps first, first + stride, ... of the K range (first and
// stride wavefront-uniform).  Lane (li, lk) reads row li of A's blocks and
// column li of B's blocks at k = 4 step + lk through pointers advanced per
// step; a lane past the matrix edge or past K reads the zero entry instead
// (a select of the address, never of the value, and no short-circuit test:
// either would put a branch around the load).
template <int TM, int TN>
struct KWalk {
  const double2* pa[TM];
  const double2* pb[TN];
  bool aok[TM], bok[TN];
  int k, dk, K;   // this lane's k, its step, the K range
  size_t da, db;  // pointer steps of A (dk columns) and B (dk rows)

  __device__ inline void load(Frag<TM, TN>& f) {
    const double2* z = &sgn_zgemm_zero_entry;
    const bool kok = k < K;
#pragma unroll
    for (int a = 0; a < TM; ++a) f.a[a] = *((kok & aok[a]) ? pa[a] : z);
#pragma unroll
    for (int b = 0; b < TN; ++b) f.b[b] = *((kok & bok[b]) ? pb[b] : z);
  }
  __device__ inline void advance() {
#pragma unroll
    for (int a = 0; a < TM; ++a) pa[a] += da;
#pragma unroll
    for (int b = 0; b < TN; ++b) pb[b] += db;
    k += dk;
  }
};

// One k-step of the complex products.  G3 (the Newton-Schulz products): the
// three-multiplication form, re += Re A Re B, im += Im A Im B,
// tx += (Re A + Im A)(Re B + Im B), turned into Re C = re - im and
// Im C = tx - re - im by finish3 (a quarter fewer matrix-core instructions;
// the extra rounding of Im C is a few units of (|Re A| + |Im A|) (|Re B| +
// |Im B|) per entry, and the iteration does not amplify rounding of that
// size).  Otherwise the four real products straight into Re C and Im C.
template <int TM, int TN, bool G3>
__device__ inline void mma(const Frag<TM, TN>& f, v4d (&re)[TM][TN], v4d (&im)[TM][TN], v4d (&tx)[TM][TN]) {
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      if constexpr (G3) {
        re[a][b] = mfma(f.a[a].x, f.b[b].x, re[a][b]);
        im[a][b] = mfma(f.a[a].y, f.b[b].y, im[a][b]);
        tx[a][b] = mfma(f.a[a].x + f.a[a].y, f.b[b].x + f.b[b].y, tx[a][b]);
      } else {
        re[a][b] = mfma(f.a[a].x, f.b[b].x, re[a][b]);
        re[a][b] = mfma(-f.a[a].y, f.b[b].y, re[a][b]);
        im[a][b] = mfma(f.a[a].x, f.b[b].y, im[a][b]);
        im[a][b] = mfma(f.a[a].y, f.b[b].x, im[a][b]);
      }
    }
}

template <int TM, int TN>
__device__ inline void finish3(v4d (&re)[TM][TN], v4d (&im)[TM][TN], const v4d (&tx)[TM][TN]) {
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const v4d r = re[a][b] - im[a][b];
      im[a][b] = tx[a][b] - re[a][b] - im[a][b];
      re[a][b] = r;
    }
}

// The k-steps with NF - 1 in flight ahead of the one being multiplied (NF =
// 3, or 2 where the register count would otherwise cost occupancy); the loop
// body is unrolled NF times so the fragments rotate through NF register sets
// without copies (a copy of a just-loaded register would wait for the load).
// Steps past K multiply zeros, which leaves the sums unchanged; the k-steps
// are multiplied in the same order for either NF.
template <int TM, int TN, bool G3, int NF = 3>
__device__ inline void kloop(const ZgArgs& g, const double2* __restrict__ A, const double2* __restrict__ B,
                             const int* ar, const bool* aok, const int* bc, const bool* bok, int lk, int first,
                             int stride, v4d (&re)[TM][TN], v4d (&im)[TM][TN], v4d (&tx)[TM][TN]) {
  const int S = (g.K + 3) / 4;
  if (first >= S) return;
  KWalk<TM, TN> w;
  w.K = g.K;
  w.k = 4 * first + lk;
  w.dk = 4 * stride;
  w.da = (size_t)w.dk * g.lda;
  w.db = (size_t)w.dk;
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    w.pa[a] = A + (size_t)(4 * first + lk) * g.lda + ar[a];
    w.aok[a] = aok[a];
  }
#pragma unroll
  for (int b = 0; b < TN; ++b) {
    w.pb[b] = B + (size_t)bc[b] * g.ldb + (4 * first + lk);
    w.bok[b] = bok[b];
  }
  static_assert(NF == 2 || NF == 3, "two or three fragment sets");
  if constexpr (NF == 3) {
    Frag<TM, TN> f0, f1, f2;
    w.load(f0);
    w.advance();
    w.load(f1);
    w.advance();
    for (int st = first; st < S; st += 3 * stride) {
      w.load(f2);
      w.advance();
      mma<TM, TN, G3>(f0, re, im, tx);
      w.load(f0);
      w.advance();
      mma<TM, TN, G3>(f1, re, im, tx);
      w.load(f1);
      w.advance();
      mma<TM, TN, G3>(f2, re, im, tx);
    }
  } else {
    Frag<TM, TN> f0, f1;
    w.load(f0);
    w.advance();
    for (int st = first; st < S; st += 2 * stride) {
      w.load(f1);
      w.advance();
      mma<TM, TN, G3>(f0, re, im, tx);
      w.load(f0);
      w.advance();
      mma<TM, TN, G3>(f1, re, im, tx);
    }
  }
}

// epilogue of one 16 x 16 block (item r of a lane holds row lk + 4 r of
// column li: the instruction's result layout, D[i][j] in lane j + 16 (i % 4),
// item i / 4); returns this lane's part of |P - I|^2 (NS_SQUARE)
template <int MODE>
__device__ inline double store_block(const ZgArgs& g, double2* __restrict__ C, int bz, int row0, int col, int lk,
                                     const v4d& re, const v4d& im, bool final_out) {
  double psum = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row0 + lk + 4 * r;
    if (row >= g.M || col >= g.N) continue;
    double vr = re[r], vi = im[r];
    if (MODE == ZG_NS_SQUARE) {
      const double dI = (row == col) ? 1.0 : 0.0;
      psum += (vr - dI) * (vr - dI) + vi * vi;
      vr = 3.0 * dI - vr;
      vi = -vi;
    } else {
      vr *= g.alpha;
      vi *= g.alpha;
    }
    C[(size_t)col * g.ldc + row] = make_double2(vr, vi);
    if (MODE == ZG_NS_UPDATE && final_out) g.F[(size_t)bz * g.fstride + (size_t)col * g.ldf + row] = make_double2(vr, vi);
  }
  return psum;
}

// Large problems: a workgroup is 2 x 2 wavefronts, each owning TM x TN blocks
// of 16 x 16 over the whole K range.
template <int TM, int TN, int MODE>
__global__ void __launch_bounds__(256) zgemm_kernel(ZgArgs g) {
  const int bz = blockIdx.z;
  if (MODE == ZG_NS_SQUARE && g.state[bz] != 0) return;
  if (MODE == ZG_NS_UPDATE && g.state[bz] > 1) return;
  const double2* __restrict__ A = g.A + (size_t)bz * g.astride;
  const double2* __restrict__ B = g.B + (size_t)bz * g.bstride;
  double2* __restrict__ C = g.C + (size_t)bz * g.cstride;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loop control
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = (blockIdx.y * 2 + (w & 1)) * (16 * TM);
  const int j0 = (blockIdx.x * 2 + (w >> 1)) * (16 * TN);

  constexpr bool G3 = MODE != ZG_PLAIN;
  v4d re[TM][TN], im[TM][TN], tx[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      re[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      im[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      tx[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  int ar[TM], bc[TN];
  bool aok[TM], bok[TN];
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int i = i0 + 16 * a + li;
    aok[a] = i < g.M;
    ar[a] = min(i, g.M - 1);
  }
#pragma unroll
  for (int b = 0; b < TN; ++b) {
    const int j = j0 + 16 * b + li;
    bok[b] = j < g.N;
    bc[b] = min(j, g.N - 1);
  }
  kloop<TM, TN, G3>(g, A, B, ar, aok, bc, bok, lk, 0, 1, re, im, tx);
  if constexpr (G3) finish3<TM, TN>(re, im, tx);

  double psum = 0.0;
  const bool final_out = MODE == ZG_NS_UPDATE && g.state[bz] == 1;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
      psum += store_block<MODE>(g, C, bz, i0 + 16 * a, j0 + 16 * b + li, lk, re[a][b], im[a][b], final_out);
  if (MODE == ZG_NS_SQUARE) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) psum += __shfl_xor(psum, off, 64);
    if (lane == 0) g.part[(size_t)bz * g.nparts + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 4 + w] = psum;
  }
}

// Small problems (one matrix of a few hundred): a workgroup owns T x T
// blocks of 16 x 16 and its four wavefronts split the k-steps (wavefront w
// takes steps w, w + 4, ...); wavefront 0 adds the four partial products in
// a fixed order from LDS.  Four times the wavefronts of one block per
// wavefront; T = 2 shares each operand fragment between two blocks (half
// the loads per matrix-core instruction).  Every entry's sum runs over the
// same k-steps in the same order for either T.
template <int MODE, int T>
__global__ void __launch_bounds__(256) zgemm_splitk_kernel(ZgArgs g) {
  const int bz = blockIdx.z;
  if (MODE == ZG_NS_SQUARE && g.state[bz] != 0) return;
  if (MODE == ZG_NS_UPDATE && g.state[bz] > 1) return;
  const double2* __restrict__ A = g.A + (size_t)bz * g.astride;
  const double2* __restrict__ B = g.B + (size_t)bz * g.bstride;
  double2* __restrict__ C = g.C + (size_t)bz * g.cstride;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loop control
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = blockIdx.y * 16 * T, j0 = blockIdx.x * 16 * T;

  constexpr bool G3 = MODE != ZG_PLAIN;
  v4d re[T][T], im[T][T], tx[T][T];
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      re[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      im[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      tx[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  int ar[T], bc[T];
  bool aok[T], bok[T];
#pragma unroll
  for (int a = 0; a < T; ++a) {
    const int i = i0 + 16 * a + li, j = j0 + 16 * a + li;
    aok[a] = i < g.M;
    ar[a] = min(i, g.M - 1);
    bok[a] = j < g.N;
    bc[a] = min(j, g.N - 1);
  }
  // 2 x 2 blocks: one fragment set in flight (three waves per SIMD, not two)
  kloop<T, T, G3, (T > 1 ? 2 : 3)>(g, A, B, ar, aok, bc, bok, lk, w, 4, re, im, tx);
  if constexpr (G3) finish3<T, T>(re, im, tx);

  // partial products of wavefronts 1..3 -> LDS [w - 1][block][item][lane]
  __shared__ double red[3][T * T][8][64];
  if (w > 0) {
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          red[w - 1][a * T + b][r][lane] = re[a][b][r];
          red[w - 1][a * T + b][4 + r][lane] = im[a][b][r];
        }
  }
  __syncthreads();
  if (w != 0) return;
  const bool final_out = MODE == ZG_NS_UPDATE && g.state[bz] == 1;
  // |P - I|^2 partials per 16 x 16 block (row-major over the blocks), the
  // same set for either T
  const int nbx = (g.N + 15) / 16;
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          re[a][b][r] += red[q][a * T + b][r][lane];
          im[a][b][r] += red[q][a * T + b][4 + r][lane];
        }
      double psum = store_block<MODE>(g, C, bz, i0 + 16 * a, j0 + 16 * b + li, lk, re[a][b], im[a][b], final_out);
      if (MODE == ZG_NS_SQUARE) {
        const int by = blockIdx.y * T + a, bx = blockIdx.x * T + b;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) psum += __shfl_xor(psum, off, 64);
        if (lane == 0 && by * 16 < g.M && bx * 16 < g.N) g.part[(size_t)bz * g.nparts + (size_t)by * nbx + bx] = psum;
      }
    }
}

// per matrix: r = sqrt(sum |P - I|^2 / n) in a fixed order, then the state
// transition of iteration `it` (see the file comment)
__global__ void __launch_bounds__(256) ns_check_kernel(const double* __restrict__ part, int nparts, int n,
                                                       int* __restrict__ state, int* __restrict__ iters, int it,
                                                       int maxit) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int st = state[b];
  __shared__ double red[256];
  if (st == 1) {
    if (tid == 0) state[b] = 2;
    return;
  }
  if (st != 0) return;
  double s = 0.0;
  for (int t = tid; t < nparts; t += 256) s += part[(size_t)b * nparts + t];
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    const double r = sqrt(red[0] / n);  // |X^2 - I|_F / sqrt(n) of the iterate before this update
    if (!isfinite(r) || r > 1e3) {
      state[b] = 3;  // diverging: left for the fallback
    } else if (r < 1e-7) {
      // the error after this update ~ (3/2) (r/2)^2 < 1e-14
      state[b] = 1;
      iters[b] = it;
    } else if (it >= maxit) {
      state[b] = 3;
    }
  }
}

template <int TM, int TN, int MODE>
void launch(const ZgArgs& g, int nb, hipStream_t s) {
  const int gx = (g.N + 32 * TN - 1) / (32 * TN);
  const int gy = (g.M + 32 * TM - 1) / (32 * TM);
  SGN_REQUIRE(gy <= 65535 && nb <= 65535, SGN_EINVAL, "zgemm: grid too large");
  hipLaunchKernelGGL((zgemm_kernel<TM, TN, MODE>), dim3(gx, gy, nb), dim3(256), 0, s, g);
  SGN_HIP(hipGetLastError());
}

template <int MODE, int T>
void launch_splitk(const ZgArgs& g, int nb, hipStream_t s) {
  const int gx = (g.N + 16 * T - 1) / (16 * T), gy = (g.M + 16 * T - 1) / (16 * T);
  SGN_REQUIRE(gy <= 65535 && nb <= 65535, SGN_EINVAL, "zgemm: grid too large");
  hipLaunchKernelGGL((zgemm_splitk_kernel<MODE, T>), dim3(gx, gy, nb), dim3(256), 0, s, g);
  SGN_HIP(hipGetLastError());
}

// launch shape by the output size of one matrix (never by the batch, so a
// matrix gets the same arithmetic alone and in any batch): 0 = split k-steps
// over the wavefronts of a workgroup (up to 2047 blocks of 16 x 16, n < 724),
// 1 = 2 x 2 wavefronts of 16 x 16 blocks, 2 = 2 x 2 wavefronts of 32 x 32
// blocks (16384 blocks and more)
int shape(int M, int N) {
  const long long blocks16 = (long long)((M + 15) / 16) * ((N + 15) / 16);
  if (blocks16 < 2048) return 0;
  if (blocks16 < 16384) return 1;
  return 2;
}

// Split-k workgroups own 2 x 2 blocks when a launch has four or more
// matrices of 256 blocks or more (enough workgroups), else one: the entries'
// sums and the residual partials are the same either way.
template <int MODE>
void launch_auto(const ZgArgs& g, int nb, hipStream_t s) {
  const long long blocks16 = (long long)((g.M + 15) / 16) * ((g.N + 15) / 16);
  switch (shape(g.M, g.N)) {
    case 0:
      if (nb >= 4 && blocks16 >= 256)
        launch_splitk<MODE, 2>(g, nb, s);
      else
        launch_splitk<MODE, 1>(g, nb, s);
      break;
    case 1: launch<1, 1, MODE>(g, nb, s); break;
    default: launch<2, 2, MODE>(g, nb, s); break;
  }
}

}  // namespace

void zgemm(int M, int N, int K, double alpha, const double2* A, int lda, size_t astride, const double2* B, int ldb,
           size_t bstride, double2* C, int ldc, size_t cstride, int nb, hipStream_t s) {
  if (M <= 0 || N <= 0 || nb <= 0) return;
  ZgArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.A = A;
  g.lda = lda;
  g.astride = astride;
  g.B = B;
  g.ldb = ldb;
  g.bstride = bstride;
  g.C = C;
  g.ldc = ldc;
  g.cstride = cstride;
  launch_auto<ZG_PLAIN>(g, nb, s);
}

int zgemm_ns_parts(int n, int nb) {
  (void)nb;
  switch (shape(n, n)) {
    case 0: {
      const int g = (n + 15) / 16;
      return g * g;
    }
    case 1: {
      const int g = (n + 31) / 32;
      return g * g * 4;
    }
    default: {
      const int g = (n + 63) / 64;
      return g * g * 4;
    }
  }
}

void zgemm_ns_square(int n, const double2* X, double2* Y, size_t stride, int nb, const int* state, double* part,
                     hipStream_t s) {
  ZgArgs g{};
  g.M = g.N = g.K = n;
  g.alpha = 1.0;
  g.A = g.B = X;
  g.lda = g.ldb = g.ldc = n;
  g.astride = g.bstride = g.cstride = stride;
  g.C = Y;
  g.state = state;
  g.part = part;
  g.nparts = zgemm_ns_parts(n, nb);
  launch_auto<ZG_NS_SQUARE>(g, nb, s);
}

void zgemm_ns_update(int n, const double2* X, const double2* Y, double2* Xn, size_t stride, int nb, const int* state,
                     double2* F, int ldf, size_t fstride, hipStream_t s) {
  ZgArgs g{};
  g.M = g.N = g.K = n;
  g.alpha = 0.5;
  g.A = X;
  g.B = Y;
  g.lda = g.ldb = g.ldc = n;
  g.astride = g.bstride = g.cstride = stride;
  g.C = Xn;
  g.state = state;
  g.F = F;
  g.ldf = ldf;
  g.fstride = fstride;
  launch_auto<ZG_NS_UPDATE>(g, nb, s);
}

void ns_check(const double* part, int nparts, int n, int* state, int* iters, int it, int maxit, int nb,
              hipStream_t s) {
  hipLaunchKernelGGL(ns_check_kernel, dim3(nb), dim3(256), 0, s, part, nparts, n, state, iters, it, maxit);
  SGN_HIP(hipGetLastError());
}
