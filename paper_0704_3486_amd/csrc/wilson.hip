// Wilson-Dirac stencil H_w(mu) = gamma5 D_w(mu) (Eq. Dw, Section 2) for gfx950.
//
// Internal layout (structure of arrays, one coalesced stream per component):
//   spinor  v[c * V + n],        c = 3 spin + colour, n = site index
//   links   U[(nu * 6 + 3 row + col) * V + n],  rows 0 and 1 only
// so that the 64 lanes of a wavefront, which own 64 consecutive sites, read
// every component with one fully coalesced 1 KiB load.  Neighbour spinors
// (8 per site) are re-read through L2 / MALL; each link is used by two sites.
// A link is an SU(3) matrix, so its third row is the complex conjugate of
// the cross product of the first two (unitarity and det U = 1; sgn_create
// checks both): the stencil stores 12 of the 18 reals and rebuilds the third
// row in registers, 24 instead of 36 link entries per site (the stencil's
// bytes fall from 60 to 48 complex numbers per site).  The antiperiodic time
// boundary is then a sign on the hops that cross it (folded into the link it
// would change the determinant); kappa and e^{+-mu} stay scalars.
//
// Spin structure (chiral basis): (1 +- gamma_nu) has rank 2, so each hop
// projects the 4-spinor onto a 2-spinor ("half spinor"), multiplies the two
// colour vectors by the link, and reconstructs the lower two spin components
// from the upper two.  In the chiral basis, with psi = (p0,p1,p2,p3):
//   (1 + g1): h = (p0 - i p3, p1 - i p2),   lower = ( i h1,  i h0)
//   (1 + g2): h = (p0 - p3,   p1 + p2),     lower = ( h1,   -h0)
//   (1 + g3): h = (p0 - i p2, p1 + i p3),   lower = ( i h0, -i h1)
//   (1 + g4): h = (p0 + p2,   p1 + p3),     lower = ( h0,    h1)
// and (1 - g_nu) flips the sign of every gamma term (lower = -(same map)).
#include <initializer_list>

#include "internal.h"

namespace {

constexpr int kWilsonBlock = 128;

// complex helpers generic over double2 / float2
template <typename C> struct Real;
template <> struct Real<double2> { using type = double; };
template <> struct Real<float2> { using type = float; };
template <typename C>
__device__ inline C mk(typename Real<C>::type x, typename Real<C>::type y) {
  C c;
  c.x = x;
  c.y = y;
  return c;
}
template <typename C> __device__ inline C tadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ inline C tsub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ inline C tscale(C a, typename Real<C>::type s) { return mk<C>(a.x * s, a.y * s); }
template <typename C> __device__ inline C tmul(C a, C b) { return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename C> __device__ inline C tfma(C a, C b, C acc) {
  return mk<C>(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}
// acc + conj(a) b
template <typename C> __device__ inline C tfmac(C a, C b, C acc) {
  return mk<C>(acc.x + a.x * b.x + a.y * b.y, acc.y + a.x * b.y - a.y * b.x);
}

// Spin-projection table of (1 + gamma_nu) in the chiral basis:
//   h0 = p0 + a0 p[i0],  h1 = p1 + a1 p[i1]      (upper two spin components)
//   lower0 = b0 chi[j0],  lower1 = b1 chi[j1]     (chi = U h, the colour-rotated half spinor)
// with a, b in {+-1, +-i} stored as (re, im) sign pairs; (1 - gamma_nu) negates a0, a1, b0, b1.
struct SpinProj {
  int i0, i1, j0, j1;
  int a0r, a0i, a1r, a1i, b0r, b0i, b1r, b1i;
};

__device__ inline SpinProj spin_proj(int nu) {
  switch (nu) {
    case 0: return SpinProj{3, 2, 1, 0, 0, -1, 0, -1, 0, 1, 0, 1};
    case 1: return SpinProj{3, 2, 1, 0, -1, 0, 1, 0, 1, 0, -1, 0};
    case 2: return SpinProj{2, 3, 0, 1, 0, -1, 0, 1, 0, 1, 0, -1};
    default: return SpinProj{2, 3, 0, 1, 1, 0, 1, 0, 1, 0, 1, 0};
  }
}

// (re, im) * sign pair (exact: entries are 0 or +-1)
template <typename C>
__device__ inline C unit_mul(int sr, int si, C v, typename Real<C>::type sg) {
  using R = typename Real<C>::type;
  return mk<C>(sg * ((R)sr * v.x - (R)si * v.y), sg * ((R)sr * v.y + (R)si * v.x));
}

// contribution of hop d (nu = d/2, forward if d even) to the 12 components of
// sum_hops at one site: the half-spinor of the neighbour m times the link
// (U_{n,nu} forward, U_{m,nu}^dag backward), times e^{+-mu} on time hops,
// expanded back to four spins
template <typename C>
__device__ inline void hop_term(const C u[9], const C* __restrict__ v, int V, int m, int d,
                                typename Real<C>::type emu, typename Real<C>::type emmu, typename Real<C>::type bc,
                                C o[4][3]) {
  using R = typename Real<C>::type;
  const int nu = d >> 1;
  const bool fwd = (d & 1) == 0;
  const R sg = fwd ? (R)1 : (R)-1;
  const R phase = (nu == 3) ? (fwd ? emu : emmu) * bc : (R)1;
  const SpinProj P = spin_proj(nu);
  C h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const C p0 = v[c * V + m];
    const C p1 = v[(3 + c) * V + m];
    const C pa = v[(3 * P.i0 + c) * V + m];
    const C pb = v[(3 * P.i1 + c) * V + m];
    h0[c] = tadd(p0, unit_mul(P.a0r, P.a0i, pa, sg));
    h1[c] = tadd(p1, unit_mul(P.a1r, P.a1i, pb, sg));
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    C s0 = mk<C>(0, 0), s1 = mk<C>(0, 0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (fwd) {
        s0 = tfma(u[3 * r + c], h0[c], s0);
        s1 = tfma(u[3 * r + c], h1[c], s1);
      } else {
        s0 = tfmac(u[3 * c + r], h0[c], s0);
        s1 = tfmac(u[3 * c + r], h1[c], s1);
      }
    }
    o[0][r] = tscale(s0, phase);
    o[1][r] = tscale(s1, phase);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const C x0 = (P.j0 == 0) ? o[0][c] : o[1][c];
    const C x1 = (P.j1 == 0) ? o[0][c] : o[1][c];
    o[2][c] = unit_mul(P.b0r, P.b0i, x0, sg);
    o[3][c] = unit_mul(P.b1r, P.b1i, x1, sg);
  }
}

constexpr int kLinkRows = 2;               // rows of an SU(3) link held in memory
constexpr int kLinkEntries = 3 * kLinkRows;  // complex entries per link and site

// the link of site ls in direction nu: rows 0 and 1 from memory, row 2 =
// conj(row 0 x row 1)
template <typename C>
__device__ inline void load_link(const C* __restrict__ links, int V, int nu, int ls, C u[9]) {
  const C* __restrict__ lp = links + (size_t)nu * kLinkEntries * V;
#pragma unroll
  for (int e = 0; e < kLinkEntries; ++e) u[e] = lp[(size_t)e * V + ls];
  // cross product of the first two rows, conjugated
  const C c0 = tsub(tmul(u[1], u[5]), tmul(u[2], u[4]));
  const C c1 = tsub(tmul(u[2], u[3]), tmul(u[0], u[5]));
  const C c2 = tsub(tmul(u[0], u[4]), tmul(u[1], u[3]));
  u[6] = mk<C>(c0.x, -c0.y);
  u[7] = mk<C>(c1.x, -c1.y);
  u[8] = mk<C>(c2.x, -c2.y);
}

// neighbour of site n (coordinates x, y, z, t) along hop d, periodic wrap
__device__ inline int hop_neighbour(int n, int d, int x, int y, int z, int t, int Lx, int Ly, int Lz, int Lt) {
  const int nu = d >> 1;
  const int L = nu == 0 ? Lx : nu == 1 ? Ly : nu == 2 ? Lz : Lt;
  const int coord = nu == 0 ? x : nu == 1 ? y : nu == 2 ? z : t;
  const int stride = nu == 0 ? 1 : nu == 1 ? Lx : nu == 2 ? Lx * Ly : Lx * Ly * Lz;
  if ((d & 1) == 0) return (coord == L - 1) ? n - (L - 1) * stride : n + stride;
  return (coord == 0) ? n + (L - 1) * stride : n - stride;
}

// Out_r = H_w(mu) In_r for RB right-hand sides per thread, one site per thread
// (blockIdx.y picks the group of RB); the link of each hop is loaded once and
// applied to all RB.  Used for several right-hand sides on large lattices.
template <typename C, int RB>
__global__ void __launch_bounds__(kWilsonBlock)
wilson_hw_kernel(const C* __restrict__ links, const C* __restrict__ in, size_t istride, C* __restrict__ out,
                 size_t ostride, int nrhs, int Lx, int Ly, int Lz, int Lt, double kappa_d, double emu_d,
                 double emmu_d) {
  using R = typename Real<C>::type;
  const int V = Lx * Ly * Lz * Lt;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int rb0 = blockIdx.y * RB;
  if (n >= V) return;
  const int x = n % Lx;
  const int y = (n / Lx) % Ly;
  const int z = (n / (Lx * Ly)) % Lz;
  const int t = n / (Lx * Ly * Lz);
  const R kappa = (R)kappa_d, emu = (R)emu_d, emmu = (R)emmu_d;

  C acc[RB][4][3];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[b][s][c] = mk<C>(0, 0);

  // The eight hops run as a rolled loop so that only one hop's neighbour
  // spinors and link are live at a time (an unrolled body spills on gfx950).
#pragma unroll 1
  for (int d = 0; d < 8; ++d) {
    const int m = hop_neighbour(n, d, x, y, z, t, Lx, Ly, Lz, Lt);
    const int ls = (d & 1) == 0 ? n : m;  // site that owns the link
    C u[9];
    load_link<C>(links, V, d >> 1, ls, u);
    // antiperiodic in time: the hops across the time boundary
    const R bc = ((d == 6 && t == Lt - 1) || (d == 7 && t == 0)) ? (R)-1 : (R)1;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      if (rb0 + b >= nrhs) break;
      C o[4][3];
      hop_term<C>(u, in + (size_t)(rb0 + b) * istride, V, m, d, emu, emmu, bc, o);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[b][s][c] = tadd(acc[b][s][c], o[s][c]);
    }
  }

#pragma unroll
  for (int b = 0; b < RB; ++b) {
    if (rb0 + b >= nrhs) break;
    const C* __restrict__ v = in + (size_t)(rb0 + b) * istride;
    C* __restrict__ o = out + (size_t)(rb0 + b) * ostride;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const R g5 = (s < 2) ? (R)1 : (R)-1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int idx = (3 * s + c) * V + n;
        // gamma5 (psi - kappa * hops)
        o[idx] = tscale(tsub(v[idx], tscale(acc[b][s][c], kappa)), g5);
      }
    }
  }
}

// Workgroup b runs on XCD b mod 8, each XCD with its own L2.  Renumber the
// blocks so that XCD x works through one contiguous range of sites (about
// 1/8 of the lattice): the neighbour spinors and backward-hop links a block
// reads were then mostly fetched into the same L2 by the blocks just before
// it.  A bijection on [0, nblk).
constexpr int kXcds = 8;
constexpr int kSiteGroup = 32;  // sites per workgroup of the stencil
__device__ inline int xcd_block(int b, int nblk) {
  const int x = b % kXcds, i = b / kXcds, q = nblk / kXcds, r = nblk % kXcds;
  return x * q + min(x, r) + i;
}

// Order in which the workgroups (16 lexicographically consecutive sites
// each) visit the lattice.  Lexicographic order puts the t-neighbours of a
// site a whole time slice of work away, beyond L2 on large lattices.  The
// blocked order walks 4D blocks of Lx x By x Bz x Bt sites (inside a block:
// 16-site segments of By rows, then z, then t; the blocks with t fastest), so
// every neighbour of a site is touched within about Lx By Bz sites of work.
// on = 0: lexicographic (lattices the blocks do not tile, or too small to care).
struct SiteOrder {
  int on = 0;
  int By = 1, Bz = 1, Bt = 1;
  int segw = 1;  // workgroups per segment: Lx By / kSiteGroup
};

// first site of logical workgroup w
__device__ inline int order_site(int w, const SiteOrder& o, int Lx, int Ly, int Lz, int Lt, int sites_per_wg) {
  if (!o.on) return w * sites_per_wg;
  const int wpb = o.segw * o.Bz * o.Bt;
  const int blk = w / wpb, in = w - blk * wpb;
  const int seg = in % o.segw, zi = (in / o.segw) % o.Bz, ti = in / (o.segw * o.Bz);
  const int ntb = Lt / o.Bt, nzb = Lz / o.Bz;
  const int tb = blk % ntb, zb = (blk / ntb) % nzb, yb = blk / (ntb * nzb);
  const int t = tb * o.Bt + ti, z = zb * o.Bz + zi, y0 = yb * o.By;
  return ((t * Lz + z) * Ly + y0) * Lx + seg * sites_per_wg;
}

template <typename C>
__device__ inline C shfl_xor_c(C v, int mask) {
  return mk<C>(__shfl_xor(v.x, mask, 64), __shfl_xor(v.y, mask, 64));
}

// Out_r = H_w(mu) In_r.  A workgroup holds kSiteGroup = 32 sites and four
// wavefronts, wavefront nu taking direction nu for all 32 sites: lanes 0..31
// the forward hop, lanes 32..63 the backward hop of the same sites.  The
// direction, its link array, spin projector and phase are then uniform over
// the wavefront; the backward lanes turn U_{m,nu} into U_{m,nu}^dag with
// selects, so both halves run one instruction stream.  One butterfly shuffle
// (xor 32) adds the two hops, p_nu = fwd_nu + bwd_nu (the same bits in both
// halves: addition is commutative); the four p_nu meet in LDS and are summed
// in direction order.  The site's own spinor entries for the second phase
// are loaded with the hop operands, so a workgroup waits on memory once.
// blockIdx.y = right-hand side (slot map).  Optional: scale = *inv_beta on
// input and output, copy_out = In * scale; with CHEB, Out_r = ca H_w In_r +
// cb Prev_r (Prev_r = prev + slot pstride; prev null: cb ignored), a step of
// a three-term polynomial recurrence.
template <typename C, bool CHEB>
__global__ void __launch_bounds__(256)
wilson_hw_dir_kernel(const C* __restrict__ links, const C* __restrict__ in, size_t istride, C* __restrict__ out,
                     size_t ostride, const double* __restrict__ inv_beta, C* __restrict__ copy_out, int Lx, int Ly,
                     int Lz, int Lt, double kappa_d, double emu_d, double emmu_d, SlotMap map, SiteOrder order,
                     const C* __restrict__ prev, size_t pstride, double ca, double cb) {
  using R = typename Real<C>::type;
  constexpr int kThreads = 256, kOut = 12 * kSiteGroup;
  const int V = Lx * Ly * Lz * Lt;
  const int lane = threadIdx.x & 63;
  const int nu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sl = lane & (kSiteGroup - 1);
  const bool fwd = lane < kSiteGroup;
  const int n0 = order_site(xcd_block(blockIdx.x, gridDim.x), order, Lx, Ly, Lz, Lt, kSiteGroup);
  const int n = n0 + sl;
  const int nc = n < V ? n : V - 1;  // lanes past the lattice work on a valid site, never written out
  const int slot = map.n > 0 ? map.slot[blockIdx.y] : (int)blockIdx.y;
  const C* __restrict__ v = in + (size_t)slot * istride;
  // second-phase outputs of this thread: p = tid + q kThreads < kOut, i.e.
  // component p / kSiteGroup of site n0 + p % kSiteGroup
  C self[2], pv[2];
  const C* __restrict__ pr = (CHEB && prev) ? prev + (size_t)slot * pstride : nullptr;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int p = threadIdx.x + q * kThreads, nn = n0 + p % kSiteGroup;
    const bool ok = p < kOut && nn < V;
    self[q] = ok ? v[(size_t)(p / kSiteGroup) * V + nn] : mk<C>(0, 0);
    // the recurrence's previous term, loaded with the operands (one wait)
    if constexpr (CHEB) pv[q] = (ok && pr) ? pr[(size_t)(p / kSiteGroup) * V + nn] : mk<C>(0, 0);
  }
  const int x = nc % Lx;
  const int y = (nc / Lx) % Ly;
  const int z = (nc / (Lx * Ly)) % Lz;
  const int t = nc / (Lx * Ly * Lz);
  const int m = hop_neighbour(nc, 2 * nu + (fwd ? 0 : 1), x, y, z, t, Lx, Ly, Lz, Lt);
  const int ls = fwd ? nc : m;  // site that owns the link
  C u[9];
  load_link<C>(links, V, nu, ls, u);
  // the matrix applied to the half spinor: U (forward) or U^dag (backward)
  C w9[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C a = u[3 * r + c], b = u[3 * c + r];
      w9[3 * r + c] = fwd ? a : mk<C>(b.x, -b.y);
    }
  const SpinProj P = spin_proj(nu);
  const R sg = fwd ? (R)1 : (R)-1;
  // e^{+-mu} on time hops, and the antiperiodic sign on the two hops across
  // the time boundary (forward from the last slice, backward from the first)
  const bool across = nu == 3 && (fwd ? t == Lt - 1 : t == 0);
  const R phase = (nu == 3) ? (fwd ? (R)emu_d : (R)emmu_d) * (across ? (R)-1 : (R)1) : (R)1;
  C h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const C p0 = v[(size_t)c * V + m];
    const C p1 = v[(size_t)(3 + c) * V + m];
    const C pa = v[(size_t)(3 * P.i0 + c) * V + m];
    const C pb = v[(size_t)(3 * P.i1 + c) * V + m];
    h0[c] = tadd(p0, unit_mul(P.a0r, P.a0i, pa, sg));
    h1[c] = tadd(p1, unit_mul(P.a1r, P.a1i, pb, sg));
  }
  C o[4][3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    C s0 = mk<C>(0, 0), s1 = mk<C>(0, 0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s0 = tfma(w9[3 * r + c], h0[c], s0);
      s1 = tfma(w9[3 * r + c], h1[c], s1);
    }
    o[0][r] = tscale(s0, phase);
    o[1][r] = tscale(s1, phase);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const C x0 = (P.j0 == 0) ? o[0][c] : o[1][c];
    const C x1 = (P.j1 == 0) ? o[0][c] : o[1][c];
    o[2][c] = unit_mul(P.b0r, P.b0i, x0, sg);
    o[3][c] = unit_mul(P.b1r, P.b1i, x1, sg);
  }
  __shared__ C part[12][4][kSiteGroup];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C pnu = tadd(o[s][c], shfl_xor_c(o[s][c], 32));
      if (fwd) part[3 * s + c][nu][sl] = pnu;
    }
  __syncthreads();
  const R kappa = (R)kappa_d;
  const R scale = inv_beta ? (R)(*inv_beta) : (R)1;
  C* __restrict__ w = out + (size_t)slot * ostride;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int p = threadIdx.x + q * kThreads;
    const int comp = p / kSiteGroup, s2 = p % kSiteGroup, nn = n0 + s2;
    if (p >= kOut || nn >= V) continue;
    C acc = mk<C>(0, 0);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc = tadd(acc, part[comp][k][s2]);
    const size_t idx = (size_t)comp * V + nn;
    // gamma5 (psi - kappa * hops), all times 1/beta
    const R g5 = comp < 6 ? (R)1 : (R)-1;
    C val = tscale(tsub(self[q], tscale(acc, kappa)), g5 * scale);
    if constexpr (CHEB) {
      val = tscale(val, (R)ca);
      if (pr) val = tadd(val, tscale(pv[q], (R)cb));
    }
    w[idx] = val;
    if (copy_out) copy_out[idx] = tscale(self[q], scale);
  }
}

__global__ void links_to_f32_kernel(const double2* __restrict__ a, float2* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// rows 0 and 1 of every link into the internal layout; bad = 1 if some link
// is not SU(3) to 1e-10 (|U U^dag - I|, |det U - 1|), since row 2 is rebuilt
__global__ void pack_links_kernel(const double2* __restrict__ g, double2* __restrict__ U, int V, int* bad) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  bool ok = true;
  for (int nu = 0; nu < 4; ++nu) {
    double2 a[9];
    for (int e = 0; e < 9; ++e) a[e] = g[((size_t)n * 4 + nu) * 9 + e];
    for (int e = 0; e < kLinkEntries; ++e) U[((size_t)nu * kLinkEntries + e) * V + n] = a[e];
    double dev = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double2 acc = make_double2(0.0, 0.0);
        for (int k = 0; k < 3; ++k) acc = cfma(a[3 * i + k], make_double2(a[3 * j + k].x, -a[3 * j + k].y), acc);
        dev = fmax(dev, fabs(acc.x - (i == j ? 1.0 : 0.0)) + fabs(acc.y));
      }
    // det = row 2 . (row 0 x row 1)
    const double2 c0 = csub(cmul(a[1], a[5]), cmul(a[2], a[4]));
    const double2 c1 = csub(cmul(a[2], a[3]), cmul(a[0], a[5]));
    const double2 c2 = csub(cmul(a[0], a[4]), cmul(a[1], a[3]));
    const double2 det = cadd(cadd(cmul(a[6], c0), cmul(a[7], c1)), cmul(a[8], c2));
    dev = fmax(dev, fabs(det.x - 1.0) + fabs(det.y));
    if (!(dev <= 1e-10)) ok = false;
  }
  if (!ok) *bad = 1;
}

// threads run over the interface layout, so the reads are contiguous; the
// writes go to 12 streams (one per component), each contiguous across the
// lanes that share a component (as in unpack_kernel, the other way round)
__global__ void pack_kernel(const double2* __restrict__ x, double2* __restrict__ v, int V) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // ABI index 12 n + c
  if (i >= 12 * V) return;
  const int n = i / 12, c = i - 12 * n;
  v[(size_t)c * V + n] = x[i];
}

__global__ void unpack_kernel(const double2* __restrict__ v, double2* __restrict__ y, int V) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // ABI index 12 n + c
  if (i >= 12 * V) return;
  const int n = i / 12, c = i - 12 * n;
  y[i] = v[c * V + n];
}

}  // namespace

void wilson_pack_links(const Lattice& lat, const double2* gauge_abi, double2* links, int* bad, hipStream_t s) {
  const int V = lat.V;
  hipLaunchKernelGGL(pack_links_kernel, dim3((V + 255) / 256), dim3(256), 0, s, gauge_abi, links, V, bad);
  SGN_HIP(hipGetLastError());
}

size_t wilson_link_entries(int V) { return (size_t)4 * kLinkEntries * V; }

void wilson_pack(const Lattice& lat, const double2* x_abi, double2* v, hipStream_t s) {
  const int n = 12 * lat.V;
  hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, x_abi, v, lat.V);
  SGN_HIP(hipGetLastError());
}

void wilson_unpack(const Lattice& lat, const double2* v, double2* y_abi, hipStream_t s) {
  const int n = 12 * lat.V;
  hipLaunchKernelGGL(unpack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, v, y_abi, lat.V);
  SGN_HIP(hipGetLastError());
}

// y = x + gamma5 y in the interface layout (component 12 n + 3 spin + colour;
// gamma5 = diag(1, 1, -1, -1) in spin): the last step of D_ov(mu) x
__global__ void overlap_finish_kernel(const double2* __restrict__ x, double2* __restrict__ y, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 xi = x[i], si = y[i];
  y[i] = (i % 12 < 6) ? make_double2(xi.x + si.x, xi.y + si.y) : make_double2(xi.x - si.x, xi.y - si.y);
}

void overlap_finish(const double2* x, double2* y, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(overlap_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
  SGN_HIP(hipGetLastError());
}

// the adjoint D_ov(mu)^dag x = x + sgn(H_w(mu))^dag gamma5 x, in the interface
// layout: y = gamma5 x before the sign, y = x + y after it
__global__ void gamma5_abi_kernel(const double2* __restrict__ x, double2* __restrict__ y, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 xi = x[i];
  y[i] = (i % 12 < 6) ? xi : make_double2(-xi.x, -xi.y);
}

__global__ void add_abi_kernel(const double2* __restrict__ x, double2* __restrict__ y, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 xi = x[i], si = y[i];
  y[i] = make_double2(xi.x + si.x, xi.y + si.y);
}

// y = a x + b g y, g = gamma5 (if g5) or 1, in the interface layout; x may be y
__global__ void axpby_abi_kernel(const double2* x, double2* y, double a, double b, int g5, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 xi = x[i], yi = y[i];
  const double bb = (g5 && i % 12 >= 6) ? -b : b;
  y[i] = make_double2(a * xi.x + bb * yi.x, a * xi.y + bb * yi.y);
}

void axpby_abi(const double2* x, double2* y, double a, double b, bool g5, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(axpby_abi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, a, b, g5 ? 1 : 0,
                     n);
  SGN_HIP(hipGetLastError());
}

void overlap_adjoint_start(const double2* x, double2* y, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(gamma5_abi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
  SGN_HIP(hipGetLastError());
}

void overlap_adjoint_finish(const double2* x, double2* y, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(add_abi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
  SGN_HIP(hipGetLastError());
}

// the blocked order when the lattice is large enough to leave L2 and its
// extents admit the blocks (Lx By a multiple of the workgroup's 16 sites)
static SiteOrder site_order(const Lattice& lat) {
  SiteOrder o;
  const int Lx = lat.L[0], Ly = lat.L[1], Lz = lat.L[2], Lt = lat.L[3];
  if (lat.blk[0] < 0) return o;
  if (lat.blk[0] > 0) {  // set by sgn_set_stencil_blocks (validated there)
    o.By = lat.blk[0];
    o.Bz = lat.blk[1];
    o.Bt = lat.blk[2];
    o.segw = Lx * o.By / kSiteGroup;
    o.on = 1;
    return o;
  }
  if (lat.V < 65536) return o;
  // preferred extents first (at 32^4, Lx x 4 x 16 x 4 walked 6 % faster than
  // Lx x 8 x 8 x 4 and 14 % faster than the natural order)
  auto pick = [](int L, std::initializer_list<int> pref, auto ok) {
    for (int b : pref)
      if (L % b == 0 && ok(b)) return b;
    return 0;
  };
  o.By = pick(Ly, {4, 8, 2, 16, 1}, [&](int b) { return (Lx * b) % kSiteGroup == 0; });
  o.Bz = pick(Lz, {16, 8, 4, 2, 1}, [](int) { return true; });
  o.Bt = pick(Lt, {4, 8, 2, 1}, [](int) { return true; });
  if (o.By == 0 || o.Bz == 0 || o.Bt == 0) return SiteOrder{};
  o.segw = Lx * o.By / kSiteGroup;
  o.on = 1;
  return o;
}

bool wilson_blocks_valid(const Lattice& lat, int By, int Bz, int Bt) {
  if (By == 0 && Bz == 0 && Bt == 0) return true;
  if (By < 0) return Bz <= 0 && Bt <= 0;
  return By >= 1 && Bz >= 1 && Bt >= 1 && lat.L[1] % By == 0 && lat.L[2] % Bz == 0 && lat.L[3] % Bt == 0 &&
         (lat.L[0] * By) % kSiteGroup == 0;
}

void wilson_apply(const Lattice& lat, const double2* links, const double2* in, double2* out,
                  const double* inv_beta, double2* copy_out, hipStream_t s, Profiler* prof) {
  const int V = lat.V;
  // algorithmic bytes: read v (12), write w (12), 4 links of 6 stored entries
  // (24) per site; + copy (12)
  const double per_site = (48.0 + (copy_out ? 12.0 : 0.0)) * 16.0;
  prof_launch(prof, K_WILSON, per_site * V, 1392.0 * V, wilson_hw_dir_kernel<double2, false>,
              dim3((V + kSiteGroup - 1) / kSiteGroup, 1), dim3(256), 0, s, links, in, (size_t)0, out, (size_t)0,
              inv_beta, copy_out, lat.L[0], lat.L[1], lat.L[2], lat.L[3], lat.kappa, lat.emu, lat.emmu, SlotMap{},
              site_order(lat), (const double2*)nullptr, (size_t)0, 1.0, 0.0);
}

void wilson_apply_cheb_slots(const Lattice& lat, const double2* links, const double2* in, size_t istride,
                             double2* out, size_t ostride, const double2* prev, size_t pstride, double ca, double cb,
                             const SlotMap& map, hipStream_t s, Profiler* prof) {
  SGN_REQUIRE(map.n >= 1 && map.n <= kMaxBatch, SGN_EINVAL, "wilson: slot map must hold 1..64 slots");
  const int V = lat.V;
  // per site: the links (24 stored entries) once, per slot read v and
  // prev, write w (12 each)
  const double bytes = (24.0 + (24.0 + (prev ? 12.0 : 0.0)) * map.n) * 16.0 * V;
  prof_launch(prof, K_WILSON, bytes, 1392.0 * V * map.n, wilson_hw_dir_kernel<double2, true>,
              dim3((V + kSiteGroup - 1) / kSiteGroup, map.n), dim3(256), 0, s, links, in, istride, out, ostride,
              (const double*)nullptr, (double2*)nullptr, lat.L[0], lat.L[1], lat.L[2], lat.L[3], lat.kappa, lat.emu,
              lat.emmu, map, site_order(lat), prev, pstride, ca, cb);
}

// several right-hand sides: one hop per thread (bitwise the single-RHS
// result) unless the lattice is large enough that one site per thread fills
// the chip, where the link is shared by up to four right-hand sides
template <typename C>
static void wilson_multi(const Lattice& lat, const C* links, const C* in, size_t istride, C* out, size_t ostride,
                         int nrhs, bool split, hipStream_t s, Profiler* prof) {
  const int V = lat.V;
  SGN_REQUIRE(nrhs >= 1, SGN_EINVAL, "wilson: nrhs must be positive");
  const int idx = prof ? prof->begin(K_WILSON) : -1;
  const dim3 blk(kWilsonBlock);
  const unsigned gx = (V + kWilsonBlock - 1) / kWilsonBlock;
  const int L0 = lat.L[0], L1 = lat.L[1], L2 = lat.L[2], L3 = lat.L[3];
  if (split || nrhs == 1) {
    hipLaunchKernelGGL((wilson_hw_dir_kernel<C, false>), dim3((V + kSiteGroup - 1) / kSiteGroup, nrhs),
                       dim3(256), 0, s, links, in, istride, out, ostride, nullptr, nullptr, L0, L1, L2,
                       L3, lat.kappa, lat.emu, lat.emmu, SlotMap{}, site_order(lat), (const C*)nullptr, (size_t)0,
                       1.0, 0.0);
  } else if (nrhs >= 4 && sizeof(C) == 8) {
    hipLaunchKernelGGL((wilson_hw_kernel<C, 4>), dim3(gx, (nrhs + 3) / 4), blk, 0, s, links, in, istride, out,
                       ostride, nrhs, L0, L1, L2, L3, lat.kappa, lat.emu, lat.emmu);
  } else {
    hipLaunchKernelGGL((wilson_hw_kernel<C, 2>), dim3(gx, (nrhs + 1) / 2), blk, 0, s, links, in, istride, out,
                       ostride, nrhs, L0, L1, L2, L3, lat.kappa, lat.emu, lat.emmu);
  }
  SGN_HIP(hipGetLastError());
  if (prof) {
    const double b = (double)sizeof(C);
    // per site: 24 spinor entries per RHS (read + write) and 36 link entries once per launch
    prof->end(idx, (24.0 * nrhs + 24.0) * b * V, 1392.0 * V * nrhs);
  }
}

template <typename C>
void wilson_apply_slots(const Lattice& lat, const C* links, const C* in, size_t istride, C* out, size_t ostride,
                        const SlotMap& map, hipStream_t s, Profiler* prof) {
  SGN_REQUIRE(map.n >= 1 && map.n <= kMaxBatch, SGN_EINVAL, "wilson: slot map must hold 1..64 slots");
  const int V = lat.V;
  // per site: the links (24 stored entries) once, per slot read v (12) and write w (12)
  const double b = (double)sizeof(C);
  prof_launch(prof, K_WILSON, (24.0 + 24.0 * map.n) * b * V, 1392.0 * V * map.n, wilson_hw_dir_kernel<C, false>,
              dim3((V + kSiteGroup - 1) / kSiteGroup, map.n), dim3(256), 0, s, links, in, istride, out, ostride,
              (const double*)nullptr, (C*)nullptr, lat.L[0], lat.L[1], lat.L[2], lat.L[3], lat.kappa, lat.emu,
              lat.emmu, map, site_order(lat), (const C*)nullptr, (size_t)0, 1.0, 0.0);
}
template void wilson_apply_slots<double2>(const Lattice&, const double2*, const double2*, size_t, double2*, size_t,
                                          const SlotMap&, hipStream_t, Profiler*);
template void wilson_apply_slots<float2>(const Lattice&, const float2*, const float2*, size_t, float2*, size_t,
                                         const SlotMap&, hipStream_t, Profiler*);

void wilson_apply_multi(const Lattice& lat, const double2* links, const double2* in, size_t istride, double2* out,
                        size_t ostride, int nrhs, bool split, hipStream_t s, Profiler* prof) {
  wilson_multi<double2>(lat, links, in, istride, out, ostride, nrhs, split, s, prof);
}

void wilson_apply_multi32(const Lattice& lat, const float2* links, const float2* in, size_t istride, float2* out,
                          size_t ostride, int nrhs, bool split, hipStream_t s, Profiler* prof) {
  wilson_multi<float2>(lat, links, in, istride, out, ostride, nrhs, split, s, prof);
}

void wilson_links_f32(const double2* links, float2* links32, int V, hipStream_t s) {
  const size_t n = wilson_link_entries(V);
  hipLaunchKernelGGL(links_to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, links, links32, n);
  SGN_HIP(hipGetLastError());
}
