// Wilson-Dirac stencil H_w(mu) = gamma5 D_w(mu) (Eq. Dw, Section 2) for gfx950.
//
// Internal layout (structure of arrays, one coalesced stream per component):
//   spinor  v[c * V + n],        c = 3 spin + colour, n = site index
//   links   U[(nu * 9 + 3 row + col) * V + n]
// so that the 64 lanes of a wavefront, which own 64 consecutive sites, read
// every component with one fully coalesced 1 KiB load.  Neighbour spinors
// (8 per site) are re-read through L2 / MALL; each link is used by two sites.
// The antiperiodic time boundary is folded into U_{n,t} of the last time
// slice, the hopping factor kappa and e^{+-mu} stay scalars.
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
#include "internal.h"

namespace {

constexpr int kWilsonBlock = 128;

// chi = U h  (u row-major 3x3)
__device__ inline void su3_mul(const double2 u[9], const double2 h[3], double2 out[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc = cfma(u[3 * r + c], h[c], acc);
    out[r] = acc;
  }
}

// chi = U^dag h
__device__ inline void su3_dagmul(const double2 u[9], const double2 h[3], double2 out[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc = cfmac(u[3 * c + r], h[c], acc);
    out[r] = acc;
  }
}

// Spin-projection table of (1 + gamma_nu) in the chiral basis:
//   h0 = p0 + a0 p[i0],  h1 = p1 + a1 p[i1]      (upper two spin components)
//   lower0 = b0 chi[j0],  lower1 = b1 chi[j1]     (chi = U h, the colour-rotated half spinor)
// with a, b in {+-1, +-i}; (1 - gamma_nu) negates a0, a1, b0, b1.
struct SpinProj {
  int i0, i1, j0, j1;
  double2 a0, a1, b0, b1;
};

__device__ inline SpinProj spin_proj(int nu) {
  const double2 one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0);
  const double2 im = make_double2(0.0, 1.0), mim = make_double2(0.0, -1.0);
  switch (nu) {
    case 0: return SpinProj{3, 2, 1, 0, mim, mim, im, im};
    case 1: return SpinProj{3, 2, 1, 0, mone, one, one, mone};
    case 2: return SpinProj{2, 3, 0, 1, mim, im, im, mim};
    default: return SpinProj{2, 3, 0, 1, one, one, one, one};
  }
}

__global__ void __launch_bounds__(kWilsonBlock)
wilson_hw_kernel(const double2* __restrict__ links, const double2* __restrict__ in, double2* __restrict__ out,
                 const double* __restrict__ inv_beta, double2* __restrict__ copy_out, int Lx, int Ly, int Lz,
                 int Lt, double kappa, double emu, double emmu) {
  const int V = Lx * Ly * Lz * Lt;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  const int x = n % Lx;
  const int y = (n / Lx) % Ly;
  const int z = (n / (Lx * Ly)) % Lz;
  const int t = n / (Lx * Ly * Lz);
  const int sy = Lx, sz = Lx * Ly, st = Lx * Ly * Lz;
  int nb[8];
  nb[0] = (x == Lx - 1) ? n - (Lx - 1) : n + 1;
  nb[1] = (x == 0) ? n + (Lx - 1) : n - 1;
  nb[2] = (y == Ly - 1) ? n - (Ly - 1) * sy : n + sy;
  nb[3] = (y == 0) ? n + (Ly - 1) * sy : n - sy;
  nb[4] = (z == Lz - 1) ? n - (Lz - 1) * sz : n + sz;
  nb[5] = (z == 0) ? n + (Lz - 1) * sz : n - sz;
  nb[6] = (t == Lt - 1) ? n - (Lt - 1) * st : n + st;
  nb[7] = (t == 0) ? n + (Lt - 1) * st : n - st;

  double2 acc[4][3];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[s][c] = make_double2(0.0, 0.0);

  // The eight hops run as a rolled loop so that only one hop's neighbour
  // spinor and link are live at a time (an unrolled body spills on gfx950).
#pragma unroll 1
  for (int d = 0; d < 8; ++d) {
    const int nu = d >> 1;
    const bool fwd = (d & 1) == 0;  // forward hop: (1 + gamma) U_{n,nu} psi_{n+nu}
    const int m = nb[d];
    const double sg = fwd ? 1.0 : -1.0;
    const double phase = (nu == 3) ? (fwd ? emu : emmu) : 1.0;
    const SpinProj P = spin_proj(nu);
    double2 h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 p0 = in[c * V + m];
      const double2 p1 = in[(3 + c) * V + m];
      const double2 pa = in[(3 * P.i0 + c) * V + m];
      const double2 pb = in[(3 * P.i1 + c) * V + m];
      h0[c] = cadd(p0, cscale(cmul(P.a0, pa), sg));
      h1[c] = cadd(p1, cscale(cmul(P.a1, pb), sg));
    }
    const int ls = fwd ? n : m;  // site that owns the link
    double2 u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = links[(nu * 9 + e) * V + ls];
    double2 c0[3], c1[3];
    if (fwd) {
      su3_mul(u, h0, c0);
      su3_mul(u, h1, c1);
    } else {
      su3_dagmul(u, h0, c0);
      su3_dagmul(u, h1, c1);
    }
    const double2 b0 = cscale(P.b0, sg * phase), b1 = cscale(P.b1, sg * phase);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      acc[0][c] = cadd(acc[0][c], cscale(c0[c], phase));
      acc[1][c] = cadd(acc[1][c], cscale(c1[c], phase));
      const double2 x0 = (P.j0 == 0) ? c0[c] : c1[c];
      const double2 x1 = (P.j1 == 0) ? c0[c] : c1[c];
      acc[2][c] = cfma(b0, x0, acc[2][c]);
      acc[3][c] = cfma(b1, x1, acc[3][c]);
    }
  }

  const double scale = inv_beta ? *inv_beta : 1.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double g5 = (s < 2) ? 1.0 : -1.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int idx = (3 * s + c) * V + n;
      const double2 self = in[idx];
      // gamma5 (psi - kappa * hops), all times 1/beta
      const double2 r = csub(self, cscale(acc[s][c], kappa));
      out[idx] = cscale(r, g5 * scale);
      if (copy_out) copy_out[idx] = cscale(self, scale);
    }
  }
}

__global__ void pack_links_kernel(const double2* __restrict__ g, double2* __restrict__ U, int V, int Lt,
                                  int st) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  const int t = n / st;
  for (int nu = 0; nu < 4; ++nu) {
    const double bc = (nu == 3 && t == Lt - 1) ? -1.0 : 1.0;
    for (int e = 0; e < 9; ++e) U[(nu * 9 + e) * V + n] = cscale(g[(n * 4 + nu) * 9 + e], bc);
  }
}

__global__ void pack_kernel(const double2* __restrict__ x, double2* __restrict__ v, int V) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // internal index c * V + n
  if (i >= 12 * V) return;
  const int c = i / V, n = i - c * V;
  v[i] = x[12 * n + c];
}

__global__ void unpack_kernel(const double2* __restrict__ v, double2* __restrict__ y, int V) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // ABI index 12 n + c
  if (i >= 12 * V) return;
  const int n = i / 12, c = i - 12 * n;
  y[i] = v[c * V + n];
}

}  // namespace

void wilson_pack_links(const Lattice& lat, const double2* gauge_abi, double2* links, hipStream_t s) {
  const int V = lat.V;
  hipLaunchKernelGGL(pack_links_kernel, dim3((V + 255) / 256), dim3(256), 0, s, gauge_abi, links, V, lat.L[3],
                     lat.L[0] * lat.L[1] * lat.L[2]);
  SGN_HIP(hipGetLastError());
}

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

void wilson_apply(const Lattice& lat, const double2* links, const double2* in, double2* out,
                  const double* inv_beta, double2* copy_out, hipStream_t s, Profiler* prof) {
  const int V = lat.V;
  const int idx = prof ? prof->begin(K_WILSON) : -1;
  hipLaunchKernelGGL(wilson_hw_kernel, dim3((V + kWilsonBlock - 1) / kWilsonBlock), dim3(kWilsonBlock), 0, s,
                     links, in, out, inv_beta, copy_out, lat.L[0], lat.L[1], lat.L[2], lat.L[3], lat.kappa,
                     lat.emu, lat.emmu);
  SGN_HIP(hipGetLastError());
  if (prof) {
    // algorithmic bytes: read v (12), write w (12), 4 links of 9 (36) per site; + copy (12)
    const double per_site = (60.0 + (copy_out ? 12.0 : 0.0)) * 16.0;
    prof->end(idx, per_site * V, 1392.0 * V);
  }
}
