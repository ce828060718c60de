// Deflation setup (Section 5.2, steps (i)-(ii); Results section): the m
// critical eigenvectors of A = H_w(mu) and the partial Schur pair (S_m, T_m).
//
// As in the paper, the eigenvalues of smallest magnitude are sought on the
// squared operator A^2, where they lie on the boundary of the convex hull of
// the spectrum, with an Arnoldi method that is restarted by keeping the wanted
// Ritz vectors ("thick restart", the Krylov-Schur form
// A^2 V_k = V_k T_k + v_{k+1} b^T with a full k x k block T_k).  The Arnoldi
// steps run on the device (two stencil applications and two classical
// Gram-Schmidt passes per step); the small projected eigenproblems are solved
// on the host (hostla.cpp).
//
// After convergence, a Rayleigh-Ritz step with A itself on the span Z of the
// converged vectors of A^2 resolves pairs +-lambda (which share lambda^2):
// G = Z^dag A Z, G W = W diag(theta).  The m Ritz values with smallest
// |Re theta| (ties: smaller |theta|, then larger Im theta) are kept; the QR
// factor of their coefficient vectors, R = Q_R G_R, gives S_m = Z Q_R and
// T_m = Q_R^dag G Q_R, upper triangular up to rounding (Eq. pSd).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <random>

#include "context.h"
#include "hostla.h"

namespace {

using hostla::cplx;

// out = in * (*inv); in and out may alias
__global__ void scale_kernel(const double2* in, double2* out, int n, const double* __restrict__ inv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cscale(in[i], *inv);
}

void dev_scale(const double2* in, double2* out, int n, const double* inv, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n, inv);
  SGN_HIP(hipGetLastError());
}

// one step of the Chebyshev recurrence on L = (A^2 - c) / e:
// out = a (hy - c y) - b yp, with hy = A^2 y (out may alias yp)
__global__ void cheb_step_kernel(const double2* hy, const double2* y, const double2* yp, double2* out, double a,
                                 double c, double b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 h = hy[i], v = y[i];
  double2 r = make_double2(a * (h.x - c * v.x), a * (h.y - c * v.y));
  if (b != 0.0) {
    const double2 q = yp[i];
    r.x -= b * q.x;
    r.y -= b * q.y;
  }
  out[i] = r;
}

void dev_cheb_step(const double2* hy, const double2* y, const double2* yp, double2* out, double a, double c, double b,
                   int n, hipStream_t s) {
  hipLaunchKernelGGL(cheb_step_kernel, dim3((n + 255) / 256), dim3(256), 0, s, hy, y, yp, out, a, c, b, n);
  SGN_HIP(hipGetLastError());
}

struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) { SGN_HIP(hipMalloc(&p, bytes)); }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <class T>
  T* as() {
    return static_cast<T*>(p);
  }
};

inline double2 to_d2(cplx z) { return make_double2(z.real(), z.imag()); }
inline cplx to_c(double2 z) { return cplx(z.x, z.y); }

// indices of the wanted entries: smallest |Re|, then |.|, then larger Im, then index
std::vector<int> select_critical(const std::vector<cplx>& lam, int m) {
  std::vector<int> idx(lam.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    const double ra = std::abs(lam[a].real()), rb = std::abs(lam[b].real());
    if (ra != rb) return ra < rb;
    const double ma = std::abs(lam[a]), mb = std::abs(lam[b]);
    if (ma != mb) return ma < mb;
    if (lam[a].imag() != lam[b].imag()) return lam[a].imag() > lam[b].imag();
    return a < b;
  });
  idx.resize(std::min<size_t>(m, idx.size()));
  return idx;
}

}  // namespace

// thrown by deflate_run when the Ritz pairs have not converged within its restarts
struct NotConverged {
  int matvecs;
};

// Krylov subspace size of the deflation eigensolver: the context's setting,
// else max(3 nev, nev + 40); at most N - 1
static int deflation_ncv(const sgn_ctx* c, int nev) {
  const int want = c->defl_ncv > 0 ? std::max(c->defl_ncv, nev + 3) : std::max(3 * nev, nev + 40);
  return std::min(want, c->N - 1);
}

struct DeflateStats {
  int ncv = 0;            // Krylov subspace size of the run that converged
  int restarts = 0;
  int matvecs = 0;
  double residual = 0.0;  // ||A S - S T||_F / ||A||
  double lower = 0.0;     // ||tril(T, -1)||_F before it is dropped
  int degree = 0;         // Chebyshev degree of the operator of the run that converged (0: A^2)
  double alpha = 0.0, beta = 0.0;  // its damped interval [alpha, beta] of A^2
};

// Operator of the eigensolver: A^2 (degree 0) or the Chebyshev polynomial
// T_d((A^2 - c) / e) of degree d, which stays within [-1, 1] on the real
// interval [alpha, beta] = [c - e, c + e] of A^2's spectrum and grows fast
// below alpha, so that the smallest-magnitude eigenvalues of A^2 become the
// largest-magnitude ones of the operator.
struct OpSpec {
  int degree = 0;
  double c = 0.0, e = 1.0;
};

// The critical Schur pair of the context's operator: S (device, internal
// layout, ldq x m) and T (host, m x m column-major, upper triangular).
static DeflateStats deflate_run(sgn_ctx* c, int m, int nev, int ncv, int max_restarts, double tol,
                                unsigned long long seed, const OpSpec& op, std::unique_ptr<DevBuf>& S_out,
                                std::vector<double2>& T_out) {
  hipStream_t s = c->stream;
  const int N = c->N;
  const size_t ldq = c->ldq;
  const int ldh = ncv + 1;
  DeflateStats st;

  DevBuf bV(sizeof(double2) * ldq * (size_t)(ncv + 1)), bVt(sizeof(double2) * ldq * (size_t)(ncv + 1));
  DevBuf bt(sizeof(double2) * ldq), bw(sizeof(double2) * ldq);
  std::unique_ptr<DevBuf> bya, byb;  // Chebyshev recurrence
  if (op.degree > 0) {
    bya = std::make_unique<DevBuf>(sizeof(double2) * ldq);
    byb = std::make_unique<DevBuf>(sizeof(double2) * ldq);
  }
  DevBuf bH(sizeof(double2) * (size_t)ldh * ldh), bcoef(sizeof(double2) * (size_t)ldh * ldh);
  DevBuf bh1(sizeof(double2) * ldh), bh2(sizeof(double2) * ldh);
  DevBuf bsc(sizeof(double) * 8), bflag(sizeof(int) * 4);
  double2* V = bV.as<double2>();
  double2* Vt = bVt.as<double2>();
  double2* t1 = bt.as<double2>();
  double2* w = bw.as<double2>();
  double2* Hd = bH.as<double2>();
  double2* coef = bcoef.as<double2>();
  double* sc = bsc.as<double>();
  int* flag = bflag.as<int>();
  GsWork g;
  gs_alloc(g, N, ldq, ldh);
  struct GsGuard {
    GsWork& g;
    ~GsGuard() { gs_free(g); }
  } guard{g};
  SGN_HIP(hipMemsetAsync(V, 0, sizeof(double2) * ldq * (ncv + 1), s));
  SGN_HIP(hipMemsetAsync(Vt, 0, sizeof(double2) * ldq * (ncv + 1), s));
  SGN_HIP(hipMemsetAsync(Hd, 0, sizeof(double2) * (size_t)ldh * ldh, s));
  SGN_HIP(hipMemsetAsync(flag, 0, sizeof(int) * 4, s));

  // deterministic start vector (the internal layout is a permutation of the
  // ABI layout, so this is simply some fixed unit vector)
  {
    std::vector<double2> v0((size_t)N);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd;
    for (auto& z : v0) z = make_double2(nd(rng), nd(rng));
    SGN_HIP(hipMemcpyAsync(w, v0.data(), sizeof(double2) * N, hipMemcpyHostToDevice, s));
    SGN_HIP(hipStreamSynchronize(s));
    gs_norm(g, N, w, &sc[0], &sc[1], flag, s, nullptr);
    dev_scale(w, V, N, &sc[1], s);
  }

  // w = operator(v): A^2 v, or T_d((A^2 - c) / e) v by the three-term
  // recurrence y_{j+1} = 2 L y_j - y_{j-1}, y_1 = L v, y_0 = v
  auto apply_op = [&](const double2* v) {
    auto sq = [&](const double2* in, double2* out) {
      wilson_apply(c->lat, c->links, in, t1, nullptr, nullptr, s, nullptr);
      wilson_apply(c->lat, c->links, t1, out, nullptr, nullptr, s, nullptr);
      st.matvecs += 2;
    };
    if (op.degree == 0) {
      sq(v, w);
      return;
    }
    double2* ya = bya->as<double2>();
    double2* yb = byb->as<double2>();
    const double ie = 1.0 / op.e;
    sq(v, w);
    if (op.degree == 1) {
      dev_cheb_step(w, v, v, w, ie, op.c, 0.0, N, s);
      return;
    }
    dev_cheb_step(w, v, v, ya, ie, op.c, 0.0, N, s);  // y_1
    const double2* prev = v;
    double2* cur = ya;
    for (int d = 2; d <= op.degree; ++d) {
      sq(cur, w);
      double2* out = (d == op.degree) ? w : (prev == v ? yb : const_cast<double2*>(prev));
      dev_cheb_step(w, cur, prev, out, 2.0 * ie, op.c, 1.0, N, s);
      prev = cur;
      cur = out;
    }
  };

  std::vector<double2> Hh((size_t)ldh * ldh);
  std::vector<cplx> Hn((size_t)ncv * ncv), theta(ncv), Y((size_t)ncv * ncv);
  int k = 0;
  bool converged = false;
  double bnorm = 1.0;
  for (int rst = 0; rst <= max_restarts; ++rst) {
    // Arnoldi extension k -> ncv on A^2 (Eq. Arnoldi with A^2 in place of A)
    for (int j = k; j < ncv; ++j) {
      double2* vj = V + (size_t)j * ldq;
      apply_op(vj);
      const int ncol = j + 1;
      gs_dot(g, V, ldq, N, ncol, w, bh1.as<double2>(), s, nullptr);
      gs_update(g, V, ldq, N, ncol, bh1.as<double2>(), w, nullptr, 0, s, nullptr);
      gs_dot(g, V, ldq, N, ncol, w, bh2.as<double2>(), s, nullptr);
      GsFinal fin{bh1.as<double2>(), Hd + (size_t)j * ldh, nullptr, &sc[1], nullptr};
      gs_update(g, V, ldq, N, ncol, bh2.as<double2>(), w, &fin, j + 1, s, nullptr);
      dev_scale(w, V + (size_t)(j + 1) * ldq, N, &sc[1], s);
    }
    SGN_HIP(hipMemcpyAsync(Hh.data(), Hd, sizeof(double2) * Hh.size(), hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < ncv; ++j)
      for (int i = 0; i < ncv; ++i) Hn[(size_t)j * ncv + i] = to_c(Hh[(size_t)j * ldh + i]);
    const double beta = Hh[(size_t)(ncv - 1) * ldh + ncv].x;
    SGN_REQUIRE(std::isfinite(beta), SGN_EDEFL, "deflation: non-finite Arnoldi coefficient");
    SGN_REQUIRE(hostla::eig(ncv, Hn.data(), theta.data(), Y.data()), SGN_EDEFL,
                "deflation: small eigenproblem did not converge");
    // order by |theta|: wanted the smallest magnitude of lambda^2 (A^2), or
    // the largest of the filter polynomial
    std::vector<int> ord(ncv);
    std::iota(ord.begin(), ord.end(), 0);
    if (op.degree == 0)
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::abs(theta[a]) < std::abs(theta[b]); });
    else
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::abs(theta[a]) > std::abs(theta[b]); });
    bnorm = 0.0;
    for (auto& t : theta) bnorm = std::max(bnorm, std::abs(t));
    int nconv = 0;
    double worst = 0.0;
    for (int i = 0; i < nev; ++i) {
      const double r = std::abs(beta) * std::abs(Y[(size_t)ord[i] * ncv + (ncv - 1)]);
      // A^2: relative to its spectral radius; the filter: relative to the
      // Ritz value itself (the wanted ones are the large ones)
      const double scale = op.degree == 0 ? bnorm : std::abs(theta[ord[i]]);
      worst = std::max(worst, r / scale);
      if (r <= tol * scale) ++nconv;
    }
    st.restarts = rst;
    const bool last = (rst == max_restarts);
    if (nconv == nev || last) {
      converged = (nconv == nev) || worst < 1e-10;
      // U = V Y[:, wanted nev]  -> Vt[:, 0..nev)
      std::vector<double2> cf((size_t)ncv * nev);
      for (int i = 0; i < nev; ++i)
        for (int r = 0; r < ncv; ++r) cf[(size_t)i * ncv + r] = to_d2(Y[(size_t)ord[i] * ncv + r]);
      SGN_HIP(hipMemcpyAsync(coef, cf.data(), sizeof(double2) * cf.size(), hipMemcpyHostToDevice, s));
      dev_zgemm_nn(c->dense, N, nev, ncv, V, (int)ldq, coef, ncv, Vt, (int)ldq, s);  // one pass over V
      SGN_HIP(hipStreamSynchronize(s));  // cf is pageable host memory
      break;
    }
    // thick restart: keep kk wanted Ritz vectors (orthonormalised)
    int kk = std::min(nev + (ncv - nev) / 2, ncv - 2);
    std::vector<cplx> Yq((size_t)ncv * kk);
    for (int i = 0; i < kk; ++i)
      for (int r = 0; r < ncv; ++r) Yq[(size_t)i * ncv + r] = Y[(size_t)ord[i] * ncv + r];
    hostla::thin_qr(ncv, kk, Yq.data(), 1e-12);
    // drop columns that became zero (numerically dependent Ritz vectors)
    {
      int w2 = 0;
      for (int i = 0; i < kk; ++i) {
        double nn = 0.0;
        for (int r = 0; r < ncv; ++r) nn += std::norm(Yq[(size_t)i * ncv + r]);
        if (nn > 0.5) {
          if (w2 != i)
            for (int r = 0; r < ncv; ++r) Yq[(size_t)w2 * ncv + r] = Yq[(size_t)i * ncv + r];
          ++w2;
        }
      }
      kk = w2;
    }
    // T_k = Yq^H H Yq, b = beta * Yq[ncv-1, :]
    std::vector<cplx> HY((size_t)ncv * kk, cplx(0.0, 0.0));
    for (int i = 0; i < kk; ++i)
      for (int l = 0; l < ncv; ++l) {
        const cplx y = Yq[(size_t)i * ncv + l];
        if (y == cplx(0.0, 0.0)) continue;
        for (int r = 0; r < ncv; ++r) HY[(size_t)i * ncv + r] += Hn[(size_t)l * ncv + r] * y;
      }
    std::fill(Hh.begin(), Hh.end(), make_double2(0.0, 0.0));
    for (int i = 0; i < kk; ++i) {
      for (int r = 0; r < kk; ++r) {
        cplx sacc = 0.0;
        for (int l = 0; l < ncv; ++l) sacc += std::conj(Yq[(size_t)r * ncv + l]) * HY[(size_t)i * ncv + l];
        Hh[(size_t)i * ldh + r] = to_d2(sacc);
      }
      Hh[(size_t)i * ldh + kk] = to_d2(beta * Yq[(size_t)i * ncv + (ncv - 1)]);
    }
    std::vector<double2> cf((size_t)ncv * kk);
    for (size_t e = 0; e < cf.size(); ++e) cf[e] = to_d2(Yq[e]);
    SGN_HIP(hipMemcpyAsync(coef, cf.data(), sizeof(double2) * cf.size(), hipMemcpyHostToDevice, s));
    dev_zgemm_nn(c->dense, N, kk, ncv, V, (int)ldq, coef, ncv, Vt, (int)ldq, s);  // one pass over V
    SGN_HIP(hipMemcpyAsync(Vt + (size_t)kk * ldq, V + (size_t)ncv * ldq, sizeof(double2) * ldq,
                           hipMemcpyDeviceToDevice, s));
    std::swap(V, Vt);
    SGN_HIP(hipMemcpyAsync(Hd, Hh.data(), sizeof(double2) * Hh.size(), hipMemcpyHostToDevice, s));
    SGN_HIP(hipStreamSynchronize(s));
    k = kk;
  }
  if (!converged) throw NotConverged{st.matvecs};

  // Z = orth(U) on the device (classical Gram-Schmidt, two passes), in Vt
  for (int i = 0; i < nev; ++i) {
    double2* u = Vt + (size_t)i * ldq;
    if (i > 0) {
      gs_dot(g, Vt, ldq, N, i, u, bh1.as<double2>(), s, nullptr);
      gs_update(g, Vt, ldq, N, i, bh1.as<double2>(), u, nullptr, 0, s, nullptr);
      gs_dot(g, Vt, ldq, N, i, u, bh2.as<double2>(), s, nullptr);
      GsFinal fin{nullptr, nullptr, &sc[0], &sc[1], nullptr};
      gs_update(g, Vt, ldq, N, i, bh2.as<double2>(), u, &fin, 0, s, nullptr);
    } else {
      gs_norm(g, N, u, &sc[0], &sc[1], nullptr, s, nullptr);
    }
    dev_scale(u, u, N, &sc[1], s);
  }
  // W = A Z (in V), G = Z^dag W
  std::vector<double2> Gd((size_t)nev * nev);
  for (int i = 0; i < nev; ++i) {
    wilson_apply(c->lat, c->links, Vt + (size_t)i * ldq, V + (size_t)i * ldq, nullptr, nullptr, s, nullptr);
    st.matvecs += 1;
    gs_dot(g, Vt, ldq, N, nev, V + (size_t)i * ldq, coef + (size_t)i * nev, s, nullptr);
  }
  SGN_HIP(hipMemcpyAsync(Gd.data(), coef, sizeof(double2) * Gd.size(), hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  std::vector<cplx> G((size_t)nev * nev), lam(nev), Wv((size_t)nev * nev);
  for (size_t e = 0; e < G.size(); ++e) G[e] = to_c(Gd[e]);
  SGN_REQUIRE(hostla::eig(nev, G.data(), lam.data(), Wv.data()), SGN_EDEFL,
              "deflation: Rayleigh-Ritz eigenproblem did not converge");
  const std::vector<int> sel = select_critical(lam, m);
  std::vector<cplx> Rq((size_t)nev * m);
  for (int j = 0; j < m; ++j)
    for (int r = 0; r < nev; ++r) Rq[(size_t)j * nev + r] = Wv[(size_t)sel[j] * nev + r];
  SGN_REQUIRE(hostla::thin_qr(nev, m, Rq.data(), 1e-10) == m, SGN_EDEFL,
              "deflation: selected eigenvectors are linearly dependent");
  // T = Rq^H G Rq
  std::vector<cplx> GR((size_t)nev * m, cplx(0.0, 0.0)), T((size_t)m * m);
  for (int j = 0; j < m; ++j)
    for (int l = 0; l < nev; ++l)
      for (int r = 0; r < nev; ++r) GR[(size_t)j * nev + r] += G[(size_t)l * nev + r] * Rq[(size_t)j * nev + l];
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      cplx sacc = 0.0;
      for (int r = 0; r < nev; ++r) sacc += std::conj(Rq[(size_t)i * nev + r]) * GR[(size_t)j * nev + r];
      T[(size_t)j * m + i] = sacc;
    }
  double low = 0.0;
  for (int j = 0; j < m; ++j)
    for (int i = j + 1; i < m; ++i) low += std::norm(T[(size_t)j * m + i]);
  st.lower = std::sqrt(low);

  // S = Z Rq (device, internal layout) and the residual ||A S - S T||_F
  auto bS = std::make_unique<DevBuf>(sizeof(double2) * ldq * (size_t)m);
  double2* Sd = bS->as<double2>();
  SGN_HIP(hipMemsetAsync(Sd, 0, sizeof(double2) * ldq * (size_t)m, s));
  std::vector<double2> cf((size_t)nev * m), cf2((size_t)m * m);
  for (size_t e = 0; e < cf.size(); ++e) cf[e] = to_d2(Rq[e]);
  SGN_HIP(hipMemcpyAsync(coef, cf.data(), sizeof(double2) * cf.size(), hipMemcpyHostToDevice, s));
  for (int j = 0; j < m; ++j)
    gs_combine(g, Vt, ldq, N, nev, coef + (size_t)j * nev, Sd + (size_t)j * ldq, nullptr, s, nullptr);
  std::vector<double2> Tkeep((size_t)m * m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) Tkeep[(size_t)j * m + i] = (i <= j) ? to_d2(T[(size_t)j * m + i]) : make_double2(0, 0);
  SGN_HIP(hipMemcpyAsync(coef + (size_t)nev * m, Tkeep.data(), sizeof(double2) * Tkeep.size(),
                         hipMemcpyHostToDevice, s));
  double res2 = 0.0;
  for (int j = 0; j < m; ++j) {
    wilson_apply(c->lat, c->links, Sd + (size_t)j * ldq, w, nullptr, nullptr, s, nullptr);
    GsFinal fin{nullptr, nullptr, &sc[0], &sc[1], nullptr};
    gs_update(g, Sd, ldq, N, m, coef + (size_t)nev * m + (size_t)j * m, w, &fin, 0, s, nullptr);
    double r = 0.0;
    SGN_HIP(hipMemcpyAsync(&r, &sc[0], sizeof(double), hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    res2 += r * r;
  }
  // ||A||: from the spectral radius of A^2 (its Ritz values), or, with the
  // filter, from the interval the filter was built on
  const double anorm = std::sqrt(op.degree == 0 ? bnorm : op.c + op.e);
  st.residual = std::sqrt(res2) / anorm;
  st.degree = op.degree;
  st.alpha = op.degree ? op.c - op.e : 0.0;
  st.beta = op.degree ? op.c + op.e : 0.0;
  SGN_REQUIRE(st.residual <= 1e-10, SGN_EDEFL,
              "deflation basis not accurate enough: ||AS - ST||_F / ||A|| = " + std::to_string(st.residual));
  S_out = std::move(bS);
  T_out = std::move(Tkeep);
  return st;
}

// Spectral radius of A^2 from a short Arnoldi run (the largest-magnitude Ritz
// values converge first): the upper end of the filter's damped interval,
// with a 10 % margin (eigenvalues above it would be amplified too).
double sq_radius_estimate(sgn_ctx* c, int steps, unsigned long long seed) {
  hipStream_t s = c->stream;
  const int N = c->N;
  const size_t ldq = c->ldq;
  steps = std::max(2, std::min(steps, N - 1));
  const int ldh = steps + 1;
  DevBuf bV(sizeof(double2) * ldq * (size_t)(steps + 1)), bt(sizeof(double2) * ldq), bw(sizeof(double2) * ldq);
  DevBuf bH(sizeof(double2) * (size_t)ldh * ldh), bh1(sizeof(double2) * ldh), bh2(sizeof(double2) * ldh),
      bsc(sizeof(double) * 4);
  double2* V = bV.as<double2>();
  double2* t1 = bt.as<double2>();
  double2* w = bw.as<double2>();
  double2* Hd = bH.as<double2>();
  double* sc = bsc.as<double>();
  GsWork g;
  gs_alloc(g, N, ldq, ldh);
  struct GsGuard {
    GsWork& g;
    ~GsGuard() { gs_free(g); }
  } guard{g};
  SGN_HIP(hipMemsetAsync(Hd, 0, sizeof(double2) * (size_t)ldh * ldh, s));
  {
    std::vector<double2> v0((size_t)N);
    std::mt19937_64 rng(seed ^ 0x9e3779b97f4a7c15ull);
    std::normal_distribution<double> nd;
    for (auto& z : v0) z = make_double2(nd(rng), nd(rng));
    SGN_HIP(hipMemcpyAsync(w, v0.data(), sizeof(double2) * N, hipMemcpyHostToDevice, s));
    SGN_HIP(hipStreamSynchronize(s));
    gs_norm(g, N, w, &sc[0], &sc[1], nullptr, s, nullptr);
    dev_scale(w, V, N, &sc[1], s);
  }
  for (int j = 0; j < steps; ++j) {
    double2* vj = V + (size_t)j * ldq;
    wilson_apply(c->lat, c->links, vj, t1, nullptr, nullptr, s, nullptr);
    wilson_apply(c->lat, c->links, t1, w, nullptr, nullptr, s, nullptr);
    gs_dot(g, V, ldq, N, j + 1, w, bh1.as<double2>(), s, nullptr);
    gs_update(g, V, ldq, N, j + 1, bh1.as<double2>(), w, nullptr, 0, s, nullptr);
    gs_dot(g, V, ldq, N, j + 1, w, bh2.as<double2>(), s, nullptr);
    GsFinal fin{bh1.as<double2>(), Hd + (size_t)j * ldh, nullptr, &sc[1], nullptr};
    gs_update(g, V, ldq, N, j + 1, bh2.as<double2>(), w, &fin, j + 1, s, nullptr);
    dev_scale(w, V + (size_t)(j + 1) * ldq, N, &sc[1], s);
  }
  std::vector<double2> Hh((size_t)ldh * ldh);
  SGN_HIP(hipMemcpyAsync(Hh.data(), Hd, sizeof(double2) * Hh.size(), hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  std::vector<cplx> Hn((size_t)steps * steps), theta(steps), Y((size_t)steps * steps);
  for (int j = 0; j < steps; ++j)
    for (int i = 0; i < steps; ++i) Hn[(size_t)j * steps + i] = to_c(Hh[(size_t)j * ldh + i]);
  SGN_REQUIRE(hostla::eig(steps, Hn.data(), theta.data(), Y.data()), SGN_EDEFL,
              "deflation: spectral estimate did not converge");
  double r = 0.0;
  for (auto& t : theta) r = std::max(r, std::abs(t));
  SGN_REQUIRE(std::isfinite(r) && r > 0.0, SGN_EDEFL, "deflation: non-finite spectral estimate");
  return 1.1 * r;
}

// deflate_run with a growing Krylov subspace: unless the context fixes ncv,
// a run that has not converged after 400 restarts is repeated with twice the
// subspace (the restart count is very sensitive to ncv on clustered spectra),
// up to N - 1; the last size gets 3000 restarts.
//
// With a filter degree set (sgn_set_deflation_filter), a filtered run comes
// first: the operator is T_d((A^2 - c) / e) on the interval [alpha, beta] =
// [cut rho, rho] of A^2's spectrum (rho its spectral radius, estimated), whose
// largest-magnitude Ritz values are sought.  It keeps the Krylov subspace
// small, so it replaces most of the restarts (each of which orthogonalises
// against the whole basis and solves a small eigenproblem on the host) by
// stencil applications.  If it has not converged within its restarts, or
// its basis fails the Schur-residual test, the unfiltered solver runs.
static DeflateStats deflate_escalating(sgn_ctx* c, int m, int nev, unsigned long long seed,
                                       std::unique_ptr<DevBuf>& S_out, std::vector<double2>& T_out) {
  int ncv = deflation_ncv(c, nev);
  SGN_REQUIRE(ncv > nev + 2, SGN_EINVAL, "lattice too small for this m");
  int spent_restarts = 0, spent_matvecs = 0;
  if (c->defl_degree > 0) {
    const double rho = sq_radius_estimate(c, 40, seed);
    spent_matvecs += 2 * std::min(40, c->N - 1);
    OpSpec op;
    op.degree = c->defl_degree;
    const double alpha = c->defl_cut * rho;
    op.c = 0.5 * (rho + alpha);
    op.e = 0.5 * (rho - alpha);
    try {
      DeflateStats st = deflate_run(c, m, nev, ncv, 300, 1e-13, seed, op, S_out, T_out);
      st.ncv = ncv;
      st.matvecs += spent_matvecs;
      return st;
    } catch (const NotConverged& e) {
      spent_restarts += 300;
      spent_matvecs += e.matvecs;
    } catch (const SgnError& e) {
      if (e.status != SGN_EDEFL) throw;
    }
  }
  for (;;) {
    const bool last = c->defl_ncv > 0 || ncv >= c->N - 1;
    try {
      DeflateStats st = deflate_run(c, m, nev, ncv, last ? 3000 : 400, 1e-13, seed, OpSpec{}, S_out, T_out);
      st.ncv = ncv;
      st.restarts += spent_restarts;
      st.matvecs += spent_matvecs;
      return st;
    } catch (const NotConverged& e) {
      SGN_REQUIRE(!last, SGN_EDEFL, "deflation: Arnoldi on A^2 did not converge");
      spent_restarts += 400;
      spent_matvecs += e.matvecs;
      ncv = std::min(2 * ncv, c->N - 1);
    }
  }
}

namespace {

// in-place inverse of a column-major n x n complex matrix (Gauss-Jordan with
// partial pivoting); false if singular
bool invert(int n, std::vector<cplx>& A) {
  std::vector<int> piv(n);
  std::vector<cplx> I((size_t)n * n, cplx(0.0, 0.0));
  for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
  auto at = [n](std::vector<cplx>& M, int r, int c) -> cplx& { return M[(size_t)c * n + r]; };
  for (int col = 0; col < n; ++col) {
    int p = col;
    for (int r = col + 1; r < n; ++r)
      if (std::abs(at(A, r, col)) > std::abs(at(A, p, col))) p = r;
    if (std::abs(at(A, p, col)) == 0.0) return false;
    if (p != col)
      for (int c2 = 0; c2 < n; ++c2) {
        std::swap(at(A, p, c2), at(A, col, c2));
        std::swap(at(I, p, c2), at(I, col, c2));
      }
    const cplx d = 1.0 / at(A, col, col);
    for (int c2 = 0; c2 < n; ++c2) {
      at(A, col, c2) *= d;
      at(I, col, c2) *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const cplx f = at(A, r, col);
      if (f == cplx(0.0, 0.0)) continue;
      for (int c2 = 0; c2 < n; ++c2) {
        at(A, r, c2) -= f * at(A, col, c2);
        at(I, r, c2) -= f * at(I, col, c2);
      }
    }
  }
  A.swap(I);
  return true;
}

// eigenvalues and eigenvectors (columns) of a host m x m column-major matrix
void host_eigvecs(int m, const std::vector<double2>& T, std::vector<cplx>& lam, std::vector<cplx>& W) {
  std::vector<cplx> A((size_t)m * m);
  for (size_t e = 0; e < A.size(); ++e) A[e] = to_c(T[e]);
  lam.assign(m, cplx(0.0, 0.0));
  W.assign((size_t)m * m, cplx(0.0, 0.0));
  SGN_REQUIRE(hostla::eig(m, A.data(), lam.data(), W.data()), SGN_EDEFL,
              "LR deflation: eigenproblem of T did not converge");
}

// the time-hop factors e^{+mu}, e^{-mu} exchanged while alive: the operator
// becomes H_w(-mu) = H_w(mu)^dag
struct MinusMu {
  Lattice& lat;
  explicit MinusMu(Lattice& l) : lat(l) { std::swap(lat.emu, lat.emmu); }
  ~MinusMu() { std::swap(lat.emu, lat.emmu); }
};

}  // namespace

extern "C" int sgn_deflate(sgn_ctx* c, int m) {
  return guarded(c, [&] {
    SGN_REQUIRE(m >= 0 && m <= c->N / 4, SGN_EINVAL, "m must satisfy 0 <= m <= N/4");
    SGN_REQUIRE(c->sessions == 0, SGN_ESTATE, "a serving session holds this field's Schur pair");
    if (m == 0) {
      install_schur_pair(c, 0, nullptr, {});
      return SGN_OK;
    }
    const int nev = std::min(m + std::max(10, m / 2), c->N / 2);
    std::unique_ptr<DevBuf> S;
    std::vector<double2> T;
    const DeflateStats st = deflate_escalating(c, m, nev, 0x5151ull, S, T);
    install_schur_pair(c, m, S->as<double2>(), T);
    c->defl_restarts = st.restarts;
    c->defl_matvecs = st.matvecs;
    c->defl_residual = st.residual;
    c->defl_used_degree = st.degree;
    c->defl_alpha = st.alpha;
    c->defl_beta = st.beta;
    return SGN_OK;
  });
}

extern "C" int sgn_set_deflation_filter(sgn_ctx* c, int degree, double cut) {
  return guarded(c, [&] {
    SGN_REQUIRE(degree >= 0 && degree <= 200, SGN_EINVAL, "degree must satisfy 0 <= degree <= 200");
    SGN_REQUIRE(cut == 0.0 || (cut > 0.0 && cut < 1.0), SGN_EINVAL, "cut must be 0 (default) or in (0, 1)");
    c->defl_degree = degree;
    c->defl_cut = cut > 0.0 ? cut : kDefaultFilterCut;
    return SGN_OK;
  });
}

extern "C" int sgn_deflate_filter_stats(const sgn_ctx* c, int* degree, double* alpha, double* beta) {
  if (!c) return SGN_ESTATE;
  if (degree) *degree = c->defl_used_degree;
  if (alpha) *alpha = c->defl_alpha;
  if (beta) *beta = c->defl_beta;
  return SGN_OK;
}

extern "C" int sgn_deflate_stats(const sgn_ctx* c, int* restarts, int* matvecs, double* residual) {
  if (!c) return SGN_ESTATE;
  if (restarts) *restarts = c->defl_restarts;
  if (matvecs) *matvecs = c->defl_matvecs;
  if (residual) *residual = c->defl_residual;
  return SGN_OK;
}

// LR-deflation setup (the LR-deflation subsection, steps (i)-(ii)): right
// eigenvectors R = S W of the critical Schur pair of H_w(mu) (T W = W Lambda),
// left eigenvectors from the critical Schur pair of H_w(-mu) = H_w(mu)^dag
// (a left eigenvector of H_w(mu) for lambda is a right eigenvector of
// H_w(-mu) for conj(lambda)), paired by eigenvalue and rescaled to
// L^dag R = I.
extern "C" int sgn_deflate_lr(sgn_ctx* c, int m) {
  return guarded(c, [&] {
    SGN_REQUIRE(m >= 1 && m <= c->N / 4, SGN_EINVAL, "m must satisfy 1 <= m <= N/4");
    SGN_REQUIRE(c->sessions == 0, SGN_ESTATE, "a serving session holds this field's deflation");
    const int nev = std::min(m + std::max(10, m / 2), c->N / 2);
    hipStream_t s = c->stream;
    const size_t ldq = c->ldq;
    const int N = c->N;
    std::unique_ptr<DevBuf> S1, S2;
    std::vector<double2> T1, T2;
    const DeflateStats st1 = deflate_escalating(c, m, nev, 0x5151ull, S1, T1);
    DeflateStats st2;
    {
      MinusMu flip(c->lat);
      st2 = deflate_escalating(c, m, nev, 0x5151ull, S2, T2);
    }
    std::vector<cplx> lam1, W1, lam2, W2;
    host_eigvecs(m, T1, lam1, W1);
    host_eigvecs(m, T2, lam2, W2);
    // pair lambda_i with the eigenvalue conj(lambda_i) of H_w(-mu)
    std::vector<int> perm(m, -1);
    std::vector<char> used(m, 0);
    for (int i = 0; i < m; ++i) {
      int best = -1;
      double bd = 0.0;
      for (int j = 0; j < m; ++j) {
        const double d = std::abs(lam2[j] - std::conj(lam1[i]));
        if (!used[j] && (best < 0 || d < bd)) best = j, bd = d;
      }
      SGN_REQUIRE(best >= 0 && bd <= 1e-8 * std::max(1.0, std::abs(lam1[i])), SGN_EDEFL,
                  "LR deflation: the critical eigenvalues of H_w(mu) and H_w(-mu) do not pair up");
      used[best] = 1;
      perm[i] = best;
    }
    GsWork g;
    gs_alloc(g, N, ldq, m);
    struct GsGuard {
      GsWork& g;
      ~GsGuard() { gs_free(g); }
    } guard{g};
    DevBuf bR(sizeof(double2) * ldq * (size_t)m), bL0(sizeof(double2) * ldq * (size_t)m),
        bL(sizeof(double2) * ldq * (size_t)m), bcoef(sizeof(double2) * (size_t)m * m);
    double2* R = bR.as<double2>();
    double2* L0 = bL0.as<double2>();
    double2* L = bL.as<double2>();
    double2* coef = bcoef.as<double2>();
    SGN_HIP(hipMemsetAsync(R, 0, sizeof(double2) * ldq * (size_t)m, s));
    SGN_HIP(hipMemsetAsync(L0, 0, sizeof(double2) * ldq * (size_t)m, s));
    SGN_HIP(hipMemsetAsync(L, 0, sizeof(double2) * ldq * (size_t)m, s));
    std::vector<double2> hc((size_t)m * m);
    auto combine = [&](const double2* Q, const std::vector<cplx>& C, double2* out) {
      for (size_t e = 0; e < hc.size(); ++e) hc[e] = to_d2(C[e]);
      SGN_HIP(hipMemcpyAsync(coef, hc.data(), sizeof(double2) * hc.size(), hipMemcpyHostToDevice, s));
      for (int j = 0; j < m; ++j) gs_combine(g, Q, ldq, N, m, coef + (size_t)j * m, out + (size_t)j * ldq, nullptr, s, nullptr);
      SGN_HIP(hipStreamSynchronize(s));
    };
    auto gram = [&](const double2* A, const double2* B) {  // A^dag B, host column-major
      for (int j = 0; j < m; ++j) gs_dot(g, A, ldq, N, m, B + (size_t)j * ldq, coef + (size_t)j * m, s, nullptr);
      SGN_HIP(hipMemcpyAsync(hc.data(), coef, sizeof(double2) * hc.size(), hipMemcpyDeviceToHost, s));
      SGN_HIP(hipStreamSynchronize(s));
      std::vector<cplx> G(hc.size());
      for (size_t e = 0; e < G.size(); ++e) G[e] = to_c(hc[e]);
      return G;
    };
    combine(S1->as<double2>(), W1, R);
    std::vector<cplx> W2p((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int r = 0; r < m; ++r) W2p[(size_t)i * m + r] = W2[(size_t)perm[i] * m + r];
    combine(S2->as<double2>(), W2p, L0);
    // L = L0 (L0^dag R)^{-dag}, so that L^dag R = I
    std::vector<cplx> M = gram(L0, R);
    SGN_REQUIRE(invert(m, M), SGN_EDEFL, "LR deflation: left and right eigenvectors are not independent");
    std::vector<cplx> X((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) X[(size_t)j * m + i] = std::conj(M[(size_t)i * m + j]);
    combine(L0, X, L);
    const std::vector<cplx> B = gram(L, R);
    double dev = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) dev = std::max(dev, std::abs(B[(size_t)j * m + i] - (i == j ? 1.0 : 0.0)));
    SGN_REQUIRE(dev <= 1e-8, SGN_EDEFL, "LR deflation: L^dag R deviates from I by " + std::to_string(dev));
    std::vector<double2> lam(m);
    for (int i = 0; i < m; ++i) lam[i] = to_d2(lam1[i]);
    install_lr_pair(c, m, R, L, lam);
    c->defl_restarts = st1.restarts + st2.restarts;
    c->defl_matvecs = st1.matvecs + st2.matvecs;
    c->defl_residual = std::max(st1.residual, st2.residual);
    c->defl_used_degree = std::min(st1.degree, st2.degree);
    c->defl_alpha = st1.alpha;
    c->defl_beta = st1.beta;
    return SGN_OK;
  });
}

extern "C" int sgn_set_deflation_krylov(sgn_ctx* c, int ncv) {
  return guarded(c, [&] {
    SGN_REQUIRE(ncv >= 0, SGN_EINVAL, "ncv must be >= 0 (0: default)");
    c->defl_ncv = ncv;
    return SGN_OK;
  });
}
