// Small dense complex linear algebra on the host, used by the deflation setup
// (Section 5.2, step (i)) for the Rayleigh-Ritz problems of size <= a few
// hundred: Hessenberg reduction by Householder reflections, the implicit
// single-shift QR algorithm with Wilkinson shifts (complex Schur form
// A = Z T Z^H), eigenvectors of the triangular factor by back substitution,
// and a thin QR factorisation (modified Gram-Schmidt, applied twice).
#include "hostla.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace hostla {

namespace {

inline double abs1(cplx z) { return std::abs(z.real()) + std::abs(z.imag()); }

// Givens rotation G = [[c, s], [-conj(s), c]] with G (x, y)^T = (r, 0)^T.
inline void givens(cplx x, cplx y, double& c, cplx& s) {
  const double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  if (ax == 0.0) {
    c = 0.0;
    s = std::conj(y) / ay;
    return;
  }
  const double nrm = std::hypot(ax, ay);
  c = ax / nrm;
  s = (x / ax) * std::conj(y) / nrm;
}

}  // namespace

// A (n x n, column-major) -> upper Hessenberg H = Q^H A Q (in place), Q accumulated.
void hessenberg(int n, cplx* H, cplx* Q) {
  auto h = [&](int i, int j) -> cplx& { return H[(size_t)j * n + i]; };
  auto q = [&](int i, int j) -> cplx& { return Q[(size_t)j * n + i]; };
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) q(i, j) = (i == j) ? 1.0 : 0.0;
  std::vector<cplx> v(n), tmp(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    double xn = 0.0;
    for (int i = 0; i < len; ++i) xn += std::norm(h(k + 1 + i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cplx x0 = h(k + 1, k);
    const cplx ph = (std::abs(x0) > 0.0) ? x0 / std::abs(x0) : cplx(1.0, 0.0);
    const cplx alpha = -ph * xn;
    for (int i = 0; i < len; ++i) v[i] = h(k + 1 + i, k);
    v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < len; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    const double tau = 2.0 / vn;
    // left: H[k+1:, k:] -= tau v (v^H H[k+1:, k:])
    for (int j = k; j < n; ++j) {
      cplx s = 0.0;
      for (int i = 0; i < len; ++i) s += std::conj(v[i]) * h(k + 1 + i, j);
      s *= tau;
      for (int i = 0; i < len; ++i) h(k + 1 + i, j) -= v[i] * s;
    }
    // right: H[:, k+1:] -= tau (H[:, k+1:] v) v^H ; same for Q
    for (int i = 0; i < n; ++i) {
      cplx s = 0.0;
      for (int l = 0; l < len; ++l) s += h(i, k + 1 + l) * v[l];
      s *= tau;
      for (int l = 0; l < len; ++l) h(i, k + 1 + l) -= s * std::conj(v[l]);
      cplx t = 0.0;
      for (int l = 0; l < len; ++l) t += q(i, k + 1 + l) * v[l];
      t *= tau;
      for (int l = 0; l < len; ++l) q(i, k + 1 + l) -= t * std::conj(v[l]);
    }
    for (int i = 2; i <= len; ++i) h(k + i, k) = 0.0;
  }
}

// Hessenberg H -> Schur form T (in place), Z updated so that A = Z T Z^H.
bool schur_from_hessenberg(int n, cplx* H, cplx* Z) {
  auto h = [&](int i, int j) -> cplx& { return H[(size_t)j * n + i]; };
  auto z = [&](int i, int j) -> cplx& { return Z[(size_t)j * n + i]; };
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = n - 1;
  int iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      const double s = abs1(h(l - 1, l - 1)) + abs1(h(l, l));
      if (abs1(h(l, l - 1)) <= eps * (s > 0 ? s : 1.0)) {
        h(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 100 * n) return false;
    ++iter;
    // Wilkinson shift from the trailing 2x2 block
    cplx mu;
    if (iter % 11 == 10) {
      mu = h(hi, hi) + cplx(std::abs(h(hi, hi - 1).real()) + std::abs(h(hi, hi - 1).imag()), 0.0);
    } else {
      const cplx a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
      const cplx half = 0.5 * (a - d);
      const cplx disc = std::sqrt(half * half + b * c);
      const cplx m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
    }
    // implicit QR sweep on the active block l..hi (bulge chase with Givens)
    cplx x = h(l, l) - mu, y = h(l + 1, l);
    for (int k = l; k < hi; ++k) {
      double c;
      cplx s;
      givens(x, y, c, s);
      const int jc = (k > l) ? k - 1 : l;
      for (int j = jc; j < n; ++j) {  // rows k, k+1
        const cplx a = h(k, j), b = h(k + 1, j);
        h(k, j) = c * a + s * b;
        h(k + 1, j) = -std::conj(s) * a + c * b;
      }
      const int ir = std::min(k + 2, hi);
      for (int i = 0; i <= ir; ++i) {  // columns k, k+1
        const cplx a = h(i, k), b = h(i, k + 1);
        h(i, k) = c * a + std::conj(s) * b;
        h(i, k + 1) = -s * a + c * b;
      }
      for (int i = 0; i < n; ++i) {
        const cplx a = z(i, k), b = z(i, k + 1);
        z(i, k) = c * a + std::conj(s) * b;
        z(i, k + 1) = -s * a + c * b;
      }
      if (k > l) h(k + 1, k - 1) = 0.0;
      if (k + 1 < hi) {
        x = h(k + 1, k);
        y = h(k + 2, k);
      }
    }
  }
  // clean the strictly lower part
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) h(i, j) = 0.0;
  return true;
}

bool eig(int n, const cplx* A, cplx* w, cplx* V) {
  std::vector<cplx> T(A, A + (size_t)n * n), Z((size_t)n * n);
  hessenberg(n, T.data(), Z.data());
  if (!schur_from_hessenberg(n, T.data(), Z.data())) return false;
  auto t = [&](int i, int j) -> cplx& { return T[(size_t)j * n + i]; };
  double tn = 0.0;
  for (auto& v : T) tn = std::max(tn, std::abs(v));
  const double small = std::numeric_limits<double>::epsilon() * (tn > 0 ? tn : 1.0);
  std::vector<cplx> X((size_t)n * n, cplx(0.0, 0.0));
  for (int i = 0; i < n; ++i) {
    w[i] = t(i, i);
    cplx* x = &X[(size_t)i * n];
    x[i] = 1.0;
    for (int j = i - 1; j >= 0; --j) {
      cplx s = 0.0;
      for (int l = j + 1; l <= i; ++l) s += t(j, l) * x[l];
      cplx d = t(j, j) - t(i, i);
      if (std::abs(d) < small) d = small;
      x[j] = -s / d;
    }
  }
  // V = Z X, unit columns
  for (int i = 0; i < n; ++i) {
    double nn = 0.0;
    for (int r = 0; r < n; ++r) {
      cplx s = 0.0;
      for (int l = 0; l <= i; ++l) s += Z[(size_t)l * n + r] * X[(size_t)i * n + l];
      V[(size_t)i * n + r] = s;
      nn += std::norm(s);
    }
    nn = std::sqrt(nn);
    for (int r = 0; r < n; ++r) V[(size_t)i * n + r] /= nn;
  }
  return true;
}

int thin_qr(int rows, int cols, cplx* A, double rank_tol) {
  auto a = [&](int i, int j) -> cplx& { return A[(size_t)j * rows + i]; };
  int rank = 0;
  for (int j = 0; j < cols; ++j) {
    double n0 = 0.0;
    for (int i = 0; i < rows; ++i) n0 += std::norm(a(i, j));
    n0 = std::sqrt(n0);
    for (int pass = 0; pass < 2; ++pass) {
      for (int k = 0; k < j; ++k) {
        cplx s = 0.0;
        for (int i = 0; i < rows; ++i) s += std::conj(a(i, k)) * a(i, j);
        for (int i = 0; i < rows; ++i) a(i, j) -= s * a(i, k);
      }
    }
    double nn = 0.0;
    for (int i = 0; i < rows; ++i) nn += std::norm(a(i, j));
    nn = std::sqrt(nn);
    if (nn <= rank_tol * (n0 > 0 ? n0 : 1.0)) {
      for (int i = 0; i < rows; ++i) a(i, j) = 0.0;
      continue;
    }
    for (int i = 0; i < rows; ++i) a(i, j) /= nn;
    ++rank;
  }
  return rank;
}

}  // namespace hostla

extern "C" int sgn_host_eig(int n, const double* A, double* w, double* V) {
  if (n < 1 || !A || !w || !V) return -1;
  try {
    const auto* a = reinterpret_cast<const hostla::cplx*>(A);
    return hostla::eig(n, a, reinterpret_cast<hostla::cplx*>(w), reinterpret_cast<hostla::cplx*>(V)) ? 0 : -5;
  } catch (...) {
    return -2;
  }
}
