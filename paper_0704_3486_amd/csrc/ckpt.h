// Checkpoint placement and stopping rule of the Krylov loop, shared by the
// single-source, batched and session drivers.
//
// The small-matrix sign (step (v)) is evaluated at even Krylov dimensions
// only (Section 4: odd k see-saws).  At a checkpoint k with a previous one at
// k' the drivers know the change of y over the span, e = |y_k - y_k'| / |y_k|
// (exact, because Q has orthonormal columns).  The paper measures only the
// error against the exact y; the stopping rule is this library's:
//   * geometric error model err(k) ~ A exp(r k), r < 0, fitted to the
//     changes of the last two spans;
//   * under it e = err(k') (1 - q) with q = exp(r (k - k')), so
//     bound = e / (1 - q) estimates the error of the earlier checkpoint k';
//   * a result is accepted when bound <= tol: the earlier checkpoint is
//     certified, and the returned y_k is a factor q more accurate still.
// A confirming checkpoint is placed so that q <= 1/2 (bound <= 2 e).  With
// no rate known yet q = 1/2 is assumed; a history whose changes do not fall
// certifies nothing (the apply then runs to kmax).
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

struct CkSpan {
  int a, b;   // checkpoints k' < k
  double e;   // change of y between them
};

struct CkModel {
  std::vector<CkSpan> hist;

  static int even_up(int k) { return (k + 1) & ~1; }

  // change over [a, a + d] relative to the error at a: 1 - exp(r d)
  static double drop(double r, int d) { return -std::expm1(r * (double)d); }

  // rate of the model from the last two spans: solves
  //   e2 / e1 = exp(r (a2 - a1)) (1 - exp(r d2)) / (1 - exp(r d1))
  // for r < 0 by bisection on [-8, -1e-9].  The right side rises
  // monotonically to d2 / d1 as r -> 0; changes that fall less than that
  // (the error does not decrease) give a positive rate (no convergence).
  // Returns fallback with fewer than two spans.
  double rate(double fallback) const {
    if (hist.size() < 2) return fallback;
    const CkSpan& s1 = hist[hist.size() - 2];
    const CkSpan& s2 = hist[hist.size() - 1];
    if (!(s1.e > 0.0) || !(s2.e > 0.0) || s2.a <= s1.a) return fallback;
    const double target = std::log(s2.e / s1.e);
    auto f = [&](double r) {
      return r * (double)(s2.a - s1.a) + std::log(drop(r, s2.b - s2.a)) - std::log(drop(r, s1.b - s1.a)) - target;
    };
    double lo = -8.0, hi = -1e-9;
    if (f(hi) < 0.0) return 1e-3;  // not converging
    if (f(lo) > 0.0) return lo;
    for (int it = 0; it < 80; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (f(mid) > 0.0)
        hi = mid;
      else
        lo = mid;
    }
    return 0.5 * (lo + hi);
  }

  // the rate predicts where the error falls (placement of checkpoints)
  static bool usable(double r) { return r < -1e-6 && std::isfinite(r); }

  // estimated error at the earlier checkpoint of a span of d steps with
  // change e: e / (1 - exp(r d)); no rate known (r = 0): q = 1/2 assumed;
  // a rate >= 0 (the error does not fall) certifies nothing
  static double bound(double e, int d, double r) {
    if (r == 0.0) return 2.0 * e;
    if (!(r < 0.0)) return HUGE_VAL;
    const double dq = drop(r, d);
    return dq > 0.0 ? e / dq : HUGE_VAL;
  }

  // span of a confirming checkpoint: exp(r span) <= 1/2
  static int confirm_span(double r) {
    if (!usable(r)) return 8;
    const double d = std::ceil(std::log(2.0) / -r);
    return even_up(std::max(4, (int)std::min(d, 1e6)));
  }

  // next checkpoint after k (no convergence yet).  hinted_first: k is the
  // first checkpoint of an apply that starts where an earlier one on the
  // field was certified, so the next one confirms it.
  int next(int k, int kmax, double tol, double r, bool hinted_first) const {
    int nk;
    if (hist.empty() && hinted_first) {
      nk = k + confirm_span(r);
    } else if (!hist.empty() && usable(r)) {
      // error at k under the model, then the k where it reaches tol (5 % margin)
      const CkSpan& s = hist.back();
      const double q = std::min(std::exp(r * (double)(s.b - s.a)), 0.999);
      const double ek = s.e * q / (1.0 - q);
      const double steps = std::log(tol / std::max(ek, 1e-300)) / r;
      const int target = k + (int)std::ceil(1.05 * std::max(steps, 0.0));
      nk = (target <= k) ? k + confirm_span(r) : std::max(target, k + 2);
    } else {
      nk = k + std::max(8, k / 2);
    }
    // the model is fitted on early checkpoints, where the error often falls
    // more slowly than later; a jump that would land on kmax leaves no later
    // checkpoint to certify the result against, so such a jump goes at most
    // as far again as the steps already taken
    if (nk >= kmax) nk = std::min(nk, 2 * k + 8);
    return std::min(kmax, even_up(std::max(nk, k + 2)));
  }
};
