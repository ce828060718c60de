"""Host logic of the checkpoint placement and stopping rule (csrc/ckpt.h).

A small C++ driver includes the header and runs the rule against synthetic
error histories err(k) = A exp(r k) (the geometric model the rule assumes),
with and without a perturbation of the rate.  The change of y between two
checkpoints is then err(k') - err(k) (the Krylov approximations move towards
the exact result).  The checks:
  * the rate fitted from two spans of different lengths is the true rate;
  * a result is accepted only once the error of the checkpoint before the
    last is at most tol, so the returned error is below tol;
  * a confirming span halves the error (q <= 1/2);
  * a hinted start (first checkpoint where an earlier source was certified)
    confirms after one span.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0704_3486_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include "ckpt.h"

// error history: err(k) = A exp(r k) for k < kb, then exp(r2 (k - kb)) slower
static double err_at(double A, double r, double r2, int kb, int k) {
  if (k <= kb) return A * std::exp(r * k);
  return A * std::exp(r * kb) * std::exp(r2 * (k - kb));
}

int main(int argc, char** argv) {
  const double A = atof(argv[1]), r = atof(argv[2]), r2 = atof(argv[3]), tol = atof(argv[4]);
  const int kb = atoi(argv[5]), kmax = atoi(argv[6]), k_hint = atoi(argv[7]);
  const double rate_hint = atof(argv[8]);
  CkModel model;
  int k = k_hint > 0 ? k_hint : 32, prev = -1, nck = 0;
  double fitted = 0.0;
  for (;;) {
    ++nck;
    const double ek = err_at(A, r, r2, kb, k);
    double rate = rate_hint;
    if (prev >= 0) {
      const double e = err_at(A, r, r2, kb, prev) - ek;  // change of y over the span
      model.hist.push_back(CkSpan{prev, k, e});
      rate = model.rate(rate_hint);
      if (model.hist.size() >= 2) fitted = rate;
      if (CkModel::bound(e, k - prev, rate) <= tol) {
        printf("accept k=%d prev=%d err=%.6e err_prev=%.6e fitted=%.8f nck=%d\n", k, prev, ek,
               err_at(A, r, r2, kb, prev), fitted, nck);
        return 0;
      }
    }
    if (k >= kmax) {
      printf("noconv k=%d err=%.6e nck=%d\n", k, ek, nck);
      return 0;
    }
    const int nk = model.next(k, kmax, tol, rate, k_hint > 0 && model.hist.empty());
    prev = k;
    k = nk;
  }
}
"""


@pytest.fixture(scope="module")
def driver():
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "drv.cpp")
    exe = os.path.join(d, "drv")
    with open(src, "w") as f:
        f.write(DRIVER)
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", CSRC, src, "-o", exe], check=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def run(exe, A=1.0, r=-0.07, r2=None, tol=1e-10, kb=10**6, kmax=2000, k_hint=0, rate_hint=0.0):
    r2 = r if r2 is None else r2
    out = subprocess.run([exe, repr(A), repr(r), repr(r2), repr(tol), str(kb), str(kmax), str(k_hint),
                          repr(rate_hint)], check=True, capture_output=True, text=True).stdout.split()
    kv = dict(t.split("=") for t in out[1:])
    return out[0], {k: float(v) for k, v in kv.items()}


@pytest.mark.parametrize("r", [-0.02, -0.07, -0.15])
def test_geometric_history_is_accepted_below_tol(driver, r):
    status, v = run(driver, r=r)
    assert status == "accept"
    assert v["err_prev"] <= 1e-10 * 1.0000001  # the certified checkpoint
    assert v["err"] <= 0.5 * 1e-10 * 1.0000001  # the returned result: one confirming span further
    assert abs(v["fitted"] - r) <= 1e-6 * abs(r)


def test_hinted_start_confirms_after_one_span(driver):
    r, tol = -0.07, 1e-10
    k_cert = int(__import__("math").ceil(__import__("math").log(tol) / r))  # err(k_cert) <= tol
    status, v = run(driver, r=r, tol=tol, k_hint=k_cert + (k_cert & 1), rate_hint=r)
    assert status == "accept" and v["nck"] == 2
    assert v["err"] <= 0.5 * tol * 1.0000001


def test_hinted_start_on_a_harder_source_needs_more(driver):
    # the remembered k suits a faster source: the rule must not accept early
    r, tol = -0.06, 1e-10
    status, v = run(driver, r=r, tol=tol, k_hint=330, rate_hint=-0.07)
    assert status == "accept"
    assert v["err_prev"] <= tol * 1.0000001 and v["err"] <= tol


def test_slowdown_after_the_fit_is_not_accepted_early(driver):
    # the error falls fast, then slows to a third of the rate: the bound must
    # still certify a checkpoint whose true error is <= tol
    status, v = run(driver, r=-0.09, r2=-0.03, kb=150, tol=1e-10)
    assert status == "accept"
    assert v["err_prev"] <= 1e-10 * 1.0000001


def test_no_decrease_ends_at_kmax(driver):
    # changes that do not fall (an error that stays put) certify nothing
    status, v = run(driver, r=-1e-9, tol=1e-12, kmax=600)
    assert status == "noconv"
