"""Write the stored exact results used by the full-size parity tests.

Calls only the oracle (and the seeded input generators).  For each case it
stores y = sgn(H_w(mu)) x for the Gaussian source x of seed 1000:
  * 4^4, mu = 0.3       -- spectral definition (full eigendecomposition)
  * 6^4, mu = 0.0       -- Hermitian eigh route
  * 6^4, mu = 0.2, 0.5  -- dense Roberts iteration (Eq. Roberts) on H_w
Each file is checked for sgn(A)^2 = I on the stored vector (|sgn(A) y - x|)
and the 4^4 case also against Roberts.  Output: c<L>_mu<mu>.npy plus
golden_meta.json with the self-checks.

Run from the repository root:  python tests/golden/make_golden.py [case ...]
The 6^4 cases each take tens of minutes on 8 cores and ~12 GB of memory.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import matfunc, wilson  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
M_W = -1.6
SOURCE_SEED = 1000

CASES = {
    "c4_mu0.3": ((4, 4, 4, 4), 0.3, "spectral"),
    "c6_mu0.0": ((6, 6, 6, 6), 0.0, "eigh"),
    "c6_mu0.2": ((6, 6, 6, 6), 0.2, "roberts"),
    "c6_mu0.5": ((6, 6, 6, 6), 0.5, "roberts"),
    "c8_mu0.3": ((8, 8, 8, 8), 0.3, "arnoldi800"),
}


def run_case(name):
    dims, mu, how = CASES[name]
    links = synth.random_links(dims, synth.GAUGE_SEED)
    x = synth.gaussian_source(dims, SOURCE_SEED)
    t0 = time.time()
    if how == "arnoldi800":
        return run_arnoldi_case(name, dims, mu, links, x)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    meta = {"dims": dims, "mu": mu, "m_w": M_W, "gauge_seed": synth.GAUGE_SEED,
            "source_seed": SOURCE_SEED, "method": how}
    if how == "spectral":
        lam, R = np.linalg.eig(A)
        y = R @ (np.sign(lam.real) * np.linalg.solve(R, x))
        Sg = (R * np.sign(lam.real)) @ np.linalg.inv(R)
        Sr, it = matfunc.sgn_roberts(A)
        meta["roberts_vs_spectral"] = float(np.linalg.norm(Sr @ x - y) / np.linalg.norm(y))
        meta["roberts_iterations"] = it
        meta["min_abs_re_lambda"] = float(np.min(np.abs(lam.real)))
        meta["cond_eigvecs"] = float(np.linalg.cond(R))
    elif how == "eigh":
        w, W = np.linalg.eigh(A)
        y = W @ (np.sign(w) * (W.conj().T @ x))
        Sg = (W * np.sign(w)) @ W.conj().T
        meta["min_abs_lambda"] = float(np.min(np.abs(w)))
    else:
        Sg, it = matfunc.sgn_roberts(A)
        y = Sg @ x
        meta["roberts_iterations"] = it
    meta["sgn2_residual"] = float(np.linalg.norm(Sg @ y - x) / np.linalg.norm(x))
    meta["seconds"] = time.time() - t0
    np.save(os.path.join(HERE, f"{name}.npy"), y, allow_pickle=False)
    return meta


def run_arnoldi_case(name, dims, mu, links, x):
    """No dense oracle fits at 8^4: the oracle's FP64 deflated Arnoldi at k = 800
    (m = 30, deflation basis from ARPACK on H_w^2), required to be self-converged."""
    from oracle import arnoldi, deflation

    t0 = time.time()
    A = wilson.hw_matrix(links, dims, mu, M_W)
    S, T, theta, low = deflation.critical_from_arpack(A, 30)
    st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, 800)
    y800 = arnoldi.approx_definition(S, T, st)
    sub = arnoldi.ArnoldiState(st.V[:, :701], st.Hbar[:701, :700], st.X[:, :700], st.beta, st.c0, 700, False)
    y700 = arnoldi.approx_definition(S, T, sub)
    self_conv = float(np.linalg.norm(y800 - y700) / np.linalg.norm(y800))
    assert self_conv <= 1e-8, self_conv
    np.save(os.path.join(HERE, f"{name}.npy"), y800, allow_pickle=False)
    return {"dims": dims, "mu": mu, "m_w": M_W, "gauge_seed": synth.GAUGE_SEED, "source_seed": SOURCE_SEED,
            "method": "oracle deflated Arnoldi, m=30 (ARPACK), k=800", "self_convergence_700_800": self_conv,
            "schur_residual": deflation.schur_residual(A, S, T), "seconds": time.time() - t0}


def main(names):
    path = os.path.join(HERE, "golden_meta.json")
    allmeta = {}
    if os.path.exists(path):
        with open(path) as f:
            allmeta = json.load(f)
    for name in names:
        print("case", name, flush=True)
        allmeta[name] = run_case(name)
        print(json.dumps(allmeta[name]), flush=True)
        with open(path, "w") as f:
            json.dump(allmeta, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
