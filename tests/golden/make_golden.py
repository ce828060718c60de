"""Write the stored exact results used by the full-size parity tests.

Calls only the oracle (and the seeded input generators).  For each case it
stores y = sgn(H_w(mu)) x for the Gaussian source x of seed 1000:
  * 4^4, mu = 0.3       -- spectral definition (full eigendecomposition)
  * 6^4, mu = 0.0       -- Hermitian eigh route
  * 6^4, mu = 0.2, 0.5  -- dense Roberts iteration (Eq. Roberts) on H_w
Each file is checked for sgn(A)^2 = I on the stored vector (|sgn(A) y - x|)
and the 4^4 case also against Roberts.  Output: c<L>_mu<mu>.npy plus
golden_meta.json with the self-checks.

Two further kinds of case store several sources at once (rows r = 0, 1, ...
hold y for the Gaussian source of seed 1000 + r):
  * c6s_mu<mu>  -- 6^4, dense Roberts, sources 1000..1015
                   (c6_mu<mu>_sources.npy, shape (16, N)); row 0 is also
                   compared with the single-source file of the same field;
  * c12_mu0.3   -- 12^4, the oracle's FP64 deflated Arnoldi at k = 800 with
                   m = 40 Schur vectors from ARPACK on H_w^2, sources 1000 and
                   1001 (c12_mu0.3_sources.npy, shape (2, N)), each required
                   to be self-converged (|y_800 - y_700| / |y_800| <= 1e-8).

Run from the repository root:  python tests/golden/make_golden.py [case ...]
The 6^4 cases each take tens of minutes on 8 cores and ~12 GB of memory; the
12^4 case a few hours (its two sources run in two processes).
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
    "c6s_mu0.0": ((6, 6, 6, 6), 0.0, "roberts_sources"),
    "c6s_mu0.2": ((6, 6, 6, 6), 0.2, "roberts_sources"),
    "c6s_mu0.5": ((6, 6, 6, 6), 0.5, "roberts_sources"),
    "c12_mu0.3": ((12, 12, 12, 12), 0.3, "arnoldi800_m40"),
}

#: sources of the multi-source cases (seeds 1000 + r)
N_SOURCES_6 = 16
N_SOURCES_12 = 2


def run_case(name):
    dims, mu, how = CASES[name]
    links = synth.random_links(dims, synth.GAUGE_SEED)
    x = synth.gaussian_source(dims, SOURCE_SEED)
    t0 = time.time()
    if how == "arnoldi800":
        return run_arnoldi_case(name, dims, mu, links, x)
    if how == "arnoldi800_m40":
        return run_arnoldi_sources_case(name, dims, mu, links)
    if how == "roberts_sources":
        return run_roberts_sources_case(name, dims, mu, links)
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


def run_roberts_sources_case(name, dims, mu, links):
    """Dense Roberts iteration (Eq. Roberts) on H_w; y for N_SOURCES_6 sources."""
    t0 = time.time()
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    Sg, it = matfunc.sgn_roberts(A)
    del A
    X = np.stack([synth.gaussian_source(dims, SOURCE_SEED + r) for r in range(N_SOURCES_6)])
    Y = (Sg @ X.T).T
    sgn2 = [float(np.linalg.norm(Sg @ Y[r] - X[r]) / np.linalg.norm(X[r])) for r in range(N_SOURCES_6)]
    meta = {"dims": dims, "mu": mu, "m_w": M_W, "gauge_seed": synth.GAUGE_SEED,
            "source_seeds": [SOURCE_SEED, SOURCE_SEED + N_SOURCES_6 - 1], "method": "roberts",
            "roberts_iterations": it, "sgn2_residual_max": max(sgn2)}
    single = os.path.join(HERE, f"c6_mu{mu}.npy")
    if os.path.exists(single):
        y0 = np.load(single, allow_pickle=False)
        meta["row0_vs_single_source_file"] = float(np.linalg.norm(Y[0] - y0) / np.linalg.norm(y0))
    meta["seconds"] = time.time() - t0
    np.save(os.path.join(HERE, f"c6_mu{mu}_sources.npy"), Y, allow_pickle=False)
    return meta


_SHARED = {}  # operator and Schur pair of the 12^4 case, inherited by the forked workers


def _arnoldi_800(x):
    """One source of the 12^4 case: y_800 and its self-convergence against y_700."""
    from oracle import arnoldi

    A, S, T = _SHARED["A"], _SHARED["S"], _SHARED["T"]
    st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, 800)
    y800 = arnoldi.approx_definition(S, T, st)
    sub = arnoldi.ArnoldiState(st.V[:, :701], st.Hbar[:701, :700], st.X[:, :700], st.beta, st.c0, 700, False)
    y700 = arnoldi.approx_definition(S, T, sub)
    return y800, float(np.linalg.norm(y800 - y700) / np.linalg.norm(y800))


def run_arnoldi_sources_case(name, dims, mu, links):
    """12^4: the oracle's FP64 deflated Arnoldi at k = 800 (m = 40 from ARPACK on
    H_w^2) for sources 1000 and 1001, one process per source."""
    import multiprocessing as mp

    from oracle import deflation

    t0 = time.time()
    A = wilson.hw_matrix(links, dims, mu, M_W)
    S, T, theta, low = deflation.critical_from_arpack(A, 40)
    t_defl = time.time() - t0
    xs = [synth.gaussian_source(dims, SOURCE_SEED + r) for r in range(N_SOURCES_12)]
    _SHARED.update(A=A, S=S, T=T)
    with mp.get_context("fork").Pool(N_SOURCES_12) as pool:
        out = pool.map(_arnoldi_800, xs)
    for _, sc in out:
        assert sc <= 1e-8, sc
    np.save(os.path.join(HERE, f"{name}_sources.npy"), np.stack([y for y, _ in out]), allow_pickle=False)
    return {"dims": dims, "mu": mu, "m_w": M_W, "gauge_seed": synth.GAUGE_SEED,
            "source_seeds": [SOURCE_SEED, SOURCE_SEED + N_SOURCES_12 - 1],
            "method": "oracle deflated Arnoldi, m=40 (ARPACK), k=800",
            "self_convergence_700_800": [sc for _, sc in out],
            "schur_residual": deflation.schur_residual(A, S, T), "schur_lower_part": low,
            "deflation_seconds": t_defl, "seconds": time.time() - t0}


def main(names):
    path = os.path.join(HERE, "golden_meta.json")
    allmeta = {}
    if os.path.exists(path):
        with open(path) as f:
            allmeta = json.load(f)
    for name in names:
        print("case", name, flush=True)
        meta = run_case(name)
        print(json.dumps(meta), flush=True)
        # other cases may have been written meanwhile by another process
        if os.path.exists(path):
            with open(path) as f:
                allmeta = json.load(f)
        allmeta[name] = meta
        with open(path, "w") as f:
            json.dump(allmeta, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
