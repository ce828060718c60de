"""The 12^4 x 32-source mixed-precision workload as configured, against the
oracle.

12^4 random-link field (seed 20070426), mu = 0.3, m_w = -1.6, the library's
own m = 40 Schur pair (sgn_deflate), sources 1000..1031 in one batched apply,
kmax 400, mixed precision (FP32 stencil and Krylov basis, FP64 elsewhere),
tol 1e-7.  Checks:
  * sources 1000 and 1001 against the oracle's FP64 deflated Arnoldi at
    k = 800 (m = 40 Schur vectors from ARPACK on H_w^2; self-converged to
    1e-8 between k = 700 and 800), stored by make_golden.py: <= 1e-6, the
    mixed-precision target;
  * every source: sgn(H)^2 x = x (the sign applied again, as a second batched
    apply) to 5e-6: two mixed applies at about 1e-7 each, times the norm of
    the non-normal sign.
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

M_W = -1.6
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


def test_12x12_batched_mixed_vs_oracle(env):
    sg, torch = env
    path = os.path.join(GOLDEN, "c12_mu0.3_sources.npy")
    if not os.path.exists(path):
        pytest.skip("golden file c12_mu0.3_sources not generated")
    gold = np.load(path, allow_pickle=False)
    dims, mu, m, nrhs = (12, 12, 12, 12), 0.3, 40, 32
    print("12^4 x 32 mixed: setup", flush=True)
    links = synth.random_links(dims, synth.GAUGE_SEED)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_set_precision(ctx, sg.SGN_PREC_MIXED)
        assert sg.sgn_deflate(ctx, m) == sg.SGN_OK
        print(sg.sgn_deflate_stats(ctx), flush=True)
        X = torch.from_numpy(np.stack([synth.gaussian_source(dims, 1000 + r) for r in range(nrhs)])).cuda()
        Y = torch.empty_like(X)
        print("12^4 x 32 mixed: apply", flush=True)
        st, infos = sg.sgn_apply_batched(ctx, X, Y, 1e-7, 400)
        assert st == sg.SGN_OK and all(i["converged"] for i in infos)
        print("k", sorted({i["k_used"] for i in infos}), flush=True)
        for r in range(gold.shape[0]):
            err = float(np.linalg.norm(Y[r].cpu().numpy() - gold[r]) / np.linalg.norm(gold[r]))
            print("source", 1000 + r, "rel err vs oracle", err, flush=True)
            assert err <= 1e-6
        print("12^4 x 32 mixed: sign applied again", flush=True)
        Z = torch.empty_like(X)
        st, _ = sg.sgn_apply_batched(ctx, Y, Z, 1e-7, 400)
        assert st == sg.SGN_OK
        dev = (torch.linalg.vector_norm(Z - X, dim=1) / torch.linalg.vector_norm(X, dim=1)).cpu().numpy()
        print("max |sgn^2 x - x| / |x|", float(dev.max()), flush=True)
        assert float(dev.max()) <= 5e-6
    finally:
        sg.sgn_destroy(ctx)
