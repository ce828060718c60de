"""Lattices beyond the dense oracle (12^4, N = 248832).

A pure-gauge field U_{n,nu} = Omega_n Omega_{n+nu}^dag is a gauge rotation of
U = 1, so sgn(H[U]) (Omega x) = Omega sgn(H[1]) x exactly, and sgn(H[1]) has
a closed form per momentum (oracle.freefield).  Its spectrum at 12^4 keeps
|Re lambda| >= 0.17, so the Krylov method converges without deflation (its
eigenvalues are highly degenerate, so a small Schur basis would cut through
degenerate eigenspaces of H_w^2; sgn_deflate rejects such a basis).
"""
import numpy as np
import pytest

import synth
from oracle import freefield

pytestmark = pytest.mark.gpu

M_W = -1.6
DIMS = (12, 12, 12, 12)
MU = 0.3


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


@pytest.fixture(scope="module")
def pure_gauge():
    om = synth.random_su3_field(DIMS, 21)
    X = np.stack([synth.gaussian_source(DIMS, 1000 + r) for r in range(4)])
    exact = np.stack([synth.gauge_transform_spinor(om, freefield.sgn_free_apply(x, DIMS, MU, M_W)) for x in X])
    Xg = np.stack([synth.gauge_transform_spinor(om, x) for x in X])
    return synth.pure_gauge_links(om), Xg, exact


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_fp64_apply_12x12_pure_gauge(env, pure_gauge):
    sg, torch = env
    links, Xg, exact = pure_gauge
    print("12^4 fp64", flush=True)
    ctx = sg.sgn_create(links, DIMS, MU, M_W)
    try:
        x = torch.from_numpy(Xg[0]).cuda()
        y = torch.empty_like(x)
        # the free-field Krylov error drops abruptly once the distinct
        # eigenvalues are captured, so certifying it needs room past that k
        st = sg.sgn_apply(ctx, x, y, 1e-11, 1200)
        info = sg.sgn_last_info(ctx)
        err = _rel(y.cpu().numpy(), exact[0])
        print(info, err, flush=True)
        assert st == sg.SGN_OK and err < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def test_batched_mixed_12x12_pure_gauge(env, pure_gauge):
    """The batched mixed-precision path (several sources per launch) at 12^4:
    every source within the 1e-6 mixed-precision target of the exact result."""
    sg, torch = env
    links, Xg, exact = pure_gauge
    print("12^4 batched mixed", flush=True)
    ctx = sg.sgn_create(links, DIMS, MU, M_W)
    try:
        sg.sgn_set_precision(ctx, sg.SGN_PREC_MIXED)
        X = torch.from_numpy(Xg).cuda()
        Y = torch.empty_like(X)
        st, infos = sg.sgn_apply_batched(ctx, X, Y, 1e-7, 1000)
        errs = [_rel(Y[r].cpu().numpy(), exact[r]) for r in range(Xg.shape[0])]
        print([i["k_used"] for i in infos], errs, flush=True)
        assert st == sg.SGN_OK
        assert max(errs) < 1e-6
    finally:
        sg.sgn_destroy(ctx)
