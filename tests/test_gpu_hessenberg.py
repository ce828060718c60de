"""The device composite matrix H = [[T, X], [0, H_k]] (Eq. eq:newH) against the
oracle's, entry by entry, for both orthogonalisation schedules."""
import numpy as np
import pytest

import synth
from oracle import arnoldi, deflation, wilson

pytestmark = pytest.mark.gpu
M_W = -1.6


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


@pytest.mark.parametrize("orth", [0, 1])
@pytest.mark.parametrize("m", [0, 6])
@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_hessenberg_matches_oracle(env, orth, m, k):
    sg, torch = env
    dims, mu = (2, 2, 2, 4), 0.3
    links = synth.random_links(dims, 44)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    x = synth.gaussian_source(dims, 7)
    S = T = None
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_set_orthogonalization(ctx, orth)
        if m:
            S, T, _, _ = deflation.critical_from_dense(A.toarray(), m)
            sg.sgn_deflate_import(ctx, torch.from_numpy(S).cuda(), T)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        sg.sgn_apply_fixed(ctx, torch.from_numpy(x).cuda(), y, k)
        n = m + k
        Hg, c0g, bg = sg.sgn_debug_hessenberg(ctx, n, m)
        st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, k)
        Hc = arnoldi.composite_h(T if m else np.zeros((0, 0)), st)
        d = np.abs(Hg - Hc)
        if orth == 1:
            d[:, n - 1] = 0  # last column gets its re-orthogonalisation on a copy
        np.set_printoptions(precision=3, linewidth=200)
        print("\north", orth, "m", m, "k", k, "beta", bg, st.beta, "\n", d.max(axis=0))
        assert abs(bg - st.beta) < 1e-12 * st.beta
        if m:
            assert np.abs(c0g - st.c0).max() < 1e-12
        assert d.max() < 1e-12
    finally:
        sg.sgn_destroy(ctx)
