"""GPU parity of the HIP path against the oracle, element by element.

Tolerance (FP64): relative 2-norm error <= 1e-10 for sgn(H)x, the bound the
method is specified to meet; building blocks are held to tighter bounds
derived from their arithmetic (stencil: summation order only, 1e-14).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import arnoldi, deflation, freefield, matfunc, wilson

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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def _make(sg, dims, mu, seed):
    links = synth.random_links(dims, seed)
    return links, sg.sgn_create(links, dims, mu, M_W)


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (3, 3, 3, 3), (4, 2, 6, 4), (4, 4, 4, 4), (6, 6, 6, 6)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_matvec_matches_oracle(env, dims, mu):
    sg, torch = env
    print("matvec", dims, mu, flush=True)
    links, ctx = _make(sg, dims, mu, 17)
    try:
        x = synth.gaussian_source(dims, 3)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        sg.sgn_matvec(ctx, _dev(torch, x), y)
        ref = wilson.hw_matrix(links, dims, mu, M_W) @ x
        assert _rel(y.cpu().numpy(), ref) < 1e-14
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("dims", [(16, 16, 16, 16), (20, 16, 16, 16), (16, 8, 32, 16), (24, 24, 24, 28)])
def test_matvec_large_pure_gauge(env, dims):
    """Lattices large enough for the blocked site order of the stencil: no
    dense oracle fits, so the exact relation H[U] (Omega x) = Omega H[1] x for
    pure-gauge links U = Omega_n Omega_{n+nu}^dag (H[1] by FFT) is checked."""
    sg, torch = env
    print("matvec pure gauge", dims, flush=True)
    om = synth.random_su3_field(dims, 11)
    ctx = sg.sgn_create(synth.pure_gauge_links(om), dims, 0.3, M_W)
    try:
        x = synth.gaussian_source(dims, 4)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        sg.sgn_matvec(ctx, _dev(torch, synth.gauge_transform_spinor(om, x)), y)
        ref = synth.gauge_transform_spinor(om, freefield.h_free_apply(x, dims, 0.3, M_W))
        assert _rel(y.cpu().numpy(), ref) < 1e-13
    finally:
        sg.sgn_destroy(ctx)


def _test_matrix(n, seed, tri=False, spread=0.3):
    rng = np.random.default_rng(seed)
    re = rng.uniform(0.2, 2.0, n) * np.where(rng.random(n) < 0.5, -1, 1)
    lam = re + 1j * spread * rng.uniform(-1.0, 1.0, n)
    if tri:
        return np.triu(0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))), 1) + np.diag(lam)
    R = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    return R @ np.diag(lam) @ np.linalg.inv(R)


@pytest.mark.parametrize("method", [0, 1])  # Newton-Schulz (with fallback), Roberts/Gauss-Jordan
@pytest.mark.parametrize("n,tri,spread", [(1, False, 0.3), (5, False, 0.3), (37, False, 0.3), (128, False, 0.3),
                                          (300, False, 0.3), (20, True, 0.3), (577, False, 0.3),
                                          (64, False, 0.05), (300, False, 0.05), (833, False, 0.05)])
def test_dense_sign_matches_oracle(env, n, tri, spread, method):
    # spread = |Im| / |Re| scale of the eigenvalues; 0.3 with |Re| down to 0.2 puts
    # some outside the Newton-Schulz region (exercising the fallback), 0.05 does not
    sg, torch = env
    print("dense sign", n, tri, spread, method, flush=True)
    links, ctx = _make(sg, (2, 2, 2, 2), 0.0, 1)
    sg.sgn_set_sign_method(ctx, method)
    try:
        A = _test_matrix(n, n, tri, spread)
        Ad = _dev(torch, A.T.copy())  # column-major
        Fd = torch.empty_like(Ad)
        it = sg.sgn_dense_sign(ctx, Ad, Fd)
        F = Fd.cpu().numpy().T
        ref = matfunc.sgn_spectral(A)
        assert np.linalg.norm(F - ref) / np.linalg.norm(ref) < 1e-11
        assert it < 70
        if tri:
            assert np.abs(np.tril(F, -1)).max() < 1e-13
    finally:
        sg.sgn_destroy(ctx)


@pytest.fixture(scope="module")
def small_problem():
    dims = (3, 3, 3, 4)
    mu = 0.3
    links = synth.random_links(dims, 32)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    S, T, lam, low = deflation.critical_from_dense(A.toarray(), 12)
    x = synth.gaussian_source(dims, 1001)
    return dims, mu, links, A, S, T, x


ORTH = [0, 1]  # SGN_ORTH_CGS2, SGN_ORTH_DELAYED


@pytest.mark.parametrize("orth", ORTH)
@pytest.mark.parametrize("m", [0, 12])
@pytest.mark.parametrize("k", [1, 2, 10, 40, 100])
def test_fixed_k_matches_oracle_arnoldi(env, small_problem, m, k, orth):
    sg, torch = env
    dims, mu, links, A, S, T, x = small_problem
    print("fixed k", m, k, orth, flush=True)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_set_orthogonalization(ctx, orth)
    try:
        Sm, Tm = (S, T) if m else (None, None)
        if m:
            sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        sg.sgn_apply_fixed(ctx, _dev(torch, x), y, k)
        st = arnoldi.modified_arnoldi(lambda v: A @ v, x, Sm, k)
        ref = arnoldi.approx_definition(Sm, Tm, st)
        assert _rel(y.cpu().numpy(), ref) < 1e-10
        info = sg.sgn_last_info(ctx)
        assert info["k_used"] == k
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("orth", ORTH)
def test_apply_converges_to_exact_small(env, small_problem, orth):
    sg, torch = env
    dims, mu, links, A, S, T, x = small_problem
    exact = matfunc.sgn_spectral_apply(A.toarray(), x)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_set_orthogonalization(ctx, orth)
    try:
        sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        st = sg.sgn_apply(ctx, _dev(torch, x), y, 1e-11, 600)
        info = sg.sgn_last_info(ctx)
        print(info, flush=True)
        assert st == sg.SGN_OK and info["converged"] == 1
        assert _rel(y.cpu().numpy(), exact) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("orth", ORTH)
def test_full_grade_is_exact(env, orth):
    # Eq. (interp): with k + m = N the composite space is everything and y is exact
    sg, torch = env
    dims, mu = (2, 2, 2, 4), 0.3
    links = synth.random_links(dims, 31)
    A = wilson.hw_matrix(links, dims, mu, M_W).toarray()
    x = synth.gaussian_source(dims, 1000)
    exact = matfunc.sgn_spectral_apply(A, x)
    S, T, _, _ = deflation.critical_from_dense(A, 8)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_set_orthogonalization(ctx, orth)
    try:
        sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        sg.sgn_apply_fixed(ctx, _dev(torch, x), y, x.size - 8)
        info = sg.sgn_last_info(ctx)
        print(info, flush=True)
        assert _rel(y.cpu().numpy(), exact) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


def _golden(name):
    path = os.path.join(GOLDEN, name + ".npy")
    if not os.path.exists(path):
        pytest.skip(f"golden file {name} not generated")
    return np.load(path, allow_pickle=False)


def test_4x4_no_deflation_vs_exact(env):
    # 4^4, mu = 0.3, m = 0, k <= 300 per the workload; at k = 300 the error is ~1e-10,
    # so the apply is allowed kmax = 400 and held to 1e-10 against the exact result.
    sg, torch = env
    dims, mu = (4, 4, 4, 4), 0.3
    exact = _golden("c4_mu0.3")
    links = synth.random_links(dims, synth.GAUGE_SEED)
    x = synth.gaussian_source(dims, 1000)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        sg.sgn_apply(ctx, _dev(torch, x), y, 1e-11, 400)
        info = sg.sgn_last_info(ctx)
        print(info, flush=True)
        assert _rel(y.cpu().numpy(), exact) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("mu", [0.0, 0.2, 0.5])
def test_6x6_deflated_vs_exact(env, mu):
    sg, torch = env
    dims = (6, 6, 6, 6)
    exact = _golden(f"c6_mu{mu}")
    links = synth.random_links(dims, synth.GAUGE_SEED)
    x = synth.gaussian_source(dims, 1000)
    A = wilson.hw_matrix(links, dims, mu, M_W)
    S, T, th, low = deflation.critical_from_arpack(A, 20)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        y = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        # the stopping rule certifies tol on the result before the last
        # checkpoint, so the stated tolerance is the asserted one
        st = sg.sgn_apply(ctx, _dev(torch, x), y, 1e-10, 500)
        info = sg.sgn_last_info(ctx)
        print(mu, info, flush=True)
        assert st == sg.SGN_OK
        assert _rel(y.cpu().numpy(), exact) < 1e-10
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("orth", ORTH)
def test_edge_cases(env, small_problem, orth):
    sg, torch = env
    dims, mu, links, A, S, T, x = small_problem
    N = x.size
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_set_orthogonalization(ctx, orth)
    try:
        sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        y = torch.empty(N, dtype=torch.complex128, device="cuda")
        # zero source -> zero result
        sg.sgn_apply(ctx, torch.zeros(N, dtype=torch.complex128, device="cuda"), y, 1e-10, 50)
        assert float(y.abs().max()) == 0.0
        # source inside the Schur space -> S sgn(T) S^dag x exactly, no Krylov step
        xs = S @ np.arange(1, 13)
        sg.sgn_apply(ctx, _dev(torch, xs), y, 1e-10, 50)
        ref = matfunc.sgn_spectral_apply(A.toarray(), xs)
        assert _rel(y.cpu().numpy(), ref) < 1e-11
        assert sg.sgn_last_info(ctx)["k_used"] == 0
        # NaN in x
        xn = x.copy()
        xn[5] = np.nan
        with pytest.raises(sg.SgnError) as e:
            sg.sgn_apply(ctx, _dev(torch, xn), y, 1e-10, 50)
        assert e.value.status == sg.SGN_EINVAL
        # kmax too small: soft failure with the kmax estimate
        st = sg.sgn_apply(ctx, _dev(torch, x), y, 1e-14, 6)
        assert st == sg.SGN_ENOCONV
        info = sg.sgn_last_info(ctx)
        assert info["converged"] == 0 and info["k_used"] == 6
        # bad arguments
        with pytest.raises(sg.SgnError):
            sg.sgn_apply(ctx, _dev(torch, x), y, -1.0, 50)
        with pytest.raises(sg.SgnError):
            sg.sgn_apply(ctx, _dev(torch, x), y, 1e-8, 1)
        # y aliasing x is allowed
        xa = _dev(torch, x)
        sg.sgn_apply_fixed(ctx, xa, xa, 20)
        y2 = torch.empty(N, dtype=torch.complex128, device="cuda")
        sg.sgn_apply_fixed(ctx, _dev(torch, x), y2, 20)
        assert torch.equal(xa, y2)
        # removing the deflation
        sg.sgn_deflate_import(ctx, None, np.zeros((0, 0)))
        assert sg.sgn_deflation_size(ctx) == 0
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("orth", ORTH)
def test_deterministic_repeat(env, small_problem, orth):
    sg, torch = env
    dims, mu, links, A, S, T, x = small_problem
    ctx = sg.sgn_create(links, dims, mu, M_W)
    sg.sgn_set_orthogonalization(ctx, orth)
    try:
        sg.sgn_deflate_import(ctx, _dev(torch, S), T)
        y1 = torch.empty(x.size, dtype=torch.complex128, device="cuda")
        y2 = torch.empty_like(y1)
        # the first apply on a field records the checkpoint schedule; from then on
        # applies are reproducible bit for bit
        sg.sgn_apply(ctx, _dev(torch, x), y1, 1e-10, 300)
        sg.sgn_apply(ctx, _dev(torch, x), y1, 1e-10, 300)
        sg.sgn_apply(ctx, _dev(torch, x), y2, 1e-10, 300)
        assert torch.equal(y1, y2)
    finally:
        sg.sgn_destroy(ctx)


@pytest.mark.parametrize("mu", [0.0, 0.2, 0.5])
def test_6x6_sources_at_tol_1e10_vs_exact(env, mu):
    # the headline configuration: the library's own m = 20 Schur pair, tol
    # 1e-10.  The first apply places the checkpoints; the later sources start
    # where it was certified, and each must still land within 1e-10 of the
    # exact result (stored for sources 1000..1015 by the oracle's dense
    # Roberts sign)
    sg, torch = env
    dims = (6, 6, 6, 6)
    Y = _golden(f"c6_mu{mu}_sources")
    links = synth.random_links(dims, synth.GAUGE_SEED)
    ctx = sg.sgn_create(links, dims, mu, M_W)
    try:
        assert sg.sgn_deflate(ctx, 20) == sg.SGN_OK
        y = torch.empty(Y.shape[1], dtype=torch.complex128, device="cuda")
        errs = []
        for r in range(Y.shape[0]):
            x = synth.gaussian_source(dims, 1000 + r)
            st = sg.sgn_apply(ctx, _dev(torch, x), y, 1e-10, 500)
            info = sg.sgn_last_info(ctx)
            e = _rel(y.cpu().numpy(), Y[r])
            errs.append(e)
            print(mu, r, info["k_used"], info["n_checkpoints"], f"{e:.3e}", flush=True)
            assert st == sg.SGN_OK
        assert max(errs) < 1e-10, errs
    finally:
        sg.sgn_destroy(ctx)


def test_create_refuses_non_su3_links(env):
    # the stencil rebuilds the third row of each link from the first two
    sg, torch = env
    dims = (2, 2, 2, 4)
    links = synth.random_links(dims, 9).copy()
    links[1, 0, 1, 0, 2] *= 1.01  # one link no longer unitary
    with pytest.raises(sg.SgnError) as e:
        sg.sgn_create(links, dims, 0.3, M_W)
    assert "SU(3)" in str(e.value)
    links = synth.random_links(dims, 9).copy()
    links[0, 1, 0, 1, 3] *= np.exp(2j * np.pi / 3 + 0.1j)  # unitary, det != 1
    with pytest.raises(sg.SgnError):
        sg.sgn_create(links, dims, 0.3, M_W)
