"""The matrix-core complex product (the small-matrix sign's Newton-Schulz
GEMM and the deflation setup's V Y) against numpy, element by element.

FP64 with a different summation order: relative Frobenius error <= 1e-14 *
sqrt(K), entries bounded by |A| |B| rounding; ragged sizes cover partial
16 x 16 blocks, partial k-steps of 4 and both tile shapes (32 x 32 and 64 x 64
workgroups)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    ctx = sg.sgn_create(synth.random_links((2, 2, 2, 2), 1), (2, 2, 2, 2), 0.0, -1.6)
    yield sg, torch, ctx
    sg.sgn_destroy(ctx)


def _cm(torch, M):
    """column-major device copy of a numpy matrix (as its transpose, contiguous)"""
    return torch.from_numpy(np.ascontiguousarray(M.T)).cuda()


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (17, 33, 5), (3, 70, 2), (100, 37, 64), (64, 64, 64),
                                   (360, 360, 360), (363, 361, 359), (4001, 150, 135), (130, 130, 0)])
def test_zgemm_matches_numpy(env, M, N, K):
    sg, torch, ctx = env
    print("zgemm", M, N, K, flush=True)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    B = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    C = torch.full((N, M), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    sg.sgn_zgemm(ctx, _cm(torch, A), _cm(torch, B), C)
    got = C.cpu().numpy().T
    ref = A @ B
    if K == 0:
        assert np.all(got == 0)
        return
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-14 * np.sqrt(K), err
    # every entry: within the rounding bound of its own sum
    bound = 4 * K * 2.2e-16 * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(got - ref) <= bound + 1e-300)


def test_zgemm_rejects_bad_sizes(env):
    sg, torch, ctx = env
    import ctypes as C

    x = torch.zeros(4, dtype=torch.complex128, device="cuda")
    p = C.c_void_p(x.data_ptr())
    assert sg._lib.sgn_zgemm(ctx, -1, 2, 2, p, 2, p, 2, p, 2) == sg.SGN_EINVAL
    assert sg._lib.sgn_zgemm(ctx, 2, 2, 2, p, 1, p, 2, p, 2) == sg.SGN_EINVAL
