"""Independent contexts driven from several host threads, each on its own
stream (the benchmark's arrangement: fields and applies in flight together):
every result is bitwise the one the same context computes alone, so the
contexts share no device scratch or library state."""
import threading

import pytest

import synth

pytestmark = pytest.mark.gpu
M_W = -1.6


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


@pytest.mark.parametrize("prec", [0, 1])
def test_threads_and_streams_match_serial(env, prec):
    sg, torch = env
    dims, m, nsrc = (4, 4, 4, 4), 8, 3
    mus = (0.0, 0.3, 0.5, 0.3)  # the last two: one field, two contexts
    links = synth.random_links(dims, 77)
    X = [torch.from_numpy(synth.gaussian_source(dims, 7700 + r)).cuda() for r in range(nsrc)]
    ctxs, streams = [], []
    try:
        for q, mu in enumerate(mus):
            c = sg.sgn_create(links, dims, mu, M_W)
            ctxs.append(c)
            st = torch.cuda.Stream()
            streams.append(st)
            sg.sgn_set_stream(c, st.cuda_stream)
            sg.sgn_set_precision(c, prec)
            if q < 3:
                sg.sgn_deflate(c, m)
            else:  # the second context of the field of context 1: its pair
                S, T, _ = sg.sgn_deflate_export(ctxs[1])
                sg.sgn_deflate_import(c, S, T)
        torch.cuda.synchronize()
        tol = 1e-10 if prec == 0 else 1e-7

        def run(q, out):
            for r in range(nsrc):
                y = torch.empty_like(X[r])
                assert sg.sgn_apply(ctxs[q], X[r], y, tol, 600) == sg.SGN_OK
                yf = torch.empty_like(X[r])
                sg.sgn_apply_fixed(ctxs[q], X[r], yf, 50)
                out.append((y, yf))

        # one apply per context first: it fixes the context's checkpoint
        # schedule (remembered k), which the serial and concurrent passes share
        for c in ctxs:
            y = torch.empty_like(X[0])
            assert sg.sgn_apply(c, X[0], y, tol, 600) == sg.SGN_OK
        serial = []
        for q in range(len(ctxs)):
            serial.append([])
            run(q, serial[q])
        torch.cuda.synchronize()
        conc = [[] for _ in ctxs]
        th = [threading.Thread(target=run, args=(q, conc[q])) for q in range(len(ctxs))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        torch.cuda.synchronize()
        for q in range(len(ctxs)):
            assert len(conc[q]) == nsrc
            for (a, af), (b, bf) in zip(serial[q], conc[q]):
                assert torch.equal(a, b) and torch.equal(af, bf)
        # the two contexts of one field agree with each other as well
        for (a, af), (b, bf) in zip(serial[1], serial[3]):
            assert torch.equal(a, b) and torch.equal(af, bf)
    finally:
        for c in ctxs:
            sg.sgn_destroy(c)
