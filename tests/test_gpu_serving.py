"""Serving scheduler: requests on two resident fields arrive from another
thread while earlier ones run; each result must be bitwise the one the same
request gives alone (a one-slot session on the same context), near the exact
sign (oracle), and a bad request must fail alone."""
import threading
import time

import numpy as np
import pytest

import synth
from oracle import matfunc, wilson

pytestmark = pytest.mark.gpu

M_W = -1.6
FIELDS = [("a", (3, 3, 3, 4), 0.3, 6, 61), ("b", (4, 4, 2, 4), 0.1, 8, 62)]


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0704_3486_amd as sg

    return sg, torch


def test_server_results_equal_single_apply(env):
    sg, torch = env
    from paper_0704_3486_amd.serving import Request, Server

    print("serving: two fields, 14 requests", flush=True)
    srv = Server(2e9, nsteps=3)
    links = {}
    try:
        for name, dims, mu, m, seed in FIELDS:
            links[name] = synth.random_links(dims, seed)
            setup = srv.add_field(name, links[name], dims, mu, M_W, m, 600, 0.5)
            assert setup["slots"] >= 1
        srv.fields["a"].max_slots = 3  # fewer slots than requests: admission waits
        reqs = []
        for q in range(14):
            name, dims = FIELDS[q % 2][0], FIELDS[q % 2][1]
            x = torch.from_numpy(synth.gaussian_source(dims, 5000 + q)).cuda()
            tol = 1e-10 if q % 3 else 1e-8
            reqs.append(Request(name, x, torch.empty_like(x), tol, 600))
        bad = reqs[5].x.clone()
        bad[7] = float("nan")
        reqs[5].x = bad
        torch.cuda.synchronize()  # the fields' streams read these
        srv.start()

        def feed():
            for q, r in enumerate(reqs):
                srv.submit(r)
                time.sleep(0.002 * (q % 4))

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        for r in reqs:
            assert r.done.wait(120), "request not completed"
        srv.stop()
        assert isinstance(reqs[5].error, sg.SgnError) and reqs[5].error.status == sg.SGN_EINVAL
        for q, r in enumerate(reqs):
            if q == 5:
                continue
            assert r.error is None and r.info["converged"] == 1, (q, r.info)
            assert r.latency is not None and r.latency >= 0
            alone = sg.Session(srv.fields[r.field].ctx, 1, 600)
            try:
                y = torch.empty_like(r.y)
                h = alone.submit(r.x, y, r.tol, r.kmax)
                while alone.poll(h) is None:
                    alone.step(5)
            finally:
                alone.destroy()
            assert torch.equal(y, r.y), q
        for q in (0, 1):
            name, dims, mu = FIELDS[q][:3]
            A = wilson.hw_matrix(links[name], dims, mu, M_W).toarray()
            exact = matfunc.sgn_spectral_apply(A, reqs[q].x.cpu().numpy())
            got = reqs[q].y.cpu().numpy()
            assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 1e-7
    finally:
        srv.close()
