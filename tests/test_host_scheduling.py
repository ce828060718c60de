"""CPU checks of the host-side scheduling around the library: the serving
worker loop (admission by free slots, first come first served, completion
and error reporting, draining on stop) and the autotuner's cache.  The
library's session and tuning calls are replaced by host stand-ins that
record what they are asked; no arithmetic of the method is involved."""
import json
import threading


class FakeSession:
    """Stand-in for a serving session: a request finishes after `work[x]`
    steps; submit rejects x == "bad"; poll raises for x == "nan"."""

    def __init__(self, max_slots, work):
        self.max_slots = max_slots
        self.work = work
        self.slots = {}
        self.next_handle = 0
        self.admitted = []
        self.peak = 0
        self.lock = threading.Lock()

    def submit(self, x, y, tol, kmax):
        with self.lock:
            if x == "bad":
                raise ValueError("bad input")
            if len(self.slots) >= self.max_slots:
                return None
            h = self.next_handle
            self.next_handle += 1
            self.slots[h] = [x, self.work.get(x, 3), False]
            self.admitted.append(x)
            self.peak = max(self.peak, len(self.slots))
            return h

    def step(self, nsteps):
        finished = 0
        with self.lock:
            for s in self.slots.values():
                if not s[2]:
                    s[1] -= nsteps
                    if s[1] <= 0:
                        s[2] = True
                        finished += 1
        return finished

    def poll(self, h):
        with self.lock:
            x, _, done = self.slots[h]
            if not done:
                return None
            del self.slots[h]
            if x == "nan":
                raise FloatingPointError("non-finite value")
            return {"converged": 1, "x": x}


def _server(max_slots, work, nsteps=1):
    from paper_0704_3486_amd import serving

    srv = serving.Server(hbm_budget=1 << 30, nsteps=nsteps)
    ses = FakeSession(max_slots, work)
    f = serving._Field("f", None, None, ses, max_slots, 100, {})
    srv.fields["f"] = f
    return srv, ses, serving


def test_serving_admits_in_order_within_the_slots():
    work = {f"r{i}": 1 + (7 * i) % 5 for i in range(20)}
    srv, ses, serving = _server(max_slots=3, work=work)
    reqs = [serving.Request("f", f"r{i}", None, 1e-8, 100) for i in range(20)]
    for r in reqs:  # queued before the worker starts: admission order is queue order
        srv.submit(r)
    srv.start()
    for r in reqs:
        assert r.done.wait(10)
    srv.stop()
    assert ses.admitted == [f"r{i}" for i in range(20)]
    assert ses.peak <= 3
    assert ses.peak == 3  # the slots were used
    for r in reqs:
        assert r.error is None and r.info == {"converged": 1, "x": r.x}
        assert r.latency is not None and r.latency >= 0
    assert srv.fields["f"].completed == 20


def test_serving_reports_errors_on_the_request():
    srv, ses, serving = _server(max_slots=2, work={})
    reqs = [serving.Request("f", x, None, 1e-8, 100) for x in ("ok1", "bad", "nan", "ok2")]
    srv.start()
    for r in reqs:
        srv.submit(r)
    for r in reqs:
        assert r.done.wait(10)
    srv.stop()
    assert isinstance(reqs[1].error, ValueError) and reqs[1].info is None
    assert isinstance(reqs[2].error, FloatingPointError) and reqs[2].info is None
    assert reqs[0].info["converged"] == 1 and reqs[3].info["converged"] == 1
    assert "bad" not in ses.admitted


def test_serving_stop_drains_the_queue():
    work = {f"r{i}": 5 for i in range(6)}
    srv, ses, serving = _server(max_slots=1, work=work)
    reqs = [serving.Request("f", f"r{i}", None, 1e-8, 100) for i in range(6)]
    srv.start()
    for r in reqs:
        srv.submit(r)
    srv.stop()  # returns only when everything queued has finished
    assert all(r.done.is_set() and r.info is not None for r in reqs)
    assert ses.peak == 1 and not ses.slots


def test_autotune_cache_hit_sets_the_stored_shape(tmp_path, monkeypatch):
    import torch

    from paper_0704_3486_amd import autotune as at

    calls = []
    monkeypatch.setattr(at, "sgn_get_dims", lambda ctx: ((6, 6, 6, 6), 15552))
    monkeypatch.setattr(at, "sgn_get_precision", lambda ctx: 0)
    monkeypatch.setattr(at, "sgn_deflation_size", lambda ctx: 20)
    monkeypatch.setattr(at, "sgn_get_tuning", lambda ctx: (8, 4, 8))
    monkeypatch.setattr(at, "sgn_set_tuning", lambda ctx, ub, cpw, uw: calls.append((ub, cpw, uw)))

    def no_timing(*a, **k):
        raise AssertionError("a cache hit must not time anything")

    monkeypatch.setattr(at, "sgn_apply_fixed", no_timing)
    monkeypatch.setattr(at, "sgn_apply_batched_fixed", no_timing)
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda *a: "TestGPU")
    key = at._key(None, 1, 300, "TestGPU")
    assert key == "6x6x6x6|15552|0|20|1|300|TestGPU"
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({key: {"update_batch": 16, "dot_cols": 1, "ms": 1.0},
                                 "other|key": {"update_batch": 4, "dot_cols": 2, "ms": 2.0}}))
    out = at.autotune(None, k=300, nrhs=1, cache=str(cache))
    assert out == {"update_batch": 16, "dot_cols": 1, "ms": None, "cached": True}
    assert calls == [(16, 1, 8)]  # the wavefronts per workgroup (uw) are kept
    # another Krylov dimension or source count is another entry
    assert at._key(None, 1, 200, "TestGPU") not in json.loads(cache.read_text())
    assert at._key(None, 32, 300, "TestGPU") != key


def test_serving_requeues_every_unsubmitted_request_in_order():
    # a session that turns one request away once (no free slot reported):
    # that request and every one admitted after it return to the queue in
    # order, and all of them finish
    work = {f"r{i}": 2 for i in range(8)}
    srv, ses, serving = _server(max_slots=4, work=work)
    inner = ses.submit
    refused = []

    def submit_refusing_once(x, y, tol, kmax):
        if x == "r1" and not refused:
            refused.append(x)
            return None
        return inner(x, y, tol, kmax)

    ses.submit = submit_refusing_once
    reqs = [serving.Request("f", f"r{i}", None, 1e-8, 100) for i in range(8)]
    for r in reqs:
        srv.submit(r)
    srv.start()
    for r in reqs:
        assert r.done.wait(10), r.x
    srv.stop()
    assert refused == ["r1"]
    assert ses.admitted == [f"r{i}" for i in range(8)]
    assert all(r.info is not None and r.error is None for r in reqs)
