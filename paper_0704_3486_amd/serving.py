"""Serving loop over resident fields: requests y = sgn(H_w(mu)) x arrive at
any time and are batched continuously.

Each field (links, Schur pair, sgn(T_m)) stays on the device in its own
context, on its own HIP stream, served by one worker thread that drives one
serving session (sgn_session_* in include/sgn.h).  A request waits in its
field's queue until the session has a free slot (admission by device memory:
a session's slot count is fixed at creation from its share of the HBM budget
and the Krylov workspace one request needs, sgn_footprint_bytes), then
advances one Arnoldi step per session step together with every other
request in flight on that field.  The sessions of different fields run
concurrently on the device.

This module only schedules: all arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import collections
import threading
import time

from . import (SGN_PREC_FP64, Session, sgn_create, sgn_deflate, sgn_deflate_stats, sgn_destroy, sgn_footprint_bytes,
               sgn_get_dims, sgn_set_precision, sgn_set_stream)

MAX_SLOTS = 64


class Request:
    """One sign request: x (device tensor), y (device tensor, written), its
    tolerance and Krylov cap, and the host times of arrival and completion."""

    def __init__(self, field, x, y, tol, kmax):
        self.field = field
        self.x, self.y = x, y
        self.tol, self.kmax = tol, kmax
        self.t_arrive = None
        self.t_done = None
        self.info = None
        self.error = None
        self.done = threading.Event()

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrive


class _Field:
    def __init__(self, name, ctx, stream, session, max_slots, kmax, setup):
        self.name = name
        self.ctx, self.stream, self.session = ctx, stream, session
        self.max_slots, self.kmax = max_slots, kmax
        self.setup = setup
        self.queue = collections.deque()
        self.cv = threading.Condition()
        self.thread = None
        self.completed = 0


class Server:
    """Resident fields and their serving sessions.

    hbm_budget: device bytes the Krylov workspaces of all fields may take;
    each field gets the share given to add_field.  nsteps: Arnoldi steps per
    session step between admissions and completions."""

    def __init__(self, hbm_budget, nsteps=4):
        import torch

        self.torch = torch
        self.budget = int(hbm_budget)
        self.nsteps = int(nsteps)
        self.fields = {}
        self._stop = False

    def add_field(self, name, links, dims, mu, m_w, m, kmax, share, prec=SGN_PREC_FP64):
        """Create the context, compute its deflation basis (m Schur vectors)
        and a session with as many slots as its share of the budget holds."""
        torch = self.torch
        t0 = time.perf_counter()
        ctx = sgn_create(links, dims, mu, m_w)
        try:
            stream = torch.cuda.Stream()
            sgn_set_stream(ctx, stream.cuda_stream)
            sgn_set_precision(ctx, prec)
            sgn_deflate(ctx, m)
            per_slot = sgn_footprint_bytes(ctx, kmax, MAX_SLOTS) / MAX_SLOTS
            slots = int(max(1, min(MAX_SLOTS, share * self.budget // per_slot)))
            ses = Session(ctx, slots, kmax)
        except Exception:
            sgn_destroy(ctx)
            raise
        torch.cuda.synchronize()
        setup = {"seconds": round(time.perf_counter() - t0, 2), "slots": slots, "kmax": kmax, "m": m,
                 "bytes_per_slot": int(per_slot), **sgn_deflate_stats(ctx)}
        self.fields[name] = _Field(name, ctx, stream, ses, slots, kmax, setup)
        return setup

    def n_sites(self, name):
        return sgn_get_dims(self.fields[name].ctx)[1]

    def start(self):
        self._stop = False
        for f in self.fields.values():
            f.thread = threading.Thread(target=self._work, args=(f,), daemon=True)
            f.thread.start()

    def submit(self, req):
        """Queue a request (its arrival time is taken now)."""
        f = self.fields[req.field]
        req.t_arrive = time.perf_counter()
        with f.cv:
            f.queue.append(req)
            f.cv.notify()

    def stop(self):
        """Finish everything queued, then end the workers."""
        self._stop = True
        for f in self.fields.values():
            with f.cv:
                f.cv.notify()
        for f in self.fields.values():
            if f.thread is not None:
                f.thread.join()
                f.thread = None

    def close(self):
        self.stop()
        for f in self.fields.values():
            f.session.destroy()
            sgn_destroy(f.ctx)
        self.fields.clear()

    def _work(self, f):
        ses = f.session
        running = {}
        while True:
            with f.cv:
                while not f.queue and not running and not self._stop:
                    f.cv.wait(0.05)
                if self._stop and not f.queue and not running:
                    return
                admit = []
                while f.queue and len(running) + len(admit) < f.max_slots:
                    admit.append(f.queue.popleft())
            for req in admit:
                try:
                    h = ses.submit(req.x, req.y, req.tol, req.kmax)
                except Exception as e:  # bad input: report on the request
                    req.error = e
                    req.t_done = time.perf_counter()
                    req.done.set()
                    continue
                if h is None:  # cannot happen with the slot count above; requeue in order
                    with f.cv:
                        f.queue.extendleft(reversed(admit[admit.index(req):]))
                    break
                running[h] = req
            if not running:
                continue
            if ses.step(self.nsteps) > 0:
                now = time.perf_counter()
                for h in list(running):
                    try:
                        info = ses.poll(h)
                    except Exception as e:  # the request failed (non-finite values)
                        info, running[h].error = None, e
                    if info is not None or running[h].error is not None:
                        req = running.pop(h)
                        req.info = info
                        req.t_done = now
                        f.completed += 1
                        req.done.set()
