"""Launch-shape autotuner for the Arnoldi step's dot and update passes.

The update pass's column-load batch (4, 8, 16) and the dot pass's columns per
wavefront (1, 2, 4) form every sum in the same order, so any of them gives
bitwise the same result; which is fastest depends on the lattice size, the
precision and the number of sources in flight.  `autotune` times each of the
nine shapes on the context itself (sgn_apply_fixed, or
sgn_apply_batched_fixed for several sources, at a given Krylov dimension),
keeps the fastest and records it in a JSON cache keyed by lattice,
precision, deflation size, sources, Krylov dimension and device, so a later
process with the same key sets it without timing.

This module only schedules and times calls of the library; all arithmetic
runs in its kernels.
"""
from __future__ import annotations

import itertools
import json
import os
import time

from . import (sgn_apply_batched_fixed, sgn_apply_fixed, sgn_deflation_size, sgn_get_dims, sgn_get_precision,
               sgn_get_tuning, sgn_matvec, sgn_set_stencil_blocks, sgn_set_tuning)

UPDATE_BATCH = (4, 8, 16)
DOT_COLS = (1, 2, 4)
# stencil walk blocks (By, Bz, Bt) tried by autotune_stencil: the default
# rule, the natural order and blocks around the default
STENCIL_BLOCKS = ((0, 0, 0), (-1, 0, 0), (4, 16, 2), (4, 16, 8), (4, 8, 8), (8, 8, 2), (8, 8, 4), (2, 8, 4),
                  (8, 4, 4))


def _key(ctx, nrhs, k, device):
    dims, n = sgn_get_dims(ctx)
    return "|".join(str(v) for v in ("x".join(map(str, dims)), n, sgn_get_precision(ctx), sgn_deflation_size(ctx),
                                        nrhs, k, device))


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def autotune(ctx, k=256, nrhs=1, cache=None, reps=3):
    """Pick the fastest bitwise-neutral launch shape for this context and set
    it.  k: Krylov dimension of the timed applies (about the k the workload
    reaches); nrhs: sources per batched apply (1: sgn_apply).  cache: JSON
    file path or None.  Returns {"update_batch", "dot_cols", "ms", "cached"}
    (ms: per apply of the chosen shape, None when taken from the cache)."""
    import torch

    device = torch.cuda.get_device_name()
    key = _key(ctx, nrhs, k, device)
    table = _load(cache)
    _, _, uw = sgn_get_tuning(ctx)
    if key in table:
        ub, cpw = table[key]["update_batch"], table[key]["dot_cols"]
        sgn_set_tuning(ctx, ub, cpw, uw)
        return {"update_batch": ub, "dot_cols": cpw, "ms": None, "cached": True}

    _, n = sgn_get_dims(ctx)
    gen = torch.Generator(device="cuda").manual_seed(12345)
    X = torch.randn(nrhs, n, dtype=torch.complex128, device="cuda", generator=gen)
    Y = torch.empty_like(X)
    torch.cuda.synchronize()  # the library reads X on the context's stream

    def run():
        if nrhs == 1:
            sgn_apply_fixed(ctx, X[0], Y[0], k)
        else:
            sgn_apply_batched_fixed(ctx, X, Y, k)

    times = {}
    for ub, cpw in itertools.product(UPDATE_BATCH, DOT_COLS):
        sgn_set_tuning(ctx, ub, cpw, uw)
        run()  # warm-up (first launches of these kernel instances)
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            run()
            best = min(best, time.perf_counter() - t0)
        times[(ub, cpw)] = best
    (ub, cpw), t = min(times.items(), key=lambda kv: kv[1])
    sgn_set_tuning(ctx, ub, cpw, uw)
    if cache:
        table = _load(cache)  # merge with what other processes wrote meanwhile
        table[key] = {"update_batch": ub, "dot_cols": cpw, "ms": round(1e3 * t, 4)}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return {"update_batch": ub, "dot_cols": cpw, "ms": round(1e3 * t, 4), "cached": False}


def autotune_stencil(ctx, reps=10):
    """Pick the fastest stencil walk (sgn_set_stencil_blocks; results are
    bitwise the same for every walk) by timing sgn_matvec on this context's
    lattice; shapes that do not fit the lattice are skipped.  Returns
    {"blocks": (By, Bz, Bt), "us": per matvec}."""
    import torch

    from . import SgnError

    _, n = sgn_get_dims(ctx)
    gen = torch.Generator(device="cuda").manual_seed(4321)
    x = torch.randn(n, dtype=torch.complex128, device="cuda", generator=gen)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    best = None
    for blocks in STENCIL_BLOCKS:
        try:
            sgn_set_stencil_blocks(ctx, *blocks)
        except SgnError:
            continue
        sgn_matvec(ctx, x, y)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sgn_matvec(ctx, x, y)
        torch.cuda.synchronize()
        us = 1e6 * (time.perf_counter() - t0) / reps
        if best is None or us < best[0]:
            best = (us, blocks)
    sgn_set_stencil_blocks(ctx, *best[1])
    return {"blocks": best[1], "us": round(best[0], 2)}
