"""Throughput of y = sgn(H_w(mu)) x on one MI355X.

Workload (one GPU): 6^4 lattice (N = 15552, complex128), random-link SU(3)
field (seed 20070426, the synthetic stand-in for the paper's quenched
ensembles), m_w = -1.6, three fields mu in {0.0, 0.2, 0.5}, m = 20 critical
Schur vectors computed once per field by the library's own deflation setup,
single right-hand side per apply, FP64, kmax = 500, tolerance 1e-10.

A step is --per-field (default 2) sgn(H_w(mu)) x per field, each a
single-source FP64 apply on a distinct Gaussian source.  The applies are
independent: every field has that many contexts, each holding the field's
links and Schur pair, on its own HIP stream and driven by its own host
thread, so their latency-bound kernels overlap on the device.  The timed region covers exactly --steps
steps with inputs resident in device memory, bracketed by device
synchronisations; value = applies per second.  Also reported:
  * latency: the same steps run one apply at a time (ms per apply);
  * kernels / roofline: a separate serial pass with the library's HIP-event
    kernel profiling on, per-kernel average duration and algorithmic bytes;
    the roofline is that of the kernel with the largest share of the time;
  * aggregate_timed_region: the Krylov passes' and the stencil's algorithmic
    bytes per apply (from the profiled pass) times the timed applies per
    second: the device-wide rate while several applies overlap;
  * stencil: H_w(mu) on a 32^4 lattice (1 GB of operands, beyond the 256 MB
    Infinity Cache), algorithmic GB/s against the HBM peak, beside a plain
    device copy timed the same way;
  * batched_mixed_12x12x12x12: 32 sources of a 12^4 field (m = 40) in one
    mixed-precision batched apply (tol 1e-7) against FP64 single-source
    applies (tol 1e-10) on the same field, with the mixed error;
  * cpu_baseline: the oracle's plain Arnoldi (numpy/scipy, FP64) on a bounded
    sample, one apply per field at the Krylov dimension the GPU used.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sgn(H_w(mu))·x applies/sec at 1e-10 rel err; stencil HBM GB/s vs peak"
HBM_PEAK_GBPS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
# profiling class -> kernel symbol (as rocprofv3 lists it)
HBM_KERNELS = {"krylov_update": "kupdate_kernel<double2>", "krylov_dot": "kdot_kernel<double2>",
               "krylov_reduce": "kred_kernel", "wilson_hw": "wilson_hw_dir_kernel<double2, false>"}
# the same for the block (s-step) process
HBM_KERNELS_BLOCK = {"block_update": "bupdate_kernel<false, 1>", "block_dot": "bdot_kernel", "block_reduce": "bred_kernel",
                     "block_factor": "bsmall_kernel<false>", "wilson_hw": "wilson_hw_dir_kernel<double2, true>"}
BLOCK_STEPS = 16  # Arnoldi steps per block of the headline applies (sgn_set_block_steps)
BATCH = 8  # sources per batched apply call of each context in the timed region
STENCIL_DIMS = (32, 32, 32, 32)
# HBM traffic of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs, stored with the hash of the source it was measured on (stale -> null)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_krylov_6x6x6x6_m20_fp64.txt")
TRAFFIC_FILE_BLOCK = os.path.join(ROOT, "profiles", "hbm_traffic_block_6x6x6x6_m20_fp64_batch8.txt")
DIMS = (6, 6, 6, 6)
MUS = (0.0, 0.2, 0.5)
M_W = -1.6
M_DEFL = 20
KMAX = 500
TOL = 1e-10
AUTOTUNE_K = 300  # about the k these fields reach at TOL (248-428)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lr", action="store_true", help="skip the LR-deflation comparison on the mu=0.2 field")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the 8^4 mixed-precision figures and the 4^4 undeflated leg")
    ap.add_argument("--no-overlap", action="store_true", help="skip the overlap-operator figures on the mu=0.2 field")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shape of the Arnoldi passes instead of timing the nine")
    ap.add_argument("--no-stencil", action="store_true", help="skip the 32^4 stencil measurement")
    ap.add_argument("--stencil-only", action="store_true",
                    help="only run the 32^4 stencil measurement and print its JSON object")
    ap.add_argument("--no-batched", action="store_true", help="skip the 12^4 x 32-source mixed batch")
    ap.add_argument("--serving", action="store_true",
                    help="only run the serving stream (Poisson arrivals over four resident fields) and print its "
                         "JSON object")
    ap.add_argument("--serving-rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--serving-requests", type=int, default=2000, help="arrivals at the offered rate")
    ap.add_argument("--serving-sustained", type=int, default=400,
                    help="arrivals of the second stream, at 70%% of the served rate")
    ap.add_argument("--serving-mixed", action="store_true", help="serve in mixed precision")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the bounded serving leg of the default run")
    ap.add_argument("--no-setup", action="store_true", help="skip the deflation-setup timings")
    ap.add_argument("--setup-scan", action="store_true",
                    help="only time the deflation setup, filtered and unfiltered, on more lattices and degrees")
    ap.add_argument("--m-scan", action="store_true",
                    help="only the deflation-size scan (setup time, k and time per apply against m) and exit")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 12^4 x 32-source mixed-precision batch and print its JSON object")
    ap.add_argument("--per-field", type=int, default=2,
                    help="contexts per field in the timed steps: one stream each, all holding the field's Schur "
                         "pair")
    ap.add_argument("--batch", type=int, default=BATCH,
                    help="sources per apply call of each context in the timed region (1: sgn_apply; more: one "
                         "sgn_apply_batched call on that many sources)")
    ap.add_argument("--block-steps", type=int, default=BLOCK_STEPS,
                    help="Arnoldi steps per block of the headline applies (sgn_set_block_steps; 0: the one-vector "
                         "process with its delayed re-orthogonalisation)")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="replay runs of this many Arnoldi steps as captured HIP graphs in the timed applies "
                         "(sgn_set_step_graphs; bitwise the same results; 0: direct launches)")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the one-source-at-a-time latency leg (for kernel-trace runs: the traced launches "
                         "are then those of the timed region and the profiled pass)")
    ap.add_argument("--serial", action="store_true",
                    help="run the timed region's lanes one after another (no overlap of the fields; for "
                         "kernel-trace runs, whose per-kernel averages then compare with the HIP-event ones)")
    ap.add_argument("--counters", action="store_true",
                    help="only one batched call per field of the headline configuration, with the library's "
                         "algorithmic bytes per launch of each kernel class (the run that rocprofv3 counter "
                         "passes wrap)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device-to-device copy of 2 GiB three times (the reference for the "
                         "HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent sources shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        calibrate_copy(torch)
        return

    import threading

    import paper_0704_3486_amd as sg
    import synth
    from paper_0704_3486_amd.autotune import autotune

    if args.stencil_only:
        print(json.dumps(stencil_leg(sg, synth, torch, tune=not args.no_autotune)))
        return
    if args.batched_only:
        print(json.dumps(batched_leg(sg, synth, torch, tune=not args.no_autotune)))
        return
    if args.m_scan:
        print(json.dumps(m_scan_leg(sg, synth, torch)))
        return
    if args.setup_scan:
        print(json.dumps(setup_leg(sg, synth, torch, SETUP_SCAN_FULL)))
        return
    if args.serving:
        print(json.dumps(serving_leg(sg, synth, torch, args.serving_rate, args.serving_requests, args.serving_sustained,
                                     sg.SGN_PREC_MIXED if args.serving_mixed else sg.SGN_PREC_FP64)))
        return

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.counters:
        print(json.dumps(counters_leg(sg, synth, torch, args.block_steps, args.batch)))
        return
    dev = torch.device("cuda:0")
    links = synth.random_links(DIMS, synth.GAUGE_SEED)
    N = 12 * int(np.prod(DIMS))

    # setup: one context, one stream and one deflation basis per field (not timed)
    ctxs, streams = [], []
    setup = {}
    for mu in MUS:
        t0 = time.perf_counter()
        ctx = sg.sgn_create(links, DIMS, mu, M_W)
        st = torch.cuda.Stream(device=dev)
        sg.sgn_set_stream(ctx, st.cuda_stream)
        sg.sgn_deflate(ctx, M_DEFL)
        torch.cuda.synchronize()
        setup[str(mu)] = {"seconds": round(time.perf_counter() - t0, 3), **sg.sgn_deflate_stats(ctx)}
        if args.block_steps:
            sg.sgn_set_block_steps(ctx, args.block_steps)
        elif not args.no_autotune:
            # launch shape of the Arnoldi passes (results are bitwise the same for every shape)
            tuned = autotune(ctx, k=AUTOTUNE_K)
            setup[str(mu)]["launch_shape"] = [tuned["update_batch"], tuned["dot_cols"]]
        log(f"setup mu={mu}: {setup[str(mu)]}")
        ctxs.append(ctx)
        streams.append(st)

    P = 1 if args.serial else max(1, args.per_field)
    B = max(1, args.batch)
    # sources: the seeds whose exact results are stored for every field
    # (1000 .. 1000 + n - 1, dense Roberts sign of the oracle), cycled; so
    # every timed apply is checked against the exact y
    gold = {}
    for f, mu in enumerate(MUS):
        path = os.path.join(GOLDEN, f"c6_mu{mu}_sources.npy")
        if os.path.exists(path):
            gold[f] = torch.from_numpy(np.load(path, allow_pickle=False)).to(dev)
    nstored = min(g.shape[0] for g in gold.values()) if len(gold) == len(MUS) else 0
    nsrc = nstored if nstored else max((args.steps + args.warmup) * P * B, 2)
    xs = [torch.from_numpy(synth.gaussian_source(DIMS, 1000 + r)).to(dev) for r in range(nsrc)]
    ys = [torch.empty(N, dtype=torch.complex128, device=dev) for _ in MUS]
    torch.cuda.synchronize()

    # accuracy on the source with stored exact results (seed 1000)
    acc = {}
    for f, mu in enumerate(MUS):
        path = os.path.join(GOLDEN, f"c6_mu{mu}.npy")
        st = sg.sgn_apply(ctxs[f], xs[0], ys[f], TOL, KMAX)
        info = sg.sgn_last_info(ctxs[f])
        entry = {"k": info["k_used"], "status": st}
        if os.path.exists(path):
            exact = np.load(path, allow_pickle=False)
            y = ys[f].cpu().numpy()
            entry["rel_err"] = float(np.linalg.norm(y - exact) / np.linalg.norm(exact))
        acc[str(mu)] = entry
        log(f"accuracy mu={mu}: {entry}")

    # further contexts per field (P applies of a field in flight): the same
    # links and Schur pair, their own stream and output; the launch shape of
    # the field's first context; one untimed apply of the seed-1000 source
    # (the first context's accuracy apply) so every context starts from the
    # same remembered checkpoint
    lanes = [(ctxs[f], ys[f]) for f in range(len(MUS))]
    extra = []
    for p in range(1, P):
        for f, mu in enumerate(MUS):
            c = sg.sgn_create(links, DIMS, mu, M_W)
            extra.append(c)
            st = torch.cuda.Stream(device=dev)
            streams.append(st)
            sg.sgn_set_stream(c, st.cuda_stream)
            S, T, _ = sg.sgn_deflate_export(ctxs[f])
            sg.sgn_deflate_import(c, S, T)
            sg.sgn_set_tuning(c, *sg.sgn_get_tuning(ctxs[f]))
            sg.sgn_set_block_steps(c, args.block_steps)
            y = torch.empty(N, dtype=torch.complex128, device=dev)
            sg.sgn_apply(c, xs[0], y, TOL, KMAX)
            lanes.append((c, y))
    if args.graph_steps:
        for c, _ in lanes:
            sg.sgn_set_step_graphs(c, args.graph_steps)
    torch.cuda.synchronize()

    unconverged = []  # applies that ended without reaching TOL (SGN_ENOCONV)

    def field_steps(f, first, count, ks):
        for r in range(first, first + count):
            if sg.sgn_apply(ctxs[f], xs[r % len(xs)], ys[f], TOL, KMAX) != sg.SGN_OK:
                unconverged.append(f)
            ks.append(sg.sgn_last_info(ctxs[f])["k_used"])

    # one output buffer per timed step and lane (the results are checked
    # after the timed region); lane q = p * len(MUS) + f takes sources
    # (r * P + p) * B + i, i < B, of step r, as one batched call when B > 1
    outs = [[torch.empty(B, N, dtype=torch.complex128, device=dev) for _ in range(args.steps)] for _ in lanes]
    src = lambda q, r: [((r * P + q // len(MUS)) * B + i) % len(xs) for i in range(B)]
    batches = {}
    if B > 1:
        for q in range(len(lanes)):
            for r in range(args.warmup + args.steps):
                batches[(q, r)] = torch.stack([xs[i] for i in src(q, r)]).contiguous()
    ybuf = [torch.empty(B, N, dtype=torch.complex128, device=dev) for _ in lanes]
    torch.cuda.synchronize()

    def lane_steps(q, first, count, ks, timed):
        c = lanes[q][0]
        for r in range(first, first + count):
            out = outs[q][r - first] if timed else ybuf[q]
            if B == 1:
                if sg.sgn_apply(c, xs[src(q, r)[0]], out[0], TOL, KMAX) != sg.SGN_OK:
                    unconverged.append(q)
                ks.append(sg.sgn_last_info(c)["k_used"])
            else:
                st, infos = sg.sgn_apply_batched(c, batches[(q, r)], out, TOL, KMAX)
                if st != sg.SGN_OK:
                    unconverged.append(q)
                ks.extend(i["k_used"] for i in infos)

    def run_concurrent(first, count, timed=False):
        ks = [[] for _ in lanes]
        th = [threading.Thread(target=lane_steps, args=(q, first, count, ks[q], timed)) for q in range(len(lanes))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        return [k for kq in ks for k in kq]

    def run_serial(first, count, timed=False):
        ks = []
        for r in range(first, first + count):
            for f in range(len(MUS)):
                field_steps(f, r, 1, ks)
        return ks

    def run_lanes_serial(first, count, timed=False):
        ks = []
        for q in range(len(lanes)):
            lane_steps(q, first, count, ks, timed)
        return ks

    runner = run_lanes_serial if args.serial else run_concurrent
    runner(0, args.warmup)
    torch.cuda.synchronize()
    unconverged.clear()
    t0 = time.perf_counter()
    ks = runner(args.warmup, args.steps, timed=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed_unconverged = len(unconverged)
    applies = args.steps * len(lanes) * B
    value = applies / elapsed
    mode = "serial" if args.serial else f"{len(lanes)} streams"
    log(f"timed ({mode}): {applies} applies in {elapsed:.3f} s -> {value:.2f} applies/s, mean k {np.mean(ks):.1f}")
    timed_acc = timed_accuracy(torch, outs, gold, nstored, P, B, args.warmup, args.steps)
    log(f"timed applies vs exact: {timed_acc}")

    latency = None
    if not args.no_latency:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_serial(args.warmup, args.steps)
        torch.cuda.synchronize()
        elapsed_serial = time.perf_counter() - t0
        n_serial = args.steps * len(MUS)
        latency = {"ms_per_apply": round(1e3 * elapsed_serial / n_serial, 3),
                   "applies_per_s_one_at_a_time": round(n_serial / elapsed_serial, 3)}
        log(f"serial: {latency}")
    for c in extra:
        sg.sgn_destroy(c)
    for c in ctxs:
        sg.sgn_set_step_graphs(c, 0)  # the profiled pass times direct launches

    # profiled pass over the same steps and calls as the timed region (B
    # sources per call), one field at a time (HIP events on each context's
    # stream)
    for c in ctxs:
        sg.sgn_profile_reset(c)
        sg.sgn_set_profiling(c, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ks_prof = []
    for q in range(len(MUS)):  # the first context of each field (the others are gone)
        lane_steps(q, args.warmup, args.steps, ks_prof, False)
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t1
    kstats = {}
    for c in ctxs:
        for name, s in sg.sgn_profile_read(c).items():
            a = kstats.setdefault(name, {"launches": 0, "ms": 0.0, "bytes": 0.0, "flops": 0.0})
            for key in a:
                a[key] += s[key]
        sg.sgn_set_profiling(c, False)
    kern = kernel_table(kstats)
    log("kernels: " + json.dumps(kern))
    kmap = HBM_KERNELS
    if args.block_steps:
        kmap = dict(HBM_KERNELS_BLOCK)
        if args.block_steps > 8:  # the three-multiplication forms of the sweeps
            kmap.update({"block_dot": "bdot3_kernel<4>" if B >= 4 else "bdot3_kernel<2>",
                         "block_update": "bupdate_kernel<true, 2>" if B >= 4 else "bupdate_kernel<true, 1>",
                         "block_factor": "bsmall_kernel<true>"})
    hbm_kernels = {k: v for k, v in kern.items() if k in kmap}
    dom = max(hbm_kernels, key=lambda k: hbm_kernels[k]["total_ms"]) if hbm_kernels else None
    roofline = None
    if dom:
        s = kstats[dom]
        achieved = s["bytes"] / (s["ms"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": stored_traffic(kmap[dom]),
                    "kernel": kmap[dom], "avg_launch_us": kern[dom]["avg_us"],
                    "bytes_per_launch": round(s["bytes"] / s["launches"], 1)}
    # the timed region's aggregate rate: the Krylov passes' and the stencil's
    # algorithmic bytes per apply (from the profiled pass) times applies per second
    aggregate = None
    nprof = len(ks_prof)
    if nprof and all(k in kstats for k in kmap):
        per_apply = sum(kstats[k]["bytes"] for k in kmap) / nprof
        gbs = per_apply * value / 1e9
        aggregate = {"GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBPS, 4),
                     "bytes_per_apply": round(per_apply), "mean_k_profiled": round(float(np.mean(ks_prof)), 1),
                     "kernels": sorted(kmap)}
    sign = None
    if "ns_gemm" in kstats and kstats["ns_gemm"]["ms"] > 0:
        s = kstats["ns_gemm"]
        tf = s["flops"] / (s["ms"] * 1e-3) / 1e12
        sign = {"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / FP64_MFMA_PEAK_TFLOPS, 4), "avg_launch_us": kern["ns_gemm"]["avg_us"],
                "kernel": "zgemm_splitk_kernel / zgemm_kernel (hand-written, v_mfma_f64_16x16x4f64), "
                          "Newton-Schulz products X^2 and X Y / 2 with their epilogues"}
    stencil_6 = None
    if "wilson_hw" in kstats and kstats["wilson_hw"]["ms"] > 0:
        s = kstats["wilson_hw"]
        gb = s["bytes"] / (s["ms"] * 1e-3) / 1e9
        stencil_6 = {"workload": "6^4 FP64 (inside the applies)", "achieved": round(gb, 1), "unit": "GB/s",
                     "frac": round(gb / HBM_PEAK_GBPS, 4), "avg_launch_us": kern["wilson_hw"]["avg_us"]}

    ov = None if args.no_overlap else overlap_leg(sg, torch, ctxs[1], MUS[1], xs)
    ovs = None if args.no_overlap else overlap_solve_leg(sg, torch, ctxs[1], MUS[1], xs)
    lrd = None if args.no_lr else lr_leg(sg, synth, torch, MUS[1], xs, latency_schur(sg, torch, ctxs[1], xs),
                                         tune=not args.no_autotune)

    pairs = []  # the Schur pairs, for the oracle baseline
    for c in ctxs:
        S, T, _ = sg.sgn_deflate_export(c)
        pairs.append((S.cpu().numpy(), T))
        sg.sgn_destroy(c)

    stencil = None if args.no_stencil else stencil_leg(sg, synth, torch, tune=not args.no_autotune)
    batched = None if args.no_batched else batched_leg(sg, synth, torch, tune=not args.no_autotune)
    mixed8 = None if args.no_mixed else mixed_leg(sg, synth, torch, tune=not args.no_autotune)
    small4 = None if args.no_mixed else undeflated_4x4_leg(sg, synth, torch)
    if stencil is not None and stencil_6 is not None:
        stencil["in_apply_6x6x6x6"] = stencil_6

    setup_times = None if args.no_setup else setup_leg(sg, synth, torch, SETUP_SCAN)
    serving = None
    if not args.no_serving:
        serving = serving_leg(sg, synth, torch, *SERVE_DEFAULT, sg.SGN_PREC_FP64)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pairs, xs[0].cpu().numpy(), [acc[str(mu)]["k"] for mu in MUS], links)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sgn(H_w(mu))x, 6^4 lattice (N=15552), m_w=-1.6, mu in {0.0,0.2,0.5}, "
                               "m=20 Schur deflation, kmax=500, tol=1e-10, FP64, 1 RHS per apply, "
                               + (f"{len(lanes) * B} applies per step (the fields one after another, {B} "
                                  f"source(s) per apply call)" if args.serial else
                                  f"{len(lanes) * B} applies per step ({P * B} per field in flight: {P} "
                                  f"context(s) and stream(s) per field, {B} source(s) per apply call)"),
                   "applies_in_flight_per_field": P * B, "contexts_per_field": P, "sources_per_call": B,
                   "graph_steps": args.graph_steps,
                   "block_steps": args.block_steps,
                   "lattice": list(DIMS), "m": M_DEFL, "kmax": KMAX, "tol": TOL, "mu": list(MUS),
                   "mean_k": round(float(np.mean(ks)), 1), "timed_unconverged": timed_unconverged},
        "accuracy": {"timed_applies": timed_acc, "seed_1000": acc},
        "latency": latency,
        "setup": setup,
        "roofline": roofline,
        "aggregate_timed_region": aggregate,
        "stencil": stencil,
        "batched_mixed_12x12x12x12": batched,
        "mixed_8x8x8x8": mixed8,
        "undeflated_4x4x4x4": small4,
        "small_sign": sign,
        "overlap": ov,
        "overlap_solve": ovs,
        "lr_deflation": lrd,
        "deflation_setup": setup_times,
        "serving": serving,
        "kernels": kern,
        "profiled_pass_seconds": round(elapsed_prof, 4),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def counters_leg(sg, synth, torch, block_steps, B):
    """One batched call of B sources per field of the headline configuration
    (profiling on: the library's algorithmic bytes per launch), for the
    rocprofv3 FETCH_SIZE / WRITE_SIZE passes that wrap this command."""
    links = synth.random_links(DIMS, synth.GAUGE_SEED)
    N = 12 * int(np.prod(DIMS))
    X = torch.stack([torch.from_numpy(synth.gaussian_source(DIMS, 1000 + r)) for r in range(B)]).cuda()
    Y = torch.empty_like(X)
    stats = {}
    for mu in MUS:
        ctx = sg.sgn_create(links, DIMS, mu, M_W)
        sg.sgn_deflate(ctx, M_DEFL)
        sg.sgn_set_block_steps(ctx, block_steps)
        sg.sgn_profile_reset(ctx)
        sg.sgn_set_profiling(ctx, True)
        sg.sgn_apply_batched(ctx, X, Y, TOL, KMAX)
        torch.cuda.synchronize()
        for name, st in sg.sgn_profile_read(ctx).items():
            a = stats.setdefault(name, {"launches": 0, "bytes": 0.0})
            a["launches"] += st["launches"]
            a["bytes"] += st["bytes"]
        sg.sgn_destroy(ctx)
    return {"workload": f"6^4, mu in {list(MUS)}, m={M_DEFL}, {B} sources per batched call, block steps "
                        f"{block_steps}, tol {TOL}, N={N}",
            "per_class": {k: {"launches": v["launches"], "algorithmic_bytes_per_launch": round(v["bytes"] / v["launches"])}
                          for k, v in stats.items() if v["launches"]}}


def timed_accuracy(torch, outs, gold, nstored, P, B, warmup, steps):
    """Relative error |y - y_exact| / |y_exact| of every timed apply (the
    Results section's measure), against the stored exact results."""
    if outs is None or not nstored:
        return None
    errs, per_mu = [], {}
    for q, lane in enumerate(outs):
        f, p = q % len(MUS), q // len(MUS)
        for i, Yb in enumerate(lane):
            r = warmup + i
            for b in range(B):
                ref = gold[f][((r * P + p) * B + b) % nstored]
                y = Yb[b]
                e = float(torch.linalg.vector_norm(y - ref) / torch.linalg.vector_norm(ref))
                errs.append(e)
                per_mu.setdefault(str(MUS[f]), []).append(e)
    return {"applies": len(errs), "max_rel_err": max(errs), "median_rel_err": float(np.median(errs)),
            "max_rel_err_per_mu": {k: max(v) for k, v in per_mu.items()},
            "sources": f"Gaussian seeds 1000..{1000 + nstored - 1}, cycled",
            "reference": "oracle dense Roberts sign of H_w(mu) (stored exact y per source and field)"}


def latency_schur(sg, torch, ctx, xs, reps=10):
    """ms per apply, one at a time, and mean k of the Schur-deflated field."""
    y = torch.empty_like(xs[0])
    ks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        sg.sgn_apply(ctx, xs[r % len(xs)], y, TOL, KMAX)
        ks.append(sg.sgn_last_info(ctx)["k_used"])
    torch.cuda.synchronize()
    return {"ms_per_apply": round(1e3 * (time.perf_counter() - t0) / reps, 3), "mean_k": float(np.mean(ks))}


M_SCAN = ((DIMS, 0.2, (0, 10, 20, 30, 40)), ((8, 8, 8, 8), 0.3, (0, 15, 30, 45, 60)))


def m_scan_leg(sg, synth, torch, reps=6):
    """Deflation size against cost (the paper's closing question: how the
    best m and the setup time depend on the volume).  Per lattice and m: the
    Schur setup time (sgn_deflate), the mean k and ms per apply at tol 1e-10
    (FP64, one at a time, kmax 1200), and the number of applies after which
    the setup has paid for itself against m = 0."""
    out = []
    for dims, mu, ms in M_SCAN:
        links = synth.random_links(dims, synth.GAUGE_SEED)
        xs = [torch.from_numpy(synth.gaussian_source(dims, 1000 + r)).cuda() for r in range(reps)]
        y = torch.empty_like(xs[0])
        rows = []
        for m in ms:
            ctx = sg.sgn_create(links, dims, mu, M_W)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if m:
                    sg.sgn_deflate(ctx, m)
                torch.cuda.synchronize()
                setup = time.perf_counter() - t0
                sg.sgn_apply(ctx, xs[0], y, TOL, 1200)  # first apply: places the checkpoints
                ks = []
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for x in xs:
                    st = sg.sgn_apply(ctx, x, y, TOL, 1200)
                    ks.append(sg.sgn_last_info(ctx)["k_used"] if st == sg.SGN_OK else None)
                torch.cuda.synchronize()
                ms_apply = 1e3 * (time.perf_counter() - t0) / len(xs)
            finally:
                sg.sgn_destroy(ctx)
            row = {"m": m, "setup_s": round(setup, 3), "mean_k": (float(np.mean(ks)) if None not in ks else None),
                   "ms_per_apply": round(ms_apply, 3)}
            rows.append(row)
            log(f"m-scan {dims} mu={mu}: {row}")
        base = rows[0]["ms_per_apply"]
        for row in rows[1:]:
            gain = base - row["ms_per_apply"]
            row["break_even_applies"] = round(1e3 * row["setup_s"] / gain, 1) if gain > 0 else None
        out.append({"lattice": list(dims), "N": 12 * int(np.prod(dims)), "mu": mu, "tol": TOL, "rows": rows})
    return {"workload": "deflation size scan, FP64, one source per apply, one at a time", "scan": out}


# deflation setup (sgn_deflate): lattice, mu, m, filter degrees timed (0 = the
# unfiltered thick-restart Arnoldi on H_w^2)
SETUP_SCAN = (((8, 8, 8, 8), 0.5, 30, (16, 0)), ((12, 12, 12, 12), 0.5, 40, (16,)),
              ((16, 16, 16, 16), 0.5, 60, (16,)))
SETUP_SCAN_FULL = (((6, 6, 6, 6), 0.2, 20, (16, 0)), ((8, 8, 8, 8), 0.5, 30, (8, 16, 24, 0)),
                   ((12, 12, 12, 12), 0.5, 40, (16, 24, 0)), ((16, 16, 16, 16), 0.5, 60, (16, 32)))


def setup_leg(sg, synth, torch, scan):
    """Deflation setup time (the Results section's initialisation cost) with
    the Chebyshev-filtered eigensolver against the unfiltered one, on the
    serving stream's mu = 0.5 fields."""
    rows = []
    for dims, mu, m, degrees in scan:
        links = synth.random_links(dims, synth.GAUGE_SEED)
        for deg in degrees:
            ctx = sg.sgn_create(links, dims, mu, M_W)
            try:
                sg.sgn_set_deflation_filter(ctx, deg)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sg.sgn_deflate(ctx, m)
                torch.cuda.synchronize()
                row = {"lattice": list(dims), "mu": mu, "m": m, "degree": deg,
                       "seconds": round(time.perf_counter() - t0, 3), **sg.sgn_deflate_stats(ctx)}
            finally:
                sg.sgn_destroy(ctx)
            rows.append(row)
            log(f"setup {dims} mu={mu} m={m} degree={deg}: {row}")
    return {"workload": "sgn_deflate (critical Schur pair), FP64", "rows": rows}


def undeflated_4x4_leg(sg, synth, torch, reps=20):
    """4^4, mu = 0.3, no deflation, exactly k = 300 Arnoldi steps (FP64), one
    source per apply: error of the seed-1000 source against its stored exact
    sign (full diagonalisation) and the rate, one at a time."""
    dims, mu, k = (4, 4, 4, 4), 0.3, 300
    ctx = sg.sgn_create(synth.random_links(dims, synth.GAUGE_SEED), dims, mu, M_W)
    try:
        x = torch.from_numpy(synth.gaussian_source(dims, 1000)).cuda()
        y = torch.empty_like(x)
        sg.sgn_apply_fixed(ctx, x, y, k)
        out = {"workload": f"4^4 (N=3072), mu={mu}, m=0, k={k} fixed, FP64, 1 RHS per apply, one at a time"}
        path = os.path.join(GOLDEN, "c4_mu0.3.npy")
        if os.path.exists(path):
            exact = np.load(path, allow_pickle=False)
            out["rel_err_vs_exact"] = float(np.linalg.norm(y.cpu().numpy() - exact) / np.linalg.norm(exact))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sg.sgn_apply_fixed(ctx, x, y, k)
        torch.cuda.synchronize()
        out["applies_per_s"] = round(reps / (time.perf_counter() - t0), 3)
    finally:
        sg.sgn_destroy(ctx)
    log(f"4^4: {out}")
    return out


def mixed_leg(sg, synth, torch, tune=True, reps=5):
    """8^4, mu = 0.3, m = 30 Schur vectors: mixed precision (FP32 stencil and
    Krylov basis, tol 1e-7) against FP64 (tol 1e-10), one source per apply,
    one at a time on the same field and Schur pair: error of the seed-1000
    source against the stored FP64 oracle result (k = 800), k and rate."""
    from paper_0704_3486_amd.autotune import autotune

    dims, mu, m = (8, 8, 8, 8), 0.3, 30
    links = synth.random_links(dims, synth.GAUGE_SEED)
    xs = [torch.from_numpy(synth.gaussian_source(dims, 1000 + r)).cuda() for r in range(reps)]
    path = os.path.join(GOLDEN, "c8_mu0.3.npy")
    ref = np.load(path, allow_pickle=False) if os.path.exists(path) else None
    out = {"workload": f"8^4 (N={12 * 8 ** 4}), mu={mu}, m={m}, 1 RHS per apply, one at a time"}
    ctxs = {}
    try:
        t0 = time.perf_counter()
        for prec, tol in ((sg.SGN_PREC_MIXED, 1e-7), (sg.SGN_PREC_FP64, 1e-10)):
            ctx = sg.sgn_create(links, dims, mu, M_W)
            ctxs[prec] = ctx
            sg.sgn_set_precision(ctx, prec)
            if prec == sg.SGN_PREC_MIXED:
                sg.sgn_deflate(ctx, m)
                out["deflation_seconds"] = round(time.perf_counter() - t0, 2)
                S, T, _ = sg.sgn_deflate_export(ctx)
            else:
                sg.sgn_deflate_import(ctx, S, T)
            if tune:
                autotune(ctx, k=300)
            y = torch.empty_like(xs[0])
            sg.sgn_apply(ctx, xs[0], y, tol, 800)
            name = "mixed" if prec == sg.SGN_PREC_MIXED else "fp64"
            entry = {"tol": tol, "k": sg.sgn_last_info(ctx)["k_used"]}
            if ref is not None:
                entry["rel_err_vs_fp64_oracle"] = float(np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for x in xs:
                sg.sgn_apply(ctx, x, y, tol, 800)
            torch.cuda.synchronize()
            entry["applies_per_s"] = round(len(xs) / (time.perf_counter() - t1), 3)
            out[name] = entry
    finally:
        for c in ctxs.values():
            sg.sgn_destroy(c)
    log(f"mixed 8^4: {out}")
    return out


def lr_leg(sg, synth, torch, mu, xs, schur, reps=10, tune=True):
    """LR-deflation (right and left critical eigenvectors, m = M_DEFL) on the
    same 6^4 field against its Schur deflation: setup time, error on the
    source with a stored exact result, ms per apply and k, one at a time."""
    t0 = time.perf_counter()
    ctx = sg.sgn_create(synth.random_links(DIMS, synth.GAUGE_SEED), DIMS, mu, M_W)
    try:
        sg.sgn_deflate_lr(ctx, M_DEFL)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        if tune:
            from paper_0704_3486_amd.autotune import autotune

            autotune(ctx, k=AUTOTUNE_K)
        y = torch.empty_like(xs[0])
        out = {"workload": f"6^4, mu={mu}, m={M_DEFL} (LR), tol={TOL}, FP64, 1 RHS per apply, one at a time",
               "setup_seconds": round(setup_s, 3), **sg.sgn_deflate_stats(ctx)}
        sg.sgn_apply(ctx, xs[0], y, TOL, KMAX)
        path = os.path.join(GOLDEN, f"c6_mu{mu}.npy")
        if os.path.exists(path):
            exact = np.load(path, allow_pickle=False)
            out["rel_err_vs_exact"] = float(np.linalg.norm(y.cpu().numpy() - exact) / np.linalg.norm(exact))
        lat = latency_schur(sg, torch, ctx, xs, reps)
        out["ms_per_apply"], out["mean_k"] = lat["ms_per_apply"], lat["mean_k"]
        out["schur_same_field"] = schur
    finally:
        sg.sgn_destroy(ctx)
    log(f"lr: {out}")
    return out


OVS_MASSES = (0.5, 0.1)


def overlap_solve_leg(sg, torch, ctx, mu, xs):
    """D(m) x = b for the massive overlap operator (1 - m/2) D_ov + m on the
    6^4 field with its m = 20 Schur pair: restarted GMRES (50) over sign
    applies (inner tol 1e-10), outer tol 1e-8, the seed-1000 source as b;
    outer steps, seconds and the true relative residual per mass."""
    b = xs[0]
    x = torch.empty_like(b)
    out = {"workload": f"6^4, mu={mu}, m={M_DEFL} Schur, D(m) = (1 - m/2) D_ov + m, GMRES(50), tol 1e-8, "
                       "inner sign tol 1e-10, FP64", "solves": []}
    for mass in OVS_MASSES:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, res = sg.sgn_overlap_solve(ctx, b, x, mass, 1e-8, max_iter=2000, restart=50, inner_tol=1e-10,
                                           inner_kmax=KMAX)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out["solves"].append({"mass": mass, "status": st, "outer_steps": it, "rel_residual": res,
                              "seconds": round(sec, 3), "ms_per_outer_step": round(1e3 * sec / max(it, 1), 3)})
    log(f"overlap solve: {out}")
    return out


def overlap_leg(sg, torch, ctx, mu, xs, reps=10):
    """D_ov(mu) x = x + gamma5 sgn(H_w(mu)) x on one 6^4 field: the error on
    the source with a stored exact sign, the Ginsparg-Wilson defect
    ||D g5 D x - (g5 D x + D g5 x)|| / ||x|| from three applies, and the rate
    of one apply at a time."""
    N = xs[0].numel()
    g5 = torch.from_numpy(np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), N // 12)).to(xs[0].device)
    y = torch.empty_like(xs[0])
    out = {"workload": f"6^4, mu={mu}, m={M_DEFL}, tol={TOL}, FP64, 1 RHS per apply, one at a time"}
    path = os.path.join(GOLDEN, f"c6_mu{mu}.npy")
    sg.sgn_overlap_apply(ctx, xs[0], y, TOL, KMAX)
    if os.path.exists(path):
        x0 = xs[0].cpu().numpy()
        exact = x0 + g5.cpu().numpy() * np.load(path, allow_pickle=False)
        out["rel_err_vs_exact"] = float(np.linalg.norm(y.cpu().numpy() - exact) / np.linalg.norm(exact))

    def D(v):
        w = torch.empty_like(v)
        sg.sgn_overlap_apply(ctx, v.contiguous(), w, TOL, KMAX)
        return w

    dx = D(xs[1])
    defect = (D(g5 * dx) - g5 * dx - D(g5 * xs[1])).norm() / xs[1].norm()
    out["gw_defect"] = float(defect)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        sg.sgn_overlap_apply(ctx, xs[r % len(xs)], y, TOL, KMAX)
    torch.cuda.synchronize()
    out["applies_per_s_one_at_a_time"] = round(reps / (time.perf_counter() - t0), 3)
    log(f"overlap: {out}")
    return out


def kernel_table(kstats):
    kern = {}
    for name, s in kstats.items():
        if s["launches"] == 0:
            continue
        kern[name] = {
            "launches": s["launches"],
            "total_ms": round(s["ms"], 3),
            "avg_us": round(1e3 * s["ms"] / s["launches"], 3),
            "GBps": round(s["bytes"] / (s["ms"] * 1e-3) / 1e9, 1) if s["ms"] > 0 else None,
            "GFLOPs": round(s["flops"] / (s["ms"] * 1e-3) / 1e9, 1) if s["ms"] > 0 else None,
        }
    return kern


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the stored rocprofv3 counter runs,
    or None if absent or measured on a different source of the kernel."""
    import hashlib

    rec = None
    for path in (TRAFFIC_FILE, TRAFFIC_FILE_BLOCK):
        if not os.path.exists(path):
            continue
        with open(path) as f:
            for line in f:
                if line.startswith("traffic_json:"):
                    r = json.loads(line.split(":", 1)[1])
                    if r.get("kernel") == kernel:
                        rec = r
    if not rec:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return rec["bytes_per_launch"]


def stencil_leg(sg, synth, torch, tune=True):
    """H_w(mu) x on a 32^4 lattice, FP64, one right-hand side: average kernel
    time from the library's HIP events and algorithmic GB/s (48 V 16 bytes:
    read v, write w, the four links of a site as the two stored rows of each
    SU(3) matrix), beside a plain 2 GiB copy.  Also the rate in the unit of
    full 3 x 3 links (60 V 16 bytes per application), which counts the
    operator's data rather than what the kernel moves."""
    dims = STENCIL_DIMS
    links = synth.random_links(dims, synth.GAUGE_SEED)
    ctx = sg.sgn_create(links, dims, 0.3, M_W)
    del links
    try:
        from paper_0704_3486_amd.autotune import autotune_stencil

        # the walk order only (results bitwise the same); else the default walk
        walk = autotune_stencil(ctx) if tune else {"blocks": (0, 0, 0)}
        x = torch.from_numpy(synth.gaussian_source(dims, 1000)).cuda()
        y = torch.empty_like(x)
        for _ in range(3):
            sg.sgn_matvec(ctx, x, y)
        torch.cuda.synchronize()
        sg.sgn_profile_reset(ctx)
        sg.sgn_set_profiling(ctx, True)
        for _ in range(20):
            sg.sgn_matvec(ctx, x, y)
        torch.cuda.synchronize()
        s = sg.sgn_profile_read(ctx)["wilson_hw"]
    finally:
        sg.sgn_destroy(ctx)
    gb = s["bytes"] / (s["ms"] * 1e-3) / 1e9
    copy = copy_rate(torch)
    out = {"workload": "32^4 (V=1048576) FP64, 1 RHS, mu=0.3", "bound": "hbm", "achieved": round(gb, 1),
           "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(gb / HBM_PEAK_GBPS, 4),
           "avg_launch_us": round(1e3 * s["ms"] / s["launches"], 2), "kernel": HBM_KERNELS["wilson_hw"],
           "bytes_per_launch": s["bytes"] / s["launches"], "plain_copy_GBps": copy,
           "frac_of_plain_copy": round(gb / copy, 4), "walk_blocks": list(walk["blocks"]),
           "full_link_equivalent_GBps": round(gb * 60.0 / 48.0, 1),
           "full_link_equivalent_frac": round(gb * 60.0 / 48.0 / HBM_PEAK_GBPS, 4)}
    log(f"stencil: {out}")
    return out


BATCH_DIMS = (12, 12, 12, 12)
BATCH_M = 40
BATCH_NRHS = 32
BATCH_KMAX = 400
BATCH_TOL = 1e-7


def batched_leg(sg, synth, torch, tune=True):
    """32 sources of one 12^4 field (mu = 0.3, m = 40) in one mixed-precision
    batched apply, against FP64 single-source applies on the same field; the
    mixed results of two sources are compared with their FP64 results.  With
    tune, each precision's launch shape is autotuned first (FP64 single
    source at k = 200; mixed, 32 sources at k = 120; one timed call per
    shape, since the shapes give bitwise the same results)."""
    from paper_0704_3486_amd.autotune import autotune

    dims = BATCH_DIMS
    N = 12 * int(np.prod(dims))
    links = synth.random_links(dims, synth.GAUGE_SEED)
    ctx = sg.sgn_create(links, dims, 0.3, M_W)
    try:
        t0 = time.perf_counter()
        sg.sgn_deflate(ctx, BATCH_M)
        torch.cuda.synchronize()
        t_defl = time.perf_counter() - t0
        X = torch.from_numpy(np.stack([synth.gaussian_source(dims, 1000 + r) for r in range(BATCH_NRHS)])).cuda()
        shapes = {}
        if tune:
            t = autotune(ctx, k=200, nrhs=1, reps=1)
            shapes["fp64"] = [t["update_batch"], t["dot_cols"]]
        # FP64, one source at a time (tol 1e-10)
        y64 = torch.empty((2, N), dtype=torch.complex128, device="cuda")
        sg.sgn_apply(ctx, X[0], y64[0], TOL, BATCH_KMAX)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ks64 = []
        for r in range(2):
            sg.sgn_apply(ctx, X[r], y64[r], TOL, BATCH_KMAX)
            ks64.append(sg.sgn_last_info(ctx)["k_used"])
        torch.cuda.synchronize()
        fp64_rate = 2 / (time.perf_counter() - t0)
        # mixed precision, all sources in one batched call (one untimed call first)
        sg.sgn_set_precision(ctx, sg.SGN_PREC_MIXED)
        if tune:
            t = autotune(ctx, k=120, nrhs=BATCH_NRHS, reps=1)
            shapes["mixed_batched"] = [t["update_batch"], t["dot_cols"]]
        Y = torch.empty_like(X)
        sg.sgn_apply_batched(ctx, X, Y, BATCH_TOL, BATCH_KMAX)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, infos = sg.sgn_apply_batched(ctx, X, Y, BATCH_TOL, BATCH_KMAX)
        torch.cuda.synchronize()
        mixed_rate = BATCH_NRHS / (time.perf_counter() - t0)
        err = [float(torch.linalg.vector_norm(Y[r] - y64[r]) / torch.linalg.vector_norm(y64[r])) for r in range(2)]
        # sources 1000, 1001 against the oracle's FP64 deflated Arnoldi at k = 800
        gpath = os.path.join(GOLDEN, "c12_mu0.3_sources.npy")
        err_oracle = None
        if os.path.exists(gpath):
            gold = torch.from_numpy(np.load(gpath, allow_pickle=False)).cuda()
            err_oracle = {"mixed_batched": [float(torch.linalg.vector_norm(Y[r] - gold[r]) /
                                                  torch.linalg.vector_norm(gold[r])) for r in range(gold.shape[0])],
                          "fp64_single": [float(torch.linalg.vector_norm(y64[r] - gold[r]) /
                                                torch.linalg.vector_norm(gold[r])) for r in range(gold.shape[0])]}
        # the same batch with captured runs of 16 steps (bitwise the same results)
        sg.sgn_set_step_graphs(ctx, 16)
        Yg = torch.empty_like(X)
        sg.sgn_apply_batched(ctx, X, Yg, BATCH_TOL, BATCH_KMAX)  # captures
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sg.sgn_apply_batched(ctx, X, Yg, BATCH_TOL, BATCH_KMAX)
        torch.cuda.synchronize()
        graph_rate = BATCH_NRHS / (time.perf_counter() - t0)
        graph_same = bool(torch.equal(Yg, Y))
        sg.sgn_set_step_graphs(ctx, 0)
    finally:
        sg.sgn_destroy(ctx)
    out = {"workload": f"12^4 (N={N}), mu=0.3, m={BATCH_M} (sgn_deflate), {BATCH_NRHS} Gaussian sources, "
                       f"kmax={BATCH_KMAX}",
           "mixed_batched_applies_per_s": round(mixed_rate, 3), "mixed_tol": BATCH_TOL, "status": st,
           "mixed_k": [i["k_used"] for i in infos], "fp64_single_applies_per_s": round(fp64_rate, 3),
           "fp64_tol": TOL, "fp64_k": ks64, "speedup": round(mixed_rate / fp64_rate, 3),
           "mixed_rel_err_vs_fp64": err, "rel_err_vs_oracle_k800": err_oracle, "deflation_seconds": round(t_defl, 2),
           "mixed_batched_graph16_applies_per_s": round(graph_rate, 3), "graph16_bitwise_same": graph_same,
           "launch_shapes": shapes or None}
    log(f"batched: {out}")
    return out


# serving stream: lattice, deflation m, session kmax, arrival weight, share of
# the HBM budget for its Krylov workspaces.  The 12^4 and 16^4 fields draw
# mu = 0.5; their deflation bases (m = 40, 60) come from the filtered setup.
SERVE_FIELDS = [((6, 6, 6, 6), 20, 500, 0.4, 0.05), ((8, 8, 8, 8), 30, 500, 0.3, 0.10),
                ((12, 12, 12, 12), 40, 600, 0.2, 0.35), ((16, 16, 16, 16), 60, 600, 0.1, 0.50)]
# the bounded serving leg of the default run: arrivals at the offered rate,
# then at 70 % of the rate served
SERVE_DEFAULT = (200.0, 200, 120)
SERVE_TOL = 1e-8
SERVE_BUDGET = 150e9


def serving_leg(sg, synth, torch, rate, nreq, nreq_sustained, prec):
    """Poisson arrivals of sgn(H)x requests over four resident fields (6^4,
    8^4, 12^4, 16^4 with weights 0.4/0.3/0.2/0.1; field seeds G+1..G+4, mu per
    field drawn once from {0.1, 0.3, 0.5} with default_rng(G+100)), tol 1e-8,
    served by one continuous-batching session per field.

    Two streams over the same resident fields: `nreq` arrivals at the offered
    `rate` (inter-arrival times from default_rng(7)), which exceeds what one
    device serves, so its served rate is the device's capacity for this mix;
    then `nreq_sustained` arrivals at 70 % of that served rate
    (default_rng(8)), whose latencies are those of a stable queue.  Latency =
    host time from a request's arrival to its completion."""
    from paper_0704_3486_amd.serving import Server

    G = synth.GAUGE_SEED
    mus = np.random.default_rng(G + 100).choice([0.1, 0.3, 0.5], size=len(SERVE_FIELDS))
    srv = Server(SERVE_BUDGET, nsteps=4)
    setup = {}
    names = []
    for i, (dims, m, kmax, _, share) in enumerate(SERVE_FIELDS):
        name = "x".join(str(d) for d in dims)
        links = synth.random_links(dims, G + 1 + i)
        setup[name] = {"mu": float(mus[i]),
                       **srv.add_field(name, links, dims, float(mus[i]), M_W, m, kmax, share, prec)}
        log(f"serving setup {name}: {setup[name]}")
        names.append(name)
    try:
        offered = _serve_stream(srv, names, synth, torch, rate, nreq, 7, 1000)
        rate2 = round(0.7 * offered["served_applies_per_s"], 3)
        sustained = _serve_stream(srv, names, synth, torch, rate2, nreq_sustained, 8, 1000 + nreq)
    finally:
        srv.close()
    out = {"workload": "Poisson arrivals over 6^4/8^4/12^4/16^4 (0.4/0.3/0.2/0.1), tol "
                       + f"{SERVE_TOL}, " + ("mixed precision" if prec == sg.SGN_PREC_MIXED else "FP64"),
           "served_applies_per_s": offered["served_applies_per_s"], "offered": offered,
           "at_70pct_of_served": sustained, "setup": setup}
    log(f"serving: {out}")
    return out


def _serve_stream(srv, names, synth, torch, rate, nreq, arrival_seed, source_seed):
    """One bounded Poisson stream through the running server; returns its
    served rate and latency percentiles, overall and per field."""
    from paper_0704_3486_amd.serving import Request

    rng = np.random.default_rng(arrival_seed)
    arrive = np.cumsum(rng.exponential(1.0 / rate, nreq))
    which = rng.choice(len(SERVE_FIELDS), size=nreq, p=[f[3] for f in SERVE_FIELDS])
    reqs = []
    for q in range(nreq):
        dims, _, kmax, _, _ = SERVE_FIELDS[which[q]]
        x = torch.from_numpy(synth.gaussian_source(dims, source_seed + q)).cuda()
        reqs.append(Request(names[which[q]], x, torch.empty_like(x), SERVE_TOL, kmax))
    torch.cuda.synchronize()
    srv.start()
    t0 = time.perf_counter()
    log(f"serving: {nreq} arrivals at {rate}/s")
    for q, req in enumerate(reqs):
        delay = t0 + arrive[q] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        srv.submit(req)
    log(f"serving: {nreq} requests submitted in {time.perf_counter() - t0:.2f} s")
    mark = max(1, nreq // 10)
    for q, req in enumerate(reqs):
        req.done.wait()
        if (q + 1) % mark == 0:
            log(f"serving: first {q + 1} requests done at {time.perf_counter() - t0:.2f} s")
    srv.stop()
    t_end = max(r.t_done for r in reqs)
    lat = np.array([r.latency for r in reqs])
    fails = sum(1 for r in reqs if r.error is not None or r.info is None or not r.info["converged"])
    per = {}
    for name in names:
        sel = [r for r in reqs if r.field == name]
        if not sel:
            continue
        lf = np.array([r.latency for r in sel])
        per[name] = {"requests": len(sel), "p50_ms": round(1e3 * float(np.percentile(lf, 50)), 2),
                     "p99_ms": round(1e3 * float(np.percentile(lf, 99)), 2),
                     "mean_k": round(float(np.mean([r.info["k_used"] for r in sel if r.info])), 1)}
    out = {"offered_per_s": rate, "requests": nreq, "served_applies_per_s": round(nreq / (t_end - t0), 3),
           "arrival_span_s": round(float(arrive[-1]), 3), "makespan_s": round(t_end - t0, 3),
           "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
           "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2), "not_converged_or_failed": fails,
           "per_field": per}
    log(f"serving stream: {out}")
    del reqs
    torch.cuda.empty_cache()
    return out


def copy_rate(torch):
    """Read + write GB/s of a plain 2 GiB device copy (torch), timed with events."""
    n = 1 << 29
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    return round(8 * n / (ms * 1e-3) / 1e9, 1)


def calibrate_copy(torch):
    """A plain copy of known size: 2 GiB read and 2 GiB written per launch."""
    n = 1 << 29  # float32 elements
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 4,
                      "ms_per_copy": round(ms, 4), "GBps_read_plus_write": round(8 * n / (ms * 1e-3) / 1e9, 1)}))


def cpu_baseline(pairs, x, ks, links):
    """The oracle's plain deflated Arnoldi on the host, one apply per field on
    the seed-1000 source, at the Krylov dimension the GPU used for it."""
    from threadpoolctl import threadpool_info

    from oracle import arnoldi, wilson

    t_total = 0.0
    for f, mu in enumerate(MUS):
        A = wilson.hw_matrix(links, DIMS, mu, M_W)
        S, T = pairs[f]
        t0 = time.perf_counter()
        st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, int(ks[f]))
        arnoldi.approx_paper(S, T, st)
        t_total += time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    cores = len(os.sched_getaffinity(0))
    log(f"cpu baseline: {len(MUS)} applies in {t_total:.2f} s")
    # the same oracle on one core (BLAS limited to one thread): the mu = 0.2 field
    from threadpoolctl import threadpool_limits

    f1 = 1
    A = wilson.hw_matrix(links, DIMS, MUS[f1], M_W)
    S, T = pairs[f1]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        st = arnoldi.modified_arnoldi(lambda v: A @ v, x, S, int(ks[f1]))
        arnoldi.approx_paper(S, T, st)
        t_one = time.perf_counter() - t0
    log(f"cpu baseline, one core: 1 apply in {t_one:.2f} s")
    return {"value": round(len(MUS) / t_total, 4), "unit": "applies/s", "cores": int(min(threads, cores)),
            "kind": "oracle",
            "sample": f"one apply per field (mu 0.0, 0.2, 0.5) on the seed-1000 source at the GPU's k {list(ks)}, "
                      f"6^4, m=20, MGS x2 Arnoldi + Roberts + Appendix A Sylvester, {t_total:.1f} s total",
            "one_core": {"value": round(1.0 / t_one, 4), "unit": "applies/s", "cores": 1,
                         "sample": f"one apply on the mu = {MUS[f1]} field at k {int(ks[f1])}, BLAS on one "
                                   f"thread, {t_one:.1f} s"}}


if __name__ == "__main__":
    main()
