#!/usr/bin/env python3
"""Graph pairs scored per second on one MI355X (commute-time anomaly detection).

One step = one graph pair end to end: for each of the two snapshots build the
Gaussian-kernel graph (distances, median bandwidth, weights, degrees), build
the inverse chain (normalise, deflate, square while the cost model says it
pays), solve the k right-hand sides until the certified embedding error is
below 1e-6 (FP64 residuals); then score all node pairs and take the top 50.
Inputs (the two n x T windows) are resident in HBM before timing.

Workload: 128 x 128 grid (n = 16384), T = 240, k = 256, chain levels in FP16
(BF16 selectable) with FP32 accumulation (the mixed form), refined in FP64;
the same pair is also timed with BF16 and FP32 chains.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "graph pairs scored/s at n=16384, mixed vs FP32 at 1e-6 rel err; MFMA % peak"
PEAK = {  # MI355X published peaks
    "fp64_mfma": 78.6e12, "fp32_mfma": 157.3e12, "bf16_mfma": 2.5e15,
    # quarter-rate 32-bit integer multiplies: 16 lanes per SIMD every 4 cycles
    "int32_mul": 256 * 4 * 16 / 4 * 2.4e9,   # 9.83e12 per second
    "hbm": 8.0e12,
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_model(name, n, k, T, prec):
    """Algorithmic work of one launch: (bound, amount, unit-per-second, peak)."""
    esz = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2}[prec]
    ld = (n + 255) // 256 * 256
    if name == "square":
        peak = {"fp64": PEAK["fp64_mfma"], "fp32": PEAK["fp32_mfma"]}.get(prec, PEAK["bf16_mfma"])
        return "mfma", float(n) * n * (n + 1), "TFLOP/s", peak          # symmetric S^2
    if name == "residual":
        return "mfma", 2.0 * n * n * k, "TFLOP/s", PEAK["fp64_mfma"]
    if name == "score":
        return "mfma", 2.0 * n * n * k, "TFLOP/s", PEAK["fp64_mfma"]      # half of n x n x 2k
    if name == "gram_dist":
        return "mfma", float(n) * n * T, "TFLOP/s", PEAK["fp64_mfma"]      # half of n x n x T
    if name in ("rhs", "rhs_pair"):
        # The signed sums run on the int8 matrix cores; what bounds the kernel
        # is the VALU's SplitMix64 sign words (one per row, neighbour and 64
        # projections; the pair's two snapshots share them), whose two 64-bit
        # products take three quarter-rate 32-bit multiplies each.
        words = float(n) * n * ((k + 63) // 64)
        return "alu", 6.0 * words, "Tops/s", PEAK["int32_mul"]
    if name == "apply":
        return "hbm", float(n) * n * esz, "GB/s", PEAK["hbm"]
    if name == "exp_degree":
        return "hbm", 2.0 * ld * ld * 8, "GB/s", PEAK["hbm"]
    if name == "normalize":
        return "hbm", float(ld) * ld * (8 + esz), "GB/s", PEAK["hbm"]
    return None   # select_median: its passes read only the keys the Gram gathers


def vendor_gemm(torch, p, n, reps=5):
    """The vendor library's dense n x n x n GEMM of the same element type
    (torch.matmul on two contiguous matrices, hipBLASLt underneath), timed with
    events: what a tuned library reaches on this chip against the same peak."""
    dt = torch.bfloat16 if p == "bf16" else torch.float16
    g = torch.Generator(device="cuda:0").manual_seed(5)
    a = torch.rand(n, n, device="cuda:0", dtype=dt, generator=g)
    b = torch.rand(n, n, device="cuda:0", dtype=dt, generator=g)
    c = torch.matmul(a, b)                                       # warm-up (algorithm choice)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c = torch.matmul(a, b)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tf = 2.0 * float(n) ** 3 / (ms * 1e-3) / 1e12
    del a, b, c
    return {"ms": round(ms, 4), "achieved_tflops": round(tf, 1), "frac_of_peak": round(tf / 2500.0, 4),
            "flop_per_launch": 2.0 * float(n) ** 3}


def vendor_gemm_residual(torch, W, k, reps=5):
    """The vendor library's FP64 GEMM of the residual product's shape: a k x m
    operand times the m x m weight matrix (torch.matmul, the padded matrix of
    the timed step's first snapshot), timed with events: the attainable mark
    for the FP64 residual on the same box."""
    m = W.shape[0]
    g = torch.Generator(device="cuda:0").manual_seed(6)
    xt = torch.rand(k, m, device="cuda:0", dtype=torch.float64, generator=g)
    c = torch.matmul(xt, W)                                      # warm-up (algorithm choice)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c = torch.matmul(xt, W)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    tf = 2.0 * k * float(m) ** 2 / (ms * 1e-3) / 1e12
    del xt, c
    return {"ms": round(ms, 4), "achieved_tflops": round(tf, 1), "frac_of_peak": round(tf / (PEAK["fp64_mfma"] / 1e12), 4),
            "shape": [k, m, m]}


def vendor_gemm_apply(torch, p, m, k, reps=10):
    """The vendor library's 16-bit GEMM of one chain application's shape (an
    m x m level times an m x k operand, and the transposed orientation k x m
    times m x m; torch.matmul), timed with events."""
    dt = torch.bfloat16 if p == "bf16" else torch.float16
    g = torch.Generator(device="cuda:0").manual_seed(7)
    a = torch.rand(m, m, device="cuda:0", dtype=dt, generator=g)
    x = torch.rand(m, k, device="cuda:0", dtype=dt, generator=g)
    xt = x.t().contiguous()
    out = {}
    for name, f in (("level_x_operand", lambda: torch.matmul(a, x)),
                    ("operand_t_x_level", lambda: torch.matmul(xt, a))):
        c = f()                                                  # warm-up (algorithm choice)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            c = f()
        e1.record()
        e1.synchronize()
        out[name + "_ms"] = round(e0.elapsed_time(e1) / reps, 4)
    del a, x, xt, c
    return out


def copy_bandwidth(cdl, torch, reps):
    """GB/s of cdl.device_copy over 1 GiB (read + write bytes / event time)."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    cdl.device_copy(src, dst)                                   # warm-up
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        cdl.device_copy(src, dst)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    nbytes = 2 * src.numel() * 8
    del src, dst
    return {"GBps": round(nbytes / ms / 1e6, 1), "bytes_per_copy": nbytes, "ms": round(ms, 4),
            "copies": reps + 1, "kernel": "k_copy16"}


def roofline(times, name, n, k, T, prec, traffic=None):
    m = kernel_model(name, n, k, T, prec)
    cnt, ms = times[name]
    avg_s = ms / cnt / 1e3
    bound, amount, unit, peak = m
    scale = 1e12 if unit in ("TFLOP/s", "Tops/s") else 1e9
    achieved = amount / avg_s
    return {"kernel": name, "bound": bound, "achieved": round(achieved / scale, 3),
            "peak": round(peak / scale, 3), "unit": unit, "frac": round(achieved / peak, 4),
            "traffic": traffic, "avg_ms": round(avg_s * 1e3, 4), "launches": cnt,
            "algorithmic_per_launch": amount}


def load_traffic(kernel):
    """HBM bytes per launch measured with rocprofv3 counters, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[kernel]
    except Exception:
        return None
    src = os.path.join(ROOT, "paper_1802_05421_amd", "csrc", rec["source"])
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    return rec["bytes_per_launch"] if sha == rec["source_sha"] else None


def sequence_section(args, cdl, gen, torch, dev, seed, DMAX):
    """Batched uneven sequence: 24 snapshots, n_t ~ U{1024..8192} on a 96 x 96
    grid, k = 128, 23 consecutive-pair scores over the common global ids:
    synchronous, two streams with no host reads, a graph replay and the one-pass
    grouped form."""
    seqin = gen.make_sequence(G=96, T=120, n_snap=24, stride=30, n_min=1024, n_max=8192,
                              onsets=(8, 16))
    Xs = [torch.from_numpy(x).to(dev) for x in seqin.X]
    gids = [torch.from_numpy(g) for g in seqin.gid]
    sp = cdl.SeqParams(k=128, seed=seed, prec=args.mixed, depth=0, depth_max=DMAX, tol=1e-8,
                       max_iter=30, top_k=50)
    Fs, tops, sinfo = cdl.score_sequence(Xs, gids, sp)        # warm-up (and workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Fs, tops, sinfo = cdl.score_sequence(Xs, gids, sp)
    torch.cuda.synchronize()
    ms_seq = time.perf_counter() - t0
    sequence = {"workload": "24 snapshots, n_t in [1024, 8192] (sum %d), T=120, k=128, %s chain, "
                            "FP64 residual 1e-8" % (sum(len(g) for g in seqin.gid), args.mixed.upper()),
                "ms_per_sequence": round(ms_seq * 1e3, 2), "pairs": sinfo.pairs,
                "pairs_per_s": round(sinfo.pairs / ms_seq, 2),
                "max_iterations": sinfo.max_iterations,
                "max_rel_residual": sinfo.max_rel_residual}
    log("sequence: %d pairs in %.1f ms" % (sinfo.pairs, ms_seq * 1e3))
    # The same sequence enqueued with no host reads, consecutive snapshots
    # on two streams, then also captured and replayed as a HIP graph:
    # every chain at the largest depth the adaptive rule picks over the
    # snapshots, every solve at the largest iteration count above (two
    # more per retry); the library rejects the call if any final residual
    # stays above 1e-8.
    dfix = 1
    for Xq in Xs:
        gb = cdl.build_graph(Xq)
        dfix = max(dfix, cdl.build_chain(gb, prec=args.mixed, depth=0, depth_max=DMAX).depth)
        del gb
    gdev = [g.to(dev) for g in gids]
    iters, err, replay = sinfo.max_iterations, None, None
    for attempt in range(3):
        spa = cdl.SeqParams(k=128, seed=seed, prec=args.mixed, depth=dfix, tol=1e-8,
                            max_iter=iters, top_k=50, asynchronous=True, graph=True)
        spe = cdl.SeqParams(k=128, seed=seed, prec=args.mixed, depth=dfix, tol=1e-8,
                            max_iter=iters, top_k=50, asynchronous=True)
        try:
            sws = torch.empty(cdl.sequence_workspace_bytes(Xs, gdev, spa), dtype=torch.uint8,
                              device=dev)
            Fa, ta, ainfo = cdl.score_sequence(Xs, gdev, spe, ws=sws, out=None)   # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                Fa, ta, ainfo = cdl.score_sequence(Xs, gdev, spe, ws=sws, out=(Fa, ta))
            torch.cuda.synchronize()
            ms_async = (time.perf_counter() - t0) / 3
            sequence["async_two_streams"] = {
                "ms_per_sequence": round(ms_async * 1e3, 2),
                "pairs_per_s": round(ainfo.pairs / ms_async, 2), "chain_depth": dfix,
                "iterations": iters, "max_rel_residual": ainfo.max_rel_residual}
            log("sequence, two streams, no host reads: %.1f ms" % (ms_async * 1e3))
            Fa, ta, ainfo = cdl.score_sequence(Xs, gdev, spa, ws=sws, out=(Fa, ta))   # eager enqueue
            Fa, ta, ainfo = cdl.score_sequence(Xs, gdev, spa, ws=sws, out=(Fa, ta))   # capture
            torch.cuda.synchronize()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                Fa, ta, ainfo = cdl.score_sequence(Xs, gdev, spa, ws=sws, out=(Fa, ta))
            torch.cuda.synchronize()
            ms_graph = (time.perf_counter() - t0) / reps
            replay = {"ms_per_sequence": round(ms_graph * 1e3, 2),
                      "pairs_per_s": round(ainfo.pairs / ms_graph, 2),
                      "chain_depth": dfix, "iterations": iters,
                      "graph_launches": ainfo.graph_launches,
                      "max_rel_residual": ainfo.max_rel_residual}
            log("sequence as a graph replay: %.1f ms (depth %d, %d iterations)" % (ms_graph * 1e3, dfix, iters))
            break
        except cdl.CdlError as e:
            err = str(e)
            log("async sequence at depth %d, %d iterations: %s" % (dfix, iters, e))
            iters += 2
    sequence["graph_replay"] = replay if replay is not None else {"error": err}
    sws = None
    # One pass: every snapshot resident, grouped launches over all
    # snapshots (squarings, each refinement step) and pairs (scores),
    # convergence on the device (max_iter only bounds it).
    pb = cdl.SeqParams(k=128, seed=seed, prec=args.mixed, depth=dfix, tol=1e-8, max_iter=20,
                       top_k=50, asynchronous=True, batched=True)
    wsb = torch.empty(cdl.sequence_workspace_bytes(Xs, gdev, pb), dtype=torch.uint8, device=dev)
    Fb, tb, binfo = cdl.score_sequence(Xs, gdev, pb, ws=wsb)          # warm-up
    torch.cuda.synchronize()
    cdl.timing(reset=True)
    cdl.set_timing(True)
    Fb, tb, binfo = cdl.score_sequence(Xs, gdev, pb, ws=wsb, out=(Fb, tb))
    torch.cuda.synchronize()
    cdl.set_timing(False)
    kb = {nm: round(v[1], 3) for nm, v in sorted(cdl.timing(reset=True).items(), key=lambda x: -x[1][1])}
    t0 = time.perf_counter()
    for _ in range(3):
        Fb, tb, binfo = cdl.score_sequence(Xs, gdev, pb, ws=wsb, out=(Fb, tb))
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) / 3
    pbg = cdl.SeqParams(k=128, seed=seed, prec=args.mixed, depth=dfix, tol=1e-8, max_iter=20,
                        top_k=50, asynchronous=True, batched=True, graph=True)
    for _ in range(2):   # eager, then captured
        Fb, tb, binfo = cdl.score_sequence(Xs, gdev, pbg, ws=wsb, out=(Fb, tb))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        Fb, tb, ginfo = cdl.score_sequence(Xs, gdev, pbg, ws=wsb, out=(Fb, tb))
    torch.cuda.synchronize()
    ms_bg = (time.perf_counter() - t0) / 3
    same = all(set(a.tolist()) == set(b.tolist()) for a, b in zip(tb, tops))
    sequence["batched_one_pass"] = {
        "ms_per_sequence": round(ms_b * 1e3, 2), "pairs_per_s": round(binfo.pairs / ms_b, 2),
        "graph_replay_ms": round(ms_bg * 1e3, 2), "graph_launches": ginfo.graph_launches,
        "chain_depth": dfix, "iterations": binfo.max_iterations,
        "max_rel_residual": binfo.max_rel_residual, "top50_equal_to_synchronous": bool(same),
        "kernels_ms": kb}
    log("sequence, one pass (grouped): %.1f ms, as a graph replay %.1f ms" % (ms_b * 1e3, ms_bg * 1e3))
    wsb = None
    return sequence


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--grid", type=int, default=128, help="grid side G (n = G*G)")
    ap.add_argument("--tol", type=float, default=-1e-6,
                    help="> 0: relative FP64 residual target; < 0: certified embedding error")
    ap.add_argument("--mixed", default="fp16", choices=("bf16", "fp16"),
                    help="element type of the mixed-precision chain (headline value)")
    ap.add_argument("--no-stress", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-sequence", action="store_true")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the two-stream pair (its kernels overlap, so per-kernel traces exclude it)")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the streamed pair (weights recomputed panel by panel)")
    ap.add_argument("--stream-grid", type=int, default=0,
                    help="also time one streamed pair on a G x G grid (e.g. 512: n = 262144)")
    ap.add_argument("--stream-only", action="store_true",
                    help="run only the streamed section (prints its results as one JSON line)")
    ap.add_argument("--sequence-only", action="store_true",
                    help="run only the 24-snapshot sequence section (prints one JSON line)")
    ap.add_argument("--square-only", default="",
                    help="profiling runs: only two chain builds of depth 2 in this type (fp16/bf16/fp32) "
                         "on the first snapshot, one squaring each (prints one JSON line)")
    ap.add_argument("--square-variant", type=int, default=-1,
                    help="with --square-only: pin the squaring's launch variant (-1: the default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="profiling runs: exactly 4 plain 1 GiB copies first (the byte counters' reference)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU only (single-GPU hot path); "
              "--gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1802_05421_amd as cdl

    # The library's plain copy kernel over 1 GiB (four times the memory-side
    # cache): the attainable HBM rate, and with --calibrate-copy the known
    # byte count that the traffic counters are scaled by.
    hbm_copy = copy_bandwidth(cdl, torch, reps=3 if args.calibrate_copy else 5)
    log("plain copy: %.0f GB/s (read + write)" % hbm_copy["GBps"])

    G, T, k, seed = args.grid, 240, 256, gen.grid.PROJ_SEED
    n = G * G
    log("generating inputs G=%d n=%d T=%d" % (G, n, T))
    pair = gen.make_pair(G, T, 4, 4)
    dev = torch.device("cuda:0")
    X = [torch.from_numpy(pair.X0).to(dev), torch.from_numpy(pair.X1).to(dev)]
    Xpair = list(X)
    if args.square_only:   # one squaring per chain build, for counters
        g0 = cdl.build_graph(X[0])
        if args.square_variant >= 0:
            cdl.force_choice("square", args.square_variant)
        for _ in range(2):
            cdl.build_chain(g0, prec=args.square_only, depth=2, depth_max=6)
        torch.cuda.synchronize()
        cdl.timing(reset=True)
        cdl.set_timing(True)
        cdl.build_chain(g0, prec=args.square_only, depth=2, depth_max=6)
        cdl.set_timing(False)
        r = roofline(cdl.timing(reset=True), "square", n, k, T, args.square_only)
        print(json.dumps({"square_only": args.square_only, "variant": args.square_variant,
                          "roofline": r}), flush=True)
        return
    if args.sequence_only:   # the sequence section alone (for kernel traces)
        print(json.dumps({"sequence_c4": sequence_section(args, cdl, gen, torch, dev, seed, 6)}),
              flush=True)
        return
    if args.stream_only:   # the streamed section alone (for kernel traces)
        print(json.dumps({"streamed": streamed_section(args, cdl, gen, torch, dev, Xpair, n, T, k,
                                                       seed, None)}), flush=True)
        return
    m = cdl.ld(n)
    graphs = [cdl.Graph(W=torch.empty((m, m), dtype=torch.float64, device=dev),
                        deg=torch.empty(n, dtype=torch.float64, device=dev),
                        stats=torch.empty(4, dtype=torch.float64, device=dev), n=n) for _ in range(2)]
    DMAX = 6
    precs = [args.mixed] + [p for p in ("bf16", "fp16") if p != args.mixed] + ([] if args.no_fp32 else ["fp32"])
    sizes = {p: cdl.workspace_bytes(n, T, k, DMAX, p) for p in precs}
    gws = torch.empty(max(v["graph"] for v in sizes.values()), dtype=torch.uint8, device=dev)
    chb = {p: [torch.empty(sizes[p]["chain"], dtype=torch.uint8, device=dev) for _ in range(2)] for p in precs}
    sws = torch.empty(max(v["solve"] for v in sizes.values()), dtype=torch.uint8, device=dev)
    scws = torch.empty(sizes[precs[0]]["score"], dtype=torch.uint8, device=dev)
    Zb = {p: [torch.empty((n, k), dtype=torch.float64, device=dev) for _ in range(2)] for p in precs}
    Fb = {p: torch.empty(n, dtype=torch.float64, device=dev) for p in precs}
    Tb = {p: torch.empty(50, dtype=torch.int32, device=dev) for p in precs}

    sws_pair = torch.empty_like(sws)

    def step(prec, sigma=None, Xs=X, tol=None, dense=False):
        # graphs and chains of both snapshots, then both solves with the
        # right-hand sides of the pair made in one sweep (shared sign words)
        tol = args.tol if tol is None else tol
        infos, chs = [], []
        for t in (0, 1):
            # no separate degree check (one host read less): the chain build
            # rejects non-finite levels, which a zero or non-finite degree gives
            cdl.build_graph(Xs[t], sigma=sigma, ws=gws, out=graphs[t], check=False)
            ch = cdl.build_chain(graphs[t], prec=prec, depth=0, depth_max=DMAX, buf=chb[prec][t])
            if dense:   # Algorithm 2's schedule: one dense P1 product per iteration
                cdl.chain_densify(ch)
            chs.append(ch)
        _, _, si0, si1 = cdl.solve_embedding_pair(graphs[0], chs[0], graphs[1], chs[1], k, seed,
                                                  tol=tol, max_iter=30, ws=(sws, sws_pair),
                                                  Z=(Zb[prec][0], Zb[prec][1]))
        for ch, si in ((chs[0], si0), (chs[1], si1)):
            infos.append({"depth": ch.info.depth, "dense_levels": ch.info.dense_levels,
                          "rho_hat": round(ch.info.rho_hat, 5),
                          "rho_bound": round(ch.info.rho_bound, 5),
                          "fro": [round(ch.info.fro[i], 7) for i in range(ch.info.depth)],
                          "iterations": si.iterations,
                          "depth_used": [si.depth_used[i] for i in range(si.iterations)],
                          "history": ["%.2e" % si.history[i] for i in range(si.iterations)],
                          "rel_residual": si.rel_residual, "kappa": round(si.kappa, 4),
                          "certified_error": si.certified_error})
        cdl.anomaly_scores(Zb[prec][0], graphs[0], Zb[prec][1], graphs[1], top_k=50, ws=scws,
                           F=Fb[prec], top=Tb[prec])
        return infos

    def timed(prec, steps, warmup, **kw):
        for i in range(warmup):
            # the first warm-up step tunes the launch configurations it meets
            cdl.set_autotune(i == 0)
            step(prec, **kw)
            cdl.set_autotune(False)
            log("warmup %s %d/%d done" % (prec, i + 1, warmup))
        # one untimed step with every kernel bracketed by events: the
        # per-kernel breakdown and the dominant kernel
        torch.cuda.synchronize()
        cdl.timing(reset=True)
        cdl.set_timing(True)
        step(prec, **kw)
        torch.cuda.synchronize()
        cdl.set_timing(False)
        breakdown = cdl.timing(reset=True)
        modeled = {nm: v for nm, v in breakdown.items() if kernel_model(nm, n, k, T, prec)}
        dom = max(modeled, key=lambda nm: modeled[nm][1])
        # the timed steps: events around the dominant kernel's launches only
        # (each timed launch adds two event records to the stream)
        cdl.set_timing(True, only=[dom])
        t0 = time.perf_counter()
        for i in range(steps):
            infos = step(prec, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cdl.set_timing(False, only=None)
        times = cdl.timing(reset=True)
        log("%s: %d pairs in %.3f s" % (prec, steps, t1 - t0))
        return (t1 - t0) / steps, infos, times, breakdown, dom

    res = {}
    res[args.mixed] = timed(args.mixed, args.steps, args.warmup)
    ms_mixed, info_mixed, times_mixed, _, dom = res[args.mixed]
    for p in precs[1:]:
        res[p] = timed(p, args.fp32_steps, 1)

    # accuracy: certificates, and agreement of the forms
    acc = {"certified_error_bound": max(i["certified_error"] for i in info_mixed),
           "mixed_rel_residual": max(i["rel_residual"] for i in info_mixed)}
    for p in precs[1:]:
        zdiff = max(float(torch.linalg.norm(Zb[args.mixed][t] - Zb[p][t]) / torch.linalg.norm(Zb[p][t]))
                    for t in (0, 1))
        fdiff = float((Fb[args.mixed] - Fb[p]).abs().max() / Fb[p].abs().max())
        acc["vs_%s" % p] = {"rel_Z": zdiff, "rel_F": fdiff,
                            "top50_equal": bool(set(Tb[args.mixed].tolist()) == set(Tb[p].tolist())),
                            "certified_error_bound": max(i["certified_error"] for i in res[p][1])}

    top_ref = Tb[args.mixed].clone()
    # the timed step's results, for the oracle comparison of the CPU leg
    gpu_ref = {"Z": [Zb[args.mixed][t].cpu().numpy() for t in (0, 1)],
               "F": Fb[args.mixed].cpu().numpy(), "top": Tb[args.mixed].cpu().numpy()}

    # The chain squaring itself (the autotuner may skip it at this spectral
    # radius): one two-level chain per type, timed on its own.
    sq = {}
    for p in precs:
        cdl.set_autotune(True)     # tune the squaring's tile variant first
        cdl.build_chain(graphs[0], prec=p, depth=2, depth_max=DMAX, buf=chb[p][0])
        cdl.set_autotune(False)
        torch.cuda.synchronize()
        cdl.timing(reset=True)
        cdl.set_timing(True)
        cdl.build_chain(graphs[0], prec=p, depth=2, depth_max=DMAX, buf=chb[p][0])
        cdl.set_timing(False)
        r = roofline(cdl.timing(reset=True), "square", n, k, T, p)
        tuned = cdl.autotune_lookup("square", p, n)
        sq[p] = {"frac_of_peak": r["frac"], "achieved_tflops": r["achieved"], "peak_tflops": r["peak"],
                 "avg_ms": r["avg_ms"], "executed_tflop_per_launch": round(float(n) ** 3 / 1e12, 3),
                 # the symmetric kernel computes the n^3 flops of the upper
                 # tiles; a dense product of the same matrices would take 2 n^3
                 "dense_equivalent_tflop_per_launch": round(2.0 * float(n) ** 3 / 1e12, 3),
                 "tuned_variant": None if tuned is None else tuned[0]}
        if p in ("bf16", "fp16"):
            sq[p]["vendor_gemm"] = vendor_gemm(torch, p, n)

    # Stress case: bandwidth 0.3 x median pushes rho(S~) to ~0.8, so deep chains
    # (many squarings) are needed - mixed vs FP32 where the squarings dominate.
    stress = None
    if not args.no_stress:
        sig = 0.3 * float(graphs[0].stats[1])
        st = {}
        for p in ([args.mixed] + ([] if args.no_fp32 else ["fp32"])):
            # ||S~||_F > 1 here, so the certificate does not apply: FP64 residual 1e-8
            msp, inf, _, tms, _ = timed(p, 1, 1, sigma=sig, tol=1e-8)
            st[p] = {"ms_per_pair": round(msp * 1e3, 2), "pairs_per_s": round(1.0 / msp, 3),
                     "chain": inf, "square_ms": round(tms.get("square", (0, 0.0))[1], 2)}
        # the paper's dense schedule on the same pair: d - 1 extra products,
        # then one application per iteration instead of d (and no repeated
        # levels)
        msd, infd, _, tmd, _ = timed(args.mixed, 1, 1, sigma=sig, tol=1e-8, dense=True)
        st["%s_dense_schedule" % args.mixed] = {
            "ms_per_pair": round(msd * 1e3, 2), "pairs_per_s": round(1.0 / msd, 3), "chain": infd,
            "chain_product_ms": round(tmd.get("chain_product", (0, 0.0))[1], 2),
            "apply_ms": round(tmd.get("apply", (0, 0.0))[1], 2)}
        stress = {"sigma": round(sig, 4), "per_prec": st}
        if "fp32" in st:
            stress["mixed_over_fp32"] = round(st["fp32"]["ms_per_pair"] / st[args.mixed]["ms_per_pair"], 3)

    # The two snapshots of a pair are independent until the score: run them
    # from two host threads on two streams (each with its own library
    # context and workspaces) and score once both are done.
    sws2 = torch.empty_like(sws)
    gws2 = torch.empty_like(gws)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def concurrent_step(prec):
        errs = []

        def snap(t):
            try:
                with torch.cuda.stream(streams[t]):
                    cdl.build_graph(X[t], ws=(gws, gws2)[t], out=graphs[t], check=True)
                    ch = cdl.build_chain(graphs[t], prec=prec, depth=0, depth_max=DMAX, buf=chb[prec][t])
                    cdl.solve_embedding(graphs[t], ch, k, seed, tol=args.tol, max_iter=30,
                                        ws=(sws, sws2)[t], Z=Zb[prec][t])
            except Exception as e:   # re-raised on the main thread
                errs.append(e)

        ths = [threading.Thread(target=snap, args=(t,)) for t in (0, 1)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        if errs:
            raise errs[0]
        cur = torch.cuda.current_stream()
        cur.wait_stream(streams[0])
        cur.wait_stream(streams[1])
        cdl.anomaly_scores(Zb[prec][0], graphs[0], Zb[prec][1], graphs[1], top_k=50, ws=scws,
                           F=Fb[prec], top=Tb[prec])

    concurrent = None
    if not args.no_concurrent:
        concurrent_step(args.mixed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            concurrent_step(args.mixed)
        torch.cuda.synchronize()
        ms_conc = (time.perf_counter() - t0) / args.steps
        concurrent = {"ms_per_pair": round(ms_conc * 1e3, 3), "pairs_per_s": round(1.0 / ms_conc, 3),
                      "prec": args.mixed,
                      "top50_equal_to_timed_step": bool(torch.equal(Tb[args.mixed], top_ref))}
        log("two-stream pair: %.2f ms" % (ms_conc * 1e3))

    # Edge-level output for the same pair: top-50 edges (exact).  The stress
    # runs left other graphs in the buffers; the two-stream section rebuilt
    # the benchmark pair, otherwise rebuild it here.
    if concurrent is None:
        step(args.mixed)
    ews = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Fe, ea, eb, ev = cdl.anomaly_edges(Zb[args.mixed][0], graphs[0], Zb[args.mixed][1], graphs[1],
                                           top_k=50, ws=ews)
        torch.cuda.synchronize()
        ms_edges = time.perf_counter() - t0
    edges = {"ms": round(ms_edges * 1e3, 3), "top_k": 50,
             "best": [int(ea[0]), int(eb[0]), float(ev[0])]}
    log("top-50 edges: %.2f ms" % (ms_edges * 1e3))

    # Amortised sequence pair: in a sequence every snapshot is embedded once,
    # so one new pair costs one graph + chain + solve and one score.
    def seq_step(prec, t):
        cdl.build_graph(X[t], ws=gws, out=graphs[t], check=True)
        ch = cdl.build_chain(graphs[t], prec=prec, depth=0, depth_max=DMAX, buf=chb[prec][t])
        cdl.solve_embedding(graphs[t], ch, k, seed, tol=args.tol, max_iter=30, ws=sws, Z=Zb[prec][t])
        cdl.anomaly_scores(Zb[prec][t ^ 1], graphs[t ^ 1], Zb[prec][t], graphs[t], top_k=50, ws=scws,
                           F=Fb[prec], top=Tb[prec])

    seq_step(args.mixed, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        seq_step(args.mixed, (i + 1) & 1)
    torch.cuda.synchronize()
    ms_amort = (time.perf_counter() - t0) / args.steps
    amortized = {"ms_per_pair": round(ms_amort * 1e3, 3), "pairs_per_s": round(1.0 / ms_amort, 3),
                 "prec": args.mixed}
    log("amortised sequence pair: %.2f ms" % (ms_amort * 1e3))

    sequence = None if args.no_sequence else sequence_section(args, cdl, gen, torch, dev, seed, DMAX)

    streamed = None
    if not args.no_stream:
        streamed = streamed_section(args, cdl, gen, torch, dev, Xpair, n, T, k, seed, top_ref)

    # dominant kernel of the mixed step, timed live over the timed steps
    roof = roofline(times_mixed, dom, n, k, T, args.mixed, load_traffic(dom))
    if dom == "residual":
        roof["vendor_gemm"] = vendor_gemm_residual(torch, graphs[0].W, (k + 63) // 64 * 64)
    # one chain application of the mixed type against the vendor GEMM of its shape
    apply_ref = None
    if args.mixed in ("fp16", "bf16"):
        tuned_apply = cdl.autotune_lookup("apply", args.mixed, n, k)
        apply_ref = {"tuned_ms": None if tuned_apply is None else round(tuned_apply[2], 4),
                     "vendor": vendor_gemm_apply(torch, args.mixed, m, (k + 63) // 64 * 64)}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: the oracle on the whole pair")
        cpu = cpu_baseline(pair, k, seed, gpu_ref)

    out = {
        "metric": METRIC, "value": round(1.0 / ms_mixed, 4), "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_mixed * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "%s/f64" % args.mixed, "data": "synthetic",
        "config": {"workload": "C3 pair: 128x128 lat/lon grid, n=16384, T=240 AR(1) windows, "
                               "4 flipped 4x4 patches, k=256 Rademacher projections, %s chain "
                               "(FP32 accum) + FP64-residual Richardson, stop at certified "
                               "embedding error %s, top-50" % (args.mixed.upper(), (
                                   "%.0e" % -args.tol) if args.tol < 0 else "residual %.0e" % args.tol),
                   "n": n, "T": T, "k": k, "tol": args.tol, "chain_depth_max": DMAX},
        "forms": {p: {"value": round(1.0 / res[p][0], 4), "ms_per_step": round(res[p][0] * 1e3, 3),
                      "steps": args.steps if p == args.mixed else args.fp32_steps} for p in precs},
        "mixed_over_fp32": None if "fp32" not in res else round(res["fp32"][0] / ms_mixed, 3),
        "roofline": roof,
        "hbm_copy": hbm_copy,
        "squaring_mfma": sq,
        "chain": {p: res[p][1] for p in precs},
        "accuracy": acc,
        "stress": stress,
        "kernels_ms_per_step": {p: {nm: round(v[1], 3)
                                    for nm, v in sorted(res[p][3].items(), key=lambda x: -x[1][1])}
                                for p in precs},
        "concurrent_snapshots": concurrent,
        "edges_top50": edges,
        "amortized_sequence_pair": amortized,
        "sequence_c4": sequence,
        "streamed": streamed,
        "cpu_baseline": cpu,
        "autotune": autotune_report(cdl, precs, n, k),
        "apply_vs_vendor": apply_ref,
    }
    print(json.dumps(out), flush=True)


def autotune_report(cdl, precs, n, k):
    """The tuner's choices and measured candidate times for the benchmark shape."""
    rep = {}
    for fam in ("square", "apply", "residual"):
        for p in (precs if fam != "residual" else ["fp64"]):
            e = cdl.autotune_lookup(fam, p, n, k)
            if e is not None:
                rep["%s/%s" % (fam, p)] = {"choice": e[0], "candidates": e[1], "ms": round(e[2], 4)}
    return rep


def streamed_section(args, cdl, gen, torch, dev, Xpair, n, T, k, seed, top_ref):
    """Streamed snapshots: the same pair with no n x n FP64 matrix stored (the
    weights recomputed from the series on every sweep), with no n x n storage
    at all or with chain level 0 stored in the mixed type; optionally a pair
    whose weight matrices exceed device memory."""
    def stream_pair(Xp, wsb, reps, level=None, cbuf=None):
        cdl.timing(reset=True)
        cdl.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            gz = [cdl.stream_embedding(x, k, seed, tol=args.tol, max_iter=30, ws=wsb, level=level,
                                       chain_buf=cbuf) for x in Xp]
            Fz, tz = cdl.anomaly_scores(gz[0][1], gz[0][0], gz[1][1], gz[1][0], top_k=50)
        torch.cuda.synchronize()
        msp = (time.perf_counter() - t0) / reps
        cdl.set_timing(False)
        tms = cdl.timing(reset=True)
        nn, TT = Xp[0].shape
        kern = {nm: {"launches": v[0] // reps, "ms": round(v[1] / reps, 3)}
                for nm, v in sorted(tms.items(), key=lambda x: -x[1][1])}
        # algorithmic FP64 work of the two MFMA kernels: 2 n^2 T per full
        # Gram sweep, 2 n^2 k per product sweep
        sweeps = sum(1 for _ in range(0, nn, min(32768, cdl.ld(nn))))
        for nm, fl in (("stream_gram", 2.0 * nn * nn * TT), ("stream_gram_exp", 2.0 * nn * nn * TT),
                       ("stream_product", 2.0 * nn * nn * k)):
            if nm in kern and kern[nm]["ms"] > 0:
                nsw = kern[nm]["launches"] / sweeps
                kern[nm]["sweeps"] = nsw
                kern[nm]["tflops"] = round(nsw * fl / (kern[nm]["ms"] * 1e-3) / 1e12, 2)
                kern[nm]["frac_fp64_peak"] = round(kern[nm]["tflops"] / 78.6, 4)
        return {"ms_per_pair": round(msp * 1e3, 2), "pairs_per_s": round(1.0 / msp, 4),
                "iterations": [z[2].iterations for z in gz],
                "certified_error": max(z[2].certified_error for z in gz),
                "kernels_ms": kern}, tz

    def both_forms(Xp, nn, reps, warm):
        out = {}
        for level in (None, args.mixed):
            wsb = torch.empty(cdl.stream_workspace_bytes(nn, T, k, 0, level), dtype=torch.uint8,
                              device=dev)
            cbuf = None if level is None else torch.empty(
                cdl.workspace_bytes(nn, 1, 1, 1, level)["chain"], dtype=torch.uint8, device=dev)
            if warm:
                stream_pair(Xp, wsb, 1, level, cbuf)
            r, tz = stream_pair(Xp, wsb, reps, level, cbuf)
            r["workspace_gib"] = round((wsb.numel() + (0 if cbuf is None else cbuf.numel())) / 2 ** 30, 2)
            if top_ref is not None and nn == n:
                r["top50_equal_to_timed_step"] = bool(set(tz.tolist()) == set(top_ref.tolist()))
            out["no_matrix" if level is None else "stored_%s_level" % level] = r
            log("streamed pair n=%d (%s): %.1f ms" % (nn, "no n x n storage" if level is None else
                                                     "stored %s level" % level, r["ms_per_pair"]))
            del wsb, cbuf
            torch.cuda.empty_cache()
        return out

    streamed = {"c3_pair": None}
    if not (args.stream_only and args.stream_grid > 0):
        streamed["c3_pair"] = both_forms(Xpair, n, args.steps, True)
    if args.stream_grid > 0:
        Gs = args.stream_grid
        log("generating the streamed pair G=%d n=%d" % (Gs, Gs * Gs))
        big = gen.make_pair(Gs, T, 4, 8)
        Xbig = [torch.from_numpy(big.X0).to(dev), torch.from_numpy(big.X1).to(dev)]
        del big
        r = both_forms(Xbig, Gs * Gs, 1, False)
        r["workload"] = ("%dx%d grid, n=%d, T=%d, four 8x8 patches, k=%d; the FP64 weight "
                         "matrix of one snapshot would take %.0f GiB" % (
                             Gs, Gs, Gs * Gs, T, k, (Gs * Gs) ** 2 * 8 / 2 ** 30))
        streamed["large_pair"] = r
        del Xbig
    torch.cuda.empty_cache()
    return streamed


def cpu_baseline(pair, k, seed, gpu=None):
    """The oracle, as it stands, timed on the whole benchmark pair.

    Per snapshot: direct-difference distances, the lower-median bandwidth,
    Gaussian weights and degrees, the right-hand sides (C loops over every
    ordered pair), Z = L^+ Y by dense Cholesky; per pair: node scores by direct
    differences and the top-50.  Each stage is timed with perf_counter.  With
    `gpu` (the timed step's embeddings, scores and top-50, copied to the host)
    the same run gives the step's errors against the oracle.
    """
    import numpy as np
    import oracle
    st = {}

    def stage(name, fn, *a):
        t = time.perf_counter()
        r = fn(*a)
        st[name] = st.get(name, 0.0) + time.perf_counter() - t
        return r

    snaps = []
    for t, X in ((0, pair.X0), (1, pair.X1)):
        D2 = stage("distances", oracle.sq_distances, X)
        sigma = stage("bandwidth", oracle.bandwidth, D2)
        W = stage("weights", oracle.gaussian_weights, D2, sigma)
        del D2
        deg, vol = stage("degrees", oracle.degrees, W)
        Y = stage("rhs", oracle.rhs, W, k, seed)
        Z = stage("solve", oracle.solve_embedding, W, Y, deg)
        del W, Y
        snaps.append((Z, vol))
        log("cpu: oracle snapshot %d done (%.1f s so far)" % (t, sum(st.values())))
    F = stage("scores", oracle.scores, snaps[0][0], snaps[0][1], snaps[1][0], snaps[1][1])
    top = stage("top_k", oracle.top_k, F, 50)
    pair_s = sum(st.values())
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    cpu_model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = None
    try:
        info = np.show_config(mode="dicts")
        blas = info.get("Build Dependencies", {}).get("blas", {}).get("name")
    except Exception:
        pass
    out = {"value": round(1.0 / pair_s, 6), "unit": "pairs/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model, "blas": blas, "host_cpus": os.cpu_count(),
           "sample": "the whole benchmark pair (both snapshots at n = %d, k = %d, scores of all "
                     "nodes), measured stage by stage" % (pair.X0.shape[0], k),
           "seconds_per_pair": round(pair_s, 2),
           "stage_seconds": {a: round(b, 2) for a, b in st.items()}}
    if gpu is not None:
        ez = [float(np.linalg.norm(gpu["Z"][t] - snaps[t][0]) / np.linalg.norm(snaps[t][0]))
              for t in (0, 1)]
        ef = float(np.abs(gpu["F"] - F).max() / np.abs(F).max())
        srt = np.sort(F)[::-1]
        out["timed_step_vs_oracle"] = {
            "e_Z": ez, "e_F_inf": ef,
            "e_F_2": float(np.linalg.norm(gpu["F"] - F) / np.linalg.norm(F)),
            "top50_gap": float((srt[49] - srt[50]) / np.abs(F).max()),
            "top50_identical": bool(set(gpu["top"].tolist()) == set(top.tolist()))}
    return out


if __name__ == "__main__":
    main()
