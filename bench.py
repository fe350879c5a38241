#!/usr/bin/env python3
"""SuCo query benchmark on one MI355X.

Workload: SIFT-like n=1,000,000 points, d=128 non-negative integers 0..255,
N_s=8 subspaces, sqrtK=50 (2,500 cells per subspace), 10,000 queries,
k=10, beta=0.005 (B=5,000 candidates).  The index is built on the GPU
(suco_build, FP64 k-means, 25 iterations).  Inputs are seeded synthetic data
resident in HBM before timing starts.

The collision ratio alpha is swept over a grid; the timed step is one pass of
the whole query path (centre distances, Dynamic Activation, collision
counting, top-B selection, re-rank) over the 10,000 queries at the smallest
grid alpha whose recall@10 reaches 0.95 (recall against exact k-NN).  The
reported value is queries per second over the timed steps, QPS at
recall@10 = 0.95 interpolated on the sweep is reported alongside.

Also printed: per-step kernel times from HIP events recorded on the query
stream, the roofline of the dominant kernel, and the FP64 CPU oracle's QPS on a
bounded sample of the same queries (host cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALPHA_GRID = (0.0005, 0.00075, 0.001, 0.0015, 0.002, 0.003, 0.005, 0.0075, 0.01, 0.02, 0.03, 0.05)
TARGET_RECALL = 0.95


def exact_topk(Xd, Qd, k, chunk=256):
    """Exact k-NN ids by (squared distance, id) on the GPU.

    For this workload every coordinate is an integer in 0..255 and d=128, so
    |x|^2, |q|^2, x.q and the squared distance are integers below 2^24: the
    FP32 product-form distances are exact whatever the summation order."""
    import torch
    n = Xd.shape[0]
    xn = (Xd * Xd).sum(dim=1)
    ids = torch.arange(n, device=Xd.device, dtype=torch.int64)
    out = []
    for s in range(0, Qd.shape[0], chunk):
        q = Qd[s:s + chunk]
        d2 = xn[None, :] + (q * q).sum(dim=1)[:, None] - 2.0 * (q @ Xd.T)
        key = d2.round().to(torch.int64) * (1 << 24) + ids[None, :]
        out.append(torch.topk(key, k, dim=1, largest=False, sorted=True).values % (1 << 24))
    return torch.cat(out).to(torch.int32)


def exact_topk_float(Xd, Qd, k, extra=64, chunk=None):
    """Exact k-NN ids by (squared distance, id) for real-valued data: the FP32
    product-form distances shortlist k + extra points per query, whose
    distances are then recomputed in FP64 from the rows and sorted by
    (distance, id).  The shortlist is exact unless the FP32 form misorders a
    true neighbour past `extra` others, far beyond its rounding error here."""
    import torch
    if chunk is None:   # about 2 GiB of FP32 distances per block of queries
        chunk = max(1, min(512, (1 << 29) // Xd.shape[0]))
    xn = (Xd * Xd).sum(dim=1)
    out = []
    for s in range(0, Qd.shape[0], chunk):
        q = Qd[s:s + chunk]
        d2 = xn[None, :] + (q * q).sum(dim=1)[:, None] - 2.0 * (q @ Xd.T)
        short = torch.topk(d2, k + extra, dim=1, largest=False).indices
        del d2
        rows = Xd[short].double()
        e = ((rows - q.double()[:, None, :]) ** 2).sum(dim=2)
        order = torch.argsort(short, dim=1)                    # ties by id: sort ids first, stably by distance
        short, e = torch.gather(short, 1, order), torch.gather(e, 1, order)
        o2 = torch.sort(e, dim=1, stable=True).indices[:, :k]
        out.append(torch.gather(short, 1, o2))
    return torch.cat(out).to(torch.int32)


def recall_at(ids, gt):
    k = gt.shape[1]
    hit = (ids[:, :, None] == gt[:, None, :]).any(dim=2).sum(dim=1)
    return float(hit.float().mean() / k)


def exact_dists(Xd, Qd, ids):
    """Euclidean distances (FP64) of the points `ids` [nq][k] to the queries."""
    rows = Xd[ids.long()].double()
    return ((rows - Qd.double()[:, None, :]) ** 2).sum(dim=2).sqrt()


def mean_relative_error(dists, gt_d):
    """Sec. 5.1's MRE: the mean over queries and ranks of (d_i - d*_i) / d*_i, zero d*_i skipped."""
    g = gt_d.double()
    m = g > 0
    r = (dists.double() - g) / g.clamp_min(1e-300)
    return float(r[m].mean()) if bool(m.any()) else 0.0


def copy_bandwidth(mib=1024, reps=5):
    """GB/s of a device-to-device copy of `mib` MiB (bytes read plus bytes written per copy)."""
    import torch
    a = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def timed_steps(fn, steps, warmup):
    """(total ms, per-step ms list) of `steps` calls after `warmup`, HIP events on the current stream."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for j in range(steps):
        fn()
        ev[j + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[j].elapsed_time(ev[j + 1]) for j in range(steps)]
    return ev[0].elapsed_time(ev[steps]), per


KERNEL_SOURCES = ("query_kernels.hip", "bf16.hip", "wave.h", "suco_impl.h")


def src_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2411_14754_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs on this
    workload, if they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    t = json.load(open(p))
    if t.get("src_hash") != src_hash():
        return None
    e = t.get("workloads", {}).get(workload, {}).get("kernels", {}).get(kernel)
    return None if e is None else e.get("bytes_per_launch")


def host_cpu():
    """(threads the oracle may use, nproc, CPU model): the GPU machine gives one GPU's share of its
    cores (16) to a job whatever nproc shows."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return max(1, min(16, avail)), os.cpu_count() or 1, model


def oracle_rate(oix, Q, k, alpha, beta, threads, budget_s, cap):
    """Queries per second of the oracle on a prefix of Q sized to take about budget_s."""
    probe = min(cap, max(threads, 32))
    t0 = time.time()
    oix.query(Q[:probe], k, alpha, beta, nthreads=threads)
    dt = time.time() - t0
    m = int(min(cap, max(probe, probe * budget_s / max(dt, 1e-6))))
    if m > probe:
        t0 = time.time()
        oix.query(Q[:m], k, alpha, beta, nthreads=threads)
        dt = time.time() - t0
    else:
        m = probe
    return m / dt, m, dt


def cpu_baseline(X, Q, alpha, beta, k, sample, log):
    """The FP64 oracle (its own index, built from the same data) timed on the host: the host's
    share of cores and one thread, each on a prefix of the queries sized to about 10 s."""
    import oracle
    threads, nproc, model = host_cpu()
    t0 = time.time()
    _, c32, asg, _ = oracle.build_index(X, 8, 50, iters=25, seed=1, nthreads=threads)
    oix = oracle.Index(X, 8, 50, c32, asg)
    log(f"oracle index built in {time.time() - t0:.1f}s on {threads} threads")
    qps, m, dt = oracle_rate(oix, Q, k, alpha, beta, threads, 10.0, min(sample, Q.shape[0]))
    qps1, m1, dt1 = oracle_rate(oix, Q, k, alpha, beta, 1, 5.0, min(sample, Q.shape[0]))
    log(f"oracle: {qps:.1f} QPS on {threads} threads ({m} queries), {qps1:.1f} QPS on 1 thread ({m1} queries)")
    return {"value": round(qps, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "value_1_thread": round(qps1, 3), "nproc": nproc, "cpu_model": model,
            "sample": f"first {m} of the 10,000 queries on {threads} threads ({dt:.1f}s) and first {m1} on one "
                      f"thread ({dt1:.1f}s), each sized to ~10 s / ~5 s of work; alpha={alpha}, beta={beta}, "
                      f"k={k}; FP64 C oracle, OpenMP over queries"}


def bench_bf16(args, log):
    """GIST-like n=1,000,000 d=960 in (0,1), N_s=20, sqrtK=50, 1,000 queries,
    k=10, beta=0.005: BF16 split precision (MFMA centre distances, BF16 re-rank
    first pass, certified survivors, FP32 re-rank of the survivors) against the
    plain FP32 path on the same index, at the smallest grid alpha reaching
    recall@10 = 0.95."""
    import torch
    import paper_2411_14754_amd as suco
    import synth

    W = synth.Workload(3)
    sp = W.spec
    n, d, ns, sk, nq, k, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["k"], sp["beta"]
    log("generating data")
    X, Q = W.data(), W.queries()
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    torch.cuda.synchronize()
    t0 = time.time()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1, flags=suco.BUILD_BF16, tile_max=args.tile_max,
                          query_chunk=args.query_chunk)
    build_s = time.time() - t0
    log(f"index built in {build_s:.2f}s")
    gt = exact_topk_float(Xd, Qd, k)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dists = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    nsurv = torch.empty((nq,), dtype=torch.int32, device="cuda")
    relerr = torch.empty((nq, k), dtype=torch.float64, device="cuda")

    def run_bf16(alpha):
        suco._check(suco.lib().suco_query_bf16(ix._h, suco._dev(Qd, torch.float32), nq, k, alpha, beta,
                                               suco.BF16_S1, suco._dev(ids, torch.int32),
                                               suco._dev(dists, torch.float32), suco._dev(nsurv, torch.int32),
                                               None, None, suco._stream(None)))

    def run_plain(alpha):
        ix.query(Qd, k, alpha, beta, out=(ids, dists))

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1)

    sweep = []
    for a in ((0.0005, 0.00075, 0.001, 0.0015, 0.002, 0.003, 0.005, 0.01, 0.02, 0.05) if args.alpha is None
              else (args.alpha,)):
        ms_b = timed(lambda: run_bf16(a), 1, 1)
        rb = recall_at(ids, gt)
        ms_p = timed(lambda: run_plain(a), 1, 1)
        rp = recall_at(ids, gt)
        sweep.append({"alpha": a, "recall_bf16": round(rb, 5), "qps_bf16": round(nq / (ms_b / 1e3), 1),
                      "recall_plain": round(rp, 5), "qps_plain": round(nq / (ms_p / 1e3), 1)})
        log(f"alpha={a}: bf16 recall={rb:.4f} qps={nq / (ms_b / 1e3):.0f} | plain recall={rp:.4f} "
            f"qps={nq / (ms_p / 1e3):.0f}")
    ok = [e for e in sweep if e["recall_bf16"] >= TARGET_RECALL]
    alpha = ok[0]["alpha"] if ok else sweep[-1]["alpha"]

    ms_plain = timed(lambda: run_plain(alpha), args.steps, args.warmup)
    plain_rec = recall_at(ids, gt)
    plain_ids, plain_d = ids.clone(), dists.clone()
    # with FP32 centre distances the BF16 re-rank must return the plain answer bit for bit
    o = ix.query_bf16(Qd, k, alpha, beta, s1_bf16=False, nsurv=False, relerr=False)
    torch.cuda.synchronize()
    same = bool(torch.equal(o["ids"], plain_ids) and torch.equal(o["dists"], plain_d))
    del o
    ms = timed(lambda: run_bf16(alpha), args.steps, args.warmup)
    value = nq * args.steps / (ms / 1e3)
    rec = recall_at(ids, gt)
    agree = recall_at(ids, plain_ids)
    surv = nsurv.double()
    log(f"bf16 timed: {ms / args.steps:.3f} ms/step, {value:.0f} QPS, recall@10={rec:.4f}; plain "
        f"{nq * args.steps / (ms_plain / 1e3):.0f} QPS recall@10={plain_rec:.4f}; FP32-S1 BF16 re-rank equals "
        f"plain: {same}; top-k overlap with plain {agree:.4f}; "
        f"survivors mean {float(surv.mean()):.1f} max {int(nsurv.max())}")
    o = ix.query_bf16(Qd, k, alpha, beta, s1_bf16=True, nsurv=False, relerr=True)
    torch.cuda.synchronize()
    rel = o["relerr"]
    aprime = None
    o = ix.query_bf16(Qd[:64], k, alpha, beta, s1_bf16=True, nsurv=False, relerr=False, debug=True)
    torch.cuda.synchronize()
    aprime = float(o["aprime"].double().sum(dim=1).mean())
    U = float((o["scores"] > 0).sum(dim=1).double().mean())
    del o
    B = suco.count_B(beta, n, k)
    R = float(surv.mean())
    step_bytes = {
        "collide": 2.0 * aprime + 2.0 * U,
        "rerank_bf16": 2.0 * B * d + 4.0 * B + 4.0 * B + 4.0 * B,   # BF16 rows, ids, error bounds, lower bounds
        "survivors": 4.0 * B + 4.0 * B + 4.0 * R,                   # ids and lower bounds read, survivors written
        "rerank": 4.0 * R * d + 4.0 * R,                            # FP32 rows of the survivors
    }
    ix.profile(True)
    ix.profile_read()
    for _ in range(args.steps):
        run_bf16(alpha)
    stage = ix.profile_read()
    ix.profile(False)
    per_kernel = {}
    for st_name, (tms, cnt) in stage.items():
        if cnt == 0:
            continue
        avg_ms = tms / cnt
        ent = {"avg_ms": round(avg_ms, 5), "launches": cnt,
               "share": round(tms / max(1e-9, sum(v[0] for v in stage.values())), 4)}
        if st_name in step_bytes:
            bytes_launch = step_bytes[st_name] * nq / max(1, cnt // args.steps)
            ent["alg_bytes_per_launch"] = bytes_launch
            ent["gbs"] = round(bytes_launch / (avg_ms * 1e-3) / 1e9, 1)
        per_kernel[st_name] = ent
    dom = max(step_bytes, key=lambda t: stage[t][0])
    kern_name = {"collide": "k_collide", "rerank_bf16": "k_rerank_bf16", "survivors": "k_survivors",
                 "rerank": "k_rerank"}[dom]
    achieved = per_kernel[dom]["gbs"]
    roofline = {"bound": "hbm", "kernel": kern_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(kern_name, "gist_like")}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = oracle_baseline(X, Q, ns, sk, alpha, beta, k, 256, "1,000 queries")
    line = {
        "metric": "QPS at recall@10=0.95, GIST-like n=1M d=960: BF16 split-precision SuCo on 1 GPU",
        "value": round(value, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": f"gist_like n={n} d={d} in (0,1), N_s={ns}, sqrtK={sk}, nq={nq}, k={k}, beta={beta}",
                   "form": "bf16 split precision", "alpha": alpha, "recall_at_10": round(rec, 5),
                   "fp32_s1_equals_plain_bitwise": same, "topk_overlap_with_plain": round(agree, 5),
                   "plain": {"qps": round(nq * args.steps / (ms_plain / 1e3), 1), "recall_at_10": round(plain_rec, 5)},
                   "survivors": {"mean": round(R, 2), "max": int(nsurv.max())},
                   "relerr_vs_fp64": {"max": float(rel.max()), "mean": float(rel.mean())},
                   "index_build_s": round(build_s, 3), "sweep": sweep},
        "kernels": per_kernel, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ix.free()


def timed_region(fn, steps, warmup):
    """Milliseconds of `steps` calls of fn after `warmup` calls, HIP events on the current stream."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)


def stage_profile(ix, fn, steps, step_bytes, nq):
    """Per-step kernel times (suco_profile) over `steps` calls and GB/s for the steps with byte counts."""
    ix.profile(True)
    ix.profile_read()
    for _ in range(steps):
        fn()
    stage = ix.profile_read()
    ix.profile(False)
    out = {}
    tot = sum(v[0] for v in stage.values())
    for name, (tms, cnt) in stage.items():
        if cnt == 0:
            continue
        avg_ms = tms / cnt
        ent = {"avg_ms": round(avg_ms, 5), "launches": cnt, "share": round(tms / max(1e-9, tot), 4)}
        if name in step_bytes:
            bytes_launch = step_bytes[name] * nq / max(1, cnt // steps)
            ent["alg_bytes_per_launch"] = bytes_launch
            ent["gbs"] = round(bytes_launch / (avg_ms * 1e-3) / 1e9, 1)
        out[name] = ent
    return stage, out


def oracle_baseline(X, Q, ns, sk, alpha, beta, k, sample, what):
    """The FP64 oracle on its own 2-iteration index, timed on the host's share of cores and on one
    thread, each on a prefix of the queries sized to about 10 s (at most `sample` queries)."""
    import oracle
    threads, nproc, model = host_cpu()
    _, c32, asg, _ = oracle.build_index(X, ns, sk, iters=2, seed=1, nthreads=threads)
    oix = oracle.Index(X, ns, sk, c32, asg)
    qps, m, dt = oracle_rate(oix, Q, k, alpha, beta, threads, 10.0, sample)
    qps1, m1, dt1 = oracle_rate(oix, Q, k, alpha, beta, 1, 5.0, sample)
    return {"value": round(qps, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "value_1_thread": round(qps1, 3), "nproc": nproc, "cpu_model": model,
            "sample": f"first {m} of the {what} on {threads} threads ({dt:.1f}s) and first {m1} on one thread "
                      f"({dt1:.1f}s); alpha={alpha}, beta={beta}, k={k}; FP64 C oracle on its own 2-iteration "
                      f"index, OpenMP over queries"}


def step_bytes_for(ix, suco, Qs, k, alpha, beta, n, d):
    """Algorithmic bytes per query of the counting, selection and re-rank steps (64-query sample)."""
    import torch
    o = ix.query_debug(Qs, k, alpha, beta, scores=True, cand=False, cells=False, feat=False)
    torch.cuda.synchronize()
    aprime = float(o["aprime"].double().sum(dim=1).mean())
    sc = o["scores"]
    U = float((sc > 0).sum(dim=1).double().mean())
    B = suco.count_B(beta, n, k)
    T = torch.sort(sc, dim=1, descending=True).values[:, B - 1:B]
    ge_T = float((sc >= T).sum(dim=1).double().mean())
    del o, sc
    return {
        "collide": 2.0 * aprime + 2.0 * U,
        "select": 2.0 * ge_T + 4.0 * B,
        "rerank": (1.0 if ix.flags() & suco.INDEX_BYTE_ROWS else 4.0) * B * d + 4.0 * B,
    }


def bench_batched_deep(args, log):
    """Deep-like n=10,000,000 d=96 unit-norm rows, N_s=8 (12 dims), sqrtK=64, a stream of 100,000 queries
    in uneven batches (sizes uniform in 1..4096), k=10, alpha=0.02, beta=0.002: the batched form (one HIP
    graph per batch-size bucket, tuned launch shapes) against the plain path on the whole stream at once."""
    import torch
    import paper_2411_14754_amd as suco
    import synth

    W = synth.Workload(4)
    sp = W.spec
    if args.nq:                      # a shorter stream (profiling runs that count every dispatch)
        sp["nq"] = args.nq
    n, d, ns, sk, nq, k, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["k"], sp["beta"]
    alpha = args.alpha if args.alpha is not None else sp["alpha"]
    log("generating data")
    X, Q = W.data(), W.queries(nq)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    torch.cuda.synchronize()
    t0 = time.time()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1, tile_max=args.tile_max, query_chunk=args.query_chunk)
    build_s = time.time() - t0
    log(f"index built in {build_s:.2f}s")
    n_gt = min(nq, 10_000)
    gt = exact_topk_float(Xd, Qd[:n_gt], k)
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dists = torch.empty((nq, k), dtype=torch.float32, device="cuda")

    def plain():
        ix.query(Qd, k, alpha, beta, out=(ids, dists))

    ms_plain = timed_region(plain, args.steps, 1)
    plain_ids, plain_d = ids.clone(), dists.clone()
    rec_plain = recall_at(ids[:n_gt], gt)
    log(f"plain: {ms_plain / args.steps:.2f} ms per {nq:,} queries, recall@10={rec_plain:.4f}")
    if args.plain_only:
        bench_deep_plain(args, log, ix, suco, Qd, X, Q, sp, alpha, ms_plain, rec_plain, plain, build_s)
        return
    sizes = W.batch_sizes(nq)
    b = suco.Batcher(ix, 4096, k, beta)

    def stream():
        s0 = 0
        for sz in sizes:
            b.query(Qd[s0:s0 + sz], alpha=alpha, out=(ids[s0:s0 + sz], dists[s0:s0 + sz]))
            s0 += sz

    t0 = time.time()
    stream()                                  # tunes every bucket met on first use
    torch.cuda.synchronize()
    tune_s = time.time() - t0
    ms = timed_region(stream, args.steps, 1)
    value = nq * args.steps / (ms / 1e3)
    same = bool(torch.equal(ids, plain_ids) and torch.equal(dists, plain_d))
    rec = recall_at(ids[:n_gt], gt)
    log(f"batched stream of {len(sizes)} batches: {ms / args.steps:.2f} ms, {value:.0f} QPS, recall@10={rec:.4f}, "
        f"bitwise equal to plain: {same}, tuning {tune_s:.1f}s")
    tuned = {}
    for j in range(13):
        try:
            tuned[str(1 << j)] = b.tuning(1 << j)
        except suco.SucoError:
            pass                               # bucket never used by this stream
    b.free()
    sb = step_bytes_for(ix, suco, Qd[:64], k, alpha, beta, n, d)
    stage, per_kernel = stage_profile(ix, plain, 1, sb, nq)
    dom = max(sb, key=lambda t: stage[t][0])
    kern_name = {"collide_sparse": "k_collide_sparse", "collide": "k_collide", "select": "k_select",
                 "rerank": "k_rerank"}[dom]
    achieved = per_kernel[dom]["gbs"]
    roofline = {"bound": "hbm", "kernel": kern_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(kern_name, "deep_like")}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = oracle_baseline(X, Q, ns, sk, alpha, beta, k, 256, f"{nq:,} queries")
    line = {
        "metric": "QPS of a stream of uneven batches, Deep-like n=10M d=96: batched persistent SuCo on 1 GPU",
        "value": round(value, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(ms / args.steps, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"deep_like n={n} d={d} unit-norm, N_s={ns}, sqrtK={sk}, nq={nq} in {len(sizes)} "
                               f"batches of 1..4096, k={k}, alpha={alpha}, beta={beta}",
                   "form": "batched", "recall_at_10_first_10000": round(rec, 5), "bitwise_equal_plain": same,
                   "plain_one_call": {"qps": round(nq * args.steps / (ms_plain / 1e3), 1),
                                      "recall_at_10_first_10000": round(rec_plain, 5)},
                   "tuning_s": round(tune_s, 2), "tuned": tuned,
                   "index_build_s": round(build_s, 3)},
        "kernels": per_kernel, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ix.free()


def bench_deep_plain(args, log, ix, suco, Qd, X, Q, sp, alpha, ms_plain, rec_plain, plain, build_s):
    """The deep_like workload through the plain path only: the whole 100,000-query stream in one call."""
    n, d, ns, sk, nq, k, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["k"], sp["beta"]
    sb = step_bytes_for(ix, suco, Qd[:64], k, alpha, beta, n, d)
    stage, per_kernel = stage_profile(ix, plain, 1, sb, nq)
    dom = max(sb, key=lambda t: stage[t][0])
    kern_name = {"collide_sparse": "k_collide_sparse", "collide": "k_collide", "select": "k_select",
                 "rerank": "k_rerank"}[dom]
    achieved = per_kernel[dom]["gbs"]
    roofline = {"bound": "hbm", "kernel": kern_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(kern_name, "deep_like")}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = oracle_baseline(X, Q, ns, sk, alpha, beta, k, 256, f"{nq:,} queries")
    line = {
        "metric": f"QPS of {nq:,} queries in one call, Deep-like n=10M d=96: plain SuCo on 1 GPU",
        "value": round(nq * args.steps / (ms_plain / 1e3), 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(ms_plain / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"deep_like n={n} d={d} unit-norm, N_s={ns}, sqrtK={sk}, nq={nq} in one call, "
                               f"k={k}, alpha={alpha}, beta={beta}",
                   "form": "plain", "recall_at_10_first_10000": round(rec_plain, 5),
                   "index_build_s": round(build_s, 3)},
        "kernels": per_kernel, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ix.free()


def bench_learned_lifted(args, log):
    """Lifted n=10,000,000 d=256, N_s=16, sqrtK=64, k=10, beta=0.003: the learned budget (trained on
    generated queries labelled by plain sweeps against exact top-10) evaluated on 10,000 held-out queries,
    in one call and as a stream of uneven batches, against plain SuCo at equal recall."""
    import torch
    import paper_2411_14754_amd as suco
    from paper_2411_14754_amd import learned
    import synth

    W = synth.Workload(5)
    sp = W.spec
    n, d, ns, sk, nq, k, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["k"], sp["beta"]
    log("generating data")
    X, Q = W.data(), W.queries()
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    torch.cuda.synchronize()
    t0 = time.time()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1, tile_max=args.tile_max, query_chunk=args.query_chunk)
    build_s = time.time() - t0
    log(f"index built in {build_s:.2f}s")
    gt = exact_topk_float(Xd, Qd, k)
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dists = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    sweep = []
    for a in (0.00001, 0.00002, 0.00005, 0.0001, 0.0002, 0.0005, 0.001, 0.002, 0.005, 0.01, 0.03):
        ms_a = timed_region(lambda: ix.query(Qd, k, a, beta, out=(ids, dists)), 1, 1)
        r = recall_at(ids, gt)
        sweep.append({"alpha": a, "recall": round(r, 5), "qps": round(nq / (ms_a / 1e3), 1)})
        log(f"plain alpha={a}: recall@10={r:.4f} qps={nq / (ms_a / 1e3):.0f}")
    ok = [e for e in sweep if e["recall"] >= TARGET_RECALL]
    alpha = ok[0]["alpha"] if ok else sweep[-1]["alpha"]
    ms_plain = timed_region(lambda: ix.query(Qd, k, alpha, beta, out=(ids, dists)), args.steps, 1)
    rec_plain = recall_at(ids, gt)
    m_tr, m_val = args.lifted_train, 10_000
    log(f"labelling {m_tr} training queries")
    t0 = time.time()
    Qt = torch.from_numpy(W.train_queries(m_tr + m_val)).cuda()
    gt_t = exact_topk_float(Xd, Qt, k)
    grid = learned.alpha_grid(0.00001, 0.01, 1.4)
    net, info = learned.train_budget_model(ix, Qt[:m_tr], gt_t[:m_tr], k, beta, grid, epochs=args.epochs)
    amin, amax = grid[0], grid[-1]
    scale = learned.calibrate_scale(ix, net, Qt[m_tr:], gt_t[m_tr:], k, beta, args.target_recall, amin, amax)
    train_s = time.time() - t0
    log(f"trained in {train_s:.1f}s, loss {info['loss'][0]:.3f} -> {info['loss'][-1]:.3f}, scale {scale:.3f}")
    ms_l1 = timed_region(lambda: suco.query_learned(ix, net, Qd, k, beta, scale, amin, amax, out=(ids, dists)),
                         args.steps, 1)
    rec_l1 = recall_at(ids, gt)
    _, _, au = suco.query_learned(ix, net, Qd, k, beta, scale, amin, amax)
    mean_alpha = float(au.double().mean())
    b = suco.Batcher(ix, 4096, k, beta)
    b.set_model(net, scale, amin, amax)
    sizes = W.batch_sizes(nq)

    def stream():
        s0 = 0
        for sz in sizes:
            b.query(Qd[s0:s0 + sz], out=(ids[s0:s0 + sz], dists[s0:s0 + sz]))
            s0 += sz

    stream()
    ms = timed_region(stream, args.steps, 1)
    value = nq * args.steps / (ms / 1e3)
    rec = recall_at(ids, gt)
    b.free()
    plain_eq = None
    for lo, hi in zip(sweep, sweep[1:]):
        if lo["recall"] < rec <= hi["recall"]:
            f = (rec - lo["recall"]) / (hi["recall"] - lo["recall"])
            plain_eq = math.exp(math.log(lo["qps"]) + f * (math.log(hi["qps"]) - math.log(lo["qps"])))
    log(f"learned one call {nq * args.steps / (ms_l1 / 1e3):.0f} QPS recall {rec_l1:.4f}; learned+batched "
        f"{value:.0f} QPS recall {rec:.4f} (mean alpha {mean_alpha:.5f}); plain at that recall {plain_eq}")
    sb = step_bytes_for(ix, suco, Qd[:64], k, alpha, beta, n, d)
    stage, per_kernel = stage_profile(ix, lambda: ix.query(Qd, k, alpha, beta, out=(ids, dists)), 1, sb, nq)
    dom = max(sb, key=lambda t: stage[t][0])
    kern_name = {"collide_sparse": "k_collide_sparse", "collide": "k_collide", "select": "k_select",
                 "rerank": "k_rerank"}[dom]
    achieved = per_kernel[dom]["gbs"]
    roofline = {"bound": "hbm", "kernel": kern_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(kern_name, "lifted256")}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = oracle_baseline(X, Q, ns, sk, alpha, beta, k, 256, "10,000 queries")
    line = {
        "metric": "QPS at recall@10=0.95, lifted n=10M d=256: learned+batched vs plain SuCo on 1 GPU",
        "value": round(value, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(ms / args.steps, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"lifted256 n={n} d={d}, N_s={ns}, sqrtK={sk}, nq={nq}, k={k}, beta={beta}",
                   "form": "learned+batched", "recall_at_10": round(rec, 5), "mean_alpha": round(mean_alpha, 6),
                   "learned_one_call": {"qps": round(nq * args.steps / (ms_l1 / 1e3), 1), "recall_at_10": round(rec_l1, 5)},
                   "plain": {"alpha": alpha, "qps": round(nq * args.steps / (ms_plain / 1e3), 1),
                             "recall_at_10": round(rec_plain, 5),
                             "qps_at_same_recall": None if plain_eq is None else round(plain_eq, 1)},
                   "train_queries": m_tr, "val_queries": m_val, "epochs": args.epochs, "scale": round(scale, 5),
                   "train_s": round(train_s, 1), "loss_first_last": [round(info["loss"][0], 4), round(info["loss"][-1], 4)],
                   "index_build_s": round(build_s, 3), "sweep": sweep},
        "kernels": per_kernel, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    net.free()
    ix.free()


def bench_sift_k50(args, log):
    """The SIFT-like workload at k = 50 (its second k): the plain path over the
    alpha grid, recall@50 against the exact top-50, and the QPS at the
    smallest grid alpha reaching recall@50 >= 0.95 (10,000 queries a call)."""
    import torch
    import paper_2411_14754_amd as suco
    import synth
    W = synth.Workload(2)
    sp = W.spec
    n, d, ns, sk, nq, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["beta"]
    k = 50
    X, Q = W.data(), W.queries()
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1)
    gt = exact_topk(Xd, Qd, k)
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dists = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    sweep = []
    for a in ALPHA_GRID:
        ms_a, _ = timed_steps(lambda: ix.query(Qd, k, a, beta, out=(ids, dists)), 1, 1)
        r = recall_at(ids, gt)
        sweep.append({"alpha": a, "recall": round(r, 5), "qps": round(nq / (ms_a / 1e3), 1)})
        log(f"k=50 alpha={a}: recall@50={r:.4f} qps={nq / (ms_a / 1e3):.0f}")
    ok = [e for e in sweep if e["recall"] >= TARGET_RECALL]
    alpha = ok[0]["alpha"] if ok else sweep[-1]["alpha"]
    ms, per = timed_steps(lambda: ix.query(Qd, k, alpha, beta, out=(ids, dists)), args.steps, args.warmup)
    rec = recall_at(ids, gt)
    value = nq * args.steps / (ms / 1e3)
    log(f"k=50 timed at alpha={alpha}: {ms / args.steps:.3f} ms/step, {value:.0f} QPS, recall@50={rec:.4f}")
    print(json.dumps({"metric": "QPS at recall@50=0.95, n=1M d=128: plain SuCo on 1 GPU", "value": round(value, 1),
                      "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(ms / args.steps, 4), "higher_is_better": True, "dtype": "f32",
                      "data": "synthetic",
                      "config": {"workload": f"sift_like n={n} d={d} int 0..255, N_s={ns}, sqrtK={sk}, nq={nq}, "
                                             f"k={k}, beta={beta}", "alpha": alpha, "recall_at_50": round(rec, 5),
                                 "sweep": sweep}}))
    ix.free()


def bench_learned_ceiling(args, log):
    """What a per-query alpha can gain on the SIFT-like workload at best: each
    evaluation query gets alphas read off its own ground truth (a perfect
    predictor), and the path is timed in one call with those alphas.  Per
    query, recall@10 over the alpha grid; the rules: `tau` (the smallest grid
    alpha at which the query reaches tau times the recall it has at the largest
    grid alpha) and `greedy` (all queries at the smallest alpha, then raised by
    recall gained per alpha spent until the mean recall reaches 0.95).  Printed
    next to plain SuCo at a few alphas."""
    import torch
    import numpy as np
    import paper_2411_14754_amd as suco
    from paper_2411_14754_amd import learned
    import synth
    W = synth.Workload(2)
    sp = W.spec
    n, d, ns, sk, nq, k, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["k"], sp["beta"]
    X, Q = W.data(), W.queries()
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1)
    gt = exact_topk(Xd, Qd, k)
    grid = learned.alpha_grid(0.0005, 0.05)
    R = torch.stack([learned.per_query_recall(ix.query(Qd, k, a, beta)[0], gt) for a in grid], 1)
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dists = torch.empty((nq, k), dtype=torch.float32, device="cuda")

    def timed(alpha=None, aq=None):
        if aq is None:
            fn = lambda: ix.query(Qd, k, alpha, beta, out=(ids, dists))
        else:
            fn = lambda: ix.query_alpha(Qd, k, aq, beta, out=(ids, dists))
        ms, _ = timed_steps(fn, args.steps, args.warmup)
        return ms / args.steps, recall_at(ids, gt)

    rows = []
    for a in (0.002, 0.0025, 0.003, 0.005, 0.0075, 0.01, 0.05):
        ms, r = timed(alpha=a)
        rows.append({"rule": "plain", "alpha": a, "ms": round(ms, 4), "recall": round(r, 5), "qps": round(nq / ms * 1e3, 1)})
        log(f"plain alpha={a}: {ms:.3f} ms, recall {r:.4f}")
    G = torch.tensor(grid, device="cuda", dtype=torch.float32)
    best = R[:, -1]
    for tau in (0.8, 0.9, 1.0):
        first = torch.argmax((R >= (best * tau - 1e-6)[:, None]).int(), dim=1)
        aq = G[first].contiguous()
        ms, r = timed(aq=aq)
        rows.append({"rule": f"tau={tau}", "mean_alpha": round(float(aq.mean()), 6), "ms": round(ms, 4),
                     "recall": round(r, 5), "qps": round(nq / ms * 1e3, 1)})
        log(f"perfect labels tau={tau}: mean alpha {float(aq.mean()):.5f}, {ms:.3f} ms, recall {r:.4f}")
    Rc, Gc = R.cpu().numpy().astype(np.float64), np.array(grid)
    gain = (Rc[:, 1:] - Rc[:, :1]) / (Gc[1:] - Gc[0])[None, :]
    jbest = np.argmax(gain, axis=1) + 1
    vbest = gain[np.arange(nq), jbest - 1]
    aq = np.full(nq, grid[0], np.float32)
    cur, target = float(Rc[:, 0].sum()), TARGET_RECALL * nq
    for q in np.argsort(-vbest):
        if cur >= target or vbest[q] <= 0:
            break
        aq[q] = grid[jbest[q]]
        cur += Rc[q, jbest[q]] - Rc[q, 0]
    ms, r = timed(aq=torch.from_numpy(aq).cuda())
    rows.append({"rule": "greedy", "mean_alpha": round(float(aq.mean()), 6), "ms": round(ms, 4), "recall": round(r, 5),
                 "qps": round(nq / ms * 1e3, 1)})
    log(f"perfect labels greedy: mean alpha {float(aq.mean()):.5f}, {ms:.3f} ms, recall {r:.4f}")
    print(json.dumps({"metric": "per-query alpha from the queries' own ground truth vs plain SuCo, n=1M d=128",
                      "value": None, "unit": "see rows", "n_gpus": 1, "steps": args.steps, "dtype": "f32",
                      "data": "synthetic", "config": {"workload": f"sift_like n={n} d={d} int 0..255, N_s={ns}, "
                                                                   f"sqrtK={sk}, nq={nq}, k={k}, beta={beta}",
                                                       "rows": rows}}))
    ix.free()


def bench_form(args, log):
    """One form of the SIFT-like query path alone, for kernel traces of it:
    `onecall` (10,000 queries in one plain call at alpha = 0.003), `batched`
    (the same queries as five uneven batches through a batcher, one launch
    each), `multi` (the five batches handed over together, one launch),
    `learned` / `learned_multi` (the five batches through a batcher with the
    trained budget model, alpha clamped to [0.0005, 0.0035], one launch each /
    together), `learned_onecall` (suco_query_learned on all 10,000).  Prints
    the per-step time."""
    import torch
    import paper_2411_14754_amd as suco
    import synth
    W = synth.Workload(2)
    sp = W.spec
    n, d, ns, sk, nq, k, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["k"], sp["beta"]
    X, Q = W.data(), W.queries()
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1)
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dists = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    sizes = W.batch_sizes(nq)
    alpha = 0.003
    starts = [sum(sizes[:j]) for j in range(len(sizes) + 1)]
    parts = [Qd[starts[j]:starts[j + 1]] for j in range(len(sizes))]
    outs = [(ids[starts[j]:starts[j + 1]], dists[starts[j]:starts[j + 1]]) for j in range(len(sizes))]
    net = scale = None
    if args.form.startswith("learned"):
        from paper_2411_14754_amd import learned
        Qt = torch.from_numpy(W.train_queries(30_000)).cuda()
        gt_t = exact_topk(Xd, Qt, k)
        grid = learned.alpha_grid(0.0005, 0.05)
        net, _ = learned.train_budget_model(ix, Qt[:20_000], gt_t[:20_000], k, beta, grid, epochs=args.epochs)
        scale = learned.calibrate_scale(ix, net, Qt[20_000:], gt_t[20_000:], k, beta, args.target_recall,
                                        grid[0], 0.0035)
    if args.form == "onecall":
        def step():
            ix.query(Qd, k, alpha, beta, out=(ids, dists))
    elif args.form == "learned_onecall":
        def step():
            suco.query_learned(ix, net, Qd, k, beta, scale, 0.0005, 0.0035, out=(ids, dists))
    else:
        together = args.form in ("multi", "learned_multi")
        b = suco.Batcher(ix, nq if together else 4096, k, beta)
        if net is not None:
            b.set_model(net, scale, 0.0005, 0.0035)

        def step():
            if together:
                b.query_multi(parts, alpha=alpha, outs=outs)
                return
            for j, q in enumerate(parts):
                b.query(q, alpha=alpha, out=outs[j])
    ms, per = timed_steps(step, args.steps, args.warmup)
    log(f"{args.form}: {ms / args.steps:.3f} ms per step of {nq} queries")
    print(json.dumps({"form": args.form, "ms_per_step": round(ms / args.steps, 4), "steps": args.steps,
                      "launches_per_step": len(sizes) if args.form in ("batched", "learned") else 1}))


def bench_build(args, log):
    """Create Index (Alg. 2) on the GPU for the SIFT-like (n=1M, d=128, N_s=8,
    sqrtK=50), Deep-like (n=10M, d=96, N_s=8, sqrtK=64) and lifted (n=10M,
    d=256, N_s=16, sqrtK=64) workloads, 25 k-means iterations: wall time with
    the data already in HBM, the device memory the index holds, and the
    k-means assignment's FP64 rate (its flops: every point's distance to every
    centre of every half, three FP64 operations per dimension)."""
    import torch
    import paper_2411_14754_amd as suco
    import synth
    rows = []
    which = (2, 4, 5) if args.build_all else (2,)
    for c in which:
        W = synth.Workload(c)
        sp = W.spec
        n, d, ns, sk = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"]
        log(f"{sp['name']}: generating data")
        Xd = torch.from_numpy(W.data()).cuda()
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        t0 = time.time()
        ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1)
        torch.cuda.synchronize()
        build_s = time.time() - t0
        free1, _ = torch.cuda.mem_get_info()
        flops_assign = 3.0 * n * d * sk          # per assignment pass, all halves
        rows.append({"workload": sp["name"], "n": n, "d": d, "n_s": ns, "sqrt_k": sk, "iters": 25,
                     "build_s": round(build_s, 4), "index_bytes": int(free0 - free1),
                     "data_bytes": 4 * n * d, "assign_flops_per_pass": flops_assign})
        log(f"{sp['name']}: built in {build_s:.3f} s, index holds {(free0 - free1) / 2**30:.2f} GiB "
            f"(data {4 * n * d / 2**30:.2f} GiB)")
        ix.free()
        del Xd
        torch.cuda.empty_cache()
    rec = {"metric": "GPU index build time (Create Index, 25 k-means iterations)", "value": rows[0]["build_s"],
           "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "higher_is_better": False, "dtype": "f64",
           "data": "synthetic", "config": {"workload": rows[0]["workload"], "rows": rows}}
    print(json.dumps(rec))


def bench_activation(args, log):
    """Dynamic Activation against Multi-sequence (Sec. 4.2, Sec. 5.2) on the
    SIFT-like index: the activation step's time and the whole query's, per
    alpha, with each rule; both activate the same cells, so recall is equal."""
    import torch
    import paper_2411_14754_amd as suco
    import synth
    W = synth.Workload(2)
    sp = W.spec
    n, d, ns, sk, nq, k, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["k"], sp["beta"]
    X, Q = W.data(), W.queries()
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1)
    out = (torch.empty((nq, k), dtype=torch.int32, device="cuda"),
           torch.empty((nq, k), dtype=torch.float32, device="cuda"))
    rows = []
    for alpha in (0.0005, 0.003, 0.01, 0.03, 0.05):
        row = {"alpha": alpha}
        ref = None
        for name, form in (("dynamic_activation", suco.ACT_DYNAMIC), ("multi_sequence", suco.ACT_MULTISEQ)):
            ix.set_activation(form)
            fn = lambda: ix.query(Qd, k, alpha, beta, out=out)
            ms, _ = timed_steps(fn, args.steps, args.warmup)
            got = out[0].clone()
            if ref is None:
                ref = got
            row[name + "_same_ids"] = bool(torch.equal(ref, got))
            ix.profile(True)
            ix.profile_read()
            for _ in range(args.steps):
                fn()
            st = ix.profile_read()
            ix.profile(False)
            row[name] = {"query_ms": round(ms / args.steps, 4), "activate_ms": round(st["activate"][0] / args.steps, 4)}
        ix.set_activation(suco.ACT_DYNAMIC)
        da, mseq = row["dynamic_activation"], row["multi_sequence"]
        row["activate_speedup"] = round(mseq["activate_ms"] / max(1e-9, da["activate_ms"]), 3)
        log(f"alpha={alpha}: activation DA {da['activate_ms']:.3f} ms, Multi-sequence {mseq['activate_ms']:.3f} ms; "
            f"query {da['query_ms']:.3f} vs {mseq['query_ms']:.3f} ms")
        rows.append(row)
    rec = {"metric": "activation step time, Dynamic Activation vs Multi-sequence, n=1M d=128, 10,000 queries",
           "value": rows[1]["activate_speedup"], "unit": "x (Multi-sequence time / Dynamic Activation time) at alpha=0.003",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"sift_like n={n} d={d} int 0..255, N_s={ns}, sqrtK={sk}, nq={nq}, k={k}, beta={beta}",
                      "rows": rows}}
    print(json.dumps(rec))
    ix.free()


def bench_sclinear(args, log):
    """SuCo against SC-Linear (Alg. 1, no index) on the SIFT-like data with the
    comparison table's parameters (alpha=0.03, beta=0.003, k=50): per-query
    time, speed-up, recall@50, and the bytes SC-Linear moves per query (its
    distance array written once and read by the threshold passes and the
    scoring pass; the rows themselves are read once per pass of queries)."""
    import torch
    import paper_2411_14754_amd as suco
    import synth
    W = synth.Workload(2)
    sp = W.spec
    n, d, ns, sk = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"]
    alpha, beta, k = 0.03, 0.003, 50
    nq_lin = 512
    X, Q = W.data(), W.queries()
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1)
    Ql = Qd[:nq_lin].contiguous()
    gt = exact_topk(Xd, Ql, k)
    out_s = (torch.empty((nq_lin, k), dtype=torch.int32, device="cuda"),
             torch.empty((nq_lin, k), dtype=torch.float32, device="cuda"))
    out_l = (torch.empty((nq_lin, k), dtype=torch.int32, device="cuda"),
             torch.empty((nq_lin, k), dtype=torch.float32, device="cuda"))
    ms_suco, _ = timed_steps(lambda: ix.query(Ql, k, alpha, beta, out=out_s), args.steps, args.warmup)
    ms_lin, per_lin = timed_steps(lambda: ix.query_sclinear(Ql, k, alpha, beta, out=out_l), max(1, args.steps // 2), 1)
    steps_lin = max(1, args.steps // 2)
    q_suco = ms_suco / args.steps / nq_lin
    q_lin = ms_lin / steps_lin / nq_lin
    r_suco, r_lin = recall_at(out_s[0], gt), recall_at(out_l[0], gt)
    # per query: n*ns FP32 distances written once, read by four radix passes, the
    # tie count and the scoring pass; n score bytes written and read twice
    lin_bytes = n * ns * 4 * (1 + 4 + 1 + 1) + 3 * n + n * d / 256.0
    gbs = lin_bytes * nq_lin / (ms_lin / steps_lin / 1e3) / 1e9
    log(f"SC-Linear: {q_lin * 1e3:.1f} us/query, recall@50={r_lin:.4f}; SuCo: {q_suco * 1e3:.2f} us/query, "
        f"recall@50={r_suco:.4f}; speed-up {q_lin / q_suco:.0f}x")
    rec = {"metric": "SuCo vs SC-Linear per-query time, n=1M d=128 (alpha=0.03, beta=0.003, k=50)",
           "value": round(q_lin / q_suco, 1), "unit": "x speed-up of SuCo over SC-Linear", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"sift_like n={n} d={d} int 0..255, N_s={ns}, sqrtK={sk}, nq={nq_lin}, k={k}, "
                                  f"alpha={alpha}, beta={beta}",
                      "suco": {"ms_per_query": round(q_suco, 6), "recall_at_50": round(r_suco, 5)},
                      "sclinear": {"ms_per_query": round(q_lin, 5), "recall_at_50": round(r_lin, 5),
                                   "step_ms": [round(x, 3) for x in per_lin],
                                   "bytes_per_query": lin_bytes, "gbs": round(gbs, 1),
                                   "frac": round(gbs / HBM_PEAK_GBS, 4)}}}
    print(json.dumps(rec))
    ix.free()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("sift_like", "sift_k50", "gist_like", "deep_like", "lifted256", "sclinear",
                                           "activation", "build", "learned_ceiling"), default="sift_like",
                    help="sift_like: the headline (plain and learned+batched SuCo); gist_like: BF16 split "
                         "precision; deep_like: batched stream at n=10M; lifted256: learned budget at n=10M; "
                         "sclinear: SuCo against SC-Linear on the SIFT-like data; activation: Dynamic Activation "
                         "against Multi-sequence; build: index build time and memory; sift_k50: the SIFT-like "
                         "workload at k=50")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=10_000, help="most queries the CPU oracle is timed on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--tile-max", type=int, default=0, help="largest collision tile (0: library default)")
    ap.add_argument("--query-chunk", type=int, default=0, help="queries per pass (0: library default)")
    ap.add_argument("--alpha", type=float, default=None, help="time this alpha and skip the sweep")
    ap.add_argument("--plain-only", action="store_true",
                    help="sift_like and deep_like: report plain SuCo only (no learned or batched form)")
    ap.add_argument("--train-queries", type=int, default=20_000)
    ap.add_argument("--val-queries", type=int, default=10_000)
    ap.add_argument("--epochs", type=int, default=25)
    ap.add_argument("--lifted-train", type=int, default=200_000, help="training queries of the lifted256 mode")
    ap.add_argument("--target-recall", type=float, default=0.951)
    ap.add_argument("--build-all", action="store_true", help="build: also the 10M-point Deep-like and lifted indexes")
    ap.add_argument("--nq", type=int, default=0, help="deep_like: queries in the stream (0: the workload's 100,000)")
    ap.add_argument("--form", choices=("onecall", "batched", "multi", "learned", "learned_multi", "learned_onecall"),
                    default=None,
                    help="sift_like: time one form of the query path alone (for kernel traces)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (a plain copy kernel of known size, used to "
                         "scale HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path shards by "
              f"queries with no exchange, see the design notes)", file=sys.stderr)
        sys.exit(2)

    def log(msg):
        if not args.quiet:
            print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.workload == "gist_like":
        bench_bf16(args, log)
        return
    if args.workload == "deep_like":
        bench_batched_deep(args, log)
        return
    if args.workload == "lifted256":
        bench_learned_lifted(args, log)
        return
    if args.workload == "sclinear":
        bench_sclinear(args, log)
        return
    if args.workload == "activation":
        bench_activation(args, log)
        return
    if args.workload == "build":
        bench_build(args, log)
        return
    if args.workload == "sift_k50":
        bench_sift_k50(args, log)
        return
    if args.workload == "learned_ceiling":
        bench_learned_ceiling(args, log)
        return

    if args.form:
        bench_form(args, log)
        return

    import torch
    import paper_2411_14754_amd as suco
    import synth

    W = synth.Workload(2)
    sp = W.spec
    n, d, ns, sk, nq, k, beta = sp["n"], sp["d"], sp["n_s"], sp["sqrt_k"], sp["nq"], sp["k"], sp["beta"]
    log("generating data")
    X, Q = W.data(), W.queries()
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    torch.cuda.synchronize()
    t0 = time.time()
    ix = suco.Index.build(Xd, ns, sk, iters=25, seed=1, tile_max=args.tile_max, query_chunk=args.query_chunk)
    build_s = time.time() - t0
    log(f"index built in {build_s:.2f}s")
    gt = exact_topk(Xd, Qd, k)
    torch.cuda.synchronize()

    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dists = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(alpha):
        ix.query(Qd, k, alpha, beta, out=(ids, dists))

    sweep = []
    for a in (ALPHA_GRID if args.alpha is None else (args.alpha,)):
        run(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run(a)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        r = recall_at(ids, gt)
        sweep.append({"alpha": a, "recall": round(r, 5), "qps": round(nq / (ms / 1e3), 1)})
        log(f"alpha={a}: recall@10={r:.4f} qps={nq / (ms / 1e3):.0f}")
    ok = [s for s in sweep if s["recall"] >= TARGET_RECALL]
    alpha = ok[0]["alpha"] if ok else sweep[-1]["alpha"]
    qps_interp = None
    for lo, hi in zip(sweep, sweep[1:]):
        if lo["recall"] < TARGET_RECALL <= hi["recall"]:
            f = (TARGET_RECALL - lo["recall"]) / (hi["recall"] - lo["recall"])
            qps_interp = math.exp(math.log(lo["qps"]) + f * (math.log(hi["qps"]) - math.log(lo["qps"])))
    if qps_interp is None and sweep[0]["recall"] >= TARGET_RECALL:
        qps_interp = sweep[0]["qps"]

    # per-step algorithmic bytes at the chosen alpha, from a 64-query sample:
    # A' (points in activated cells), U (points of non-zero score) and the
    # points at or above the score threshold
    o = ix.query_debug(Qd[:64], k, alpha, beta, scores=True, cand=False, cells=False, feat=False)
    torch.cuda.synchronize()
    aprime = float(o["aprime"].double().sum(dim=1).mean())
    sc = o["scores"].to(torch.int32)
    U = float((sc > 0).sum(dim=1).double().mean())
    B = suco.count_B(beta, n, k)
    srt = torch.sort(sc, dim=1, descending=True).values
    T = srt[:, B - 1:B]
    ge_T = float((sc >= T).sum(dim=1).double().mean())
    del o, sc, srt
    rows_b = 1.0 if ix.flags() & suco.INDEX_BYTE_ROWS else 4.0
    # algorithmic bytes per query of each step in the index's own layout: the
    # sparse step reads the activated cells' 32-bit ids once (the survey's S3
    # term 4*A'*N_s) and writes B candidate ids, everything else in LDS; the
    # tiled step reads the 16-bit tile-local ids and writes the non-zero-score
    # ids by level, the selection reads the levels at or above the threshold;
    # the re-rank reads the candidates' rows as stored (one byte per coordinate
    # when the index keeps the byte copy) and their ids
    step_bytes = {
        "collide_sparse": 4.0 * aprime + 4.0 * B,
        "collide": 2.0 * aprime + 2.0 * U,
        "select": 2.0 * ge_T + 4.0 * B,
        "rerank": rows_b * B * d + 4.0 * B,
    }
    # the survey's per-query figures for the same steps (S3: 4*A'*N_s, S5: 4*B*d FP32 rows)
    survey_bytes = {"collide_sparse": 4.0 * aprime, "collide": 4.0 * aprime, "rerank": 4.0 * B * d + 4.0 * B}

    ms_plain, per_step = timed_steps(lambda: run(alpha), args.steps, args.warmup)
    plain_value = nq * args.steps / (ms_plain / 1e3)
    plain_rec = recall_at(ids, gt)
    plain_mre = mean_relative_error(dists, exact_dists(Xd, Qd, gt))
    log(f"plain timed: {ms_plain / args.steps:.3f} ms/step (median {sorted(per_step)[len(per_step) // 2]:.3f}), "
        f"{plain_value:.0f} QPS, recall@10={plain_rec:.4f}, MRE={plain_mre:.2e}")

    # same steps again with every launch bracketed by HIP events on the query stream
    ix.profile(True)
    ix.profile_read()
    for _ in range(args.steps):
        run(alpha)
    stage = ix.profile_read()
    ix.profile(False)
    launches = stage["collide"][1] // args.steps
    per_kernel = {}
    for sname, (tms, cnt) in stage.items():
        if cnt == 0:
            continue
        avg_ms = tms / cnt
        ent = {"avg_ms": round(avg_ms, 5), "launches": cnt,
               "share": round(tms / max(1e-9, sum(v[0] for v in stage.values())), 4)}
        if sname in ("collide", "select") and stage.get("collide_sparse", (0, 0))[1]:
            # with the sparse step these take only the few queries it leaves: no per-query byte figure
            ent["note"] = "tiled step: only the queries the sparse step leaves"
        elif sname in step_bytes:
            # launches cover `chunk` queries except a ragged last one: use the per-step total
            bytes_launch = step_bytes[sname] * nq / max(1, cnt // args.steps)
            ent["alg_bytes_per_launch"] = bytes_launch
            ent["gbs"] = round(bytes_launch / (avg_ms * 1e-3) / 1e9, 1)
            if sname in survey_bytes:
                sb_launch = survey_bytes[sname] * nq / max(1, cnt // args.steps)
                ent["survey_bytes_per_launch"] = sb_launch
                ent["survey_gbs"] = round(sb_launch / (avg_ms * 1e-3) / 1e9, 1)
        per_kernel[sname] = ent
    dom = max((t for t in step_bytes if stage[t][1] and "gbs" in per_kernel.get(t, {})), key=lambda t: stage[t][0])
    kern_name = {"collide_sparse": "k_collide_sparse", "collide": "k_collide", "select": "k_select",
                 "rerank": "k_rerank"}[dom]
    achieved = per_kernel[dom]["gbs"]
    copy_gbs = copy_bandwidth()
    roofline = {"bound": "hbm", "kernel": kern_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(kern_name, "sift_like"),
                "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "survey_bytes": {t: {"gbs": per_kernel[t].get("survey_gbs"),
                                     "frac": round(per_kernel[t]["survey_gbs"] / HBM_PEAK_GBS, 4)}
                                 for t in survey_bytes if t in per_kernel and "survey_gbs" in per_kernel[t]}}

    # learned + batched: labels from plain sweeps on training queries, FP32
    # training, scale calibrated on held-out queries, then the evaluation queries
    # as a stream of uneven batches through a batcher with the model attached
    learned_info = None
    value, ms, rec, form = plain_value, ms_plain, plain_rec, "plain"
    if not args.plain_only:
        from paper_2411_14754_amd import learned
        t0 = time.time()
        Qt = torch.from_numpy(W.train_queries(args.train_queries + args.val_queries)).cuda()
        gt_t = exact_topk(Xd, Qt, k)
        m_tr = args.train_queries
        grid = learned.alpha_grid(0.0005, 0.05)
        net, info = learned.train_budget_model(ix, Qt[:m_tr], gt_t[:m_tr], k, beta, grid, epochs=args.epochs)
        # the predicted alpha is clamped to [0.0005, amax]; amax is chosen on the held-out queries (not the
        # evaluation ones) as the fastest of a few clamps whose calibrated scale reaches the target recall
        # there: a query whose activated points outgrow one CU's LDS leaves the sparse collision step for
        # the slower tiled one, so a tighter clamp can pay more than the recall it costs
        amin = grid[0]
        Qv, gt_v = Qt[m_tr:], gt_t[m_tr:]
        best_clamp = None
        for amax_c in (0.0025, 0.003, 0.0035, 0.005, 0.01):
            sc = learned.calibrate_scale(ix, net, Qv, gt_v, k, beta, args.target_recall, amin, amax_c)
            ids_v, _, _ = suco.query_learned(ix, net, Qv, k, beta, sc, amin, amax_c)
            rec_v = recall_at(ids_v, gt_v)
            ms_c, _ = timed_steps(lambda: suco.query_learned(ix, net, Qv, k, beta, sc, amin, amax_c), 3, 1)
            log(f"clamp {amax_c}: scale {sc:.3f}, held-out recall@10 {rec_v:.4f}, {ms_c / 3:.3f} ms per "
                f"{Qv.shape[0]} held-out queries")
            if rec_v >= args.target_recall and (best_clamp is None or ms_c < best_clamp[0]):
                best_clamp = (ms_c, amax_c, sc)
        if best_clamp is None:      # no clamp reaches the target: the widest one
            best_clamp = (ms_c, amax_c, sc)
        _, amax, scale = best_clamp
        train_s = time.time() - t0
        log(f"learned budget: trained in {train_s:.1f}s, loss {info['loss'][0]:.3f} -> {info['loss'][-1]:.3f}, "
            f"scale {scale:.3f}")
        b = suco.Batcher(ix, 4096, k, beta)
        sizes = W.batch_sizes(nq)

        def plain_stream():
            s0 = 0
            for sz in sizes:
                b.query(Qd[s0:s0 + sz], alpha=alpha, out=(ids[s0:s0 + sz], dists[s0:s0 + sz]))
                s0 += sz

        ms_pb, _ = timed_steps(plain_stream, args.steps, max(1, args.warmup))
        log(f"plain batched stream: {ms_pb / args.steps:.3f} ms/step, {nq * args.steps / (ms_pb / 1e3):.0f} QPS")
        # the same uneven batches handed over together: one launch for all of them
        bt = suco.Batcher(ix, nq, k, beta)
        starts = [sum(sizes[:j]) for j in range(len(sizes) + 1)]
        parts = [Qd[starts[j]:starts[j + 1]] for j in range(len(sizes))]
        outs = [(ids[starts[j]:starts[j + 1]], dists[starts[j]:starts[j + 1]]) for j in range(len(sizes))]
        ms_pt, _ = timed_steps(lambda: bt.query_multi(parts, alpha=alpha, outs=outs), args.steps, max(1, args.warmup))
        log(f"plain batched, {len(sizes)} batches in one launch: {ms_pt / args.steps:.3f} ms/step, "
            f"{nq * args.steps / (ms_pt / 1e3):.0f} QPS")
        b.set_model(net, scale, amin, amax)
        bt.set_model(net, scale, amin, amax)

        def stream_pass():
            s0 = 0
            for sz in sizes:
                b.query(Qd[s0:s0 + sz], out=(ids[s0:s0 + sz], dists[s0:s0 + sz]))
                s0 += sz

        ms_ls, _ = timed_steps(stream_pass, args.steps, max(1, args.warmup))
        rec_stream = recall_at(ids, gt)
        log(f"learned+batched, one launch per batch: {ms_ls / args.steps:.3f} ms/step, "
            f"{nq * args.steps / (ms_ls / 1e3):.0f} QPS, recall@10={rec_stream:.4f}")
        ids.zero_()
        ms_l, per_step = timed_steps(lambda: bt.query_multi(parts, outs=outs), args.steps, max(1, args.warmup))
        value = nq * args.steps / (ms_l / 1e3)
        rec = recall_at(ids, gt)
        learned_mre = mean_relative_error(dists, exact_dists(Xd, Qd, gt))
        ms_l1, _ = timed_steps(lambda: suco.query_learned(ix, net, Qd, k, beta, scale, amin, amax,
                                                          out=(ids, dists)), args.steps, max(1, args.warmup))
        log(f"learned, one call: {ms_l1 / args.steps:.3f} ms/step, {nq * args.steps / (ms_l1 / 1e3):.0f} QPS")
        _, _, au = suco.query_learned(ix, net, Qd, k, beta, scale, amin, amax)
        mean_alpha = float(au.double().mean())
        # plain SuCo at the same recall, interpolated on the sweep
        plain_eq = None
        for lo, hi in zip(sweep, sweep[1:]):
            if lo["recall"] < rec <= hi["recall"]:
                f = (rec - lo["recall"]) / (hi["recall"] - lo["recall"])
                plain_eq = math.exp(math.log(lo["qps"]) + f * (math.log(hi["qps"]) - math.log(lo["qps"])))
        ms, form = ms_l, f"learned+batched ({len(sizes)} uneven batches in one launch)"
        log(f"learned+batched: {ms_l / args.steps:.3f} ms/step, {value:.0f} QPS, recall@10={rec:.4f}, "
            f"mean alpha {mean_alpha:.5f}; plain at that recall {plain_eq}")
        # a higher target: the same network with its scale calibrated for recall 0.99 on the
        # held-out queries (clamp 0.05), against plain SuCo at the same recall
        t99 = 0.99
        sc99 = learned.calibrate_scale(ix, net, Qv, gt_v, k, beta, t99, amin, 0.05)
        ms99, _ = timed_steps(lambda: suco.query_learned(ix, net, Qd, k, beta, sc99, amin, 0.05,
                                                         out=(ids, dists)), args.steps, max(1, args.warmup))
        rec99 = recall_at(ids, gt)
        plain99 = None
        for lo, hi_ in zip(sweep, sweep[1:]):
            if lo["recall"] < rec99 <= hi_["recall"]:
                f = (rec99 - lo["recall"]) / (hi_["recall"] - lo["recall"])
                plain99 = math.exp(math.log(lo["qps"]) + f * (math.log(hi_["qps"]) - math.log(lo["qps"])))
        hi99 = {"target": t99, "scale": round(sc99, 5), "qps": round(nq * args.steps / (ms99 / 1e3), 1),
              "recall_at_10": round(rec99, 5), "plain_qps_at_same_recall": None if plain99 is None else round(plain99, 1)}
        log(f"learned at recall {rec99:.4f} (one call): {hi99['qps']:.0f} QPS; plain at that recall {plain99}")
        learned_info = {"plain_batched_stream_qps": round(nq * args.steps / (ms_pb / 1e3), 1),
                        "plain_batched_one_launch_qps": round(nq * args.steps / (ms_pt / 1e3), 1),
                        "learned_batched_stream_qps": round(nq * args.steps / (ms_ls / 1e3), 1),
                        "learned_batched_stream_recall_at_10": round(rec_stream, 5),
                        "learned_one_call_qps": round(nq * args.steps / (ms_l1 / 1e3), 1),
                        "at_recall_0.99": hi99,
                        "train_queries": m_tr, "val_queries": args.val_queries, "epochs": args.epochs,
                        "scale": round(scale, 5), "alpha_clamp": [amin, amax], "mean_alpha": round(mean_alpha, 6),
                        "train_s": round(train_s, 2),
                        "batch_sizes": sizes, "plain_qps_at_same_recall": None if plain_eq is None else round(plain_eq, 1),
                        "mre": learned_mre,
                        "loss_first_last": [round(info["loss"][0], 4), round(info["loss"][-1], 4)]}
        b.free()
        bt.free()
        net.free()
    ms_step = ms / args.steps
    log(f"reported: {form}, {value:.0f} QPS, recall@10={rec:.4f}")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(X, Q, alpha, beta, k, args.cpu_sample, log)

    line = {
        "metric": "QPS at recall@10=0.95, n=1M d=128: learned+batched vs plain SuCo on 1 GPU",
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_median": round(sorted(per_step)[len(per_step) // 2], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"sift_like n={n} d={d} int 0..255, N_s={ns}, sqrtK={sk}, nq={nq}, k={k}, "
                               f"beta={beta}",
                   "form": form, "recall_at_10": round(rec, 5),
                   "plain": {"alpha": alpha, "qps": round(plain_value, 1), "recall_at_10": round(plain_rec, 5),
                             "mre": plain_mre,
                             "qps_at_recall_0.95_interp": None if qps_interp is None else round(qps_interp, 1)},
                   "learned": learned_info,
                   "launches_per_step": launches, "index_build_s": round(build_s, 3), "sweep": sweep},
        "kernels": per_kernel,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ix.free()


if __name__ == "__main__":
    main()
