#!/usr/bin/env python3
"""Benchmark: walk steps/s and HBM GB/s of the DGRW hot path on one MI355X.

One step = one full pass of the hot path over the workload's query set: every
hop of every query (degree lookup, on-the-fly transition weights, total,
draw, inverse-CDF locate, emit), in one launch of the walker.  Inputs (graph,
starts, output buffer) are resident in HBM before the timed region.

Prints one JSON line (see the keys below).  The CPU baseline is the oracle
(plain single-threaded C walker) run over a bounded sample of the same
queries on the host's cores, sharded by query.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "walk steps/sec + HBM GB/s (node2vec, power-law graph); p50/p99 query latency"
PEAK_HBM_GBPS = 8000.0

WORKLOADS = {
    "rmat22_n2v": "R-MAT scale 22 (a=.57 b=.19 c=.19), edge factor 16, symmetrised, self-loops "
                  "and duplicates removed, sorted rows, ids relabelled; uint32 weights Zipf(1.2) "
                  "clipped to [1,65535]; node2vec p=1 q=2 (integer factors 2,2,1); one query per "
                  "vertex (4,194,304), 80 hops, Philox seed 42, uint64 offsets",
    "rmat22_deepwalk": "same graph as rmat22_n2v; weighted DeepWalk; one query per vertex, 80 hops",
    "rmat12_n2v": "R-MAT scale 12, edge factor 8; uint32 weights U[1,255]; node2vec p=2 q=1/2 "
                  "(factors 1,2,4); one query per vertex (4096), 20 hops, seed 42",
    "chunglu24_metapath": "Chung-Lu 2^24 vertices, gamma 2.1, ~253M stored edges, d_max ~0.94M; "
                          "labels U{0..4}, no weights; MetaPath schema [0,1,2,3,4] cycled; one "
                          "query per vertex (16,777,216), 20 hops",
    "rmat22_ppr": "same graph as rmat22_n2v; PPR with stop chance 1/5 per hop, all 4,194,304 "
                  "queries from the vertex of largest degree, at most 80 hops",
    "chunglu227m_n2v": "Chung-Lu 227M vertices, gamma 2.0, ~2.7B stored edges; weights U[1,1000]; "
                       "node2vec p=1/2 q=2 (factors 4,2,1); 10M uniform starts, 80 hops",
}

# Bytes a hop must read/write (excluding N(prev), re-read from cache): per
# attempted hop from v of degree d, offsets (16 B) plus `scan` bytes per
# neighbour; per realised hop, `emit` more bytes.
def byte_model(algo: str, weighted: bool, labelled: bool):
    if algo in ("deepwalk", "ppr"):
        # PPR's stop coin reads nothing: only hops that move are counted.
        return dict(scan=4 if weighted else 0, emit=8, moving_only=algo == "ppr")
    if algo == "node2vec":
        return dict(scan=8 if weighted else 4, emit=4)
    return dict(scan=(1 + (4 if weighted else 0)), emit=8)


# Sources the persistent walker kernel is compiled from; its compiler flags
# are hashed with them.
WALKER_SOURCES = ["csrc/fw_device.h", "csrc/fw_wave_sampler.h", "csrc/fw_kernels.h",
                  "csrc/fw_persistent.hip"]


def kernel_source_hash() -> str:
    from paper_2404_08364_amd import build
    h = hashlib.sha1()
    for rel in WALKER_SOURCES:
        h.update((ROOT / "paper_2404_08364_amd" / rel).read_bytes())
    h.update(" ".join(build.HIPCC_FLAGS).encode())
    return h.hexdigest()[:12]


def recipe_params(fw, recipe):
    walk = recipe["walk"]
    algo = walk["algo"]
    if algo == "node2vec":
        (pn, pd), (qn, qd) = walk["p"], walk["q"]
        return algo, fw.make_params(fw.node2vec_factors(pn, pd, qn, qd)), walk
    if algo == "metapath":
        return algo, fw.make_params(schema=walk["schema"]), walk
    if algo == "ppr":
        return algo, fw.make_params(stop=tuple(walk["stop"])), walk
    return algo, None, walk


def oracle_params(prm, algo):
    import oracle
    if prm is None:
        return oracle.params()
    return oracle.params(prm.f_ret, prm.f_in, prm.f_out,
                         schema=list(prm.schema)[:prm.schema_len],
                         stop=(prm.stop_num, prm.stop_den))


def account(torch, paths, deg, model):
    """Realised hops, attempted hops, scanned neighbours and algorithmic bytes
    of one pass; `prev_bytes` is what reading N(prev) once per node2vec hop
    (t >= 1: its two offsets and its adjacency slice) would add."""
    L = paths.shape[1] - 1
    hops = 0
    attempts = 0
    scanned = 0
    prev_scanned = 0
    prev_hops = 0
    for t in range(L):
        cur = paths[:, t]
        live = cur != -1
        n_live = int(live.sum())
        if n_live == 0:
            break
        moved = paths[:, t + 1] != -1
        if model.get("moving_only"):
            live = moved
        attempts += int(live.sum())
        scanned += int(deg[cur[live].long()].sum())
        hops += int(moved.sum())
        if t >= 1:
            prev_hops += n_live
            prev_scanned += int(deg[paths[:, t - 1][live].long()].sum())
    total = attempts * 16 + scanned * model["scan"] + hops * model["emit"]
    return dict(hops=hops, attempts=attempts, scanned=scanned, bytes=total,
                prev_bytes=prev_hops * 16 + prev_scanned * 4)


def roofline_record(achieved, traffic, traffic_source):
    """The dominant kernel against the HBM peak.  Algorithmic bytes count a
    row once per walk that scans it; rows that many walks scan (hubs) come
    partly from the L2 and Infinity caches, so the fraction can pass 1 and is
    then no statement about HBM: the note says so."""
    r = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
         "frac": achieved / PEAK_HBM_GBPS, "traffic": traffic,
         "traffic_source": traffic_source}
    if r["frac"] > 1:
        r["note"] = ("algorithmic bytes above the HBM peak: rows rescanned by many walks are "
                     "served from cache; only the counter traffic measures HBM")
    return r


def device_facts(torch, dev):
    """What the runtime reports for the device (hipGetDeviceProperties)."""
    p = torch.cuda.get_device_properties(dev)
    facts = dict(name=p.name, compute_units=p.multi_processor_count,
                 hbm_bytes=p.total_memory)
    for k in ("gcnArchName", "L2_cache_size", "max_threads_per_multi_processor",
              "warp_size", "shared_memory_per_block", "clock_rate"):
        v = getattr(p, k, None)
        if v is not None:
            facts[k] = v
    return facts


def copy_bandwidth(torch, dev, nbytes=2 << 30, reps=5):
    """Device-to-device copy rate (read + write bytes per second), median of
    `reps` timed copies: the achievable streaming bandwidth on this device."""
    a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (float(np.median(ms)) / 1e3) / 1e9


def _cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "" where unreadable."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(g, algo, oprm, starts, L, seed, n, target_s, gpu_rows_fn):
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    # Calibrate on a small single-threaded sample, then size the real sample.
    stride_q = np.arange(0, n, max(1, n // 4096), dtype=np.uint64)[:64]
    t0 = time.perf_counter()
    rows = oracle.walk_ids(g, algo, oprm, starts, stride_q, L, seed)
    dt = max(time.perf_counter() - t0, 1e-4)
    per_query = dt / len(stride_q)
    m = int(min(n, max(64, target_s * threads / per_query)))
    step = max(1, n // m)
    qids = np.arange(0, n, step, dtype=np.uint64)[:m]
    t0 = time.perf_counter()
    rows = oracle.walk_ids_threaded(g, algo, oprm, starts, qids, L, seed, threads)
    wall = time.perf_counter() - t0
    hops = int((rows[:, 1:] != oracle.END).sum())
    ok = bool(np.array_equal(gpu_rows_fn(qids), rows))
    # One host thread on a sixth of that sample (every 6th of its queries).
    q1 = qids[::6]
    t0 = time.perf_counter()
    rows1 = oracle.walk_ids(g, algo, oprm, starts, q1, L, seed)
    wall1 = time.perf_counter() - t0
    hops1 = int((rows1[:, 1:] != oracle.END).sum())
    return dict(value=hops / wall, unit="walk steps/s", cores=threads, kind="oracle",
                sample=f"{len(qids)} queries (every {step}-th query id), {hops} hops, "
                       f"{wall:.1f} s wall on {threads} host threads",
                cpu_model=_cpu_model(), host_cpus=os.cpu_count(),
                parity_on_sample=ok,
                one_core=dict(value=hops1 / wall1, queries=len(q1), hops=hops1,
                              seconds=wall1))


def serve_phase(fw, synth, workload: str, rates, seconds: float, max_requests: int,
                budget: int, log, mix: str = "mixed", graph=None, inflight: int = 3,
                ceiling_requests: int = 4000, check_every: int = 64, batch: int = 512,
                small: int = 0, express: int = 0):
    """Poisson request streams against the served form, one per offered rate
    (each for `seconds` of arrivals, capped at `max_requests` requests);
    returns latency and throughput per rate, and the served form's ceiling
    on the same mix: `ceiling_requests` requests submitted at once, steps /
    makespan.  Latency = completion (server clock) minus the request's
    scheduled arrival time (both CLOCK_MONOTONIC); steps are the realised
    hops the device counted per request.  Every `check_every`-th request's
    rows are compared with the batch walker's rows for the same starts and
    seed (a request's walks are the same alone and in the mix).  mix "mixed":
    DeepWalk, node2vec and MetaPath requests of lengths U{10..80}; "recipe":
    every request is the workload's own walk.  graph = (host graph, uploaded
    handle) of the same workload, reused instead of generated again."""
    import threading
    import torch
    if graph is None:
        g = synth.load_recipe_graph(workload)
        G = fw.Graph.of(g)
    else:
        g, G = graph
    if mix == "recipe":
        r_algo, r_prm, r_walk = recipe_params(fw, synth.RECIPES[workload])
        params = [(r_algo, r_prm)]
        mix_text = (f"sizes floor(log-uniform[1,65536]), every request the workload's "
                    f"{r_algo} walk of length {r_walk['length']}, Poisson arrivals")
    else:
        params = [(("deepwalk"), None),
                  ("node2vec", fw.make_params(fw.node2vec_factors(2, 1, 1, 2))),
                  ("metapath", fw.make_params(schema=[0, 1, 2]))]
        mix_text = ("sizes floor(log-uniform[1,65536]), algorithm uniform over "
                    "{DeepWalk, node2vec p=2 q=1/2, MetaPath [0,1,2]}, length U{10..80}, "
                    "Poisson arrivals")

    def stream(k, rate, n_req):
        rng = np.random.default_rng(2024 + k)
        arrivals = (np.cumsum(rng.exponential(1.0 / rate, n_req)) if rate > 0
                    else np.zeros(n_req))
        sizes = np.floor(np.exp(rng.uniform(0, np.log(65536), n_req))).astype(np.int64)
        kinds = rng.integers(0, len(params), n_req)
        lengths = rng.integers(10, 81, n_req)
        if mix == "recipe":
            lengths[:] = r_walk["length"]
        seeds = rng.integers(0, 1 << 62, n_req)
        starts_all = synth.uniform_ids(int(sizes.sum()), g.n_vertices, 77 + k)
        offs = np.concatenate([[0], np.cumsum(sizes)])
        srv = fw.Server(G, mem_budget_bytes=budget, max_inflight=inflight,
                        max_batch_requests=batch, small_max_queries=small,
                        express_max_queries=express)
        tickets = [None] * n_req
        sched_ns = [0] * n_req
        lat = np.zeros(n_req)
        hops = np.zeros(n_req, dtype=np.int64)
        kept = {}

        def submitter(t0):
            for i in range(n_req):
                target = t0 + int(arrivals[i] * 1e9)
                now = time.monotonic_ns()
                if target > now:
                    time.sleep((target - now) / 1e9)
                algo, prm = params[kinds[i]]
                sched_ns[i] = target
                tickets[i] = srv.submit(algo, prm, starts_all[offs[i]:offs[i + 1]],
                                        int(lengths[i]), int(seeds[i]))

        t0 = time.monotonic_ns() + 50_000_000
        th = threading.Thread(target=submitter, args=(t0,))
        th.start()
        done = 0
        while done < n_req:
            while tickets[done] is None:
                time.sleep(0.0005)
            keep = check_every > 0 and done % check_every == 0
            paths, st = srv.wait(tickets[done], rows=keep)
            lat[done] = (st["done_ns"] - sched_ns[done]) / 1e6
            hops[done] = int(st["steps"])
            if keep:
                kept[done] = paths
            done += 1
        th.join()
        t_end = time.monotonic_ns()
        srv.close()
        # The kept requests again, alone, through the batch walker.
        same = True
        for i, paths in kept.items():
            algo, prm = params[kinds[i]]
            st_dev = torch.from_numpy(starts_all[offs[i]:offs[i + 1]].view(np.int32)).cuda()
            alone = fw.walk(G, algo, prm, st_dev, int(lengths[i]), int(seeds[i]),
                            mode="persistent")
            torch.cuda.synchronize()
            same &= bool(np.array_equal(alone.cpu().numpy().view(np.uint32), paths))
            same &= int(hops[i]) == int((paths[:, 1:] != 0xFFFFFFFF).sum())
        wall = (t_end - t0) / 1e9
        span = float(arrivals[-1])
        offered = float(hops.sum()) / span if span > 0 else float("nan")
        served = float(hops.sum()) / wall
        return dict(offered_rate_per_s=rate if rate > 0 else None, requests=n_req,
                    arrival_span_s=span, duration_s=wall,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    mean_ms=float(lat.mean()), offered_steps_per_s=offered,
                    served_steps_per_s=served, served_queries=int(sizes.sum()),
                    steps=int(hops.sum()), keeps_up=bool(wall <= 1.1 * span + 0.5),
                    rows_checked=len(kept), rows_match_alone=same)

    ceiling = None
    if ceiling_requests > 0:
        ceiling = stream(999, 0.0, ceiling_requests)
        log(f"serve ceiling (all {ceiling_requests} requests at once): {ceiling}")
    out = []
    for k, rate in enumerate(rates):
        n_req = max(1, min(max_requests, int(seconds * rate)))
        r = stream(k, rate, n_req)
        if ceiling:
            r["served_over_ceiling"] = r["served_steps_per_s"] / ceiling["served_steps_per_s"]
        log(f"serve @ {rate}/s: {r}")
        out.append(r)
    if graph is None:
        G.free()
    kept = [r for r in out if r["keeps_up"]]
    head = max(kept, key=lambda r: r["offered_rate_per_s"]) if kept else out[0]
    return dict(workload=workload, mem_budget_bytes=budget,
                max_inflight=inflight, max_batch_requests=batch,
                small_max_queries=small, express_max_queries=express, request_mix=mix_text,
                p50_ms=head["p50_ms"], p99_ms=head["p99_ms"],
                at_rate_per_s=head["offered_rate_per_s"],
                note="p50/p99 at the highest offered rate the server kept up with",
                ceiling=ceiling, sweep=out)


def large_record(fw, synth, torch, log, workload="chunglu227m_n2v"):
    """One timed persistent pass of the largest workload (227M vertices,
    ~2.7G stored edges, node2vec from all 10,000,000 starts) with the default
    configuration, generated without the disk cache; the graph is freed
    afterwards.  Counter traffic comes from profiles/ when the kernel
    sources match."""
    t0 = time.time()
    g = synth.load_recipe_graph(workload, use_cache=False)
    log(f"graph {workload}: V={g.n_vertices} E={g.n_edges} ({time.time() - t0:.1f} s)")
    G = fw.Graph.of(g)
    algo, prm, walk = recipe_params(fw, synth.RECIPES[workload])
    L, seed = walk["length"], walk["seed"]
    starts_np = synth.recipe_starts(workload, g)
    n = starts_np.shape[0]
    st = torch.from_numpy(starts_np.view(np.int32)).cuda()
    out = torch.empty((n, L + 1), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    fw.walk(G, algo, prm, st, L, seed, out=out, mode="persistent", stream=stream, async_=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3
    fw.sync(G, stream)
    ms = e0.elapsed_time(e1)
    deg = torch.from_numpy(np.diff(np.asarray(g.offsets)).astype(np.int64)).cuda()
    acc = account(torch, out, deg, byte_model(algo, g.weights is not None, g.labels is not None))
    del deg, out, st
    G.free()
    del g
    torch.cuda.empty_cache()
    achieved = acc["bytes"] / (ms / 1e3) / 1e9
    traffic, traffic_source = None, None
    tfile = ROOT / "profiles" / f"traffic_{workload}_persistent.json"
    if tfile.exists():
        t = json.loads(tfile.read_text())
        if t.get("kernel_source") == kernel_source_hash():
            traffic = t.get("hbm_bytes_per_launch")
            traffic_source = (f"profiles/{tfile.name}: counters of an earlier profiled run of "
                              f"the same kernel sources ({t['kernel_source']})")
    r = dict(workload=workload, description=WORKLOADS[workload], mode="persistent",
             queries=n, length=L, ms_per_pass=ms, wall_ms=wall_ms,
             value=acc["hops"] / (ms / 1e3), unit="walk steps/s", hops=acc["hops"],
             neighbours_scanned=acc["scanned"], algorithmic_bytes_per_launch=acc["bytes"],
             hbm_gbps_algorithmic=achieved,
             roofline=roofline_record(achieved, traffic, traffic_source),
             traffic_gbps=traffic / (ms / 1e3) / 1e9 if traffic else None)
    log(f"{workload}: {ms:.1f} ms per pass, {r['value'] / 1e6:.2f} M steps/s, "
        f"{achieved:.0f} GB/s algorithmic")
    return r


def sampler_sweep():
    """One hop from the hub of a star graph (d leaves, weights U[1,255]) for
    every query, in the plain walker (one wavefront per query), with each
    sampler: the per-hop cost of ITS (two passes, one draw), DPRS (one pass,
    a scan and a ballot per 256 entries, one word per entry) and ZPRS (two
    passes, one scan, one word per entry) as the degree grows."""
    import torch
    from paper_2404_08364_amd import flowwalk as fw
    rng = np.random.default_rng(99)
    rows = []
    for k in range(2, 21):
        d = 1 << k
        off = np.concatenate([[0], d + np.arange(d + 1, dtype=np.uint64)]).astype(np.uint64)
        adj = np.concatenate([np.arange(1, d + 1), np.zeros(d)]).astype(np.uint32)
        w = rng.integers(1, 256, 2 * d).astype(np.uint32)
        G = fw.Graph.upload(off, adj, w, None)
        n = int(min(1 << 20, max(16384, (1 << 30) // d)))
        st = torch.zeros(n, dtype=torch.int32, device="cuda")
        out = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        res = dict(degree=d, queries=n)
        for smp in ["its", "dprs", "zprs"]:
            ms = []
            for rep in range(4):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fw.walk(G, "deepwalk", None, st, 1, 7 + rep, out=out, mode="plain", sampler=smp)
                e1.record()
                torch.cuda.synchronize()
                if rep:
                    ms.append(e0.elapsed_time(e1))
            t = float(np.median(ms))
            res[smp] = dict(ms=t, ns_per_hop=t * 1e6 / n, gelem_per_s=n * d / (t / 1e3) / 1e9)
        G.free()
        rows.append(res)
        print(json.dumps(res), flush=True)
    return rows


def task_sweep(total_log2=28):
    """Sampler microbenchmark: 2^28 uint32 weights (1 GiB) split into tasks
    of 2^k entries, one pick per task, for each sampler; weights U[1,255]
    and log-normal (mu 0, sigma 1, 2, 3; scaled by 16) as in the comparison
    with rejection sampling.  The alias table is built on one lane, so it
    runs up to 2^12 entries only."""
    import torch
    from paper_2404_08364_amd import flowwalk as fw
    rng = np.random.default_rng(5)
    n_all = 1 << total_log2
    dists = {"uniform": rng.integers(1, 256, n_all).astype(np.uint32)}
    for sg in (1, 2, 3):
        x = np.minimum(np.floor(rng.lognormal(0, sg, n_all) * 16), 2**32 - 1)
        dists[f"lognormal{sg}"] = np.maximum(x, 1).astype(np.uint32)
    rows = []
    for name, w in dists.items():
        wt = torch.from_numpy(w.view(np.int32)).cuda()
        for k in range(4, 21, 2):
            size = 1 << k
            res = dict(weights=name, size=size, tasks=n_all // size)
            for smp in ["its", "dprs", "zprs", "its_buffered", "alias", "rejection"]:
                if smp == "alias" and size > 4096:
                    continue
                if name != "uniform" and smp not in ("its", "dprs", "rejection"):
                    continue
                picks = torch.empty(n_all // size, dtype=torch.int32, device="cuda")
                ms = []
                for rep in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    fw.sample_tasks(smp, wt, size, 11 + rep, picks=picks)
                    e1.record()
                    torch.cuda.synchronize()
                    if rep:
                        ms.append(e0.elapsed_time(e1))
                t = float(np.median(ms))
                res[smp] = dict(ms=t, gelem_per_s=n_all / (t / 1e3) / 1e9)
            rows.append(res)
            print(json.dumps(res), flush=True)
        del wt
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22_n2v", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="persistent", choices=["plain", "persistent", "auto", "staged"])
    ap.add_argument("--compare-plain", type=int, default=1)
    ap.add_argument("--plain-slices", type=int, default=1,
                    help="run the plain comparison as this many launches over consecutive "
                         "query ranges (same rows), logging each")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--use-graph", type=int, default=1)
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--autotune-sample", type=int, default=0,
                    help="queries the autotuner times (0 = every k-th query, at least "
                         "262144 and 1/16 of the workload: a sample must hold many times "
                         "the 32,768 queries the resident wavefronts keep in flight, or "
                         "the tail of its last walks decides the timings)")
    ap.add_argument("--serve-seconds", type=float, default=8.0,
                    help="seconds of arrivals per offered rate (0 = no serve phase)")
    ap.add_argument("--serve-rates", default="250,500,1000,2000",
                    help="offered request rates (requests/s), comma-separated")
    ap.add_argument("--serve-max-requests", type=int, default=100000)
    ap.add_argument("--serve-ceiling", type=int, default=4000,
                    help="requests submitted at once to measure the served form's ceiling "
                         "on the same mix (0 = skip)")
    ap.add_argument("--serve-workload", default="rmat24_serve")
    ap.add_argument("--serve-batch", type=int, default=512,
                    help="requests per batch of the server (max_batch_requests, <= 4096)")
    ap.add_argument("--serve-small", type=int, default=0,
                    help="requests of at most this many queries complete in their batch's "
                         "first phase (0 = one phase)")
    ap.add_argument("--serve-express", type=int, default=0,
                    help="requests of at most this many queries may take the server's "
                         "express lane (0 = none)")
    ap.add_argument("--serve-variants", default="",
                    help="comma-separated server settings B:F:S:E (requests per batch, "
                         "batches in flight, small_max_queries, express_max_queries) run "
                         "after the main serve phase on the same graph and request streams")
    ap.add_argument("--serve-inflight", type=int, default=3,
                    help="batches the server keeps on the GPU at once (1..16)")
    ap.add_argument("--serve-mix", default="mixed", choices=["mixed", "recipe"],
                    help="mixed: DeepWalk / node2vec / MetaPath requests; recipe: every "
                         "request is the serve workload's own walk")
    ap.add_argument("--queries", type=int, default=0,
                    help="time only the first N queries of the workload (0 = all)")
    ap.add_argument("--forms", default="",
                    help="comma-separated extra launches over the same queries after the "
                         "timed pass, each timed once and its rows compared with the pass's: "
                         "staged (default staged configuration), staged-WG-DT (workgroup size "
                         "WG, hub threshold DT), sparse-R (persistent, sparse-N(prev) ratio R), "
                         "sparse-never")
    ap.add_argument("--large", type=int, default=1,
                    help="also time one persistent pass of the 227M-vertex Chung-Lu node2vec "
                         "workload from all 10M starts (the 'large' record; 0 = skip)")
    ap.add_argument("--host-batches", type=int, default=0,
                    help="also time fw_walk_host (rows to host memory) in this many batches")
    ap.add_argument("--task-sweep", action="store_true",
                    help="only run the sampler microbenchmark (2^28 weights split into tasks)")
    ap.add_argument("--sampler-sweep", action="store_true",
                    help="only time ITS / DPRS / ZPRS hops by degree on star graphs")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only copy this many bytes device-to-device (HBM counter calibration)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy // 4
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.copy_(a)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(json.dumps({"calibrate_copy_bytes": n * 4, "seconds": dt,
                          "gbps": 2 * n * 4 / dt / 1e9}), flush=True)
        return

    if args.sampler_sweep:
        sampler_sweep()
        return
    if args.task_sweep:
        task_sweep()
        return

    if args.gpus != 1:
        print(json.dumps({"error": "the walker runs on one GPU per process; --gpus must be 1 "
                                   "(queries are independent and keyed by their global id: "
                                   "split the query range across GPUs)"}))
        sys.exit(2)

    import torch
    import synth
    from paper_2404_08364_amd import flowwalk as fw

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731

    t0 = time.time()
    recipe = synth.RECIPES[args.workload]
    g = synth.load_recipe_graph(args.workload)
    log(f"graph {args.workload}: V={g.n_vertices} E={g.n_edges} ({time.time() - t0:.1f} s)")
    G = fw.Graph.of(g)
    info = G.info()
    algo, prm, walk = recipe_params(fw, recipe)
    L, seed = walk["length"], walk["seed"]
    starts_np = synth.recipe_starts(args.workload, g)
    if args.queries:
        starts_np = starts_np[: args.queries]
    n = starts_np.shape[0]
    starts = torch.from_numpy(starts_np.view(np.int32)).to(dev)
    out = torch.empty((n, L + 1), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    log(f"uploaded: {info['device_bytes'] / 1e9:.2f} GB; n={n} L={L} algo={algo}")

    def run_pass(mode):
        fw.walk(G, algo, prm, starts, L, seed, out=out, mode=mode, stream=stream, async_=True,
                use_graph=bool(args.use_graph))

    def timed(mode, steps, warmup):
        for _ in range(warmup):
            run_pass(mode)
        fw.sync(G, stream)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        t_start = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            run_pass(mode)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        fw.sync(G, stream)
        kern_ms = [a.elapsed_time(b) for a, b in evs]
        return wall * 1e3 / steps, float(np.mean(kern_ms)), kern_ms

    tuned = None
    if args.autotune and args.mode in ("persistent", "auto", "staged"):
        want = args.autotune_sample or max(262144, n // 16)
        sample = starts[:: max(1, n // want)].contiguous()
        t_at = time.time()
        tuned = fw.autotune(G, algo, prm, sample, L, seed, stream=stream)
        log(f"autotune ({sample.shape[0]} queries, {time.time() - t_at:.1f} s): {tuned}")

    ms_step, kern_ms, all_ms = timed(args.mode, args.steps, args.warmup)
    log(f"{args.mode}: {ms_step:.1f} ms/step, kernel {kern_ms:.1f} ms ({all_ms})")

    deg = torch.from_numpy(np.diff(np.asarray(g.offsets)).astype(np.int64)).to(dev)
    model = byte_model(algo, g.weights is not None, g.labels is not None)
    acc = account(torch, out, deg, model)
    hops, attempts, scanned, alg_bytes = acc["hops"], acc["attempts"], acc["scanned"], acc["bytes"]
    paths_main = out.clone()
    value = hops / (ms_step / 1e3)
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    log(f"hops={hops} attempts={attempts} scanned={scanned} bytes={alg_bytes / 1e9:.1f} GB "
        f"-> {value / 1e6:.1f} M steps/s, {achieved:.0f} GB/s algorithmic")

    plain = None
    if args.compare_plain and args.mode != "plain" and args.plain_slices > 1:
        # The plain walker over consecutive slices of the query set (query ids
        # kept by qid_base, so the rows are those of one launch), one launch
        # and one log line per slice.
        out.fill_(-7)
        bounds = np.linspace(0, n, args.plain_slices + 1).astype(np.int64)
        total_ms = 0.0
        for k in range(args.plain_slices):
            lo, hi = int(bounds[k]), int(bounds[k + 1])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fw.walk(G, algo, prm, starts[lo:hi], L, seed, out=out[lo:hi], mode="plain",
                    stream=stream, async_=True, qid_base=lo)
            e1.record(stream)
            torch.cuda.synchronize()
            fw.sync(G, stream)
            total_ms += e0.elapsed_time(e1)
            log(f"plain slice {k + 1}/{args.plain_slices}: queries {lo}..{hi}, "
                f"{e0.elapsed_time(e1):.1f} ms")
        same = bool(torch.equal(out, paths_main))
        plain = dict(ms_per_step=total_ms, value=hops / (total_ms / 1e3), identical_paths=same,
                     slices=args.plain_slices)
        log(f"plain: {total_ms:.1f} ms in {args.plain_slices} slices, identical={same}")
    elif args.compare_plain and args.mode != "plain":
        ms_p, kern_p, _ = timed("plain", max(1, min(args.steps, 2)), 0)
        same = bool(torch.equal(out, paths_main))
        plain = dict(ms_per_step=ms_p, value=hops / (ms_p / 1e3), identical_paths=same)
        log(f"plain: {ms_p:.1f} ms/step, identical={same}")

    forms = []
    for spec in [x for x in args.forms.split(",") if x]:
        parts = spec.split("-")
        if parts[0] == "staged":
            mode = "staged"
            tune = (fw.make_tune(wg_size=int(parts[1]), hub_min=int(parts[2]))
                    if len(parts) == 3 else None)
        elif parts[0] == "sparse" and len(parts) == 2:
            mode = "persistent"
            tune = fw.make_tune(sparse_ratio=0xFFFFFFFF if parts[1] == "never" else int(parts[1]))
        else:
            raise SystemExit(f"unknown form {spec}")
        out.fill_(-7)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fw.walk(G, algo, prm, starts, L, seed, out=out, mode=mode, stream=stream, async_=True,
                tune=tune)
        e1.record(stream)
        torch.cuda.synchronize()
        fw.sync(G, stream)
        f_ms = e0.elapsed_time(e1)
        same = bool(torch.equal(out, paths_main))
        forms.append(dict(form=spec, ms=f_ms, value=hops / (f_ms / 1e3), identical_paths=same))
        log(f"form {spec}: {f_ms:.1f} ms, {hops / (f_ms / 1e3) / 1e6:.2f} M steps/s, "
            f"identical={same}")

    host = None
    if args.host_batches:
        L1 = L + 1
        budget = -(-n // args.host_batches) * 2 * (L + 2) * 4
        fw.walk_host(G, algo, prm, starts_np[: min(n, 65536)], L, seed)  # warm
        t_h = time.perf_counter()
        rows_h, B, nb = fw.walk_host(G, algo, prm, starts_np, L, seed, device_budget_bytes=budget)
        dt_h = time.perf_counter() - t_h
        same_h = bool(np.array_equal(rows_h, paths_main.cpu().numpy().view(np.uint32)))
        host = dict(ms=dt_h * 1e3, value=hops / dt_h, batch_queries=B, batches=nb,
                    result_bytes=n * L1 * 4, identical_paths=same_h,
                    note="rows to pageable host memory through two pinned staging buffers "
                         "(PCIe-inclusive); not the headline value")
        del rows_h
        log(f"host batches: {host}")

    copy_gbps = copy_bandwidth(torch, dev)
    log(f"device copy: {copy_gbps:.0f} GB/s (read + write)")

    # HBM bytes per launch from rocprofv3 counters (FETCH_SIZE, WRITE_SIZE)
    # of an earlier run of the same kernel sources, recorded under profiles/;
    # this run does not read counters itself.
    traffic = None
    traffic_source = None
    tfile = ROOT / "profiles" / f"traffic_{args.workload}_{args.mode}.json"
    if tfile.exists():
        t = json.loads(tfile.read_text())
        if t.get("kernel_source") == kernel_source_hash():
            traffic = t.get("hbm_bytes_per_launch")
            traffic_source = (f"profiles/{tfile.name}: counters of an earlier profiled run of "
                              f"the same kernel sources ({t['kernel_source']})")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oprm = oracle_params(prm, algo)
        host_paths = paths_main.cpu().numpy().view(np.uint32)
        cpu = cpu_baseline(g, algo, oprm, starts_np, L, seed, n, args.cpu_seconds,
                           lambda q: host_paths[q.astype(np.int64)])
        log(f"cpu baseline: {cpu}")

    latency = None
    if args.serve_seconds > 0:
        del out
        torch.cuda.empty_cache()
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        same = (g, G) if args.serve_workload == args.workload else None
        if same is None and args.serve_variants:
            sg = synth.load_recipe_graph(args.serve_workload)
            same = (sg, fw.Graph.of(sg))
        latency = serve_phase(fw, synth, args.serve_workload, rates, args.serve_seconds,
                              args.serve_max_requests, 4 << 30, log, args.serve_mix, same,
                              args.serve_inflight, args.serve_ceiling, batch=args.serve_batch,
                              small=args.serve_small, express=args.serve_express)
        # Other server settings on the same graph and request streams.
        variants = []
        for spec in [x for x in args.serve_variants.split(",") if x]:
            vb, vf, vs, ve = (int(x) for x in spec.split(":"))
            r = serve_phase(fw, synth, args.serve_workload, rates, args.serve_seconds,
                            args.serve_max_requests, 4 << 30, log, args.serve_mix, same, vf,
                            args.serve_ceiling, 0, batch=vb, small=vs, express=ve)
            variants.append(dict(max_batch_requests=vb, max_inflight=vf, small_max_queries=vs,
                                 express_max_queries=ve,
                                 ceiling_steps_per_s=(r["ceiling"] or {}).get("served_steps_per_s"),
                                 sweep=[{k: x[k] for k in ("offered_rate_per_s", "p50_ms", "p99_ms",
                                                           "served_steps_per_s", "keeps_up")}
                                        for x in r["sweep"]]))
            log(f"serve variant {spec}: {variants[-1]}")
        if variants:
            latency["variants"] = variants

    large = None
    if args.large and args.workload != "chunglu227m_n2v":
        G.free()
        torch.cuda.empty_cache()
        large = large_record(fw, synth, torch, log)

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "mode": args.mode, "queries": n, "length": L,
                   "n_vertices": g.n_vertices, "n_edges": g.n_edges,
                   "max_degree": info["max_degree"]},
        "hbm_gbps_algorithmic": achieved,
        "roofline": roofline_record(achieved, traffic, traffic_source),
        "kernel_ms": kern_ms,
        "hops": hops,
        "attempted_hops": attempts,
        "neighbours_scanned": scanned,
        "edges_scanned_per_s": scanned / (kern_ms / 1e3),
        "algorithmic_bytes_per_launch": alg_bytes,
        "prev_row_bytes_per_launch": acc["prev_bytes"] if algo == "node2vec" else 0,
        "hbm_gbps_incl_prev_row": ((alg_bytes + acc["prev_bytes"]) / (kern_ms / 1e3) / 1e9
                                   if algo == "node2vec" else achieved),
        "copy_gbps": copy_gbps,
        "traffic_gbps": traffic / (kern_ms / 1e3) / 1e9 if traffic else None,
        "device": device_facts(torch, dev),
        "plain": plain,
        "forms": forms or None,
        "host_batches": host,
        "cpu_baseline": cpu,
        "latency": latency,
        "large": large,
        "tuned": tuned,
        "kernel_source": kernel_source_hash(),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
