#!/usr/bin/env python3
"""Throughput of GFD validation on one MI355X.

One step = one gfd_validate call over the workload's whole GFD set: candidate
filtering and CPI construction, core-first enumeration, the fused X -> Y check
and first-K selection for every GFD, with the graph already resident in HBM.

Default workload: the 4M-vertex / 20M-edge knowledge-graph-shaped graph with
256 GFDs of 2-8 vertices, validated in batched form; the same 256 GFDs are
also timed one at a time (256 sequential single-GFD calls) for the
batched-vs-one-at-a-time ratio.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload kg_4m_batch256|kg_4m|powerlaw_1m|twitch_trio]
    python bench.py --workload kg_4m_serving [--serve-seconds S] [--serve-rates R1,R2,..]

The serving workload replays Poisson arrivals (200 requests/s, each 1-4 GFDs
of 3-8 vertices, taken in order from a pool of 4,000 walk-sampled GFDs)
against gfd_server_* with continuous batching and reports p50/p99 latency
beside throughput, then the same at each rate of a sweep of offered loads.
"""
from __future__ import annotations

import argparse
import json
import statistics
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "embeddings/s and GFDs validated/s, batched vs one-at-a-time; % HBM peak"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
K_REPORT = 1024


# HBM traffic of the dominant kernel, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this workload scaled by the same counters on a plain
# 1 GiB copy-like kernel (bench.py --copy-probe); see profiles/.  Valid only
# for the kernel sources it was measured on (sha256 of the two files below).
TRAFFIC = {
    "sources_sha256": "e17cd3e18361270f28fdf57df0686bc5f1e05d216f1b6519571bccc497f90f78",
    "workload": "kg_4m_batch256",
    "kernel_class": "extend_last",  # k_ext_run<true, false, 8>
    "semantics": "induced",
    "count_only": False,
    # (638.27 MB read + 39.77 MB written) per dispatch, calibrated (x1.9999, x1.0)
    "bytes_per_launch": 6.7804e+08,
}
# Units of work of the dominant kernel class per step (one validate call),
# from the counting build (bench.py --units; see profiles/), and the
# algorithmic bytes the per-unit model gives them: 4 B per attempt, 8 B per
# source, 4 B per search step of ceil(log2 d) over a row of d entries for a
# one-direction probe and twice that for a check of both directions, 4 B per
# attribute value a literal reads.  Per step, not per launch: a call may add a
# small threshold re-run launch or not, which leaves the work per step as it
# is.  Valid only for the kernel sources it was counted on.
UNITS = {
    "sources_sha256": "e17cd3e18361270f28fdf57df0686bc5f1e05d216f1b6519571bccc497f90f78",
    "workload": "kg_4m_batch256",
    "kernel_class": "extend_last",
    "semantics": "induced",
    "count_only": False,
    "per_step": {"attempts": 158480914, "sources": 12614816, "injective": 158469327,
                 "checks_both": 416611439, "table_free": 361637571, "table_hit": 8274566,
                 "short_row": 46699302, "both_steps": 205912408, "both_log2d": 3856520308,
                 "checks_one": 0, "one_steps": 0, "one_log2d": 0, "matches": 147891222,
                 "literal_reads": 162874008, "violations": 68082422, "inner_attempts": 19555525},
    "model_bytes_per_step": 3.22385e10,
}
TRAFFIC_SOURCES = ("paper_2608_02321_amd/csrc/gfd_kernels.hip", "paper_2608_02321_amd/csrc/gfd_internal.h")


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def copy_gbs(torch):
    """Achievable HBM rate on this device: a plain elementwise int32 kernel
    reading 1 GiB and writing 1 GiB, best of five launches timed with events."""
    n = 1 << 28
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    best = None
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        torch.neg(src, out=dst)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 8.0 * n / (best * 1e-3) / 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(g, gfds, semantics, frac, threads):
    """The oracle (naive backtracking) on a bounded sample of the same job:
    every GFD, with the first pattern variable restricted to the first `frac`
    of the vertex ids, on `threads` host threads (split by root ranges); and
    on one thread over a sixteenth of that sample."""
    from oracle import oracle as O
    og = O.OracleGraph(g)

    def run(fr, th):
        hi = max(1, int(g.n * fr))
        t = time.perf_counter()
        matches = 0
        for d in gfds:
            r = O.validate(og, d, semantics, K=K_REPORT, root_range=(0, hi), threads=th)
            matches += r["match_count"]
        dt = time.perf_counter() - t
        return {"value": matches / dt, "unit": "embeddings/s", "cores": th, "kind": "oracle",
                "sample": f"all {len(gfds)} GFDs, first variable restricted to vertex ids "
                          f"[0, {hi}) ({fr:.2%} of {g.n}); {matches} matches in {dt:.2f} s",
                "gfds_per_s": len(gfds) * fr / dt}

    out = run(frac, threads)
    out["single_thread"] = run(frac / 16, 1)
    return out


def unit_report(args, P, gh, gfds, stream, batched):
    """Unit counts of the last enumeration level (the dominant kernel class)
    from the counting build, per launch, and the algorithmic bytes they imply
    under the per-unit model: 4 B per attempt (its CPI entry), 8 B per source
    (its list's offsets), 4 B per search step of ceil(log2 d) over a row of d
    entries for a one-direction probe and twice that for a check of both
    directions, 4 B per attribute value a literal reads.  Printed beside the
    bytes the kernels count on the device, which price what they touch: table
    bounds and one byte per fingerprint slot instead of a row search."""
    K = 0 if args.count_only else K_REPORT
    flags = (P.GFD_FLAG_COUNT_ONLY if args.count_only else 0) | P.GFD_FLAG_NO_GRAPH
    pc = P.PreparedCall(gh, gfds, K=K, semantics=args.semantics, stream=stream, batched=batched)
    pc.run(flags=flags)
    st = pc.run(flags=flags | P.GFD_FLAG_TIMING)
    assert st["units_counted"], "GFD_LIBRARY did not load the counting build"
    u = st["units"]
    n = max(1, st["class_launches"]["extend_last"])
    model = (4 * u["attempts"] + 8 * u["sources"] + 8 * u["both_log2d"] + 4 * u["one_log2d"]
             + 4 * u["literal_reads"])
    dev = st["class_bytes"]["extend_last"]
    ms = st["class_ms"]["extend_last"]
    out = {"units_per_step": u, "extend_last_launches": n,
           "units_per_launch": {k: v / n for k, v in u.items()},
           "model_bytes_per_step": model, "model_bytes_per_launch": model / n,
           "device_bytes_per_launch": dev / n,
           "extend_last_ms_per_step": ms, "matches_per_step": pc.match_count(),
           "config": {"workload": args.workload, "semantics": args.semantics,
                      "count_only": bool(args.count_only), "library": "libgfd_count.so"}}
    if ms > 0:
        out["model_gbs"] = model / (ms * 1e-3) / 1e9
        out["device_gbs"] = dev / (ms * 1e-3) / 1e9
    log(json.dumps(out, indent=1))
    print(json.dumps(out), flush=True)


class ServingRig:
    """Poisson arrivals of requests (1-4 GFDs each, taken in order from the
    4,000-GFD walk-sampled pool) against gfd_server_* with continuous
    batching; every served result is checked against the same GFD validated
    alone (one single-GFD call, cached per pool position)."""

    def __init__(self, P, g, gh, semantics, workers):
        from synth import configs
        self.P, self.g, self.gh, self.semantics, self.workers = P, g, gh, semantics, workers
        self.configs = configs
        self.pool = [{k: v for k, v in d.items() if k != "meta"} for d in configs.serving_pool(g)]
        self.alone = {}

    def alone_result(self, i):
        if i not in self.alone:
            q = self.P.PreparedCall(self.gh, [self.pool[i]], K=K_REPORT, semantics=self.semantics)
            q.run(stats=False, flags=self.P.GFD_FLAG_NO_GRAPH)
            self.alone[i] = q.results()[0]
        return self.alone[i]

    def run(self, rate, seconds, seed):
        import threading
        import numpy as np
        P, pool = self.P, self.pool
        reqs = self.configs.serving_requests(self.g, rate=rate, duration_s=seconds, seed=seed,
                                             pool=pool)
        # pool positions of each request's GFDs (taken in order, wrapping)
        idx, at = [], 0
        for r in reqs:
            idx.append([(at + j) % len(pool) for j in range(len(r["gfds"]))])
            at += len(r["gfds"])
        srv = P.Server(self.gh, K=K_REPORT, semantics=self.semantics, workers=self.workers)
        for w in range(3):  # warm-up: workspaces and first launches
            srv.wait(srv.submit(reqs[w]["gfds"]))
        done = [None] * len(reqs)
        ids = [None] * len(reqs)
        ready = [threading.Event() for _ in reqs]

        def waiter():
            for j in range(len(reqs)):
                ready[j].wait()
                done[j] = srv.wait(ids[j])

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for j, r in enumerate(reqs):
            dt = t0 + r["t"] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            ids[j] = srv.submit(r["gfds"])
            ready[j].set()
        th.join()
        srv.close()
        lat = np.array([(info["done_ns"] - info["submit_ns"]) / 1e6 for _, info in done])
        wall = (max(i["done_ns"] for _, i in done) - min(i["submit_ns"] for _, i in done)) / 1e9
        matches = 0
        for (res, _), ix in zip(done, idx):
            assert res == [self.alone_result(i) for i in ix], "a served result differs from the GFD alone"
            matches += sum(r["match_count"] for r in res)
        batches = {info["batch_id"]: info["batch_gfds"] for _, info in done}
        ngfd = sum(len(x) for x in idx)
        return {"rate_per_s": rate, "seconds": seconds, "requests": len(reqs), "gfds": ngfd,
                "distinct_gfds": len({i for x in idx for i in x}),
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_ms": float(lat.max()), "gfds_per_s": ngfd / wall,
                "embeddings_per_s": matches / wall, "batches": len(batches),
                "mean_batch_gfds": float(np.mean(list(batches.values()))),
                "workers": self.workers, "identical_to_alone": True}


def serve(args, torch, P, g, gh):
    """The serving workload: the headline rate, then each rate of a sweep."""
    rig = ServingRig(P, g, gh, args.semantics, args.serve_workers)
    head = rig.run(args.serve_rate, args.serve_seconds, 4)
    log(f"serving at {args.serve_rate:g}/s: {head['requests']} requests, p50 {head['p50_ms']:.1f} ms, "
        f"p99 {head['p99_ms']:.1f} ms, {head['gfds_per_s']:.0f} GFDs/s, {head['batches']} batches")
    sweep = []
    for k, rate in enumerate(args.serve_rates):
        row = rig.run(rate, args.sweep_seconds, 40 + k)
        log(f"  offered {rate:g}/s: p50 {row['p50_ms']:.1f} ms, p99 {row['p99_ms']:.1f} ms, "
            f"{row['gfds_per_s']:.0f} GFDs/s, mean batch {row['mean_batch_gfds']:.1f} GFDs")
        sweep.append(row)
    out = {"metric": METRIC, "value": head["embeddings_per_s"], "unit": "embeddings/s", "n_gpus": 1,
           "steps": head["requests"], "warmup": 3, "ms_per_step": head["p50_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic", "gfds_per_s": head["gfds_per_s"],
           "config": {"workload": "kg_4m_serving", "mode": "serving", "n": g.n, "m": g.m,
                      "rate_per_s": args.serve_rate, "seconds": args.serve_seconds,
                      "pool_gfds": len(rig.pool), "semantics": args.semantics, "K": K_REPORT,
                      "workers": args.serve_workers, "parallelism": "single_gpu"},
           "serving": head, "sweep": sweep, "roofline": None}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="kg_4m_batch256")
    ap.add_argument("--mode", choices=["batched", "plain"], default=None,
                    help="default: batched for the 256-GFD workload, plain otherwise")
    ap.add_argument("--semantics", default="induced", choices=["induced", "mono"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rates", type=lambda x: [float(v) for v in x.split(",") if v],
                    default=[100.0, 400.0, 800.0, 1600.0, 3200.0],
                    help="offered loads (requests/s) of the sweep after the headline rate")
    ap.add_argument("--sweep-seconds", type=float, default=3.0)
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the short serving leg of the default workload")
    ap.add_argument("--serving-leg-seconds", type=float, default=3.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-workers", type=int, default=2)
    ap.add_argument("--cpu-frac", type=float, default=None)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the one-at-a-time comparison")
    ap.add_argument("--no-timing", action="store_true",
                    help="no HIP events at all (no roofline line)")
    ap.add_argument("--count-only", action="store_true",
                    help="counts and satisfied flags only (K = 0, no fingerprints): postponed "
                         "leaves are counted, not enumerated (with --semantics mono)")
    ap.add_argument("--k", type=int, default=None, metavar="K",
                    help="violations listed per GFD (default 1024, or 0 with --count-only; "
                         "a count-only call with K > 0 lists the first K from the window its "
                         "counts bound)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB read + 1 GiB write elementwise kernel "
                         "(int32 negation) three times: the calibration run for HBM counters")
    ap.add_argument("--sources-sha256", action="store_true",
                    help="print the hash of the kernel sources that counter figures are keyed on")
    ap.add_argument("--mem-budget", type=int, default=0, metavar="BYTES",
                    help="device bytes a call may use for its workspace (0: the library's "
                         "default); implies --no-tune")
    ap.add_argument("--no-tune", action="store_true",
                    help="run with the library's default launch shapes (no autotuning)")
    ap.add_argument("--units", action="store_true",
                    help="measurement run on the unit-counting build (libgfd_count.so): the "
                         "dominant class's unit counts per launch and the byte model priced "
                         "from them, beside the device-counted algorithmic bytes")
    ap.add_argument("--per-gfd", type=int, default=0, metavar="N",
                    help="diagnostic: validate each GFD alone with statistics and print the "
                         "N slowest to stderr")
    args = ap.parse_args()
    if args.sources_sha256:
        print(sources_sha256())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; how the path would shard "
                                   "across GPUs is a design note, not an implemented path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    mode = args.mode or ("batched" if args.workload.endswith("batch256") else "plain")

    import torch
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = 1 << 28  # int32 elements: 1 GiB in, 1 GiB out per launch
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe": {"launches": 3, "read_bytes_per_launch": 4 * n,
                                         "write_bytes_per_launch": 4 * n}}), flush=True)
        return
    if args.units:  # before the package loads its library
        os.environ["GFD_LIBRARY"] = os.path.join(ROOT, "paper_2608_02321_amd", "libgfd_count.so")
    import paper_2608_02321_amd as P
    from paper_2608_02321_amd._binding import KERNEL_CLASSES
    from synth import configs

    t = time.perf_counter()
    g = configs.graph(configs.CONFIG_GRAPH[args.workload])
    gfds = [] if args.workload == "kg_4m_serving" else \
        [{k: v for k, v in d.items() if k != "meta"} for d in configs.gfds(args.workload, g)]
    log(f"inputs: {args.workload} n={g.n} m={g.m} gfds={len(gfds)} ({time.perf_counter() - t:.1f}s)")
    stream = torch.cuda.current_stream()
    free0 = torch.cuda.mem_get_info()[0]
    t = time.perf_counter()
    gh = P.load(g, stream=stream)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t
    if args.workload == "kg_4m_serving":
        serve(args, torch, P, g, gh)
        gh.free()
        return
    batched = mode == "batched"

    if args.units:
        unit_report(args, P, gh, gfds, stream, batched)
        gh.free()
        return

    # specs, options and result buffers are marshalled once; a step is one
    # gfd_validate_ex call through the C ABI
    K = args.k if args.k is not None else (0 if args.count_only else K_REPORT)
    base_flags = P.GFD_FLAG_COUNT_ONLY if args.count_only else 0
    # launch shapes: the autotuner's choice for this call shape (tried and
    # checked for identical results on this graph, or read from its cache)
    tuning, tune_info = None, None
    if not args.no_tune and not args.mem_budget:
        from paper_2608_02321_amd import tune as T
        t = time.perf_counter()
        tune_info = T.tune(gh, gfds, g.sha256(), K=K, semantics=args.semantics, batched=batched,
                           count_only=args.count_only, stream=stream, log=log)
        tuning = tune_info["tuning"]
        gh.trim()  # the candidates' workspaces go: what is held is what the chosen shapes need
        torch.cuda.empty_cache()  # and torch's allocator returns them to the device
        log(f"tuning: {tuning} ({'cached' if tune_info['cached'] else 'tuned'} in "
            f"{time.perf_counter() - t:.1f} s): {tune_info['tuned_ms']:.2f} ms against "
            f"{tune_info['default_ms']:.2f} ms with the defaults")
    pc = P.PreparedCall(gh, gfds, K=K, semantics=args.semantics, stream=stream,
                        batched=batched, tuning=tuning, mem_budget_bytes=args.mem_budget)

    # warm-up (the first step captures the batch's main pass as a graph, later
    # ones replay it); the last warm-up step runs eagerly with events on every
    # kernel class to find the dominant one
    for w in range(max(1, args.warmup)):
        st = pc.run(flags=base_flags | (0 if args.no_timing or w < args.warmup - 1
                                        else P.GFD_FLAG_TIMING))
    torch.cuda.synchronize()
    # the library keeps its workspaces between calls, so what the device lost
    # since before the load is the graph plus the largest workspace: the peak
    held_bytes = free0 - torch.cuda.mem_get_info()[0]
    res = pc.results()
    dom = None
    enum_rate = None
    if not args.no_timing:
        dom = max(range(8), key=lambda c: st["class_ms"][KERNEL_CLASSES[c]])
        log("warm-up per class: " + ", ".join(
            f"{k} {v:.2f} ms/{st['class_launches'][k]} launches/"
            f"{st['class_bytes'][k] / max(v, 1e-9) / 1e6:.0f} GB/s"
            for k, v in st["class_ms"].items()))
        log(f"warm-up: wall {st['wall_ms']:.1f} ms, kernel time {sum(st['class_ms'].values()):.1f} ms, "
            f"chunked {st['chunked_gfds']}, threshold {st['threshold_gfds']}/{st['threshold_passes']}, "
            f"counted leaves {st['leaf_gfds']} ({st['leaf_split_gfds']} split), regrown {st['regrown_gfds']}, "
            f"batches {st['batches']}, graphs "
            f"{st['graph_captures']} captured / {st['graph_replays']} replayed, frontier pool "
            f"{st['front_pool_bytes'] / 1e6:.0f} MB, CPI arena {st['cpi_arena_bytes'] / 1e6:.0f} MB")
        enum_ms = st["class_ms"]["extend"] + st["class_ms"]["extend_last"]
        if enum_ms > 0:
            enum_rate = sum(r["match_count"] for r in res) / (enum_ms * 1e-3)
    # the timed steps call as a user who asks for no statistics does (no
    # device byte counters, nothing read back for them); such a call is a
    # shape of its own, so two untimed ones first: the second captures the
    # graph the timed steps replay
    for _ in range(2):
        pc.run(flags=base_flags, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        pc.run(flags=base_flags, stats=False)  # synchronous: returns with the results on the host
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    assert pc.results() == res, "results changed between steps"
    # (the log's launch counts come from the last warm-up step's statistics)
    # the dominant kernel's launches, timed with HIP events on the call's
    # stream over further steps run eagerly (events around kernels inside a
    # replayed graph are not available); the kernels are the same
    agg_ms = agg_bytes = agg_launch = 0.0
    roof_steps = 0
    if dom is not None:
        roof_steps = max(3, min(args.steps, 10))
        name = KERNEL_CLASSES[dom]
        for _ in range(roof_steps):
            s2 = pc.run(flags=base_flags | P.GFD_FLAG_NO_GRAPH | (1 << (8 + dom)))
            agg_ms += s2["class_ms"][name]
            agg_bytes += s2["class_bytes"][name]
            agg_launch += s2["class_launches"][name]
        assert pc.results() == res, "eager results differ from the replayed ones"
    matches = sum(r["match_count"] for r in res)
    value = matches * args.steps / elapsed
    gfds_per_s = len(gfds) * args.steps / elapsed
    fixed_ms = None
    if tuning and any(tuning.values()):  # the same steps with the default launch shapes
        pf = P.PreparedCall(gh, gfds, K=K, semantics=args.semantics, stream=stream,
                            batched=batched)
        for _ in range(3):
            pf.run(flags=base_flags)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            pf.run(flags=base_flags)
        torch.cuda.synchronize()
        fixed_ms = (time.perf_counter() - t1) * 1e3 / args.steps
        assert pf.results() == res, "default launch shapes changed a result"
    log(f"{mode}: step {ms_per_step:.3f} ms, {matches} matches, {value:.4g} embeddings/s, "
        f"{gfds_per_s:.1f} GFDs/s, launches/step {st['launches']}, "
        f"bounded re-runs {st['chunked_gfds']}")

    roofline = None
    if dom is not None and agg_launch:
        name = KERNEL_CLASSES[dom]
        avg_ms = agg_ms / agg_launch
        dev_per_launch = agg_bytes / agg_launch  # counted on the device
        gbs = lambda b: b / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0  # noqa: E731

        def valid(tab):
            return (tab["kernel_class"] == name and tab["workload"] == args.workload
                    and tab["semantics"] == args.semantics
                    and tab["count_only"] == bool(args.count_only) and args.k is None
                    and tab["sources_sha256"] == sources_sha256())
        traffic = TRAFFIC["bytes_per_launch"] if valid(TRAFFIC) else None
        # algorithmic bytes: the per-unit model over the units one launch
        # processes (counting build), else the bytes counted on the device
        if valid(UNITS):  # the step's model bytes over this run's launches per step
            per_launch = UNITS["model_bytes_per_step"] / (agg_launch / roof_steps)
            basis = "per-unit model x counted units"
        else:
            per_launch, basis = dev_per_launch, "device-counted bytes (unit counts stale)"
        ach = gbs(per_launch)
        copy = copy_gbs(torch)
        roofline = {"bound": "hbm", "kernel_class": name, "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                    "basis": basis,
                    # the bytes the kernel as built touches (tables instead of
                    # row searches), counted on the device over the same launches
                    "device_bytes_per_launch": dev_per_launch,
                    "device_frac": gbs(dev_per_launch) / HBM_PEAK_GBS,
                    # measured HBM bytes (rocprofv3 counters, calibrated) over the same time
                    "measured_frac": (gbs(traffic) / HBM_PEAK_GBS if traffic else None),
                    "avg_launch_ms": avg_ms, "alg_bytes_per_launch": per_launch,
                    "launches_per_step": agg_launch / roof_steps,
                    "timed_over": f"{roof_steps} eager steps after the timed ones, HIP events "
                                  f"around each launch of the class on the call's stream",
                    "copy_gbs": copy, "frac_of_copy": ach / copy}

    if args.per_gfd:
        rows = []
        for i, d in enumerate(gfds):
            r, s1 = P.validate(gh, [d], K=K_REPORT, semantics=args.semantics, stream=stream,
                               flags=P.GFD_FLAG_TIMING, stats=True)
            rows.append((s1["wall_ms"], i, d, r[0], s1))
        rows.sort(key=lambda x: -x[0])
        log(f"per-GFD (alone, with events), total {sum(x[0] for x in rows):.1f} ms")
        for wall, i, d, r, s1 in rows[:args.per_gfd]:
            cm = " ".join(f"{k}={v:.2f}" for k, v in s1["class_ms"].items() if v >= 0.05)
            log(f"  #{i} k={d['k']} e={len(d['edges'])} wall={wall:.2f}ms match={r['match_count']} "
                f"viol={r['violation_count']} att={s1['attempts']} part={s1['partials']} "
                f"cand={s1['cpi_candidates']} cpi={s1['cpi_entries']} chunked={s1['chunked_gfds']} "
                f"thr={s1['threshold_gfds']}/{s1['threshold_passes']} | {cm}")

    # the serving form on the same graph, briefly (the kg_4m_serving workload
    # runs it at length and sweeps the offered load)
    serving = None
    if args.workload == "kg_4m_batch256" and not args.no_serving and not args.count_only:
        rig = ServingRig(P, g, gh, args.semantics, args.serve_workers)
        serving = rig.run(args.serve_rate, args.serving_leg_seconds, 4)
        log(f"serving leg at {args.serve_rate:g}/s: {serving['requests']} requests, "
            f"p50 {serving['p50_ms']:.1f} ms, p99 {serving['p99_ms']:.1f} ms, "
            f"{serving['gfds_per_s']:.0f} GFDs/s")

    compare = None
    if batched and not args.no_compare:
        # the same GFDs, one gfd_validate call each (one-at-a-time), marshalled
        # up front like the batched call
        one = [P.PreparedCall(gh, [d], K=K, semantics=args.semantics, stream=stream)
               for d in gfds]
        for _ in range(2):  # warm: each call's main pass runs once, is captured, then replayed
            for q in one:
                q.run(flags=base_flags, stats=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for q in one:
            q.run(flags=base_flags, stats=False)
        torch.cuda.synchronize()
        dt1 = time.perf_counter() - t1
        seq = [q.results()[0] for q in one]
        assert seq == res, "one-at-a-time results differ from the batched call"
        compare = {"one_at_a_time_s": dt1, "one_at_a_time_gfds_per_s": len(gfds) / dt1,
                   "one_at_a_time_embeddings_per_s": matches / dt1,
                   "batched_over_one_at_a_time": (len(gfds) * args.steps / elapsed) / (len(gfds) / dt1)}
        log(f"one-at-a-time: {dt1 * 1e3:.1f} ms for {len(gfds)} calls; ratio "
            f"{compare['batched_over_one_at_a_time']:.2f}x")

    out = {"metric": METRIC, "value": value, "unit": "embeddings/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic", "gfds_per_s": gfds_per_s, "matches_per_step": matches,
           "config": {"workload": args.workload, "mode": mode, "n": g.n, "m": g.m,
                      "gfds": len(gfds), "semantics": args.semantics, "K": K,
                      "count_only": bool(args.count_only), "mem_budget_bytes": args.mem_budget,
                      "parallelism": "single_gpu"},
           "ms_per_step_median": statistics.median(step_ms), "ms_per_step_min": min(step_ms),
           "enumeration_embeddings_per_s": enum_rate,
           "device_bytes": {"graph": gh.info["device_bytes"], "held": held_bytes},
           "load_s": load_s, "roofline": roofline, "compare": compare, "serving": serving,
           "tuning": None if tune_info is None else {
               "choice": tuning, "cached": tune_info["cached"],
               "tuned_ms_per_step": ms_per_step,
               "fixed_ms_per_step": fixed_ms if fixed_ms is not None else ms_per_step,
               "tuner_ms": {"tuned": tune_info["tuned_ms"], "default": tune_info["default_ms"]}}}
    if not args.no_cpu_baseline:
        threads = min(os.cpu_count() or 1, 16)
        frac = args.cpu_frac if args.cpu_frac is not None else (
            0.12 if args.workload.endswith("batch256") else 0.25)
        out["cpu_baseline"] = cpu_baseline(g, gfds, args.semantics, frac, threads)
    gh.free()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
