"""Launch-shape autotuner.

For a GFD set on a loaded graph it times the validate call under candidate
gfd_tuning choices -- coordinate descent over the block count of the
enumeration launches and of their scans, the last level's probe-ahead form
and the violation staging per GFD -- checks that every choice gives exactly
the results of the defaults, and keeps the fastest.  The choice is cached in
a JSON file keyed by the graph's sha256, the sha256 of the HIP sources and
of the loaded library file, and the call's shape class (batched or not, number of GFDs, largest pattern,
reading, K, counts only).  Only how the work is spread over the GPU changes,
never a result (the tests check every candidate against the oracle).
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
import time

from . import _binding as B

PKG = os.path.dirname(os.path.abspath(__file__))
CANDIDATES = {
    "flat_grid": [0, 1024, 4096, 8192],
    "scan_grid": [0, 512, 4096],
    "probe_ahead": [0, 1, 2],
    "staging_log2": [0, 16, 20],
    "ext_occupancy": [0, 1, 2],
}
DEFAULTS = {k: 0 for k in CANDIDATES}


def sources_sha256() -> str:
    """sha256 of the library's HIP sources and internal header."""
    h = hashlib.sha256()
    csrc = os.path.join(PKG, "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def library_sha256() -> str:
    """sha256 of the loaded library file (another build of the same sources,
    e.g. one chosen with GFD_LIBRARY, keeps its own choices)."""
    h = hashlib.sha256()
    with open(B.LIB_PATH, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def shape_class(gfds, K, semantics, batched, count_only) -> str:
    n = len(gfds)
    nb = 1 if n == 1 else (16 if n <= 16 else 256)
    kmax = max(int(d["k"]) for d in gfds) if gfds else 0
    return f"n{nb}:k{kmax}:{semantics}:K{K}:{'batched' if batched else 'plain'}:{'count' if count_only else 'full'}"


def cache_path() -> str:
    return os.environ.get("GFD_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                           "gfd_tuning.json")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def measure(gh, gfds, tuning, K, semantics, batched, flags, stream, reps):
    """Median wall ms of `reps` calls after warm-up (the first run of a shape
    runs eagerly, the second captures its graph), and the results."""
    pc = B.PreparedCall(gh, gfds, K=K, semantics=semantics, stream=stream, batched=batched,
                        tuning=tuning)
    for _ in range(2):
        pc.run(flags=flags, stats=False)
    ms = []
    for _ in range(reps):
        t = time.perf_counter()
        pc.run(flags=flags, stats=False)
        ms.append((time.perf_counter() - t) * 1e3)
    return statistics.median(ms), pc.results()


def tune(gh, gfds, graph_sha256, K=1024, semantics="induced", batched=True, count_only=False,
         stream=None, reps=3, path=None, retune=False, log=None):
    """The tuned gfd_tuning dict for this call shape (from the cache when it
    holds one for this graph and these sources), with the default and tuned
    times and every candidate tried."""
    path = path or cache_path()
    key = (f"{graph_sha256}:{sources_sha256()}:{library_sha256()[:16]}:"
           f"{shape_class(gfds, K, semantics, batched, count_only)}")
    cache = _load(path)
    if not retune and key in cache:
        return dict(cache[key], cached=True)
    flags = B.GFD_FLAG_COUNT_ONLY if count_only else 0
    base_ms, ref = measure(gh, gfds, DEFAULTS, K, semantics, batched, flags, stream, reps)
    best, best_ms = dict(DEFAULTS), base_ms
    tried = [{"tuning": dict(DEFAULTS), "ms": base_ms}]
    for knob, values in CANDIDATES.items():
        for v in values:
            if v == best[knob]:
                continue
            cand = dict(best, **{knob: v})
            ms, res = measure(gh, gfds, cand, K, semantics, batched, flags, stream, reps)
            if res != ref:
                raise AssertionError(f"tuning {cand} changed a result")
            tried.append({"tuning": cand, "ms": ms})
            if log:
                log(f"tune: {cand} {ms:.3f} ms (best {best_ms:.3f})")
            if ms < best_ms * 0.98:  # keep a change only when it clearly pays
                best, best_ms = cand, ms
    if best != DEFAULTS:
        # confirm against the defaults, measured in turn (the first shapes
        # measured run on a colder device, which favours later candidates)
        a, b = [], []
        for _ in range(2):
            a.append(measure(gh, gfds, DEFAULTS, K, semantics, batched, flags, stream, reps)[0])
            b.append(measure(gh, gfds, best, K, semantics, batched, flags, stream, reps)[0])
        base_ms, best_ms = statistics.median(a), statistics.median(b)
        tried.append({"confirm": {"default_ms": a, "tuned_ms": b}})
        if not best_ms < base_ms * 0.98:
            best, best_ms = dict(DEFAULTS), base_ms
    out = {"tuning": best, "tuned_ms": best_ms, "default_ms": base_ms, "tried": tried}
    cache[key] = out
    _save(path, cache)
    return dict(out, cached=False)
