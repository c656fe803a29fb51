"""The five named workloads, as seeded synthetic inputs.

    small_uniform      2,000 vertices / 8,000 uniform edges, one 3-vertex GFD
    powerlaw_1m        Chung-Lu 1M / 5M (gamma 2.1), 8 shape GFDs of 3-6 vertices
    kg_4m              Chung-Lu 4M / 20M (gamma 2.1), 16 walk GFDs of 4-8 vertices
    kg_4m_batch256     the kg_4m graph, 256 walk GFDs of 2-8 vertices
    kg_4m_serving      the kg_4m graph, Poisson request stream (1-4 GFDs each)
    twitch_trio        undirected Chung-Lu 20,000 vertices / 92,798 edges (each as two
                       antiparallel edges), two language labels, boolean 'abandoned'
                       and 'affiliate'; the paper's path, star and triangle GFDs

The paper measures on a public social graph (Twitch Gamers) that is not
available here; these synthetic inputs stand in for it.  Every array comes from
numpy PCG64 sub-streams of the stated seed.  Generated inputs are cached as
.npz/.json under $GFD_SYNTH_CACHE (default /tmp/gfd_synth_cache), keyed by the
generator version, and always re-verified against their sha256.
"""
from __future__ import annotations

import json
import os
import hashlib

import numpy as np

from .graphs import Graph, make_graph
from . import patterns as P

GEN_VERSION = 1

GRAPHS = {
    "small_uniform": dict(seed=0, n=2_000, m=8_000, model="uniform", n_vlabels=5, n_elabels=3,
                          label_zipf=None, n_attrs=1, attr_values=50, attr_zipf=None),
    "powerlaw_1m": dict(seed=1, n=1_000_000, m=5_000_000, model="chung_lu", n_vlabels=30,
                        n_elabels=10, label_zipf=1.1, n_attrs=3, attr_values=10_000,
                        attr_zipf=1.1),
    "kg_4m": dict(seed=2, n=4_000_000, m=20_000_000, model="chung_lu", n_vlabels=100,
                  n_elabels=40, label_zipf=1.2, n_attrs=4, attr_values=100_000, attr_zipf=1.2),
    # vertex labels: 0 = EN, 1 = RU; attributes: 0 = abandoned, 1 = affiliate (0 = F, 1 = T)
    "twitch_20k": dict(seed=5, n=20_000, m=2 * 92_798, model="chung_lu_sym", n_vlabels=2,
                       n_elabels=1, label_zipf=None, n_attrs=2, attr_values=2, attr_zipf=None),
}

CONFIG_GRAPH = {"small_uniform": "small_uniform", "powerlaw_1m": "powerlaw_1m",
                "kg_4m": "kg_4m", "kg_4m_batch256": "kg_4m", "kg_4m_serving": "kg_4m",
                "twitch_trio": "twitch_20k"}
CONFIG_ORDER = ["small_uniform", "powerlaw_1m", "kg_4m", "kg_4m_batch256", "kg_4m_serving",
                "twitch_trio"]


def cache_dir() -> str:
    d = os.environ.get("GFD_SYNTH_CACHE", "/tmp/gfd_synth_cache")
    os.makedirs(d, exist_ok=True)
    return d


def _save_graph(path, g: Graph):
    np.savez(path, n=g.n, m=g.m, row_ptr=g.row_ptr, col=g.col, vlabel=g.vlabel,
             elabel=g.elabel, attrs=g.attrs, meta=json.dumps(g.meta))


def _load_graph(path) -> Graph:
    z = np.load(path, allow_pickle=False)
    return Graph(n=int(z["n"]), m=int(z["m"]), row_ptr=z["row_ptr"], col=z["col"],
                 vlabel=z["vlabel"], elabel=z["elabel"], attrs=z["attrs"],
                 meta=json.loads(str(z["meta"])))


def graph(name: str, use_cache: bool = True) -> Graph:
    """The named graph (regenerated, or read from the cache and re-hashed)."""
    spec = dict(GRAPHS[name])
    seed = spec.pop("seed")
    n, m = spec.pop("n"), spec.pop("m")
    key = hashlib.sha256(json.dumps([GEN_VERSION, name, seed, n, m, spec], sort_keys=True)
                         .encode()).hexdigest()[:16]
    path = os.path.join(cache_dir(), f"{name}_{key}.npz")
    if use_cache and os.path.exists(path):
        g = _load_graph(path)
        if g.sha256() == g.meta.get("sha256"):
            return g
    g, _ = make_graph(seed, n, m, **spec)
    g.meta["sha256"] = g.sha256()
    if use_cache:
        tmp = path + ".tmp.npz"
        _save_graph(tmp, g)
        os.replace(tmp, path)
    return g


def gfd_stream(name: str):
    spec = GRAPHS[CONFIG_GRAPH[name]]
    seed = {"small_uniform": 0, "powerlaw_1m": 1, "kg_4m": 2, "kg_4m_batch256": 3,
            "kg_4m_serving": 4, "twitch_trio": 5}[name]
    ss = np.random.SeedSequence(seed).spawn(5)
    return np.random.Generator(np.random.PCG64(ss[4])), spec


def _gfds_uncached(name: str, g: Graph):
    rng, spec = gfd_stream(name)
    av, az = spec["attr_values"], spec["attr_zipf"]
    if name == "small_uniform":
        # x -[e0]-> y, x -[e0]-> z with labels (L0, L1, L1); {} -> y.name = z.name
        return [{"k": 3, "vlabels": [0, 1, 1], "edges": [[0, 1, 0], [0, 2, 0]], "x": [],
                 "y": [{"kind": "var", "var": 1, "attr": 0, "var2": 2, "attr2": 0}],
                 "y_false": False, "meta": {"fixed": True}}]
    if name == "twitch_trio":
        return twitch_trio()
    view = P.GraphView(g)
    out = []
    if name == "powerlaw_1m":
        for shape, krange in (("path", (3, 6)), ("star", (3, 6)), ("triangle", (3, 6)),
                              ("cycle4", (4, 6))):
            for _ in range(2):
                k = int(rng.integers(krange[0], krange[1] + 1))
                out.append(P.sample_shape_gfd(rng, view, shape, k, (1, 2), av, az,
                                              label_zipf=spec["label_zipf"],
                                              n_vlabels=spec["n_vlabels"],
                                              n_elabels=spec["n_elabels"]))
        return out
    if name == "kg_4m":
        for _ in range(16):
            out.append(P.sample_walk_gfd(rng, view, (4, 8), (1, 3), av, az, core_range=(3, 5)))
        return out
    if name == "kg_4m_batch256":
        for _ in range(256):
            out.append(P.sample_walk_gfd(rng, view, (2, 8), (1, 3), av, az, cyc_range=(0, 3)))
        return out
    raise ValueError(name)


def _undirected(pairs, label=0):
    """Pattern edges of undirected pairs: one antiparallel pair each."""
    return [e for a, b in pairs for e in ([a, b, label], [b, a, label])]


def twitch_trio():
    """The three queries of the paper's evaluation (Section V): on a followship
    graph with language labels EN (0) / RU (1) and boolean attributes abandoned
    (0) and affiliate (1), T = 1, F = 0.  Each also appears as X -> false."""
    T, F = 1, 0
    ab = lambda v, c: {"kind": "const", "var": v, "attr": 0, "value": c}  # noqa: E731
    af = lambda v, c: {"kind": "const", "var": v, "attr": 1, "value": c}  # noqa: E731
    path = {"k": 3, "vlabels": [0, 0, 0], "edges": _undirected([(0, 1), (1, 2)]),
            "x": [ab(0, T), ab(1, T), ab(2, T)], "y": [af(1, T)], "y_false": False}
    star = {"k": 4, "vlabels": [1, 1, 1, 1], "edges": _undirected([(0, 1), (0, 2), (0, 3)]),
            "x": [], "y": [ab(0, F)], "y_false": False}
    tri = {"k": 3, "vlabels": [0, 0, 0], "edges": _undirected([(0, 1), (1, 2), (0, 2)]),
           "x": [ab(0, T), ab(1, T)], "y": [ab(2, T)], "y_false": False}
    out = [path, star, tri]
    out += [dict(d, y=[], y_false=True) for d in (path, star, tri)]
    return out


FROZEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def frozen_path(name: str) -> str:
    return os.path.join(FROZEN_DIR, f"gfds_{name}.json")


def freeze(name: str) -> str:
    """Store the sampled GFD list next to this module (sampling the larger
    workloads takes minutes); gfds() reads it back when the graph matches."""
    g = graph(CONFIG_GRAPH[name])
    gl = gfds(name, g, use_frozen=False)
    os.makedirs(FROZEN_DIR, exist_ok=True)
    with open(frozen_path(name), "w") as f:
        json.dump({"workload": name, "gen_version": GEN_VERSION, "graph_sha256": g.sha256(),
                   "gfds": gl}, f)
    return frozen_path(name)


def gfds(name: str, g: Graph | None = None, use_cache: bool = True, use_frozen: bool = True):
    """The named config's GFD list (JSON dicts), generated from its seed."""
    if g is None:
        g = graph(CONFIG_GRAPH[name], use_cache=use_cache)
    if use_frozen and os.path.exists(frozen_path(name)):
        with open(frozen_path(name)) as f:
            d = json.load(f)
        if d.get("gen_version") == GEN_VERSION and d.get("graph_sha256") == g.sha256():
            return d["gfds"]
    path = os.path.join(cache_dir(), f"gfds_{name}_v{GEN_VERSION}_{g.sha256()[:16]}.json")
    if use_cache and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    out = _gfds_uncached(name, g)
    if use_cache:
        with open(path + ".tmp", "w") as f:
            json.dump(out, f)
        os.replace(path + ".tmp", path)
    return out


def gfds_sha256(gl) -> str:
    strip = [{k: v for k, v in d.items() if k != "meta"} for d in gl]
    return hashlib.sha256(json.dumps(strip, sort_keys=True).encode()).hexdigest()


SERVING_POOL = 4000  # walk-sampled GFDs the serving requests draw from, in order
SERVING_PARTS = 8    # independently seeded parts, sampled in parallel


def _serving_part(part: int, n: int):
    g = graph(CONFIG_GRAPH["kg_4m_serving"])
    spec = GRAPHS[CONFIG_GRAPH["kg_4m_serving"]]
    ss = np.random.SeedSequence(4).spawn(5)[4].spawn(SERVING_PARTS)[part]
    rng = np.random.Generator(np.random.PCG64(ss))
    view = P.GraphView(g)
    return [P.sample_walk_gfd(rng, view, (3, 8), (1, 3), spec["attr_values"], spec["attr_zipf"],
                              cyc_range=(0, 3)) for _ in range(n)]


def serving_pool_path() -> str:
    return os.path.join(FROZEN_DIR, "gfds_kg_4m_serving_pool.json.gz")


def serving_pool(g: Graph | None = None, procs: int = SERVING_PARTS):
    """SERVING_POOL walk-sampled GFDs (3-8 vertices, 1-3 literals, cyclomatic
    number 0-3) on the serving graph: SERVING_PARTS parts of equal size, each
    from its own seed.  Read from its frozen file when it matches the graph
    (sampling takes minutes)."""
    import gzip
    if g is None:
        g = graph(CONFIG_GRAPH["kg_4m_serving"])
    path = serving_pool_path()
    if os.path.exists(path):
        with gzip.open(path, "rt") as f:
            d = json.load(f)
        if d.get("gen_version") == GEN_VERSION and d.get("graph_sha256") == g.sha256():
            return d["gfds"]
    from concurrent.futures import ProcessPoolExecutor
    per = SERVING_POOL // SERVING_PARTS
    with ProcessPoolExecutor(max_workers=procs) as ex:
        parts = list(ex.map(_serving_part, range(SERVING_PARTS), [per] * SERVING_PARTS))
    out = [d for part in parts for d in part]
    os.makedirs(FROZEN_DIR, exist_ok=True)
    with gzip.open(path + ".tmp", "wt") as f:
        json.dump({"workload": "kg_4m_serving", "gen_version": GEN_VERSION,
                   "graph_sha256": g.sha256(), "gfds": out}, f)
    os.replace(path + ".tmp", path)
    return out


def serving_requests(g: Graph, rate: float = 200.0, duration_s: float = 60.0, seed: int = 4,
                     pool=None, start: int = 0):
    """Poisson arrivals of `rate` requests per second over `duration_s`; each
    request holds 1-4 GFDs, taken in order from the walk-sampled serving pool
    (from position `start`, wrapping around), so requests rarely repeat a GFD."""
    rng = np.random.default_rng(seed)
    pool = serving_pool(g) if pool is None else pool
    t, reqs, at = 0.0, [], start
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration_s:
            break
        nq = int(rng.integers(1, 5))
        reqs.append({"t": t, "gfds": [pool[(at + j) % len(pool)] for j in range(nq)]})
        at += nq
    return reqs


if __name__ == "__main__":
    import sys
    if len(sys.argv) >= 3 and sys.argv[1] == "freeze":
        for nm in sys.argv[2:]:
            print(freeze(nm))
    if len(sys.argv) >= 2 and sys.argv[1] == "serving-pool":
        print(len(serving_pool()), serving_pool_path())
