"""Writes tests/golden/expected_<workload>.json: the CPU oracle's results for
the full-size workloads (both matching readings, K = 1024), with the graph's
sha256 and the exact GFD list they were computed for.  Calls only the seeded
generators and oracle/.

    python tests/golden/make_expected.py powerlaw_1m kg_4m

kg_4m_serving stores a 1% sample of the serving pool (every 100th GFD) with
its positions' stride, for the serving test's oracle check.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from synth import configs  # noqa: E402


SERVING_SAMPLE_STRIDE = 100  # every 100th GFD of the serving pool: a 1% sample


def _gfds_of(name, g):
    if name == "kg_4m_serving":
        pool = configs.serving_pool(g)
        return [{k: v for k, v in pool[i].items() if k != "meta"}
                for i in range(0, len(pool), SERVING_SAMPLE_STRIDE)]
    return [{k: v for k, v in d.items() if k != "meta"} for d in configs.gfds(name, g)]


def main(names, K=1024, threads=os.cpu_count() or 1):
    for name in names:
        g = configs.graph(configs.CONFIG_GRAPH[name])
        gfds = _gfds_of(name, g)
        og = O.OracleGraph(g)
        out = {"workload": name, "graph_sha256": g.sha256(), "K": K, "gfds": gfds,
               "results": {}, "oracle_threads": threads}
        if name == "kg_4m_serving":
            out["pool_stride"] = SERVING_SAMPLE_STRIDE
        for sem in ("induced", "mono"):
            t = time.time()
            out["results"][sem] = [O.validate(og, d, sem, K=K, threads=threads) for d in gfds]
            print(name, sem, f"{time.time() - t:.1f}s", flush=True)
        text = json.dumps(out, separators=(",", ":"))
        if len(text) > 1 << 20:  # large result sets are stored compressed
            import gzip
            with gzip.open(os.path.join(HERE, f"expected_{name}.json.gz"), "wt") as f:
                f.write(text)
        else:
            with open(os.path.join(HERE, f"expected_{name}.json"), "w") as f:
                f.write(text)


if __name__ == "__main__":
    main(sys.argv[1:] or ["powerlaw_1m", "kg_4m"])
