"""bench.py's command-line contract on the host: more than one GPU is refused
with a message, and the kernel-sources hash that keys the stored HBM traffic
figures is printed on request."""
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, cwd=ROOT, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_sources_hash():
    r = _bench("--sources-sha256")
    assert r.returncode == 0
    assert re.fullmatch(r"[0-9a-f]{64}", r.stdout.strip())


def test_cpu_baseline_fields():
    """The oracle leg of the bench line on the 2,000-vertex configuration:
    the contract's fields, a multi-threaded figure and a one-thread one."""
    sys.path.insert(0, ROOT)
    import bench
    from synth import configs
    g = configs.graph(configs.CONFIG_GRAPH["small_uniform"])
    gfds = [{k: v for k, v in d.items() if k != "meta"} for d in configs.gfds("small_uniform", g)]
    out = bench.cpu_baseline(g, gfds, "induced", 0.5, 2)
    for leg, cores in ((out, 2), (out["single_thread"], 1)):
        assert leg["kind"] == "oracle" and leg["unit"] == "embeddings/s"
        assert leg["cores"] == cores and leg["value"] >= 0 and leg["sample"]


def test_stored_tables_agree():
    """The stored model bytes are the per-unit model over the stored units,
    and the units are consistent with one another."""
    sys.path.insert(0, ROOT)
    import bench
    u = bench.UNITS["per_step"]
    model = (4 * u["attempts"] + 8 * u["sources"] + 8 * u["both_log2d"] + 4 * u["one_log2d"]
             + 4 * u["literal_reads"])
    assert abs(model - bench.UNITS["model_bytes_per_step"]) <= 1e-5 * model
    # checks of both directions end in a table slot, a fingerprint match or a short row
    assert u["table_free"] + u["table_hit"] + u["short_row"] == u["checks_both"]
    assert u["matches"] <= u["injective"] <= u["attempts"]
