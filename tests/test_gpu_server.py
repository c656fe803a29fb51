"""The serving form through the C ABI (gfd_server_*): requests queued while
others run are batched together, and every request's results equal the
oracle's and those of validating it alone -- exactly (the path is integer
work, so the tolerance is zero)."""
import gzip
import json
import os
import threading

import numpy as np
import pytest

from oracle import oracle as O
from synth import configs
from synth.small import random_gfd, random_graph

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_02321_amd as P
    return P


def _requests(rng, pool, n, lo=1, hi=4):
    return [[int(i) for i in rng.integers(0, len(pool), size=int(rng.integers(lo, hi + 1)))]
            for _ in range(n)]


@pytest.mark.parametrize("sem", ["induced", "mono"])
def test_served_equals_alone_and_oracle(P, sem):
    g = random_graph(21, 1200, 12000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4,
                     absent_frac=0.1)
    rng = np.random.default_rng(21)
    pool = [random_gfd(2100 + j, int(rng.integers(1, 7)), n_vlabels=2, n_elabels=2, n_attrs=2,
                       attr_values=4, wildcard_frac=0.15, extra_edge_frac=0.3)
            for j in range(20)]
    og = O.OracleGraph(g)
    exp = [O.validate(og, d, sem, K=40, threads=4) for d in pool]
    gh = P.load(g)
    alone = [P.validate(gh, [d], K=40, semantics=sem)[0] for d in pool]
    assert alone == exp
    srv = P.Server(gh, K=40, semantics=sem, workers=2, max_batch_gfds=16)
    reqs = _requests(rng, pool, 60)
    ids = [srv.submit([pool[i] for i in r]) for r in reqs]
    mixed = 0
    for rid, r in zip(ids, reqs):
        got, info = srv.wait(rid)
        assert got == [exp[i] for i in r], (rid, r)
        assert info["batch_gfds"] <= 16 and info["start_ns"] >= info["submit_ns"]
        mixed += info["batch_requests"] > 1
    assert mixed > 0, "no batch held more than one request"
    srv.close()
    gh.free()


def test_concurrent_submitters_and_wait_timeouts(P):
    g = random_graph(22, 800, 8000, n_vlabels=2, n_elabels=1, n_attrs=1, attr_values=3)
    pool = [random_gfd(2200 + j, 3 + j % 3, n_vlabels=2, n_elabels=1, n_attrs=1, attr_values=3)
            for j in range(8)]
    og = O.OracleGraph(g)
    exp = [O.validate(og, d, "induced", K=16, threads=4) for d in pool]
    gh = P.load(g)
    srv = P.Server(gh, K=16, workers=3, max_batch_gfds=8)
    errors = []

    def client(seed):
        rng = np.random.default_rng(seed)
        try:
            for r in _requests(rng, pool, 15, 1, 3):
                rid = srv.submit([pool[i] for i in r])
                out = None
                while out is None:  # polling with a timeout returns None until done
                    out = srv.wait(rid, timeout_ms=5)
                assert out[0] == [exp[i] for i in r]
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    th = [threading.Thread(target=client, args=(s,)) for s in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    with pytest.raises(P.GfdError) as ei:
        srv.wait(12345678)
    assert ei.value.code == -1
    bad = {"k": 2, "vlabels": [0, 0], "edges": [[0, 0, 0]], "x": [], "y": []}
    with pytest.raises(P.GfdError):
        srv.submit([bad])
    srv.close()
    gh.free()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_serving_full_size_against_stored_oracle(P):
    """Requests drawn from the 256-GFD pool on the 4M-vertex graph, served with
    continuous batching; every result equals the stored oracle result, under
    the default per-worker budget and under one small enough that admission
    by estimated device bytes splits the queue into smaller batches."""
    with gzip.open(os.path.join(GOLDEN, "expected_kg_4m_batch256.json.gz"), "rt") as f:
        exp = json.load(f)
    g = configs.graph("kg_4m")
    assert g.sha256() == exp["graph_sha256"]
    pool = exp["gfds"]
    ref = exp["results"]["induced"]
    rng = np.random.default_rng(4)
    gh = P.load(g)
    reqs = _requests(rng, pool, 120)
    batches = {}
    # the default per-worker budget, then one so small that the estimated
    # device bytes of a few requests fill it: the queue is then split into
    # many smaller batches, with the same results
    for budget in (0, 1 << 30):
        srv = P.Server(gh, K=exp["K"], workers=1, mem_budget_bytes=budget)
        ids = [srv.submit([pool[i] for i in r]) for r in reqs]
        sizes = {}
        for rid, r in zip(ids, reqs):
            got, info = srv.wait(rid)
            assert got == [ref[i] for i in r], (budget, r)
            sizes[info["batch_id"]] = info["batch_gfds"]
        srv.close()
        batches[budget] = sizes
    big, small = batches[0], batches[1 << 30]
    assert len(small) > len(big), (len(small), len(big))
    assert max(small.values()) < max(big.values()), (max(small.values()), max(big.values()))
    gh.free()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_serving_sampled_requests_against_oracle(P):
    """Requests as the serving bench makes them (1-4 GFDs each, taken in order
    from the pool of 4,000 walk-sampled GFDs): every served result equals the
    same GFD validated alone, and the GFDs at every 100th pool position (a 1%
    sample) equal the stored oracle results, in both readings."""
    with open(os.path.join(GOLDEN, "expected_kg_4m_serving.json")) as f:
        exp = json.load(f)
    g = configs.graph("kg_4m")
    assert g.sha256() == exp["graph_sha256"]
    pool = [{k: v for k, v in d.items() if k != "meta"} for d in configs.serving_pool(g)]
    stride = exp["pool_stride"]
    assert [pool[i] for i in range(0, len(pool), stride)] == exp["gfds"]
    reqs = configs.serving_requests(g, rate=200.0, duration_s=4.0, seed=4, pool=pool)
    idx, at = [], 0
    for r in reqs:
        idx.append([(at + j) % len(pool) for j in range(len(r["gfds"]))])
        at += len(r["gfds"])
    gh = P.load(g)
    for sem in ("induced", "mono"):
        ref = exp["results"][sem]
        srv = P.Server(gh, K=exp["K"], semantics=sem, workers=2)
        ids = [srv.submit(r["gfds"]) for r in reqs]
        served = {}
        for rid, ix in zip(ids, idx):
            got, _ = srv.wait(rid)
            served.update(zip(ix, got))
        srv.close()
        sampled = [i for i in served if i % stride == 0]
        assert len(sampled) >= 15, len(sampled)
        for i in sampled:
            assert served[i] == ref[i // stride], (sem, i)
        if sem == "induced":
            for i, r in served.items():
                assert r == P.validate(gh, [pool[i]], K=exp["K"], semantics=sem)[0], i
    gh.free()
