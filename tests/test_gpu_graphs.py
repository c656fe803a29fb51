"""Captured main passes (HIP graphs): the first batch of a shape is captured,
later ones replay it.  Every replay -- with other calls, eager and captured,
and host synchronisations between the replays -- gives exactly the eager
result (GFD_FLAG_NO_GRAPH), which itself equals the CPU oracle, including
on the paths that follow the main pass (threshold re-runs, radix select,
bounded re-runs)."""
import numpy as np
import pytest

from oracle import oracle as O
from synth.small import random_graph, random_gfd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_02321_amd as P
    return P


def _gfds(seed, count, n_vlabels=2, kmax=7):
    rng = np.random.default_rng(seed)
    return [random_gfd(seed * 100 + j, int(rng.integers(1, kmax)), n_vlabels=n_vlabels, n_elabels=2,
                       n_attrs=2, attr_values=4, wildcard_frac=0.15, extra_edge_frac=0.3)
            for j in range(count)]


def test_replays_equal_eager_and_oracle(P):
    import torch
    g = random_graph(41, 2000, 24000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=4,
                     absent_frac=0.1)
    og = O.OracleGraph(g)
    gh = P.load(g)
    batch, other = _gfds(41, 24), _gfds(42, 6)
    # patterns of two components (a cross-product level) in the captured pass
    batch += [{"k": 3, "vlabels": [0, 1, 1], "edges": [[1, 2, 0]], "x": [],
               "y": [{"kind": "var", "var": 0, "attr": 0, "var2": 2, "attr2": 0}], "y_false": False},
              {"k": 2, "vlabels": [0, 1], "edges": [],
               "x": [{"kind": "const", "var": 0, "attr": 1, "value": 2}], "y": [], "y_false": True}]
    cases = [dict(K=64, semantics="induced", batched=True),
             dict(K=64, semantics="mono", batched=True),
             dict(K=16, semantics="induced", batched=True, violation_cap=40),   # threshold re-runs
             dict(K=16, semantics="mono", batched=False),                       # one GFD per batch
             dict(K=8, semantics="induced", batched=True, frontier_cap=300)]    # bounded re-runs
    for kw in cases:
        eager = P.validate(gh, batch, flags=P.GFD_FLAG_NO_GRAPH, **kw)
        exp = [O.validate(og, d, kw["semantics"], K=kw["K"], threads=4) for d in batch]
        assert eager == exp, kw
        for rep in range(5):
            got, st = P.validate(gh, batch, stats=True, **kw)
            assert got == eager, (kw, rep)
            # a shape runs eagerly the first time, is captured the second
            # time and replayed from then on
            if rep == 0:
                assert st["graph_captures"] == 0 and st["graph_replays"] == 0, (kw, st)
            elif rep == 1:
                assert st["graph_captures"] >= 1, (kw, st)
            else:
                assert st["graph_captures"] == 0 and st["graph_replays"] >= 1, (kw, rep, st)
            # other work between the replays: eager and captured calls of
            # other shapes, and a host synchronisation
            P.validate(gh, other, K=8, semantics="mono", batched=True, flags=P.GFD_FLAG_NO_GRAPH)
            P.validate(gh, other[:3], K=8, semantics="induced", batched=True)
            torch.cuda.synchronize()
    gh.free()


def test_select_path_under_replay(P):
    """More than 2,048 staged violations (radix select of the first K) on a
    replayed main pass."""
    g = random_graph(8, 400, 12000, n_vlabels=1, n_elabels=1, n_attrs=1, attr_values=50,
                     absent_frac=0.0)
    gfd = {"k": 3, "vlabels": [0, 0, 0], "edges": [[0, 1, 0], [0, 2, 0]], "x": [],
           "y": [{"kind": "var", "var": 1, "attr": 0, "var2": 2, "attr2": 0}], "y_false": False}
    gh = P.load(g)
    exp = O.validate(O.OracleGraph(g), gfd, "mono", K=1024, threads=4)
    assert exp["violation_count"] > 2048
    for _ in range(4):
        assert P.validate(gh, [gfd], K=1024, semantics="mono") == [exp]
    gh.free()
