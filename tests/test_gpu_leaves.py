"""Leaf postponement in count-only calls (GFD_FLAG_COUNT_ONLY): the last leaves
of the matching order are counted, not enumerated.  Counts and satisfied flags
must equal the oracle's exactly; fingerprints are 0 and no tuples are listed.
Statistics show which GFDs took the counting path."""
import json
import os

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


def c(var, attr, value):
    return {"kind": "const", "var": var, "attr": attr, "value": value}


def v(var, attr, var2, attr2):
    return {"kind": "var", "var": var, "attr": attr, "var2": var2, "attr2": attr2}


def und(pairs, label=0):
    return [e for a, b in pairs for e in ([a, b, label], [b, a, label])]


# (gfd, whether its last leaves qualify for counting under the non-induced reading)
CASES = [
    # star, 3 identical leaves, literals on the centre and on single leaves
    ({"k": 4, "vlabels": [0, 1, 1, 1], "edges": [[0, 1, 0], [0, 2, 0], [0, 3, 0]],
      "x": [c(0, 0, 1), c(1, 0, 2)], "y": [c(2, 1, 0), v(3, 0, 3, 1)], "y_false": False}, True),
    # star with 2 leaves, X -> false
    ({"k": 3, "vlabels": [1, 0, 0], "edges": [[1, 0, 1], [2, 0, 1]],
      "x": [c(1, 1, 1)], "y": [], "y_false": True}, True),
    # path: one end is the last leaf; the variable literal pairs the inner vertices
    ({"k": 4, "vlabels": [0, 1, 0, 1], "edges": [[0, 1, 0], [1, 2, 1], [2, 3, 0]],
      "x": [v(1, 0, 2, 0)], "y": [c(3, 1, 2)], "y_false": False}, True),
    # undirected star (antiparallel pattern edges), wildcard leaves
    ({"k": 4, "vlabels": [1, -1, -1, -1], "edges": und([(0, 1), (0, 2), (0, 3)]),
      "x": [], "y": [c(0, 0, 0), c(1, 1, 3)], "y_false": False}, True),
    # triangle with a pendant leaf
    ({"k": 4, "vlabels": [0, 0, 1, 1], "edges": [[0, 1, 0], [1, 2, 0], [2, 0, 1], [2, 3, 2]],
      "x": [c(3, 0, 1)], "y": [c(0, 1, 1)], "y_false": False}, True),
    # a literal tying a leaf to the centre: enumerated
    ({"k": 3, "vlabels": [0, 1, 1], "edges": [[0, 1, 0], [0, 2, 0]],
      "x": [], "y": [v(1, 0, 0, 0)], "y_false": False}, False),
    # leaves of different labels: only the identical tail is postponed
    ({"k": 4, "vlabels": [0, 1, 2, 2], "edges": [[0, 1, 0], [0, 2, 0], [0, 3, 0]],
      "x": [], "y": [c(1, 0, 1)], "y_false": False}, True),
]


# Triangles (matched first, as the core) with one leaf on each of two corners:
# the last two leaves of the order hang from different parents and are counted
# together as the product of their lists' counts less the shared vertices.
TRI = [[0, 1, 0], [1, 2, 0], [2, 0, 1]]
SPLIT_CASES = [
    # same label and edge form on both leaves: shared list vertices are common;
    # literals on each leaf and on an inner vertex
    {"k": 5, "vlabels": [0, 0, 1, 1, 1], "edges": TRI + [[0, 3, 2], [1, 4, 2]],
     "x": [c(3, 0, 1)], "y": [c(4, 1, 2), c(2, 0, 0)], "y_false": False},
    # wildcard leaves on undirected edges: matched inner vertices sit in the
    # lists; a variable literal on one leaf alone
    {"k": 5, "vlabels": [0, 1, 0, -1, -1], "edges": TRI + und([(0, 3), (1, 4)]),
     "x": [c(4, 0, 2)], "y": [v(3, 0, 3, 1)], "y_false": False},
    # leaf edges in opposite directions, X -> false
    {"k": 5, "vlabels": [0, 0, 1, 1, 1], "edges": TRI + [[3, 0, 1], [1, 4, 1]],
     "x": [c(3, 1, 0), c(4, 1, 0)], "y": [], "y_false": True},
    # leaves of different labels: the lists share nothing
    {"k": 5, "vlabels": [0, 0, 1, 1, 0], "edges": TRI + [[0, 3, 0], [1, 4, 0]],
     "x": [], "y": [c(3, 0, 1), c(4, 0, 2)], "y_false": False},
    # a literal tying one leaf to an inner vertex: only the other is counted
    {"k": 5, "vlabels": [0, 0, 1, 1, 1], "edges": TRI + [[0, 3, 2], [1, 4, 2]],
     "x": [v(3, 0, 2, 1)], "y": [c(4, 1, 2)], "y_false": False},
]
SPLIT_COUNTED = 4  # the first four have both leaves counted together


def _oracle_counts(og, d, sem):
    r = O.validate(og, d, sem, K=0, threads=4)
    return {"match_count": r["match_count"], "violation_count": r["violation_count"],
            "satisfied": r["satisfied"], "match_fp": 0, "violation_fp": 0, "violations": []}


@pytest.mark.parametrize("batched", [False, True])
def test_counted_leaves_match_oracle(P, batched):
    g = random_graph(31, 500, 9000, n_vlabels=3, n_elabels=3, n_attrs=2, attr_values=4,
                     absent_frac=0.1, reciprocal_frac=0.3)
    og = O.OracleGraph(g)
    gh = P.load(g)
    gfds = [d for d, _ in CASES]
    for sem in ("mono", "induced"):
        got, st = P.validate(gh, gfds, K=0, semantics=sem, flags=P.GFD_FLAG_COUNT_ONLY,
                             stats=True, batched=batched)
        for i, (d, r) in enumerate(zip(gfds, got)):
            assert r == _oracle_counts(og, d, sem), (sem, i)
        want = sum(q for _, q in CASES) if sem == "mono" else 0
        assert st["leaf_gfds"] == want, (sem, st["leaf_gfds"])
    # the same GFDs enumerated (no flag) give the same counts
    full = P.validate(gh, gfds, K=0, semantics="mono", batched=batched)
    cnt = P.validate(gh, gfds, K=0, semantics="mono", flags=P.GFD_FLAG_COUNT_ONLY,
                     batched=batched)
    for a, b in zip(full, cnt):
        assert (a["match_count"], a["violation_count"]) == (b["match_count"], b["violation_count"])
    gh.free()


@pytest.mark.parametrize("batched", [False, True])
def test_split_leaves_match_oracle(P, batched):
    """Two last leaves under different parents: counts equal the oracle's and
    those of the same GFDs enumerated; the statistics show which GFDs took the
    split form."""
    g = random_graph(33, 250, 12000, n_vlabels=2, n_elabels=3, n_attrs=2, attr_values=3,
                     absent_frac=0.1, reciprocal_frac=0.4)
    og = O.OracleGraph(g)
    # not vacuous: the two leaves merged into one vertex on both corners has
    # matches, so the lists of the first two GFDs share vertices and the count
    # of pairs must take out the pairs of one vertex to agree with the oracle
    for d in SPLIT_CASES[:2]:
        assert d["vlabels"][3] == d["vlabels"][4]
        merged = {"k": 4, "vlabels": d["vlabels"][:4], "x": [], "y": [], "y_false": False,
                  "edges": [[min(a, 3), min(b, 3), lab] for a, b, lab in d["edges"]]}
        assert O.validate(og, merged, "mono", K=0, threads=4)["match_count"] > 0
    gh = P.load(g)
    for sem in ("mono", "induced"):
        got, st = P.validate(gh, SPLIT_CASES, K=0, semantics=sem, flags=P.GFD_FLAG_COUNT_ONLY,
                             stats=True, batched=batched)
        for i, (d, r) in enumerate(zip(SPLIT_CASES, got)):
            assert r == _oracle_counts(og, d, sem), (sem, i)
        assert st["leaf_split_gfds"] == (SPLIT_COUNTED if sem == "mono" else 0), (sem, st)
        assert st["leaf_gfds"] == (len(SPLIT_CASES) if sem == "mono" else 0), (sem, st)
    full = P.validate(gh, SPLIT_CASES, K=0, semantics="mono", batched=batched)
    cnt = P.validate(gh, SPLIT_CASES, K=0, semantics="mono", flags=P.GFD_FLAG_COUNT_ONLY,
                     batched=batched)
    for a, b in zip(full, cnt):
        assert (a["match_count"], a["violation_count"]) == (b["match_count"], b["violation_count"])
    gh.free()


def test_count_only_random_shapes(P):
    """Count-only calls over seeded random connected GFDs (k = 3..7,
    wildcards, extra edges), batched, in both readings: every count equals the
    oracle's, whichever form (common-parent leaves, split leaves, enumeration)
    the planner picked for it."""
    g = random_graph(34, 300, 3000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=3,
                     absent_frac=0.1, reciprocal_frac=0.3)
    og = O.OracleGraph(g)
    gh = P.load(g)
    gfds = [random_gfd(3400 + j, 3 + j % 5, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=3,
                       wildcard_frac=0.2, extra_edge_frac=0.2)
            for j in range(60)]
    for sem in ("mono", "induced"):
        got, st = P.validate(gh, gfds, K=0, semantics=sem, flags=P.GFD_FLAG_COUNT_ONLY,
                             stats=True, batched=True)
        for i, (d, r) in enumerate(zip(gfds, got)):
            assert r == _oracle_counts(og, d, sem), (sem, i)
        if sem == "mono":
            assert st["leaf_gfds"] > 10 and st["leaf_split_gfds"] > 0, st
    gh.free()


def _oracle_first_k(og, d, sem, K):
    return dict(O.validate(og, d, sem, K=K, threads=4), match_fp=0, violation_fp=0)


@pytest.mark.parametrize("batched", [False, True])
def test_counted_leaf_with_first_k(P, batched):
    """Count-only calls that also list the first K violations: the last leaf
    is counted, then only the window of partial matches whose variable-0
    vertex is at most that of the K-th violation is enumerated.  Counts,
    flags and the listed violations equal the oracle's (fingerprints are 0)
    for K below, near and above the violation counts, in both readings."""
    g = random_graph(33, 250, 12000, n_vlabels=2, n_elabels=3, n_attrs=2, attr_values=3,
                     absent_frac=0.1, reciprocal_frac=0.4)
    og = O.OracleGraph(g)
    gh = P.load(g)
    gfds = [d for d, _ in CASES] + SPLIT_CASES
    viol = [O.validate(og, d, "mono", K=0, threads=4)["violation_count"] for d in gfds]
    assert sum(v > 2048 for v in viol) >= 3 and sum(0 < v < 2048 for v in viol) >= 3, viol
    for K in (1, 7, 100, 2048):
        for sem in ("mono", "induced"):
            got, st = P.validate(gh, gfds, K=K, semantics=sem, flags=P.GFD_FLAG_COUNT_ONLY,
                                 stats=True, batched=batched)
            for i, (d, r) in enumerate(zip(gfds, got)):
                assert r == _oracle_first_k(og, d, sem, K), (K, sem, i)
            if sem == "mono":  # the counted last leaf with its window
                assert st["leaf_gfds"] >= 6 and st["leaf_split_gfds"] == 0, (K, st)
    if batched:  # the same call again: captured, then replayed as a graph
        exp = [_oracle_first_k(og, d, "mono", 100) for d in gfds]
        replays = 0
        for _ in range(3):
            got, st = P.validate(gh, gfds, K=100, semantics="mono", flags=P.GFD_FLAG_COUNT_ONLY,
                                 stats=True, batched=True)
            assert got == exp
            replays += st["graph_replays"]
        assert replays > 0
    gh.free()


def test_counted_leaf_window_past_the_staging(P):
    """A window whose violations overflow the (small, testing) staging runs
    the threshold re-runs over the deferred last level: still exact."""
    g = random_graph(33, 250, 12000, n_vlabels=2, n_elabels=3, n_attrs=2, attr_values=3,
                     absent_frac=0.1, reciprocal_frac=0.4)
    og = O.OracleGraph(g)
    gh = P.load(g)
    gfds = [d for d, q in CASES if q] + SPLIT_CASES[:SPLIT_COUNTED]
    for K, cap in ((5, 6), (40, 41), (300, 512)):
        got, st = P.validate(gh, gfds, K=K, semantics="mono", flags=P.GFD_FLAG_COUNT_ONLY,
                             violation_cap=cap, stats=True, batched=True)
        for i, (d, r) in enumerate(zip(gfds, got)):
            assert r == _oracle_first_k(og, d, "mono", K), (K, i)
        assert st["threshold_passes"] > 0, st
    gh.free()


def test_counted_leaves_under_frontier_overflow(P):
    """A job whose inner frontier overflows is redone on the bounded path,
    which enumerates everything: counts stay exact."""
    g = random_graph(32, 400, 8000, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=3)
    og = O.OracleGraph(g)
    gh = P.load(g)
    gfds = [d for d, q in CASES if q] + SPLIT_CASES[:SPLIT_COUNTED]
    got = P.validate(gh, gfds, K=0, semantics="mono", flags=P.GFD_FLAG_COUNT_ONLY,
                     frontier_cap=50, batched=True)
    for d, r in zip(gfds, got):
        assert r == _oracle_counts(og, d, "mono")
    gh.free()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_twitch_star_counted(P):
    """The paper's star query on the Twitch-shaped graph: 394M matches counted
    from the leaves' candidate lists, equal to the stored oracle counts."""
    exp = json.load(open(os.path.join(GOLDEN, "expected_twitch_trio.json")))
    g = configs.graph(configs.CONFIG_GRAPH["twitch_trio"])
    assert g.sha256() == exp["graph_sha256"]
    gh = P.load(g)
    got, st = P.validate(gh, exp["gfds"], K=0, semantics="mono", flags=P.GFD_FLAG_COUNT_ONLY,
                         stats=True)
    for r, e in zip(got, exp["results"]["mono"]):
        assert (r["match_count"], r["violation_count"], r["satisfied"]) == \
            (e["match_count"], e["violation_count"], e["satisfied"])
    assert st["leaf_gfds"] >= 2  # both star forms
    gh.free()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_counted_leaf_windows_full_size_batch(P):
    """The 256-GFD workload under the non-induced reading, count-only with
    the first K listed: counts, flags and the first K violations of every GFD
    equal the stored oracle results."""
    import gzip
    with gzip.open(os.path.join(GOLDEN, "expected_kg_4m_batch256.json.gz"), "rt") as f:
        exp = json.load(f)
    g = configs.graph("kg_4m")
    assert g.sha256() == exp["graph_sha256"]
    gh = P.load(g)
    got, st = P.validate(gh, exp["gfds"], K=exp["K"], semantics="mono",
                         flags=P.GFD_FLAG_COUNT_ONLY, stats=True, batched=True)
    for i, (r, e) in enumerate(zip(got, exp["results"]["mono"])):
        assert r == dict(e, match_fp=0, violation_fp=0), i
    assert st["leaf_gfds"] > 50
    # under a 1 GiB budget: GFDs overflow the capped pool and arena and run
    # again; the next calls run in batches formed from what each asked
    for call in range(3):
        got, st = P.validate(gh, exp["gfds"], K=exp["K"], semantics="mono", mem_budget_bytes=1 << 30,
                             flags=P.GFD_FLAG_COUNT_ONLY, stats=True, batched=True)
        for i, (r, e) in enumerate(zip(got, exp["results"]["mono"])):
            assert r == dict(e, match_fp=0, violation_fp=0), (call, i)
    gh.free()


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_counted_leaves_full_size_batch(P):
    """The 256-GFD workload under the non-induced reading in one batched
    count-only call: over half the GFDs have their last leaves counted; all
    counts equal the stored oracle results."""
    import gzip
    with gzip.open(os.path.join(GOLDEN, "expected_kg_4m_batch256.json.gz"), "rt") as f:
        exp = json.load(f)
    g = configs.graph("kg_4m")
    assert g.sha256() == exp["graph_sha256"]
    gh = P.load(g)
    got, st = P.validate(gh, exp["gfds"], K=0, semantics="mono", flags=P.GFD_FLAG_COUNT_ONLY,
                         stats=True, batched=True)
    for i, (r, e) in enumerate(zip(got, exp["results"]["mono"])):
        assert (r["match_count"], r["violation_count"], r["satisfied"]) == \
            (e["match_count"], e["violation_count"], e["satisfied"]), i
    assert st["leaf_gfds"] > 100
    # and under a 256 MiB budget, the second call in batches formed from the first
    for call in range(2):
        got, st = P.validate(gh, exp["gfds"], K=0, semantics="mono", flags=P.GFD_FLAG_COUNT_ONLY,
                             mem_budget_bytes=256 << 20, stats=True, batched=True)
        for i, (r, e) in enumerate(zip(got, exp["results"]["mono"])):
            assert (r["match_count"], r["violation_count"], r["satisfied"]) == \
                (e["match_count"], e["violation_count"], e["satisfied"]), (call, i)
    gh.free()
