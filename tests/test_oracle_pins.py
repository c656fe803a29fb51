"""Pins for the CPU oracle, against things other than itself.

  * the paper's St. Petersburg example (Sections I-II), hand-derived values;
  * exhaustive brute force over V^k on tiny graphs (an independent transcription);
  * networkx's VF2 matchers (induced = subgraph isomorphism, non-induced =
    monomorphism) with label matchers;
  * closed forms: the two-out-neighbour pattern of the small uniform workload,
    trace of a label-restricted A^3 for directed triangles, the typing
    constraint of Section II, single-edge patterns;
  * identities and invariants: X -> false vs {} -> l, automorphism
    divisibility, induced within non-induced, monotonicity in X, relabelling.
"""
import itertools
import json
import os

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from oracle.brute import brute_validate, tuple_hash
from synth import configs, from_edge_list
from synth.small import random_graph, random_gfd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SEMS = ("induced", "mono")


def x1_graph(extra=()):
    d = json.load(open(os.path.join(GOLDEN, "x1_st_petersburg.json")))
    gr = d["graph"]
    g = from_edge_list(gr["n"], [tuple(e) for e in gr["edges"]] + [tuple(e) for e in extra],
                       gr["vlabel"], [gr["name"]])
    return d, g


@pytest.mark.parametrize("sem", SEMS)
def test_x1_st_petersburg(sem):
    d, g = x1_graph()
    r = O.validate(O.OracleGraph(g), d["gfd"], sem)
    exp = d["expected"][sem]
    for key in ("match_count", "violation_count", "satisfied", "violations"):
        assert r[key] == exp[key], key
    v = d["variant_contains_place"]
    _, g2 = x1_graph(v["extra_edges"])
    r2 = O.validate(O.OracleGraph(g2), d["gfd"], sem)
    for key in ("match_count", "violation_count", "satisfied", "violations"):
        assert r2[key] == v["expected"][sem][key], key


def _cases(count, seed0=0):
    out = []
    for s in range(count):
        rng = np.random.default_rng(10_000 + seed0 + s)
        n = int(rng.integers(3, 8))
        m = int(rng.integers(n, n * (n - 1) + 1))
        k = int(rng.integers(1, min(4, n) + 1))
        g = random_graph(seed0 + s, n, m, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=3)
        gfd = random_gfd(seed0 + s, k, n_vlabels=2, n_elabels=2, n_attrs=2, attr_values=3,
                         connected=bool(rng.random() < 0.85))
        out.append((g, gfd))
    return out


BRUTE_CASES = _cases(160)


@pytest.mark.parametrize("idx", range(len(BRUTE_CASES)))
def test_brute_force(idx):
    g, gfd = BRUTE_CASES[idx]
    og = O.OracleGraph(g)
    for sem in SEMS:
        for K in (0, 2, 1024):
            b = brute_validate(g, gfd, sem, K)
            r = O.validate(og, gfd, sem, K)
            assert r == b, (sem, K, gfd)


def _to_nx(g):
    G = nx.DiGraph()
    for v in range(g.n):
        G.add_node(v, label=int(g.vlabel[v]))
    for s in range(g.n):
        for e in range(g.row_ptr[s], g.row_ptr[s + 1]):
            G.add_edge(s, int(g.col[e]), label=int(g.elabel[e]))
    return G


def _pattern_nx(gfd):
    Q = nx.DiGraph()
    for i, l in enumerate(gfd["vlabels"]):
        Q.add_node(i, label=l)
    for a, b, l in gfd["edges"]:
        Q.add_edge(a, b, label=l)
    return Q


def _nx_matches(g, gfd, sem):
    GM = nx.algorithms.isomorphism.DiGraphMatcher(
        _to_nx(g), _pattern_nx(gfd),
        node_match=lambda d, q: q["label"] in (-1, d["label"]),
        edge_match=lambda d, q: q["label"] in (-1, d["label"]))
    it = GM.subgraph_isomorphisms_iter() if sem == "induced" else GM.subgraph_monomorphisms_iter()
    out = []
    for mp in it:
        inv = {q: d for d, q in mp.items()}
        out.append(tuple(inv[i] for i in range(gfd["k"])))
    return out


def _literal(g, t, l):
    a = int(g.attrs[l["attr"], t[l["var"]]])
    if l["kind"] == "const":
        return a != -1 and a == l["value"]
    b = int(g.attrs[l["attr2"], t[l["var2"]]])
    return a != -1 and b != -1 and a == b


@pytest.mark.parametrize("sem", SEMS)
def test_networkx_small_uniform(sem):
    g = configs.graph("small_uniform")
    gfd = configs.gfds("small_uniform", g)[0]
    ms = _nx_matches(g, gfd, sem)
    r = O.validate(O.OracleGraph(g), gfd, sem)
    assert r["match_count"] == len(ms)
    viol = sorted(list(t) for t in ms if not all(_literal(g, t, l) for l in gfd["y"]))
    assert r["violation_count"] == len(viol)
    assert r["violations"] == viol[:1024]
    mask = (1 << 64) - 1
    assert r["match_fp"] == sum(tuple_hash(t) for t in ms) & mask


@pytest.mark.parametrize("seed", range(12))
def test_networkx_random(seed):
    g = random_graph(500 + seed, 40, 200, n_vlabels=2, n_elabels=2, n_attrs=1, attr_values=3)
    gfd = random_gfd(500 + seed, 3 + seed % 2, n_vlabels=2, n_elabels=2, n_attrs=1,
                     attr_values=3, wildcard_frac=0.3)
    og = O.OracleGraph(g)
    for sem in SEMS:
        ms = _nx_matches(g, gfd, sem)
        r = O.validate(og, gfd, sem, K=10 ** 6)
        assert r["match_count"] == len(ms), sem
        X = lambda t: all(_literal(g, t, l) for l in gfd["x"])  # noqa: E731
        Y = lambda t: (not gfd["y_false"]) and all(_literal(g, t, l) for l in gfd["y"])  # noqa
        viol = sorted(list(t) for t in ms if X(t) and not Y(t))
        assert r["violations"] == viol, sem


def _two_out_forms(g):
    """Closed forms for x(L0) -e0-> y(L1), x -e0-> z(L1), {} -> y.name = z.name."""
    E = set()
    for s in range(g.n):
        for e in range(g.row_ptr[s], g.row_ptr[s + 1]):
            E.add((s, int(g.col[e])))
    mono_m = mono_v = ind_m = ind_v = 0
    for x in range(g.n):
        if g.vlabel[x] != 0:
            continue
        N = [int(g.col[e]) for e in range(g.row_ptr[x], g.row_ptr[x + 1])
             if g.elabel[e] == 0 and g.vlabel[g.col[e]] == 1]
        d = len(N)
        names = [int(g.attrs[0, y]) for y in N]
        c = {}
        for a in names:
            c[a] = c.get(a, 0) + 1
        mono_m += d * (d - 1)
        mono_v += d * d - sum(v * v for v in c.values())
        Np = [y for y in N if (y, x) not in E]
        for y, z in itertools.permutations(Np, 2):
            if (y, z) not in E and (z, y) not in E:
                ind_m += 1
                ind_v += g.attrs[0, y] != g.attrs[0, z]
    return mono_m, mono_v, ind_m, ind_v


@pytest.mark.parametrize("dense", [False, True])
def test_two_out_closed_forms(dense):
    if dense:
        from synth.graphs import make_graph
        g, _ = make_graph(7, 300, 9000, model="uniform", n_vlabels=2, n_elabels=2,
                          label_zipf=None, n_attrs=1, attr_values=4, attr_zipf=None)
    else:
        g = configs.graph("small_uniform")
    gfd = configs.gfds("small_uniform", configs.graph("small_uniform"))[0]
    mono_m, mono_v, ind_m, ind_v = _two_out_forms(g)
    og = O.OracleGraph(g)
    r = O.validate(og, gfd, "mono", K=0)
    assert (r["match_count"], r["violation_count"]) == (mono_m, mono_v)
    r = O.validate(og, gfd, "induced", K=0)
    assert (r["match_count"], r["violation_count"]) == (ind_m, ind_v)
    if dense:
        assert ind_m < mono_m  # the dense case separates the two readings


def test_directed_triangle_trace():
    from synth.graphs import make_graph
    g, _ = make_graph(11, 200, 3000, model="uniform", n_vlabels=2, n_elabels=2,
                      label_zipf=None, n_attrs=1, attr_values=4, attr_zipf=None)
    src = g.src()
    og = O.OracleGraph(g)
    for labs in [(0, 0, 0), (0, 1, 1), (1, 0, 1)]:
        for elabs in [(0, 0, 0), (1, 0, 1)]:
            D = [sp.diags((g.vlabel == L).astype(float)) for L in labs]
            A = [sp.csr_matrix(((g.elabel == l).astype(float), (src, g.col)), shape=(g.n, g.n))
                 for l in elabs]
            T = (D[0] @ A[0] @ D[1] @ A[1] @ D[2] @ A[2]).diagonal().sum()
            gfd = {"k": 3, "vlabels": list(labs),
                   "edges": [[0, 1, elabs[0]], [1, 2, elabs[1]], [2, 0, elabs[2]]],
                   "x": [], "y": [], "y_false": False}
            r = O.validate(og, gfd, "mono", K=0)
            assert r["match_count"] == int(round(T)) and T > 0


def test_typing_constraint():
    g = random_graph(3, 60, 200, n_vlabels=3, n_attrs=2, attr_values=4, absent_frac=0.3)
    og = O.OracleGraph(g)
    for L in range(3):
        for A in range(2):
            gfd = {"k": 1, "vlabels": [L], "edges": [], "x": [],
                   "y": [{"kind": "var", "var": 0, "attr": A, "var2": 0, "attr2": A}],
                   "y_false": False}
            for sem in SEMS:
                r = O.validate(og, gfd, sem, K=0)
                assert r["match_count"] == int((g.vlabel == L).sum())
                assert r["violation_count"] == int(((g.vlabel == L) & (g.attrs[A] == -1)).sum())


def test_single_edge():
    g = random_graph(4, 50, 400, n_vlabels=2, n_elabels=3, reciprocal_frac=0.5)
    og = O.OracleGraph(g)
    src = g.src()
    E = set(zip(src.tolist(), g.col.tolist()))
    for a, b, l in [(0, 1, 2), (1, 1, 0), (0, 0, -1), (-1, 1, 1)]:
        gfd = {"k": 2, "vlabels": [a, b], "edges": [[0, 1, l]], "x": [], "y": [],
               "y_false": False}
        ok = ((a == -1) | (g.vlabel[src] == a)) & ((b == -1) | (g.vlabel[g.col] == b)) & \
             ((l == -1) | (g.elabel == l))
        recip = np.array([(int(d), int(s)) in E for s, d in zip(src, g.col)])
        assert O.validate(og, gfd, "mono", K=0)["match_count"] == int(ok.sum())
        assert O.validate(og, gfd, "induced", K=0)["match_count"] == int((ok & ~recip).sum())


def test_x_false_identity():
    """viol({} -> l) + viol(l -> false) = matches, for every literal l."""
    for s in range(20):
        g = random_graph(40 + s, 30, 150, n_attrs=2, attr_values=3)
        gfd = random_gfd(40 + s, 3, n_attrs=2, attr_values=3)
        og = O.OracleGraph(g)
        rng = np.random.default_rng(s)
        from synth.small import random_literal
        l = random_literal(rng, 3, 2, 3)
        a = dict(gfd, x=[], y=[l], y_false=False)
        b = dict(gfd, x=[l], y=[], y_false=True)
        for sem in SEMS:
            ra, rb = O.validate(og, a, sem, K=0), O.validate(og, b, sem, K=0)
            assert ra["violation_count"] + rb["violation_count"] == ra["match_count"]
            assert (ra["violation_fp"] + rb["violation_fp"]) % (1 << 64) == ra["match_fp"]


def _automorphisms(gfd):
    k = gfd["k"]
    QE = {(a, b): l for a, b, l in gfd["edges"]}
    cnt = 0
    for p in itertools.permutations(range(k)):
        if any(gfd["vlabels"][i] != gfd["vlabels"][p[i]] for i in range(k)):
            continue
        if all(QE.get((p[a], p[b]), "none") == QE.get((a, b), "none")
               for a in range(k) for b in range(k) if a != b):
            cnt += 1
    return cnt


def test_automorphism_divisibility():
    g = random_graph(77, 40, 500, n_vlabels=2, n_elabels=1)
    og = O.OracleGraph(g)
    pats = [
        {"k": 4, "vlabels": [0, 1, 1, 1], "edges": [[0, 1, 0], [0, 2, 0], [0, 3, 0]]},
        {"k": 3, "vlabels": [0, 0, 0], "edges": [[0, 1, 0], [1, 2, 0], [2, 0, 0]]},
        {"k": 4, "vlabels": [1, 1, 1, 1], "edges": [[0, 1, 0], [1, 2, 0], [2, 3, 0], [3, 0, 0]]},
        {"k": 3, "vlabels": [-1, -1, -1], "edges": [[0, 1, 0], [0, 2, 0]]},
    ]
    for p in pats:
        p.update(x=[], y=[], y_false=False)
        aut = _automorphisms(p)
        assert aut >= 2
        for sem in SEMS:
            r = O.validate(og, p, sem, K=0)
            assert r["match_count"] % aut == 0
            assert r["match_count"] > 0 or sem == "induced"


def test_induced_within_mono_and_monotone_x():
    for s in range(25):
        g = random_graph(200 + s, 12, 50, n_attrs=2, attr_values=2)
        gfd = random_gfd(200 + s, 3, n_attrs=2, attr_values=2)
        og = O.OracleGraph(g)
        big = 10 ** 6
        ri, rm = O.validate(og, gfd, "induced", big), O.validate(og, gfd, "mono", big)
        assert ri["match_count"] <= rm["match_count"]
        assert set(map(tuple, ri["violations"])) <= set(map(tuple, rm["violations"]))
        for r in (ri, rm):
            assert r["violation_count"] <= r["match_count"]
        from synth.small import random_literal
        more = dict(gfd, x=gfd["x"] + [random_literal(np.random.default_rng(s), 3, 2, 2)])
        for sem in SEMS:
            assert O.validate(og, more, sem, 0)["violation_count"] <= \
                O.validate(og, gfd, sem, 0)["violation_count"]


def test_relabelling_invariance():
    g = random_graph(9, 25, 120, n_attrs=2, attr_values=3)
    rng = np.random.default_rng(9)
    pi = rng.permutation(g.n)
    src = g.src()
    edges = [(int(pi[s]), int(pi[d]), int(l)) for s, d, l in zip(src, g.col, g.elabel)]
    inv = np.argsort(pi)
    g2 = from_edge_list(g.n, edges, g.vlabel[inv], g.attrs[:, inv])
    og, og2 = O.OracleGraph(g), O.OracleGraph(g2)
    for s in range(10):
        gfd = random_gfd(900 + s, 3, n_attrs=2, attr_values=3)
        for sem in SEMS:
            a, b = O.validate(og, gfd, sem, 10 ** 6), O.validate(og2, gfd, sem, 10 ** 6)
            assert a["match_count"] == b["match_count"]
            assert a["violation_count"] == b["violation_count"]
            mapped = sorted([int(pi[v]) for v in t] for t in a["violations"])
            assert mapped == b["violations"]
            assert sum(tuple_hash(t) for t in mapped) % (1 << 64) == b["violation_fp"]


def test_root_partition_and_threads():
    g = configs.graph("small_uniform")
    gfd = configs.gfds("small_uniform", g)[0]
    og = O.OracleGraph(g)
    for sem in SEMS:
        full = O.validate(og, gfd, sem, K=5)
        thr = O.validate(og, gfd, sem, K=5, threads=4)
        assert thr == full
        parts = [O.validate(og, gfd, sem, K=5, root_range=(a, b))
                 for a, b in [(0, 700), (700, 1500), (1500, g.n)]]
        assert sum(p["match_count"] for p in parts) == full["match_count"]
        assert sum(p["violation_fp"] for p in parts) % (1 << 64) == full["violation_fp"]
        assert sorted(v for p in parts for v in p["violations"])[:5] == full["violations"]
